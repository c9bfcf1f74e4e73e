"""Pins of the oracle's staggered-mass Hasenbusch split (Sec. 5.1) that do not reuse its code (no GPU).

* determinant identity: the kernels K_i of the n+1 terms, read back from the oracle's
  actions by polarisation, satisfy sum_i log det K_i = -log det(M M^dag), the
  Gaussian-integral statement that the split leaves det(M M^dag) unchanged;
* heat-bath: every term evaluated at the heat-bath pseudofermion equals rho_i^dag rho_i
  (the exact Gaussian draw);
* equal masses mu_i = mu_{i-1}: xi_i = chi_i, the ratio force vanishes and the
  ratio action is chi_i^dag chi_i (the reduction the paper notes after eq. (def_xi_i));
* the summed force against central differences of the summed action at fixed chi;
* one mass equal to the base operator's reduces the last term to the plain
  pseudofermion action of eq. (hamiltonian) solved by LU.
"""
import numpy as np
import pytest

import oracle
from oracle import hasenbusch as hb
from oracle.operator import Lattice, build_M
from workloads import HASENBUSCH, draw_hasenbusch


def _rng(seed):
    return np.random.default_rng(seed)


def _cplx(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * np.sqrt(0.5)


def _kernel_from_actions(lat, phi, mts, i):
    """Hermitian K with S_i(chi) = chi^dag K chi, recovered by polarisation of the oracle's action."""
    n = lat.n

    def S(v):
        return hb.term(lat, phi, mts, v.reshape(lat.shape), i)[0]

    e = np.eye(n, dtype=np.complex128)
    diag = np.array([S(e[k]) for k in range(n)])
    K = np.diag(diag).astype(np.complex128)
    for k in range(n):
        for l in range(k + 1, n):
            re = (S(e[k] + e[l]) - diag[k] - diag[l]) / 2
            im = -(S(e[k] + 1j * e[l]) - diag[k] - diag[l]) / 2
            K[k, l] = re + 1j * im
            K[l, k] = re - 1j * im
    return K


def test_determinant_identity_of_the_split():
    lat = Lattice(2, 2, 2, 0.4)
    rng = _rng(1)
    phi = rng.normal(0, 0.8, lat.shape)
    mts = [0.15, 0.6]
    logdet = 0.0
    for i in range(len(mts) + 1):
        K = _kernel_from_actions(lat, phi, mts, i)
        assert np.allclose(K, K.conj().T, atol=1e-12)
        sign, ld = np.linalg.slogdet(K)
        assert abs(sign - 1) < 1e-10  # Hermitian positive definite
        logdet += ld
    Md = build_M(lat, phi).toarray()
    _, ld_full = np.linalg.slogdet(Md @ Md.conj().T)
    assert abs(logdet + ld_full) < 1e-9 * max(1.0, abs(ld_full))


def test_determinant_identity_fails_for_swapped_masses():
    # the identity is not automatic: swapping the roles of numerator and denominator breaks it
    lat = Lattice(2, 2, 2, 0.4)
    rng = _rng(2)
    phi = rng.normal(0, 0.8, lat.shape)
    mts = [0.15, 0.6]
    ld = [np.linalg.slogdet(_kernel_from_actions(lat, phi, mts, i))[1] for i in range(3)]
    Md = build_M(lat, phi).toarray()
    ld_full = np.linalg.slogdet(Md @ Md.conj().T)[1]
    assert abs(sum(ld) + ld_full) < 1e-9 * abs(ld_full)
    assert abs(-ld[0] - ld[1] + ld[2] + ld_full) > 1e-3


@pytest.mark.parametrize("name", ["hb_tiny"])
def test_heatbath_gives_rho_norm(name):
    hw = HASENBUSCH[name]
    w = hw.base
    lat = Lattice(w.L1, w.L2, w.Nt, w.kappa_t, w.ms_t)
    phi, rho = draw_hasenbusch(hw)
    chi = hb.heatbath(lat, phi, hw.mts, rho)
    S, _ = hb.actions_and_forces(lat, phi, hw.mts, chi)
    for i in range(hw.nterms):
        r2 = np.vdot(rho[i].ravel(), rho[i].ravel()).real
        assert abs(S[i] - r2) < 1e-10 * r2, (i, S[i], r2)


def test_heatbath_solves_the_defining_equation():
    lat = Lattice(3, 3, 6, 0.3)
    rng = _rng(3)
    phi = rng.normal(0, 0.7, lat.shape)
    mts = [0.1, 0.35, 0.9]
    rho = _cplx(rng, (4,) + lat.shape)
    chi = hb.heatbath(lat, phi, mts, rho)
    masses = [0.0] + mts
    # M_{mu_i} chi_i = M_{mu_{i-1}} rho_i (matrices built directly from eq. (ferm_op))
    for i in range(3):
        Mi = build_M(Lattice(3, 3, 6, 0.3, masses[i + 1]), phi)
        Mp = build_M(Lattice(3, 3, 6, 0.3, masses[i]), phi)
        lhs = Mi @ chi[i].ravel()
        rhs = Mp @ rho[i].ravel()
        assert np.linalg.norm(lhs - rhs) < 1e-12 * np.linalg.norm(rhs)
    Mn = build_M(Lattice(3, 3, 6, 0.3, mts[-1]), phi)
    assert np.allclose(chi[3].ravel(), Mn @ rho[3].ravel(), atol=1e-14)


def test_equal_masses_give_zero_ratio_force():
    lat = Lattice(3, 3, 8, 0.5)
    rng = _rng(4)
    phi = rng.normal(0, 0.9, lat.shape)
    mts = [0.2, 0.2]
    chi = _cplx(rng, lat.shape)
    S, F, eta, xi = hb.term(lat, phi, mts, chi, 1)
    assert np.linalg.norm(xi - chi) < 1e-12 * np.linalg.norm(chi)
    assert np.abs(F).max() < 1e-12
    assert abs(S - np.vdot(chi.ravel(), chi.ravel()).real) < 1e-12 * S
    # and a distinct pair of masses gives a force of order one
    S2, F2, _, _ = hb.term(lat, phi, [0.05, 0.5], chi, 1)
    assert np.abs(F2).max() > 1e-2


@pytest.mark.parametrize("i", [0, 1, 2])
def test_force_against_central_differences(i):
    lat = Lattice(3, 3, 4, 0.45)
    rng = _rng(10 + i)
    phi = rng.normal(0, 0.8, lat.shape)
    mts = [0.12, 0.5]
    chi = _cplx(rng, lat.shape)
    _, F, _, _ = hb.term(lat, phi, mts, chi, i)
    h = 1e-5
    flat = phi.ravel()
    for k in rng.choice(lat.n, 10, replace=False):
        pp = flat.copy(); pp[k] += h
        pm = flat.copy(); pm[k] -= h
        Sp = hb.term(lat, pp.reshape(lat.shape), mts, chi, i)[0]
        Sm = hb.term(lat, pm.reshape(lat.shape), mts, chi, i)[0]
        fd = (Sp - Sm) / (2 * h)
        assert abs(fd - F.ravel()[k]) < 1e-7 * max(1.0, abs(fd)), (i, k, fd, F.ravel()[k])


def test_last_term_is_the_plain_action_when_its_mass_is_the_base():
    lat = Lattice(3, 3, 8, 0.5)
    rng = _rng(5)
    phi = rng.normal(0, 0.9, lat.shape)
    chi = _cplx(rng, lat.shape)
    S, F, eta, _ = hb.term(lat, phi, [0.0], chi, 1)
    Md = build_M(lat, phi).toarray()
    eta_lu = np.linalg.solve(Md @ Md.conj().T, chi.ravel())
    assert abs(S - np.vdot(chi.ravel(), eta_lu).real) < 1e-10 * abs(S)
    assert np.allclose(F, oracle.force(lat, phi, eta_lu.reshape(lat.shape)), atol=1e-10)
