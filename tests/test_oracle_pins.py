"""Pins of the CPU oracle against facts that do not reuse its code (no GPU).

Each test fixes a part of the oracle by a closed form, an invariance, a special case
that reduces to a library routine, brute force, or a number the paper prints:

* eq. (ferm_op) entries: loop builder vs vectorised builder, and hand-written
  entries at the antiperiodic wrap;
* free field (phi = 0): plane waves are eigenvectors of M with a 2x2 symbol whose
  normal form gives the spectrum {4 sin^2(w/2)(1-m~)... } in closed form;
* gauge covariance M[phi'] = D M[phi] D^dagger for time-dependent phases;
* Sec. 3: M M^dagger Hermitian positive definite (and != M^dagger M);
* solve: CG vs LU vs eigendecomposition; chi = M rho gives M^dagger x = rho;
* CG iterates: the k-th iterate is the Galerkin solution on the Krylov space
  K_k(A, b), and the complex64 inner CG follows the FP64 one to single precision;
* eqs. (p_dot), (eta_xi): force vs cancellation-free central differences;
* Algorithm A.1 method oracle reaches the requested true residual, and without
  inner solves one cycle of it is GMRES(m): the minimal residual over K_m(A, b);
* Sec. 6.1: the non-interacting largest eigenvalue sits inside the paper's fit.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle.operator import Lattice, NormalOperator, build_M, build_M_dense_loops
from workloads import WORKLOADS, draw_inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def lat_of(w):
    return Lattice(w.L1, w.L2, w.Nt, w.kappa_t, w.ms_t)


def rand_phi(rng, lat, scale=1.0):
    return rng.normal(0.0, scale, size=lat.shape)


def rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


SMALL_LATS = [
    Lattice(3, 3, 8, 0.5, 0.0),
    Lattice(2, 2, 4, 0.3, 0.0),
    Lattice(2, 3, 5, 0.7, 0.2),    # L1 != L2, odd N_t, staggered mass
    Lattice(1, 1, 3, 0.4, 0.1),    # L = 1: the three bonds coincide, entries add
    Lattice(2, 2, 1, 0.25, 0.0),   # N_t = 1: both temporal hops wrap onto the same slice
    Lattice(4, 1, 2, 0.6, 0.0),
]


@pytest.mark.parametrize("lat", SMALL_LATS, ids=lambda l: f"{l.L1}x{l.L2}x{l.Nt}")
def test_vectorised_builder_equals_loop_builder(lat):
    rng = np.random.default_rng(11)
    phi = rand_phi(rng, lat)
    np.testing.assert_allclose(build_M(lat, phi).toarray(), build_M_dense_loops(lat, phi), rtol=0, atol=1e-15)


def test_entries_by_hand_at_the_wrap():
    """Individual entries of eq. (ferm_op) written out for a 2x2x3 lattice."""
    lat = Lattice(2, 2, 3, 0.3, 0.1)
    rng = np.random.default_rng(1)
    phi = rand_phi(rng, lat)
    M = build_M(lat, phi).toarray()
    idx = lambda t, s, i, j: ((t * 2 + s) * 2 + i) * 2 + j
    # A at t = 0 hops to t = N_t - 1 with the antiperiodic sign.
    assert np.isclose(M[idx(0, 0, 1, 0), idx(2, 0, 1, 0)], -(np.exp(1j * phi[0, 0, 1, 0]) - 0.1))
    # A at t = 2 hops to t = 1 with the plain sign.
    assert np.isclose(M[idx(2, 0, 0, 1), idx(1, 0, 0, 1)], np.exp(1j * phi[2, 0, 0, 1]) - 0.1)
    # B at t = N_t - 1 hops to t = 0 with the antiperiodic sign.
    assert np.isclose(M[idx(2, 1, 1, 1), idx(0, 1, 1, 1)], +(np.exp(-1j * phi[2, 1, 1, 1]) - 0.1))
    assert np.isclose(M[idx(0, 1, 1, 1), idx(1, 1, 1, 1)], -(np.exp(-1j * phi[0, 1, 1, 1]) - 0.1))
    # diagonals
    assert M[idx(1, 0, 0, 0), idx(1, 0, 0, 0)] == -1.0
    assert M[idx(1, 1, 0, 0), idx(1, 1, 0, 0)] == 1.0
    # A(1,1) bonds to B(1,1), B(0,1), B(1,0) only; with L = 2 these are distinct.
    nbrs = sorted(k for k in range(lat.n) if M[idx(1, 0, 1, 1), k] == -0.3)
    assert nbrs == sorted([idx(1, 1, 1, 1), idx(1, 1, 0, 1), idx(1, 1, 1, 0)])
    # hopping is symmetric and does not connect slices
    H = M.copy()
    np.fill_diagonal(H, 0)
    for (r, c) in zip(*np.nonzero(np.isclose(H, -0.3))):
        assert np.isclose(M[c, r], -0.3)
        assert r // 8 == c // 8  # same slice


def _plane_wave(lat, n1, n2, n, uA, uB):
    th1 = 2 * math.pi * n1 / lat.L1
    th2 = 2 * math.pi * n2 / lat.L2
    om = math.pi * (2 * n + 1) / lat.Nt
    t, i, j = np.meshgrid(np.arange(lat.Nt), np.arange(lat.L1), np.arange(lat.L2), indexing="ij")
    ph = np.exp(1j * (th1 * i + th2 * j + om * t))
    psi = np.zeros(lat.shape, dtype=np.complex128)
    psi[:, 0] = uA * ph
    psi[:, 1] = uB * ph
    return psi, ph, th1, th2, om


@pytest.mark.parametrize("lat", [Lattice(3, 3, 8, 0.5, 0.0), Lattice(4, 3, 6, 0.35, 0.15), Lattice(12, 12, 32, 0.25, 0.0)],
                         ids=["C1", "4x3x6-ms", "C2"])
def test_free_field_plane_wave_symbol(lat):
    """phi = 0: M acts on u e^{i(th1 i + th2 j + w t)} as [[a, -k f], [-k conj f, -conj a]],
    a = (1 - m~) e^{-iw} - 1, f = 1 + e^{-i th1} + e^{-i th2}, w = pi (2n+1)/N_t."""
    phi = np.zeros(lat.shape)
    M = build_M(lat, phi)
    rng = np.random.default_rng(5)
    for trial in range(6):
        n1, n2, n = rng.integers(lat.L1), rng.integers(lat.L2), rng.integers(lat.Nt)
        uA, uB = rand_c(rng, ()), rand_c(rng, ())
        psi, ph, th1, th2, om = _plane_wave(lat, n1, n2, n, uA, uB)
        a = (1 - lat.ms_t) * np.exp(-1j * om) - 1
        f = 1 + np.exp(-1j * th1) + np.exp(-1j * th2)
        k = lat.kappa_t
        want = np.zeros_like(psi)
        want[:, 0] = (a * uA - k * f * uB) * ph
        want[:, 1] = (-k * np.conj(f) * uA - np.conj(a) * uB) * ph
        got = (M @ psi.ravel()).reshape(lat.shape)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)
        # and M^dagger by the conjugate-transposed symbol
        wantd = np.zeros_like(psi)
        wantd[:, 0] = (np.conj(a) * uA - k * f * uB) * ph
        wantd[:, 1] = (-k * np.conj(f) * uA - a * uB) * ph
        gotd = oracle.apply_Mdag(lat, phi, psi)
        np.testing.assert_allclose(gotd, wantd, rtol=0, atol=1e-13)


def free_spectrum(lat, mu2=0.0):
    """Closed-form spectrum of M M^dagger + mu^2 at phi = 0: |a|^2 + k^2 |f|^2 + mu^2, twice."""
    ev = []
    for n1 in range(lat.L1):
        for n2 in range(lat.L2):
            f = 1 + np.exp(-2j * math.pi * n1 / lat.L1) + np.exp(-2j * math.pi * n2 / lat.L2)
            for n in range(lat.Nt):
                a = (1 - lat.ms_t) * np.exp(-1j * math.pi * (2 * n + 1) / lat.Nt) - 1
                lam = abs(a) ** 2 + lat.kappa_t ** 2 * abs(f) ** 2 + mu2
                ev += [lam, lam]
    return np.sort(np.array(ev))


@pytest.mark.parametrize("lat,mu2", [(Lattice(3, 3, 8, 0.5), 0.0), (Lattice(2, 3, 5, 0.7, 0.2), 0.3)])
def test_free_field_spectrum_by_exact_diagonalisation(lat, mu2):
    A = NormalOperator(lat, np.zeros(lat.shape), mu2).dense()
    ev = np.linalg.eigvalsh(A)
    np.testing.assert_allclose(ev, free_spectrum(lat, mu2), rtol=0, atol=1e-12)


def test_free_field_extremes_of_the_workloads():
    """lambda_min = 4 sin^2(pi/(2 N_t)) when L is divisible by 3 (Dirac point f = 0)."""
    for w in WORKLOADS.values():
        lat = lat_of(w)
        ev = free_spectrum(Lattice(w.L1 if w.L1 <= 12 else 12, w.L2 if w.L2 <= 12 else 12, w.Nt, w.kappa_t))
        assert math.isclose(ev[0], 4 * math.sin(math.pi / (2 * w.Nt)) ** 2, rel_tol=1e-12)


def test_gauge_covariance():
    """phi'_{A,t} = phi_{A,t} + al_t - al_{t-1}, phi'_{B,t} = phi_{B,t} + al_{t+1} - al_t
    gives M[phi'] = D M[phi] D^dagger with D = diag(e^{i al_t}) (al periodic in t).
    Holds at m~ = 0 only: the staggered mass is not carried by the phase."""
    lat = Lattice(3, 2, 6, 0.45, 0.0)
    rng = np.random.default_rng(3)
    phi = rand_phi(rng, lat)
    al = rng.normal(size=lat.Nt)
    phi2 = phi.copy()
    for t in range(lat.Nt):
        phi2[t, 0] += al[t] - al[(t - 1) % lat.Nt]
        phi2[t, 1] += al[(t + 1) % lat.Nt] - al[t]
    d = np.exp(1j * np.repeat(al, 2 * lat.L1 * lat.L2))
    M1 = build_M(lat, phi).toarray()
    M2 = build_M(lat, phi2).toarray()
    np.testing.assert_allclose(M2, d[:, None] * M1 * np.conj(d)[None, :], atol=1e-14)


def test_pure_gauge_field_has_the_free_spectrum():
    lat = Lattice(3, 3, 8, 0.5)
    rng = np.random.default_rng(4)
    al = rng.normal(size=lat.Nt) * 2
    phi = np.zeros(lat.shape)
    for t in range(lat.Nt):
        phi[t, 0] = al[t] - al[(t - 1) % lat.Nt]
        phi[t, 1] = al[(t + 1) % lat.Nt] - al[t]
    ev = np.linalg.eigvalsh(NormalOperator(lat, phi, 0.0).dense())
    np.testing.assert_allclose(ev, free_spectrum(lat), atol=1e-12)


def test_normal_operator_hermitian_positive_and_not_MdagM():
    lat = Lattice(3, 3, 8, 0.5)
    rng = np.random.default_rng(6)
    phi = rand_phi(rng, lat)
    for mu2 in (0.0, 0.05, 0.5):
        A = NormalOperator(lat, phi, mu2).dense()
        np.testing.assert_allclose(A, A.conj().T, atol=1e-14)
        assert np.linalg.eigvalsh(A).min() >= mu2 - 1e-12
        assert np.linalg.eigvalsh(A).min() > 0
    Md = build_M(lat, phi).toarray()
    assert np.abs(Md @ Md.conj().T - Md.conj().T @ Md).max() > 1e-2


def test_twelve_nonzeros_per_row_of_the_normal_operator():
    """M M^dagger couples each site to itself, t+-1, six second neighbours and three
    opposite-sublattice neighbours in one adjacent slice (same-slice A-B terms cancel)."""
    lat = Lattice(4, 4, 6, 0.3)
    rng = np.random.default_rng(8)
    A = NormalOperator(lat, rand_phi(rng, lat), 0.0).dense()
    nnz = (np.abs(A) > 1e-14).sum(axis=1)
    assert (nnz == 12).all()


def test_cg_lu_and_eigendecomposition_agree():
    w = WORKLOADS["tiny"]
    lat = lat_of(w)
    phi, eta = draw_inputs(w)
    chi = oracle.apply_Mdag(lat, phi, eta[0])
    for mu2 in (0.0, 0.05):
        A = NormalOperator(lat, phi, mu2)
        Ad = A.dense()
        x_lu = np.linalg.solve(Ad, chi.ravel())
        lam, U = np.linalg.eigh(Ad)
        x_ed = U @ ((U.conj().T @ chi.ravel()) / lam)
        x_cg, its, res = oracle.cg(A, chi.ravel(), tol=1e-13)
        assert res <= 1e-13
        np.testing.assert_allclose(x_cg, x_lu, rtol=0, atol=1e-10 * np.abs(x_lu).max())
        np.testing.assert_allclose(x_ed, x_lu, rtol=0, atol=1e-10 * np.abs(x_lu).max())


def test_heatbath_source_gives_xi_equal_rho():
    """chi = M rho (Sec. 2) at mu^2 = 0: eta = (M M^dagger)^{-1} M rho, so xi = M^dagger eta = rho
    and S = chi^dagger eta = |rho|^2 (eq. (eta_xi))."""
    w = WORKLOADS["small16"]
    lat = lat_of(w)
    phi, rho = draw_inputs(w, batch=1)
    chi = oracle.apply_M(lat, phi, rho[0])
    x, res = oracle.solve(lat, phi, 0.0, chi, tol=1e-13)
    assert res <= 1e-13
    xi = oracle.xi_from_eta(lat, phi, x)
    assert np.linalg.norm((xi - rho[0]).ravel()) <= 1e-9 * np.linalg.norm(rho[0].ravel())
    S = oracle.action(chi, x)
    assert math.isclose(S, np.vdot(rho[0], rho[0]).real, rel_tol=1e-11)


def _krylov_basis(Ad, b, k):
    """Orthonormal basis of span{b, A b, ..., A^{k-1} b} from the normalised power
    sequence and a QR factorisation (no Arnoldi recurrence)."""
    K = [b / np.linalg.norm(b)]
    for _ in range(k - 1):
        v = Ad @ K[-1]
        K.append(v / np.linalg.norm(v))
    return np.linalg.qr(np.stack(K, axis=1))[0]


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_cg_iterate_is_the_krylov_galerkin_solution(k):
    """From x0 = 0 the k-th CG iterate minimises the A-norm of the error over
    K_k(A, b): x_k = V (V^H A V)^{-1} V^H b for an orthonormal basis V of K_k."""
    lat = Lattice(3, 3, 8, 0.5)
    rng = np.random.default_rng(7)
    A = NormalOperator(lat, rand_phi(rng, lat), 0.05)
    Ad = A.dense()
    b = rand_c(rng, lat.n)
    V = _krylov_basis(Ad, b, k)
    want = V @ np.linalg.solve(V.conj().T @ Ad @ V, V.conj().T @ b)
    x, its, _ = oracle.cg(A, b, tol=0.0, maxiter=k)
    assert its == k
    assert np.linalg.norm(x - want) <= 1e-10 * np.linalg.norm(want)


def test_complex64_inner_cg_follows_the_fp64_cg():
    """The inner CG of Algorithm A.1 is the same recurrence in complex64: its first
    iterates agree with the FP64 CG's to single precision."""
    from oracle.solve import _spcg_c64
    lat = Lattice(3, 3, 8, 0.5)
    rng = np.random.default_rng(17)
    A = NormalOperator(lat, rand_phi(rng, lat), 0.05)
    A32 = lambda v: (A.M.astype(np.complex64) @ (A.Mh.astype(np.complex64) @ v)
                     + np.float32(0.05) * v)
    b = rand_c(rng, lat.n)
    for k in (1, 2, 4, 6):
        z, its = _spcg_c64(A32, 0.05, b, 0.0, k)
        x, _, _ = oracle.cg(A, b, tol=0.0, maxiter=k)
        assert its == k and z.dtype == np.complex64
        assert np.linalg.norm(z - x) <= 1e-5 * np.linalg.norm(x)


def _fd_force(lat, phi, mu2, chi, k, h):
    """Central difference of S in phi_k, cancellation free:
    S(+) - S(-) = x+^dagger (A- - A+) x-, x+- = A+-^{-1} chi."""
    php = phi.copy().ravel(); php[k] += h
    phm = phi.copy().ravel(); phm[k] -= h
    Ap = NormalOperator(lat, php.reshape(lat.shape), mu2)
    Am = NormalOperator(lat, phm.reshape(lat.shape), mu2)
    xp, _ = oracle.solve(lat, php, mu2, chi.ravel(), tol=1e-14, A=Ap)
    xm, _ = oracle.solve(lat, phm, mu2, chi.ravel(), tol=1e-14, A=Am)
    dS = np.vdot(xp, Am(xm) - Ap(xm)).real
    return dS / (2 * h)


@pytest.mark.parametrize("wname,mu2,nsite", [("tiny", 0.0, 40), ("tiny", 0.3, 12), ("small16", 0.05, 6)])
def test_force_against_central_differences(wname, mu2, nsite):
    w = WORKLOADS[wname]
    lat = Lattice(w.L1, w.L2, w.Nt, w.kappa_t, 0.1 if wname == "tiny" else 0.0)
    phi, eta = draw_inputs(w, batch=1)
    chi = oracle.apply_Mdag(lat, phi, eta[0])
    x, _ = oracle.solve(lat, phi, mu2, chi, tol=1e-14)
    F = oracle.force(lat, phi, x).ravel()
    rng = np.random.default_rng(9)
    for k in rng.choice(lat.n, size=nsite, replace=False):
        fd = _fd_force(lat, phi, mu2, chi, int(k), 1e-4)
        assert abs(fd - F[k]) <= 1e-6 * max(1.0, np.abs(F).max()), (k, fd, F[k])


def test_force_gauge_invariant():
    lat = Lattice(3, 3, 8, 0.5)
    rng = np.random.default_rng(12)
    phi = rand_phi(rng, lat)
    chi = rand_c(rng, lat.shape)
    al = rng.normal(size=lat.Nt)
    phi2 = phi.copy()
    for t in range(lat.Nt):
        phi2[t, 0] += al[t] - al[(t - 1) % lat.Nt]
        phi2[t, 1] += al[(t + 1) % lat.Nt] - al[t]
    chi2 = chi * np.exp(1j * al)[:, None, None, None]
    x1, _ = oracle.solve(lat, phi, 0.1, chi)
    x2, _ = oracle.solve(lat, phi2, 0.1, chi2)
    np.testing.assert_allclose(oracle.force(lat, phi2, x2), oracle.force(lat, phi, x1), atol=1e-10)
    assert math.isclose(oracle.action(chi2, x2), oracle.action(chi, x1), rel_tol=1e-12)


def test_force_mass_independent_of_shift_formula():
    """The shift mu^2 changes eta only: F(mu2) equals the contraction with eta(mu2)."""
    lat = Lattice(3, 3, 8, 0.5)
    rng = np.random.default_rng(13)
    phi = rand_phi(rng, lat)
    chi = rand_c(rng, lat.shape)
    for mu2 in (0.0, 0.5):
        x, _ = oracle.solve(lat, phi, mu2, chi)
        xi = oracle.apply_Mdag(lat, phi, x)
        np.testing.assert_allclose(oracle.force(lat, phi, x, xi), oracle.force(lat, phi, x), atol=1e-14)


@pytest.mark.parametrize("mu2", [0.0, 0.05])
def test_alg_a1_method_oracle_reaches_tolerance(mu2):
    w = WORKLOADS["small16"]
    lat = lat_of(w)
    phi, eta = draw_inputs(w, batch=1)
    chi = oracle.apply_Mdag(lat, phi, eta[0])
    x, info = oracle.fgmres_alg_a1(lat, phi, mu2, chi, TOL=1e-10)
    assert info["true_rel_resid"] <= 1e-10
    xref, _ = oracle.solve(lat, phi, mu2, chi, tol=1e-13)
    assert np.linalg.norm((x - xref).ravel()) <= 1e-6 * np.linalg.norm(xref.ravel())
    assert info["inner_solves"] >= 2


def test_alg_a1_without_inner_solves_is_gmres():
    """With a = 1e25 the test TOL a |b| / ERR < 1 never holds (z_j = v_j) and the
    initial spCG stops before its first step (x0 = 0), so one restart cycle of
    Algorithm A.1 is GMRES(m): x minimises |b - A x| over K_k(A, b), k the number of
    Arnoldi steps taken."""
    lat = Lattice(3, 3, 8, 0.5)
    rng = np.random.default_rng(7)
    phi = rand_phi(rng, lat)
    Ad = NormalOperator(lat, phi, 0.05).dense()
    b = rand_c(rng, lat.n)
    x, info = oracle.fgmres_alg_a1(lat, phi, 0.05, b, TOL=1e-10, a=1e25, max_outer=1)
    assert info["outer"] == 1 and info["inner_iters"] == 0 and info["arnoldi"] == 10
    V = _krylov_basis(Ad, b, info["arnoldi"])
    want = V @ np.linalg.lstsq(Ad @ V, b, rcond=None)[0]
    assert np.linalg.norm(x - want) <= 1e-9 * np.linalg.norm(want)


@pytest.mark.parametrize("mu2", [0.0, 0.05])
def test_alg_a1_cycle_minimises_the_residual_over_the_z_vectors(mu2):
    """Flexible GMRES: each restart cycle ends at the x in x0 + span{z_1 .. z_k} with
    the least |b - A x| (the z_j are the spCG outputs), and the v_j are orthonormal.
    A complex Hessenberg entry with a wrong conjugation or a missing projection
    breaks this although the restarted solver may still converge."""
    w = WORKLOADS["tiny"]
    lat = lat_of(w)
    phi, eta = draw_inputs(w, batch=1)
    chi = oracle.apply_Mdag(lat, phi, eta[0]).ravel()
    Ad = NormalOperator(lat, phi, mu2).dense()
    cycles = []
    x, info = oracle.fgmres_alg_a1(lat, phi, mu2, chi, TOL=1e-10, record=cycles)
    assert info["true_rel_resid"] <= 1e-10 and len(cycles) == info["outer"] >= 1
    ends = [c["x0"] for c in cycles[1:]] + [x]
    for c, x1 in zip(cycles, ends):
        V, Z = np.stack(c["V"], axis=1), np.stack(c["Z"], axis=1)
        assert np.abs(V.conj().T @ V - np.eye(V.shape[1])).max() <= 1e-8   # classical Gram-Schmidt
        r0 = chi - Ad @ c["x0"]
        best = c["x0"] + Z @ np.linalg.lstsq(Ad @ Z, r0, rcond=None)[0]
        assert np.linalg.norm(chi - Ad @ x1) <= (1 + 1e-6) * np.linalg.norm(chi - Ad @ best) + 1e-14 * np.linalg.norm(chi)
        assert np.linalg.norm(x1 - best) <= 1e-6 * np.linalg.norm(best)


@pytest.mark.parametrize("mu2", [0.0, 0.05])
def test_alg_a1_residual_estimate_is_the_cycle_residual(mu2):
    """The residual estimate ERR after Arnoldi step j of a cycle is the true residual of
    the best iterate of the cycle so far, |b - A (x0 + Z_j y)| minimised over y with
    Z_j = [z_0 .. z_j], recomputed here from the dense operator (not from h).  A
    product of subdiagonal entries in its place, or a missed update, fails it."""
    w = WORKLOADS["tiny"]
    lat = lat_of(w)
    phi, eta = draw_inputs(w, batch=1)
    chi = oracle.apply_Mdag(lat, phi, eta[0]).ravel()
    Ad = NormalOperator(lat, phi, mu2).dense()
    cycles = []
    oracle.fgmres_alg_a1(lat, phi, mu2, chi, TOL=1e-10, inner_floor=1e-2, m=4, record=cycles)
    steps = 0
    for c in cycles:
        r0 = chi - Ad @ c["x0"]
        for j, err in enumerate(c["err"]):
            Z = np.stack(c["Z"][: j + 1], axis=1)
            best = c["x0"] + Z @ np.linalg.lstsq(Ad @ Z, r0, rcond=None)[0]
            want = np.linalg.norm(chi - Ad @ best)
            assert abs(err - want) <= 1e-6 * want + 1e-14 * np.linalg.norm(chi), (j, err, want)
            steps += 1
    assert steps >= 4


def test_alg_a1_has_no_crawl_on_the_12x12x32_batch():
    """On the 12x12, N_t = 32 workload (mu^2 = 0) the first cycle ends close to TOL;
    with ERR the cycle's least-squares residual the solve then needs at most two
    restart cycles (the printed product estimate took 21-26 one-step cycles there)."""
    w = WORKLOADS["small16"]
    lat = lat_of(w)
    phi, eta = draw_inputs(w, batch=2)
    for k in range(2):
        chi = oracle.apply_Mdag(lat, phi, eta[k])
        x, info = oracle.fgmres_alg_a1(lat, phi, 0.0, chi, TOL=1e-10)
        assert info["true_rel_resid"] <= 1e-10 and info["outer"] <= 2, info


def _read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=")
                vals[k.strip()] = float(v)
    return vals


def test_largest_eigenvalue_inside_the_papers_fit():
    """Sec. 6.1 fits lambda_max = 4.1 +- 0.2 for M M^dagger at beta*kappa = 8, N_t = 256,
    U/kappa = 3.5, and notes the non-interacting limit is close to it for graphene.
    A graphene sheet at those couplings (free and with a hot-start field) must land there."""
    g = _read_golden("spectral_fit.txt")
    Nt, L = int(g["Nt"]), 6
    lat = Lattice(L, L, Nt, g["beta_kappa"] / Nt)
    free_max = free_spectrum(lat)[-1]
    assert abs(free_max - g["lambda_max"]) <= g["lambda_max_err"]
    rng = np.random.default_rng(21)
    phi = rng.normal(0.0, math.sqrt(g["U_over_kappa"] * g["beta_kappa"] / Nt), size=lat.shape)
    A = NormalOperator(lat, phi, 0.0)
    v = rand_c(rng, lat.n)
    for _ in range(300):
        v = A(v)
        v /= np.linalg.norm(v)
    lam = np.vdot(v, A(v)).real
    assert abs(lam - g["lambda_max"]) <= g["lambda_max_err"]
