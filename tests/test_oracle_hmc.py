"""Pins of the oracle's HMC trajectory (Sec. 2, 4, 5.2) that do not reuse its code (no GPU).

* harmonic oscillator H = p^2/2 + w^2 q^2/2: the integrator converges to the exact
  flow q0 cos wt + (p0/w) sin wt with error O(dt^2) (the second order of the Omelyan
  scheme), single-level and nested over three time scales with even and odd
  step ratios (the paper's half-step rule);
* nesting with every N_k = 1 equals one level kicking with the summed force, and
  with the outer forces switched off a nested trajectory is the innermost
  integrator run N_MD times (the odd half steps join next to the middle kick);
* on a lattice: reversibility (pi -> -pi retraces phi), symplecticity
  (J^T Omega J = Omega for the finite-difference Jacobian of the map), and
  dH = O(dt^2);
* the Metropolis decision and the rejection path.
"""
import math

import numpy as np
import pytest

from oracle import hasenbusch as ohb
from oracle import hmc
from oracle.operator import Lattice

ZETA = 0.1931833275037836


def _oscillator(N, n_md, omegas, q0=0.7, p0=-0.3, t=1.0, zeta=ZETA):
    st = {"q": q0, "p": p0}

    def kick(level, eps):
        st["p"] -= eps * omegas[level] ** 2 * st["q"]

    def drift(eps):
        st["q"] += eps * st["p"]

    hmc.Integrator(N, n_md, t, zeta).run(kick, drift)
    w = math.sqrt(sum(o * o for o in omegas))
    q_ex = q0 * math.cos(w * t) + p0 / w * math.sin(w * t)
    p_ex = -q0 * w * math.sin(w * t) + p0 * math.cos(w * t)
    return math.hypot(st["q"] - q_ex, st["p"] - p_ex)


@pytest.mark.parametrize("zeta", [ZETA, 0.0])
def test_oscillator_second_order_single_level(zeta):
    e = [_oscillator([], n, [2.0], zeta=zeta) for n in (10, 20, 40, 80)]
    for a, b in zip(e, e[1:]):
        assert 3.6 < a / b < 4.4, e
    assert e[-1] < 1e-3


@pytest.mark.parametrize("N", [[4, 2], [3, 1], [6, 3], [2, 2]])
def test_oscillator_second_order_nested(N):
    om = [0.8, 1.3, 2.1]
    base = N[0]
    e = [_oscillator(N, base * m, om) for m in (4, 8, 16, 32)]
    for a, b in zip(e, e[1:]):
        assert 3.5 < a / b < 4.5, e


def test_nesting_with_unit_factors_is_one_level_with_summed_force():
    om = [0.8, 1.3, 2.1]
    for n_md in (3, 7):
        tr = {}
        for name, N, oms in (("nested", [1, 1], om), ("single", [], [math.sqrt(sum(o * o for o in om))])):
            st = {"q": 0.4, "p": 0.9}

            def kick(level, eps, oms=oms, st=st):
                st["p"] -= eps * oms[level] ** 2 * st["q"]

            def drift(eps, st=st):
                st["q"] += eps * st["p"]

            hmc.Integrator(N, n_md, 1.3, ZETA).run(kick, drift)
            tr[name] = (st["q"], st["p"])
        assert np.allclose(tr["nested"], tr["single"], rtol=0, atol=1e-14)


@pytest.mark.parametrize("N", [[3], [5], [4], [6, 3], [3, 1]])
def test_switched_off_slow_force_leaves_consecutive_inner_steps(N):
    # with the forces of the outer levels switched off, one trajectory of the nested integrator
    # is the innermost integrator run N_MD times: the odd half steps join up (Sec. 5.2)
    om_inner = 1.7
    n_md = 2 * N[0]
    res = []
    for NN, oms in ((N, [0.0] * len(N) + [om_inner]), ([], [om_inner])):
        st = {"q": 0.4, "p": 0.9}

        def kick(level, eps, oms=oms, st=st):
            st["p"] -= eps * oms[level] ** 2 * st["q"]

        def drift(eps, st=st):
            st["q"] += eps * st["p"]

        hmc.Integrator(NN, n_md, 1.1, ZETA).run(kick, drift)
        res.append((st["q"], st["p"]))
    assert np.allclose(res[0], res[1], rtol=0, atol=1e-14)


def _max_energy_violation(n_md, zeta, t=10.0, w=1.0):
    st = {"q": 1.0, "p": 0.0}

    def kick(level, eps):
        st["p"] -= eps * w * w * st["q"]

    def drift(eps):
        st["q"] += eps * st["p"]

    worst = 0.0
    for _ in range(n_md):  # one step at a time, energy after each
        hmc.Integrator([], 1, t / n_md, zeta).run(kick, drift)
        worst = max(worst, abs(0.5 * st["p"] ** 2 + 0.5 * w * w * st["q"] ** 2 - 0.5 * w * w))
    return worst


@pytest.mark.parametrize("n", [50, 100])
def test_omelyan_beats_leapfrog_at_equal_cost(n):
    # Sec. 4: two force evaluations per Omelyan step, so compare with leapfrog (zeta = 0) at
    # twice the steps; the paper's generic estimate of the error ratio is 0.4
    ratio = _max_energy_violation(n, ZETA) / _max_energy_violation(2 * n, 0.0)
    assert ratio < 0.4


def _lattice_case(seed=0, L=(3, 3, 4)):
    lat = Lattice(L[0], L[1], L[2], 0.35)
    rng = np.random.default_rng(seed)
    U_t = 0.6
    phi = rng.normal(0, math.sqrt(U_t), lat.shape)
    pi = rng.normal(0, 1, lat.shape)
    mts = [0.08, 0.3]
    rho = (rng.standard_normal((3,) + lat.shape) + 1j * rng.standard_normal((3,) + lat.shape)) * math.sqrt(0.5)
    chi = ohb.heatbath(lat, phi, mts, rho)
    return lat, U_t, phi, pi, mts, chi


def test_reversibility_on_a_lattice():
    lat, U_t, phi, pi, mts, chi = _lattice_case(1)
    phi1, pi1 = hmc.trajectory(lat, U_t, phi, pi, mts, chi, [2, 1], 4, t=0.5)
    phi2, pi2 = hmc.trajectory(lat, U_t, phi1, -pi1, mts, chi, [2, 1], 4, t=0.5)
    assert np.abs(phi2 - phi).max() < 1e-11
    assert np.abs(pi2 + pi).max() < 1e-11
    assert np.abs(phi1 - phi).max() > 1e-2  # it moved


def test_symplectic_map_on_a_tiny_lattice():
    lat = Lattice(2, 2, 2, 0.4)
    rng = np.random.default_rng(7)
    U_t = 0.5
    phi = rng.normal(0, 0.7, lat.shape)
    pi = rng.normal(0, 1, lat.shape)
    mts = [0.2]
    rho = (rng.standard_normal((2,) + lat.shape) + 1j * rng.standard_normal((2,) + lat.shape)) * math.sqrt(0.5)
    chi = ohb.heatbath(lat, phi, mts, rho)
    n = lat.n

    def flow(z):
        p1, q1 = hmc.trajectory(lat, U_t, z[:n].reshape(lat.shape), z[n:].reshape(lat.shape), mts, chi, [1], 3,
                                t=0.6)
        return np.concatenate([p1.ravel(), q1.ravel()])

    z0 = np.concatenate([phi.ravel(), pi.ravel()])
    h = 1e-5
    J = np.empty((2 * n, 2 * n))
    for k in range(2 * n):
        zp = z0.copy(); zp[k] += h
        zm = z0.copy(); zm[k] -= h
        J[:, k] = (flow(zp) - flow(zm)) / (2 * h)
    Om = np.block([[np.zeros((n, n)), np.eye(n)], [-np.eye(n), np.zeros((n, n))]])
    assert np.abs(J.T @ Om @ J - Om).max() < 1e-6
    assert np.abs(J - np.eye(2 * n)).max() > 1e-2  # a nontrivial map


def test_energy_violation_is_second_order():
    lat, U_t, phi, pi, mts, chi = _lattice_case(3)
    H0 = hmc.hamiltonian(lat, U_t, phi, pi, mts, chi)
    dH = []
    for n_md in (16, 32, 64):
        p1, q1 = hmc.trajectory(lat, U_t, phi, pi, mts, chi, [2, 1], n_md, t=1.0)
        dH.append(abs(hmc.hamiltonian(lat, U_t, p1, q1, mts, chi) - H0))
    assert 3.4 < dH[0] / dH[1] < 4.6 and 3.4 < dH[1] / dH[2] < 4.6, dH


def test_metropolis_decision_and_rejection():
    lat, U_t, phi, pi, mts, _ = _lattice_case(4)
    rng = np.random.default_rng(9)
    rho = (rng.standard_normal((3,) + lat.shape) + 1j * rng.standard_normal((3,) + lat.shape)) * math.sqrt(0.5)
    p_acc, acc, dH, H0, H1, _ = hmc.hmc_update(lat, U_t, phi, pi, rho, mts, [1, 1], 4, u=0.0, t=0.5)
    assert acc and not np.array_equal(p_acc, phi)
    assert abs(H1 - H0 - dH) < 1e-12
    # at the start every pseudofermion term equals |rho_i|^2
    r2 = sum(float(np.vdot(r.ravel(), r.ravel()).real) for r in rho)
    assert abs(H0 - hmc.gauge_action(phi, U_t) - hmc.kinetic(pi) - r2) < 1e-10 * r2
    p_rej, acc2, dH2, _, _, _ = hmc.hmc_update(lat, U_t, phi, pi, rho, mts, [1, 1], 4, u=math.exp(-dH) * 1.0001,
                                               t=0.5)
    assert not acc2 and np.array_equal(p_rej, phi) and dH2 == dH
    _, acc3, dH3, _, _, _ = hmc.hmc_update(lat, U_t, phi, pi, rho, mts, [1, 1], 4, u=math.exp(-dH) * 0.9999, t=0.5)
    assert acc3 and dH3 == dH
