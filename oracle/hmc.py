"""Hybrid Monte Carlo trajectory (oracle, test-only).

Sec. 2: the Hamiltonian of eq. (hamiltonian),
    H = phi^T phi / (2 U~) + sum_i S_i(phi) + pi^T pi / 2,
with the pseudofermion terms S_i of the (staggered-mass Hasenbusch) split of
Sec. 5.1; momenta pi and heat-bath vectors rho are drawn by the caller; a trajectory
is accepted with probability min(1, e^{-dH}).

Sec. 5.2: the molecular dynamics is the second-order Omelyan integrator with the
force updates on the outside,
    T(h) = T_F(zeta h) T_pi(h/2) T_F((1 - 2 zeta) h) T_pi(h/2) T_F(zeta h),
where T_F(e) moves pi by -e dS/dphi and T_pi(e) moves phi by e pi, nested over time
scales: level k < n kicks with the force of term k and replaces each T_pi(h/2) by
the integration of level k+1 over h/2; level n kicks with the gauge force and term
n and drifts phi.  Level k takes steps of N_k innermost steps (N_n = 1); when a half
step of level k holds an odd number of level-(k+1) steps, the half step of level
k+1 next to the middle kick is split as the paper prescribes.  zeta = 0 is the
leapfrog integrator.  Every kick recomputes its force (no reuse between kicks).
"""
from __future__ import annotations

import numpy as np

from . import hasenbusch as hb
from .operator import Lattice


class Integrator:
    """Nested Omelyan integrator over levels 0..n (n = len(N)); N[k] innermost steps per level-k step."""

    def __init__(self, N, n_md: int, t: float = 1.0, zeta: float = 0.1931833275037836):
        self.N = list(N)
        self.n = len(self.N)
        self.n_md = int(n_md)
        self.t = float(t)
        self.zeta = float(zeta)
        full = self.N + [1]
        for k in range(self.n):
            if full[k] % full[k + 1] != 0:
                raise ValueError("N_{k+1} must divide N_k")
        if self.n and self.n_md % self.N[0] != 0:
            raise ValueError("N_0 must divide N_MD")
        self.dt = self.t / self.n_md
        self.H = [f * self.dt for f in full]  # step size per level

    def run(self, kick, drift):
        """kick(level, eps): pi -= eps dS_level/dphi; drift(eps): phi += eps pi."""
        self.kick, self.drift = kick, drift
        steps = self.n_md // (self.N[0] if self.n else 1)
        for _ in range(steps):
            self._step(0, self.H[0])

    def _step(self, k, h):
        z = self.zeta
        self.kick(k, z * h)
        self._half(k, h, first=True)
        self.kick(k, (1 - 2 * z) * h)
        self._half(k, h, first=False)
        self.kick(k, z * h)

    def _half(self, k, h, first):
        """Integrate over h/2 with what sits inside a level-k step."""
        if k == self.n:
            self.drift(h / 2)
            return
        r = int(round(h / self.H[k + 1]))
        j, odd = divmod(r, 2)
        if first:
            for _ in range(j):
                self._step(k + 1, self.H[k + 1])
            if odd:
                self._half_step(k + 1, self.H[k + 1], first=True)
        else:
            if odd:
                self._half_step(k + 1, self.H[k + 1], first=False)
            for _ in range(j):
                self._step(k + 1, self.H[k + 1])

    def _half_step(self, k, h, first):
        z = self.zeta
        if first:
            self.kick(k, z * h)
            self._half(k, h, first=True)
            self.kick(k, (1 - 2 * z) * h / 2)
        else:
            self.kick(k, (1 - 2 * z) * h / 2)
            self._half(k, h, first=False)
            self.kick(k, z * h)


def gauge_action(phi, U_t: float) -> float:
    p = np.asarray(phi, dtype=np.float64)
    return 0.5 * float(np.sum(p * p)) / U_t


def kinetic(pi) -> float:
    p = np.asarray(pi, dtype=np.float64)
    return 0.5 * float(np.sum(p * p))


def hamiltonian(lat: Lattice, U_t: float, phi, pi, mts, chi) -> float:
    S, _ = hb.actions_and_forces(lat, phi, mts, chi)
    return gauge_action(phi, U_t) + float(np.sum(S)) + kinetic(pi)


def level_force(lat: Lattice, U_t: float, phi, mts, chi, level: int) -> np.ndarray:
    """dS/dphi of one level: term `level` for level < n, gauge + term n for the last level."""
    n = len(mts)
    _, F, _, _ = hb.term(lat, phi, mts, chi[level], level)
    if level == n:
        F = F + np.asarray(phi) / U_t
    return F


def trajectory(lat: Lattice, U_t: float, phi0, pi0, mts, chi, N, n_md: int, t: float = 1.0,
               zeta: float = 0.1931833275037836):
    """(phi, pi) after one molecular-dynamics trajectory of length t."""
    if len(N) != len(mts):
        raise ValueError("one time-scale factor per Hasenbusch mass")
    phi = np.array(phi0, dtype=np.float64)
    pi = np.array(pi0, dtype=np.float64)
    state = {"phi": phi, "pi": pi}

    def kick(level, eps):
        state["pi"] = state["pi"] - eps * level_force(lat, U_t, state["phi"], mts, chi, level)

    def drift(eps):
        state["phi"] = state["phi"] + eps * state["pi"]

    Integrator(N, n_md, t, zeta).run(kick, drift)
    return state["phi"], state["pi"]


def hmc_update(lat: Lattice, U_t: float, phi0, pi0, rho, mts, N, n_md: int, u: float, t: float = 1.0,
               zeta: float = 0.1931833275037836):
    """One HMC update (Sec. 2): heat-bath chi from rho, trajectory, Metropolis with the uniform u.
    Returns (phi, accepted, dH, H0, H1, pi_end)."""
    chi = hb.heatbath(lat, phi0, mts, rho)
    H0 = hamiltonian(lat, U_t, phi0, pi0, mts, chi)
    phi1, pi1 = trajectory(lat, U_t, phi0, pi0, mts, chi, N, n_md, t, zeta)
    H1 = hamiltonian(lat, U_t, phi1, pi1, mts, chi)
    dH = H1 - H0
    accepted = bool(u < np.exp(-dH))
    return (phi1 if accepted else np.array(phi0, dtype=np.float64)), accepted, dH, H0, H1, pi1
