"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module holds no arithmetic of the method: it only names the workloads
(lattice shape and the couplings kappa, U, beta), forms the step-size-weighted
constants the fermion operator takes (delta = beta/N_t, kappa~ = delta*kappa,
U~ = delta*U, Sec. 2 of the paper), and draws seeded random fields:

* the Hubbard field phi_{x,t} ~ N(0, U~) (Gaussian weight exp(-phi^2/(2 delta U)),
  eq. (hamiltonian)), float64, layout [N_t][2][L1][L2];
* complex Gaussian vectors with weight exp(-rho^dagger rho) (Sec. 2, heat-bath),
  i.e. Re and Im i.i.d. N(0, 1/2), complex128, layout [batch][N_t][2][L1][L2].

Thermalised HMC ensembles of the paper are not available; these hot-start fields
stand in for them at the paper's lattice shapes.  Draw order is fixed: phi first,
then each right-hand side in order, real part before imaginary part.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = ["Workload", "WORKLOADS", "HasenbuschWorkload", "HASENBUSCH", "draw_phi", "draw_gaussian_c128",
           "draw_inputs", "draw_hasenbusch", "draw_hmc"]


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload: an L1 x L2 honeycomb with N_t time slices."""

    name: str
    L1: int
    L2: int
    Nt: int
    kappa: float
    U: float
    beta: float
    ms: float = 0.0
    nrhs: int = 1
    mu2: tuple = (0.0,)
    tol: float = 1e-10
    seed: int = 0

    @property
    def delta(self) -> float:
        return self.beta / self.Nt

    @property
    def kappa_t(self) -> float:
        """kappa~ = delta * kappa, the hopping entry of M^{AB}."""
        return self.delta * self.kappa

    @property
    def U_t(self) -> float:
        """U~ = delta * U, the variance of the Hubbard field."""
        return self.delta * self.U

    @property
    def ms_t(self) -> float:
        """m~ = delta * m_s, the staggered mass inside the temporal hop."""
        return self.delta * self.ms

    @property
    def nsites(self) -> int:
        """Number of complex unknowns per system, 2 * L1 * L2 * N_t."""
        return 2 * self.L1 * self.L2 * self.Nt

    @property
    def shape(self) -> tuple:
        return (self.Nt, 2, self.L1, self.L2)

    @property
    def batch(self) -> int:
        return max(self.nrhs, len(self.mu2))

    def mu2_list(self) -> list:
        """Per-system shift list of length `batch` (a single shift is broadcast)."""
        if len(self.mu2) == self.batch:
            return [float(m) for m in self.mu2]
        return [float(self.mu2[0])] * self.batch


# Workloads at the shapes of the paper's graphene runs (N_t = 64, L up to 102).
WORKLOADS = {
    # 3x3 cells, N_t = 8, kappa = 1, U = 2, beta = 4: CPU-sized, one right-hand side.
    "tiny": Workload("tiny", 3, 3, 8, 1.0, 2.0, 4.0, nrhs=1, mu2=(0.0,), tol=1e-12, seed=0),
    # 12x12 cells, N_t = 32, U = 3, beta = 8: sixteen right-hand sides sharing phi.
    "small16": Workload("small16", 12, 12, 32, 1.0, 3.0, 8.0, nrhs=16, mu2=(0.0,), seed=2),
    # 48x48 cells, N_t = 64, U = 3.5, beta = 12: three Hasenbusch shifts in one launch.
    "medium3": Workload("medium3", 48, 48, 64, 1.0, 3.5, 12.0, nrhs=3, mu2=(0.5, 0.05, 0.0), seed=3),
    # 102x102 cells, N_t = 64, U = 3.8, beta = 12: the largest lattice of the paper.
    "large2": Workload("large2", 102, 102, 64, 1.0, 3.8, 12.0, nrhs=2, mu2=(0.1, 0.0), seed=4),
}


@dataclasses.dataclass(frozen=True)
class HasenbuschWorkload:
    """A lattice with n staggered Hasenbusch masses mu_0 < ... < mu_{n-1} (units of kappa)."""

    base: Workload
    masses: tuple

    @property
    def mts(self) -> list:
        """m~_i = delta * mu_i, the parameter of M(m_s = mu_i)."""
        return [self.base.delta * m for m in self.masses]

    @property
    def nterms(self) -> int:
        return len(self.masses) + 1


# The masses of the paper's auto-tuned two-mass runs (Table tab_nmds): at 12x12 and
# 102x102 with N_t = 64; the small case uses the 12x12 pair on the 12x12, N_t = 32 lattice.
HASENBUSCH = {
    "hb_tiny": HasenbuschWorkload(Workload("hb_tiny", 3, 3, 8, 1.0, 2.0, 4.0, seed=20), (0.514011, 1.61581)),
    "hb_small": HasenbuschWorkload(Workload("hb_small", 12, 12, 32, 1.0, 3.0, 8.0, seed=21), (0.514011, 1.61581)),
    "hb_large": HasenbuschWorkload(Workload("hb_large", 102, 102, 64, 1.0, 3.8, 12.0, seed=22), (0.4054, 1.09624)),
}


def draw_phi(rng: np.random.Generator, w: Workload) -> np.ndarray:
    """phi ~ N(0, U~), float64 [N_t][2][L1][L2]."""
    return rng.normal(0.0, math.sqrt(w.U_t), size=w.shape)


def draw_gaussian_c128(rng: np.random.Generator, shape) -> np.ndarray:
    """Complex Gaussian with weight exp(-|z|^2): Re, Im i.i.d. N(0, 1/2)."""
    re = rng.standard_normal(size=shape)
    im = rng.standard_normal(size=shape)
    return (re + 1j * im) * math.sqrt(0.5)


def draw_inputs(w: Workload, seed: int | None = None, batch: int | None = None):
    """Return (phi, eta) for a workload: phi [N_t,2,L1,L2] float64 and
    eta [batch,N_t,2,L1,L2] complex128, drawn phi first then eta_0, eta_1, ..."""
    rng = np.random.default_rng(w.seed if seed is None else seed)
    phi = draw_phi(rng, w)
    nb = w.batch if batch is None else batch
    eta = np.stack([draw_gaussian_c128(rng, w.shape) for _ in range(nb)])
    return phi, eta


def draw_hasenbusch(hw: HasenbuschWorkload, seed: int | None = None):
    """Return (phi, rho) for a Hasenbusch workload: rho [n+1, N_t, 2, L1, L2] holds the
    heat-bath vectors rho_0 .. rho_n (drawn phi first, then rho_0, rho_1, ...)."""
    return draw_inputs(hw.base, seed=seed, batch=hw.nterms)


def draw_hmc(hw: HasenbuschWorkload, seed: int | None = None):
    """Return (phi, pi, rho) for one HMC update: phi as in draw_phi, momenta pi ~ N(0, 1)
    (weight exp(-pi^2/2)) float64 [N_t, 2, L1, L2], then rho_0 .. rho_n (drawn in that order)."""
    w = hw.base
    rng = np.random.default_rng(w.seed if seed is None else seed)
    phi = draw_phi(rng, w)
    pi = rng.standard_normal(size=w.shape)
    rho = np.stack([draw_gaussian_c128(rng, w.shape) for _ in range(hw.nterms)])
    return phi, pi, rho


def serving_stream(n: int, seed: int = 5, rate: float = 200.0,
                   Ls=(6, 12, 24, 48, 102), Nts=(16, 32, 64), mu2s=(0.5, 0.1, 0.01, 0.0)):
    """Seeded Poisson stream of request descriptors for the serving workload.

    Each request draws L from `Ls`, N_t from `Nts`, U ~ U[1, 4] with beta = N_t/4
    (so kappa~ = 0.25 and U~ = U/4), and a shift from `mu2s`.  Returns a list of
    dicts with the arrival time (seconds), the Workload and a per-request seed."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += rng.exponential(1.0 / rate)
        L = int(rng.choice(Ls))
        Nt = int(rng.choice(Nts))
        U = float(rng.uniform(1.0, 4.0))
        mu2 = float(rng.choice(mu2s))
        w = Workload(f"req{k}", L, L, Nt, 1.0, U, Nt / 4.0, nrhs=1, mu2=(mu2,), seed=int(rng.integers(1 << 31)))
        out.append({"t": t, "workload": w})
    return out
