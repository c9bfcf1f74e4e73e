"""Single-particle correlators from the fermion matrix and their exponential fits (oracle, test-only).

Sec. 7.2 extracts quasi-particle energies from correlators C(tau) ~ e^{-E tau} by
exponential fits in fixed windows (tau kappa in [0.2, 1] for Gamma, [0.6, 2] for M).
On one field phi the correlator of a time-slice vector v (one entry per site of a
slice, ordered as the slice's layout) is

  C_v(tau_k) = -(1/|S|) sum_{t0 in S} s(t0 + k) v^dag [M^{-1}]_{(t0 + k), (t0)} v,

with the slices taken mod N_t and s = -1 when t0 + k wraps (the antiperiodic
boundary of eq. (ferm_op)); averaging over phi gives the ensemble correlator.  With
the sign conventions of eq. (ferm_op) the Gamma channel of the 2 x 1-cell lattice is
v = (1, 1, 1, 1)/2 and the M channel v = (1, -1, 1, -1)/2 over (A0, A1, B0, B1):
in the free field they decay with the free energies 3 kappa and kappa.
"""
from __future__ import annotations

import numpy as np

from .operator import Lattice, build_M

GAMMA = np.array([1.0, 1.0, 1.0, 1.0]) / 2
M_POINT = np.array([1.0, -1.0, 1.0, -1.0]) / 2


def propagator_correlator(lat: Lattice, phi, v, t0s=None) -> np.ndarray:
    """C_v(tau_k), k = 0..N_t-1, on one field by dense inversion (small lattices)."""
    ns = 2 * lat.L1 * lat.L2
    v = np.asarray(v, dtype=np.complex128)
    Minv = np.linalg.inv(build_M(lat, phi).toarray())
    t0s = range(lat.Nt) if t0s is None else t0s
    C = np.zeros(lat.Nt)
    for t0 in t0s:
        src = np.zeros(lat.n, dtype=np.complex128)
        src[t0 * ns:(t0 + 1) * ns] = v
        col = Minv @ src
        for k in range(lat.Nt):
            t = (t0 + k) % lat.Nt
            sgn = -1.0 if t0 + k >= lat.Nt else 1.0
            C[k] += -sgn * float(np.vdot(v, col[t * ns:(t + 1) * ns]).real)
    return C / len(t0s)


def fit_energy(C, delta: float, window) -> float:
    """E of the least-squares fit log C = log A - E tau over tau in the window (tau = k delta)."""
    C = np.asarray(C, dtype=np.float64)
    tau = np.arange(len(C)) * delta
    sel = (tau >= window[0] - 1e-12) & (tau <= window[1] + 1e-12) & (C > 0)
    slope, _ = np.polyfit(tau[sel], np.log(C[sel]), 1)
    return float(-slope)
