"""Pseudofermion action and its derivative dS/dphi (oracle, test-only).

eq. (hamiltonian): S = chi^dagger (M M^dagger)^{-1} chi (plus the shift mu^2 of the
Hasenbusch term, Sec. 5.1).  eqs. (p_dot), (eta_xi): with eta = (M M^dagger)^{-1} chi
and xi = M^dagger eta, the molecular-dynamics force of the pseudofermion term is
2 Re(eta^dagger dM/dphi xi) = -dS/dphi.  This module returns +dS/dphi.

dM/dphi_{x,t} has a single nonzero entry, the derivative of the temporal hop of
eq. (ferm_op) that carries phi_{x,t}:

  A site: d/dphi [ s (e^{i phi} - m~) ]   = i s e^{i phi}    at [(t,A,x), (t-1,A,x)]
  B site: d/dphi [ -s (e^{-i phi} - m~) ] = i s e^{-i phi}   at [(t,B,x), (t+1,B,x)]

with s = -1 on the hop that wraps the antiperiodic temporal boundary.  m~ drops out.
"""
from __future__ import annotations

import numpy as np

from .operator import Lattice, apply_Mdag, site_index


def action(chi: np.ndarray, eta: np.ndarray) -> np.ndarray:
    """S = Re chi^dagger eta per system; chi, eta shaped [batch, ...] or a single vector."""
    c = np.asarray(chi, dtype=np.complex128)
    e = np.asarray(eta, dtype=np.complex128)
    if c.ndim <= 4:
        return np.vdot(c.ravel(), e.ravel()).real
    return np.array([np.vdot(c[k].ravel(), e[k].ravel()).real for k in range(c.shape[0])])


def xi_from_eta(lat: Lattice, phi, eta) -> np.ndarray:
    """xi = M^dagger eta (eq. (eta_xi))."""
    return apply_Mdag(lat, phi, eta)


def dM_dphi_entries(lat: Lattice, phi):
    """For every component k of phi (flat, same order as the sites) the single nonzero
    entry of dM/dphi_k as arrays (row, col, value)."""
    phi = np.asarray(phi, dtype=np.float64).reshape(lat.shape)
    t, s, i, j = np.meshgrid(np.arange(lat.Nt), np.arange(2), np.arange(lat.L1), np.arange(lat.L2),
                             indexing="ij")
    t, s, i, j = t.ravel(), s.ravel(), i.ravel(), j.ravel()
    row = site_index(lat, t, s, i, j)
    ph = phi.ravel()
    isA = s == 0
    # A: link to t-1, sign -1 when t == 0; B: link to t+1, sign -1 when t == N_t-1.
    tcol = np.where(isA, (t - 1) % lat.Nt, (t + 1) % lat.Nt)
    sign = np.where(isA, np.where(t == 0, -1.0, 1.0), np.where(t == lat.Nt - 1, -1.0, 1.0))
    col = site_index(lat, tcol, s, i, j)
    val = np.where(isA, 1j * sign * np.exp(1j * ph), 1j * sign * np.exp(-1j * ph))
    return row, col, val


def force(lat: Lattice, phi, eta, xi=None) -> np.ndarray:
    """dS/dphi = -2 Re(eta^dagger dM/dphi xi), shaped like phi (or [batch, ...] for batched eta)."""
    eta = np.asarray(eta, dtype=np.complex128)
    if xi is None:
        xi = xi_from_eta(lat, phi, eta)
    xi = np.asarray(xi, dtype=np.complex128)
    row, col, val = dM_dphi_entries(lat, phi)
    e = eta.reshape(-1, lat.n)
    x = xi.reshape(-1, lat.n)
    F = -2.0 * (np.conj(e[:, row]) * val[None, :] * x[:, col]).real
    return F.reshape(eta.shape[:-4] + lat.shape) if eta.ndim > 4 else F.reshape(lat.shape)
