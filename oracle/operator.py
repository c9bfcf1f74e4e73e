"""The fermion matrix M[phi] of eq. (ferm_op), built entry by entry (oracle, test-only).

Sec. 2 of the paper defines, for sites x, y of the honeycomb and slices t, t':

  M^{AA}_{(x,t)(y,t')} = delta_xy ( -delta_{tt'} + (e^{i phi_{x,t}} - m~) delta_{t-1,t'} )
  M^{BB}_{(x,t)(y,t')} = delta_xy ( +delta_{tt'} - (e^{-i phi_{x,t}} - m~) delta_{t+1,t'} )
  M^{AB} = M^{BA}      = -kappa~ delta_<x,y> delta_{tt'}

with kappa~ = delta*kappa, m~ = delta*m_s.  Readings taken where the paper is silent:

* temporal boundary antiperiodic: the A hop out of t = 0 lands on t = N_t - 1 with
  a factor -1, the B hop out of t = N_t - 1 lands on t = 0 with a factor -1;
* the phase on a temporal hop is phi of the row's own site and slice, for both
  sublattices, exactly as the equation is printed;
* site map: unit cell (i, j) with i, j mod L1, L2 along the two oblique axes; the
  A site of cell (i, j) is bonded to the B sites of cells (i, j), (i-1, j) and
  (i, j-1); flat index ((t*2 + s)*L1 + i)*L2 + j with s = 0 for A, 1 for B;
* entries add, which matters only for L = 1 or N_t = 1 where links coincide.

M^dagger is the conjugate transpose of that matrix.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass(frozen=True)
class Lattice:
    L1: int
    L2: int
    Nt: int
    kappa_t: float
    ms_t: float = 0.0

    @property
    def n(self) -> int:
        return 2 * self.L1 * self.L2 * self.Nt

    @property
    def shape(self) -> tuple:
        return (self.Nt, 2, self.L1, self.L2)


def site_index(lat: Lattice, t, s, i, j):
    """Flat index of site (t, s, i, j); accepts integers or integer arrays."""
    return ((t * 2 + s) * lat.L1 + i) * lat.L2 + j


def build_M_dense_loops(lat: Lattice, phi: np.ndarray) -> np.ndarray:
    """Dense M from eq. (ferm_op) with plain Python loops (small lattices only)."""
    phi = np.asarray(phi, dtype=np.float64).reshape(lat.shape)
    N = lat.n
    M = np.zeros((N, N), dtype=np.complex128)
    for t in range(lat.Nt):
        for i in range(lat.L1):
            for j in range(lat.L2):
                a = site_index(lat, t, 0, i, j)
                b = site_index(lat, t, 1, i, j)
                # M^{AA}: -1 on the diagonal, (e^{i phi} - m~) towards slice t-1.
                M[a, a] += -1.0
                tm = t - 1
                sign = 1.0
                if tm < 0:
                    tm += lat.Nt
                    sign = -1.0
                M[a, site_index(lat, tm, 0, i, j)] += sign * (np.exp(1j * phi[t, 0, i, j]) - lat.ms_t)
                # M^{BB}: +1 on the diagonal, -(e^{-i phi} - m~) towards slice t+1.
                M[b, b] += 1.0
                tp = t + 1
                sign = 1.0
                if tp >= lat.Nt:
                    tp -= lat.Nt
                    sign = -1.0
                M[b, site_index(lat, tp, 1, i, j)] += -sign * (np.exp(-1j * phi[t, 1, i, j]) - lat.ms_t)
                # M^{AB} = M^{BA}: -kappa~ on each of the three bonds of A(i, j).
                for (ii, jj) in ((i, j), ((i - 1) % lat.L1, j), (i, (j - 1) % lat.L2)):
                    nb = site_index(lat, t, 1, ii, jj)
                    M[a, nb] += -lat.kappa_t
                    M[nb, a] += -lat.kappa_t
    return M


def build_M(lat: Lattice, phi: np.ndarray) -> sp.csr_matrix:
    """Sparse M (CSR) from eq. (ferm_op): the same entries as the loop builder,
    generated with vectorised index arithmetic so that the largest lattices fit."""
    phi = np.asarray(phi, dtype=np.float64).reshape(lat.shape)
    t, i, j = np.meshgrid(np.arange(lat.Nt), np.arange(lat.L1), np.arange(lat.L2), indexing="ij")
    t, i, j = t.ravel(), i.ravel(), j.ravel()
    a = site_index(lat, t, 0, i, j)
    b = site_index(lat, t, 1, i, j)
    rows, cols, vals = [], [], []
    # M^{AA}
    rows.append(a); cols.append(a); vals.append(np.full(a.shape, -1.0 + 0j))
    tm = (t - 1) % lat.Nt
    sgn_m = np.where(t == 0, -1.0, 1.0)
    rows.append(a); cols.append(site_index(lat, tm, 0, i, j))
    vals.append(sgn_m * (np.exp(1j * phi[t, 0, i, j]) - lat.ms_t))
    # M^{BB}
    rows.append(b); cols.append(b); vals.append(np.full(b.shape, 1.0 + 0j))
    tp = (t + 1) % lat.Nt
    sgn_p = np.where(t == lat.Nt - 1, -1.0, 1.0)
    rows.append(b); cols.append(site_index(lat, tp, 1, i, j))
    vals.append(-sgn_p * (np.exp(-1j * phi[t, 1, i, j]) - lat.ms_t))
    # M^{AB} = M^{BA}
    for (ii, jj) in ((i, j), ((i - 1) % lat.L1, j), (i, (j - 1) % lat.L2)):
        nb = site_index(lat, t, 1, ii, jj)
        hop = np.full(a.shape, -lat.kappa_t + 0j)
        rows.append(a); cols.append(nb); vals.append(hop)
        rows.append(nb); cols.append(a); vals.append(hop)
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(lat.n, lat.n))
    return M.tocsr()  # duplicates are summed


def _flat(x: np.ndarray, n: int) -> np.ndarray:
    x = np.asarray(x, dtype=np.complex128)
    return x.reshape(-1, n)


def apply_M(lat: Lattice, phi, x, M=None) -> np.ndarray:
    """y = M[phi] x for x of shape [..., N_t, 2, L1, L2] (or flat)."""
    M = build_M(lat, phi) if M is None else M
    xs = _flat(x, lat.n)
    return (M @ xs.T).T.reshape(np.shape(x))


def apply_Mdag(lat: Lattice, phi, x, M=None) -> np.ndarray:
    """y = M[phi]^dagger x (conjugate transpose of the matrix above)."""
    M = build_M(lat, phi) if M is None else M
    Mh = M.conj().T.tocsr()
    xs = _flat(x, lat.n)
    return (Mh @ xs.T).T.reshape(np.shape(x))


class NormalOperator:
    """A = M M^dagger + mu^2 I applied as two sparse products (Sec. 3, shift of Sec. 5.1)."""

    def __init__(self, lat: Lattice, phi, mu2: float = 0.0, M=None):
        self.lat = lat
        self.M = build_M(lat, phi) if M is None else M
        self.Mh = self.M.conj().T.tocsr()
        self.mu2 = float(mu2)

    def __call__(self, x: np.ndarray) -> np.ndarray:
        return self.M @ (self.Mh @ x) + self.mu2 * x

    def dense(self) -> np.ndarray:
        Md = self.M.toarray()
        return Md @ Md.conj().T + self.mu2 * np.eye(self.lat.n)


def normal_apply(lat: Lattice, phi, mu2, x) -> np.ndarray:
    """q = (M M^dagger + mu^2) x for one flat or shaped vector."""
    A = NormalOperator(lat, phi, mu2)
    xf = np.asarray(x, dtype=np.complex128).ravel()
    return A(xf).reshape(np.shape(x))
