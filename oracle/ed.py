"""Exact diagonalisation of the Hubbard Hamiltonian on a small honeycomb (oracle, test-only).

Sec. 7.2 benchmarks the HMC against direct diagonalisation on a 4-site hexagonal
system at U/kappa = 4, beta kappa = 8.  The 4 sites are read as the honeycomb of
2 x 1 unit cells with the bonds of eq. (ferm_op) and periodic wrap (the bond to
cell (i, j-1) lands on cell (i, j) when L2 = 1, so that pair is bonded twice); its
free single-particle energies are +-3 kappa and +-1 kappa, the Gamma and M points.

  H = sum_sigma sum_{x,y} h_{xy} c^dag_{x sigma} c_{y sigma}
      + U sum_x (n_{x up} - 1/2)(n_{x down} - 1/2),
  h_{xy} = -kappa per bond (x, y) between the sublattices (coinciding bonds add).

Sites are ordered as one time slice of the operator's layout: (s, i, j) with flat
index (s L1 + i) L2 + j.  The Fock space of 2 n_s modes (spin up: modes 0..n_s-1)
uses the Jordan-Wigner sign convention; everything is dense complex128 / float64.

* `hopping`        - h;
* `hamiltonian`    - H and the particle-number operator on the Fock space;
* `quasiparticle_energies` - for each single-particle orbital of h with energy > 0,
                     the excitation energy E_n - E_0 of the level (degenerate states
                     summed) that carries the largest weight |<n| c^dag |0>|^2 when
                     one spin-up particle is added to the orbital on the ground state;
* `thermal_correlator` - C_v(tau) = Tr[e^{-(beta - tau) H} c_v e^{-tau H} c_v^dag] / Z
                     for c_v = sum_x v_x c_{x up}.
"""
from __future__ import annotations

import numpy as np


def hopping(L1: int, L2: int, kappa: float) -> np.ndarray:
    P = L1 * L2
    h = np.zeros((2 * P, 2 * P))
    for i in range(L1):
        for j in range(L2):
            a = i * L2 + j
            for (ii, jj) in ((i, j), ((i - 1) % L1, j), (i, (j - 1) % L2)):
                b = P + ii * L2 + jj
                h[a, b] -= kappa
                h[b, a] -= kappa
    return h


def _annihilators(nmodes: int):
    dim = 1 << nmodes
    ops = []
    states = np.arange(dim)
    for m in range(nmodes):
        C = np.zeros((dim, dim))
        occ = (states >> m) & 1
        lower = states & ((1 << m) - 1)
        sign = np.array([(-1) ** bin(int(x)).count("1") for x in lower])
        src = states[occ == 1]
        C[src ^ (1 << m), src] = sign[occ == 1]
        ops.append(C)
    return ops


def hamiltonian(h: np.ndarray, U: float):
    """(H, N, annihilators) on the Fock space of the two spin species."""
    ns = h.shape[0]
    C = _annihilators(2 * ns)
    dim = C[0].shape[0]
    H = np.zeros((dim, dim))
    for sp in range(2):
        for x in range(ns):
            for y in range(ns):
                if h[x, y] != 0.0:
                    H += h[x, y] * C[sp * ns + x].T @ C[sp * ns + y]
    n = [c.T @ c for c in C]
    I = np.eye(dim)
    for x in range(ns):
        H += U * (n[x] - 0.5 * I) @ (n[ns + x] - 0.5 * I)
    return H, sum(n), C


def quasiparticle_energies(L1: int, L2: int, kappa: float, U: float):
    """[(orbital energy, E_n - E_0, weight)] for the orbitals of h with positive energy."""
    h = hopping(L1, L2, kappa)
    H, _, C = hamiltonian(h, U)
    ev, V = np.linalg.eigh(H)
    g = V[:, 0]
    e1, u1 = np.linalg.eigh(h)
    out = []
    for k in range(len(e1)):
        if e1[k] <= 1e-12:
            continue
        cdag = sum(u1[x, k] * C[x].T for x in range(h.shape[0]))
        w = (V.T @ (cdag @ g)) ** 2
        # group degenerate levels
        levels = []
        for j in np.argsort(ev):
            if levels and abs(ev[j] - levels[-1][0]) <= 1e-9:
                levels[-1][1] += w[j]
            else:
                levels.append([ev[j], w[j]])
        E, wt = max(levels, key=lambda lv: lv[1])
        out.append((float(e1[k]), float(E - ev[0]), float(wt)))
    return out


def thermal_correlator(L1: int, L2: int, kappa: float, U: float, beta: float, v, taus):
    h = hopping(L1, L2, kappa)
    H, _, C = hamiltonian(h, U)
    ev, V = np.linalg.eigh(H)
    ev = ev - ev[0]
    c = sum(v[x] * C[x] for x in range(h.shape[0]))
    cm = V.T @ c @ V                     # <m| c_v |n>
    Z = np.sum(np.exp(-beta * ev))
    out = []
    for tau in taus:
        # sum_{m,n} e^{-(beta - tau) E_m} |<m|c|n>|^2 e^{-tau E_n}
        wm = np.exp(-(beta - tau) * ev)
        wn = np.exp(-tau * ev)
        out.append(float(wm @ (cm ** 2) @ wn) / Z)
    return np.array(out)
