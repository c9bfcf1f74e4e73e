"""The paper's staggered-mass Hasenbusch split (oracle, test-only).

Sec. 5.1 replaces the single pseudofermion term by n+1 terms built from the
operators M_mu = M(m_s = mu) of eq. (ferm_op) with staggered masses
mu_0, ..., mu_{n-1}; M_{mu_{-1}} is the operator without mass (here: the base
lattice's own m~, zero in the paper).  In terms of the kernels

    term n   : S_n = chi_n^dag (M_{n-1} M_{n-1}^dag)^{-1} chi_n
    term i<n : S_i = (M_i chi_i)^dag (M_{i-1} M_{i-1}^dag)^{-1} (M_i chi_i)

(M_i short for M_{mu_i}).  The heat-bath draws rho_i with density e^{-rho^dag rho}
and sets chi_n = M_{n-1} rho_n and chi_i = M_i^{-1} M_{i-1} rho_i, so that every
term equals rho_i^dag rho_i at the start of a trajectory.  With
eta_i = (M_{i-1} M_{i-1}^dag)^{-1} M_i chi_i and xi_i = M_{i-1}^dag eta_i (eq.
(def_xi_i)) the molecular-dynamics force of a ratio term is
2 Re(eta_i^dag dM/dphi (xi_i - chi_i)) (eq. (f_chi_i)); dM/dphi does not depend on
the staggered mass.  This module returns dS_i/dphi, the negative of that force.

Masses are passed as m~ values (delta * mu), the parameter of `Lattice.ms_t`.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse.linalg as spla

from .force import force
from .operator import Lattice, apply_M, apply_Mdag, build_M
from .solve import solve


def lattice_with_mass(lat: Lattice, mt: float) -> Lattice:
    return dataclasses.replace(lat, ms_t=float(mt))


def mass_of(lat: Lattice, mts, i: int) -> float:
    """m~ of M_{mu_i}; i = -1 is the base operator."""
    return lat.ms_t if i < 0 else float(mts[i])


def solve_M(lat: Lattice, phi, b, tol: float = 1e-13, direct_limit: int = 20000):
    """x = M^{-1} b: sparse LU for small N, else x = M^dag (M M^dag)^{-1} b by certified CG."""
    bf = np.asarray(b, dtype=np.complex128)
    if lat.n <= direct_limit:
        x = spla.spsolve(build_M(lat, phi).tocsc(), bf.ravel())
        return x.reshape(bf.shape)
    y, _ = solve(lat, phi, 0.0, bf, tol=tol)
    return apply_Mdag(lat, phi, y)


def heatbath(lat: Lattice, phi, mts, rho) -> np.ndarray:
    """chi_i for i = 0..n from rho_i (rho shaped [n+1, Nt, 2, L1, L2])."""
    n = len(mts)
    rho = np.asarray(rho, dtype=np.complex128)
    assert rho.shape[0] == n + 1
    chi = np.empty_like(rho)
    chi[n] = apply_M(lattice_with_mass(lat, mass_of(lat, mts, n - 1)), phi, rho[n])
    for i in range(n):
        rhs = apply_M(lattice_with_mass(lat, mass_of(lat, mts, i - 1)), phi, rho[i])
        chi[i] = solve_M(lattice_with_mass(lat, mass_of(lat, mts, i)), phi, rhs)
    return chi


def term(lat: Lattice, phi, mts, chi_i, i: int, tol: float = 1e-13):
    """(S_i, dS_i/dphi, eta_i, xi_i) of term i for the pseudofermion chi_i."""
    n = len(mts)
    chi_i = np.asarray(chi_i, dtype=np.complex128)
    den = lattice_with_mass(lat, mass_of(lat, mts, (n - 1) if i == n else (i - 1)))
    if i == n:
        w = chi_i
    else:
        w = apply_M(lattice_with_mass(lat, mass_of(lat, mts, i)), phi, chi_i)
    eta, _ = solve(den, phi, 0.0, w, tol=tol)
    xi = apply_Mdag(den, phi, eta)
    S = float(np.vdot(w.ravel(), eta.ravel()).real)
    F = force(den, phi, eta, xi if i == n else xi - chi_i)
    return S, F, eta, xi


def actions_and_forces(lat: Lattice, phi, mts, chi, terms=None, tol: float = 1e-13):
    """Per-term actions [n+1] and the summed dS/dphi over `terms` (default: all)."""
    n = len(mts)
    terms = range(n + 1) if terms is None else terms
    S = np.zeros(n + 1)
    F = np.zeros(lat.shape)
    for i in terms:
        S[i], Fi, _, _ = term(lat, phi, mts, chi[i], i, tol=tol)
        F += Fi
    return S, F
