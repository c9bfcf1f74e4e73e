"""Pins of the exact-diagonalisation oracle for the 4-site benchmark (no GPU).

* the paper's exact quasi-particle energies E_Gamma = 3.429 kappa, E_M = 1.565 kappa
  at U/kappa = 4 (Table tab:fit results, `tests/golden/four_site_ed.txt`);
* U = 0: the excitation energies are the free orbital energies 3 kappa and kappa
  with unit weight, and the thermal correlator is e^{-eps tau} / (1 + e^{-beta eps});
* H is real symmetric and conserves the particle number; the half-filled ground
  state holds 4 particles;
* the hopping matrix of the 2 x 1 cells has the free spectrum +-3, +-1.
"""
import math
import os

import numpy as np
import pytest

from oracle import ed

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "four_site_ed.txt")


def _golden():
    vals = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, v, tol = line.split()
        vals[name] = (float(v), float(tol))
    return vals


def test_paper_exact_energies():
    g = _golden()
    qp = {round(e): E for e, E, _ in ed.quasiparticle_energies(2, 1, 1.0, 4.0)}
    assert abs(qp[3] - g["E_Gamma"][0]) <= g["E_Gamma"][1]
    assert abs(qp[1] - g["E_M"][0]) <= g["E_M"][1]


def test_free_limit():
    for e, E, w in ed.quasiparticle_energies(2, 1, 1.0, 0.0):
        assert abs(E - e) < 1e-12 and abs(w - 1.0) < 1e-12
    h = ed.hopping(2, 1, 1.0)
    e1, u1 = np.linalg.eigh(h)
    assert np.allclose(e1, [-3, -1, 1, 3])
    beta = 8.0
    taus = np.linspace(0, 8, 9)
    for k in (2, 3):
        C = ed.thermal_correlator(2, 1, 1.0, 0.0, beta, u1[:, k], taus)
        eps = e1[k]
        assert np.allclose(C, np.exp(-eps * taus) / (1 + np.exp(-beta * eps)), rtol=0, atol=1e-12)


def test_hamiltonian_structure():
    H, N, _ = ed.hamiltonian(ed.hopping(2, 1, 1.0), 4.0)
    assert np.allclose(H, H.T)
    assert np.allclose(H @ N, N @ H)
    ev, V = np.linalg.eigh(H)
    assert abs(V[:, 0] @ N @ V[:, 0] - 4.0) < 1e-10


def test_hopping_bonds():
    h = ed.hopping(2, 1, 1.0)
    # sites A0, A1, B0, B1: A_i bonds B_i twice (L2 = 1 wrap) and B_{i-1} once
    assert np.array_equal(h[:2, 2:], -np.array([[2.0, 1.0], [1.0, 2.0]]))
    assert np.array_equal(h[:2, :2], np.zeros((2, 2))) and np.array_equal(h, h.T)
    # a 3x3 honeycomb: three distinct bonds per site
    h3 = ed.hopping(3, 3, 1.0)
    assert np.all((h3 != 0).sum(axis=1) == 3) and np.all(h3.sum(axis=1) == -3)
