"""Pins of the oracle's multi-shift CG and spectral bounds (no GPU).

* CG-M: every shifted iterate equals the dense LU solution of its own system;
* the Lanczos matrix of a converged CG has the extreme eigenvalues of A (dense eigh),
  and in the free field the closed forms lambda_min = 4 sin^2(pi/(2 N_t)) (L a
  multiple of 3) and the largest eigenvalue of the closed-form free spectrum;
* the ARPACK path of `spectrum_extremes` agrees with dense eigh;
* eq. (mu_i_eqn): masses geometric between lambda_min and lambda_max.
"""
import math

import numpy as np
import pytest

from oracle import multishift as ms
from oracle.operator import Lattice, NormalOperator
from tests.test_oracle_pins import free_spectrum


def _case(L1, L2, Nt, kt, seed=0, amp=0.8):
    lat = Lattice(L1, L2, Nt, kt)
    rng = np.random.default_rng(seed)
    phi = rng.normal(0, amp, lat.shape)
    b = rng.standard_normal(lat.n) + 1j * rng.standard_normal(lat.n)
    return lat, phi, b


@pytest.mark.parametrize("mu0", [0.0, 0.02])
def test_multishift_iterates_equal_dense_solves(mu0):
    lat, phi, b = _case(3, 3, 8, 0.5, seed=1)
    A0 = NormalOperator(lat, phi, mu0)
    sig = [0.0, 0.01, 0.3, 2.5]
    xs, al, be, k = ms.cg_multishift(A0, b, sig, tol=1e-12)
    Ad = A0.dense()
    for s, x in zip(sig, xs):
        ref = np.linalg.solve(Ad + s * np.eye(lat.n), b)
        assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref), s
    assert k == len(al) == len(be)


def test_shifted_systems_stop_early():
    lat, phi, b = _case(3, 3, 8, 0.5, seed=2)
    A0 = NormalOperator(lat, phi, 0.0)
    xs, _, _, k = ms.cg_multishift(A0, b, [5.0], tol=1e-10)
    # the shifted solution meets its own tolerance
    Ad = A0.dense() + 5.0 * np.eye(lat.n)
    assert np.linalg.norm(b - Ad @ xs[0]) <= 1.5e-10 * np.linalg.norm(b)


def test_ritz_extremes_of_converged_cg_equal_eigh():
    lat, phi, b = _case(3, 3, 8, 0.5, seed=3)
    A0 = NormalOperator(lat, phi, 0.0)
    _, al, be, _ = ms.cg_multishift(A0, b, [], tol=1e-13)
    lo, hi = ms.ritz_extremes(al, be)
    ev = np.linalg.eigvalsh(A0.dense())
    assert abs(lo - ev[0]) <= 1e-8 * ev[0]
    assert abs(hi - ev[-1]) <= 1e-10 * ev[-1]


def test_ritz_extremes_free_field_closed_form():
    # phi = 0, m~ = 0, L a multiple of 3: lambda_min = 4 sin^2(pi / (2 N_t)); the largest
    # eigenvalue is |1 - e^{i w}|^2 + ... at the top of the free band, from the dense spectrum
    lat = Lattice(6, 6, 8, 0.25)
    phi = np.zeros(lat.shape)
    rng = np.random.default_rng(4)
    b = rng.standard_normal(lat.n) + 1j * rng.standard_normal(lat.n)
    A0 = NormalOperator(lat, phi, 0.0)
    _, al, be, _ = ms.cg_multishift(A0, b, [], tol=1e-13)
    lo, hi = ms.ritz_extremes(al, be)
    assert abs(lo - 4 * math.sin(math.pi / 16) ** 2) <= 1e-9
    # the top of the closed-form free spectrum |a|^2 + kappa~^2 |f|^2 (pinned in test_oracle_pins)
    top = free_spectrum(lat)[-1]
    assert abs(hi - top) <= 1e-9 * top


def test_arpack_path_agrees_with_dense():
    lat, phi, _ = _case(3, 3, 10, 0.4, seed=5)
    d = ms.spectrum_extremes(lat, phi, 0.01)
    a = ms.spectrum_extremes(lat, phi, 0.01, dense_limit=10)
    assert abs(d[0] - a[0]) <= 1e-8 * d[0] and abs(d[1] - a[1]) <= 1e-8 * d[1]


def test_hasenbusch_masses_are_geometric():
    lo, hi = 0.054, 4.1  # the paper's fit values (Sec. 6.1)
    for n in (1, 2, 3):
        mu = ms.hasenbusch_masses(lo, hi, n)
        seq = [lo] + mu + [hi]
        ratios = [b / a for a, b in zip(seq, seq[1:])]
        assert np.allclose(ratios, ratios[0], rtol=1e-12)
        assert len(mu) == n and all(lo < m < hi for m in mu)
