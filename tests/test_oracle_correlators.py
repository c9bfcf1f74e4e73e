"""Pins of the correlator measurement (no GPU).

* free field: the Gamma and M projections of M^{-1} decay with the free energies
  3 kappa and kappa, with an O(delta^2) time-discretisation error of the fitted
  energy (halving delta quarters it), and approach the exact free thermal correlator
  of the ED oracle;
* time translation: on a field rolled by s slices the correlator from source slice
  s equals the one from slice 0 on the original field at every separation, the
  separations that wrap the antiperiodic boundary included;
* the exponential fit returns E exactly for a pure exponential.
"""
import numpy as np

from oracle import correlators as oc
from oracle import ed
from oracle.operator import Lattice

BETA = 8.0


def _free(Nt):
    d = BETA / Nt
    lat = Lattice(2, 1, Nt, d)
    phi = np.zeros(lat.shape)
    return d, lat, oc.propagator_correlator(lat, phi, oc.GAMMA, t0s=[0, Nt // 2]), \
        oc.propagator_correlator(lat, phi, oc.M_POINT, t0s=[0, Nt // 2])


def test_free_energies_converge_quadratically_in_delta():
    errs = {}
    for Nt in (128, 256):
        d, lat, cg, cm = _free(Nt)
        errs[Nt] = (oc.fit_energy(cg, d, (0.2, 1.0)) - 3.0, oc.fit_energy(cm, d, (0.6, 2.0)) - 1.0)
    for k in range(2):
        assert abs(errs[256][k]) < 0.002
        assert 3.6 < errs[128][k] / errs[256][k] < 4.4, errs


def test_free_correlator_approaches_ed():
    d, lat, cg, cm = _free(256)
    e1, u1 = np.linalg.eigh(ed.hopping(2, 1, 1.0))
    taus = np.arange(1, lat.Nt) * d
    for C, k in ((cg, 3), (cm, 2)):
        exact = ed.thermal_correlator(2, 1, 1.0, 0.0, BETA, u1[:, k], taus)
        sel = taus <= 2.0
        assert np.max(np.abs(C[1:][sel] - exact[sel])) < 0.03


def test_fit_of_a_pure_exponential():
    tau = np.arange(64) * 0.125
    assert abs(oc.fit_energy(2.5 * np.exp(-1.7 * tau), 0.125, (0.2, 1.0)) - 1.7) < 1e-12


def test_time_translation_with_the_antiperiodic_wrap():
    lat = Lattice(2, 1, 16, 0.5)
    phi = np.random.default_rng(3).normal(0.0, 0.8, size=lat.shape)
    for v in (oc.GAMMA, oc.M_POINT):
        ref = oc.propagator_correlator(lat, phi, v, t0s=[0])
        for s in (3, 8, 13):
            got = oc.propagator_correlator(lat, np.roll(phi, s, axis=0), v, t0s=[s])
            np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)
