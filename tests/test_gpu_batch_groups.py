"""Batched public operators with the per-site phase shared by a group of vectors.

The public M, M^dagger, (M M^dagger + mu^2) and force kernels give a workgroup a
group of several vectors of the batch (phi, its phase and the site indices are
evaluated once per site for the group) once the lattice alone has enough
workgroups; small lattices keep one vector per workgroup.  On a 48x48x16 lattice a
batch of 15 takes the grouped kernels with groups of 2 and a last group of 1; every
vector is compared with the oracle element by element (bars as in the other
operator parity tests: 1e-13 relative to max(1, max|y|)).
"""
import numpy as np
import pytest

import oracle
from paper_1804_07195_amd import binding as hb
from tests.gpu_helpers import dev, host, lattices, rel_max

pytestmark = pytest.mark.gpu

SHAPE = (48, 48, 16, 0.3, 0.05)
BATCH = 15


@pytest.fixture(scope="module")
def hub():
    ctx = hb.Context(0)
    yield ctx
    ctx.close()


@pytest.fixture(scope="module")
def inputs():
    hl, ol = lattices(*SHAPE)
    rng = np.random.default_rng(21)
    phi = rng.normal(0.0, 1.0, size=ol.shape)
    x = rng.standard_normal((BATCH,) + ol.shape) + 1j * rng.standard_normal((BATCH,) + ol.shape)
    return hl, ol, phi, x, oracle.build_M(ol, phi)


def test_apply_M_and_Mdag_grouped(hub, inputs):
    hl, ol, phi, x, M = inputs
    y = host(hb.hub_apply_M(hub, hl, dev(phi), dev(x)))
    yd = host(hb.hub_apply_Mdag(hub, hl, dev(phi), dev(x)))
    want = oracle.apply_M(ol, phi, x, M=M)
    want_d = oracle.apply_Mdag(ol, phi, x, M=M)
    for b in range(BATCH):
        assert rel_max(y[b], want[b]) <= 1e-13
        assert rel_max(yd[b], want_d[b]) <= 1e-13


def test_apply_normal_grouped(hub, inputs):
    hl, ol, phi, x, M = inputs
    mu2 = [0.01 * b for b in range(BATCH)]
    y = host(hb.hub_apply_normal(hub, hl, dev(phi), mu2, dev(x)))
    for b in range(BATCH):
        assert rel_max(y[b], oracle.normal_apply(ol, phi, mu2[b], x[b])) <= 1e-13


def test_force_grouped(hub, inputs):
    hl, ol, phi, x, M = inputs
    rng = np.random.default_rng(22)
    xi = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
    F = host(hb.hub_force(hub, hl, dev(phi), dev(x), dev(xi)))
    want = oracle.force(ol, phi, x, xi)
    for b in range(BATCH):
        assert rel_max(F[b], want[b]) <= 1e-13


def test_solve_and_apply_over_several_fields(hub):
    """hub_solve_fields / hub_apply_fields: systems k of a batch use field k // per.  Three
    fields with two shifts each, both solvers: every solution meets the oracle's true
    residual on its own field, and M^dagger x_k matches the oracle's."""
    hl, ol = lattices(12, 12, 16, 0.25)
    rng = np.random.default_rng(61)
    phis = rng.normal(0.0, 0.8, size=(3,) + ol.shape)
    b = rng.standard_normal((6,) + ol.shape) + 1j * rng.standard_normal((6,) + ol.shape)
    mu2 = [0.0, 0.1] * 3
    for solver in ("cg", "fgmres"):
        x, info, st = hb.hub_solve_fields(hub, hl, dev(phis), mu2, dev(b), opts=hb.default_opts(solver=solver))
        assert st == hb.HUB_OK
        xs = host(x)
        for k in range(6):
            assert info[k]["converged"] == 1
            assert oracle.true_rel_residual(ol, phis[k // 2], mu2[k], b[k], xs[k]) <= 1e-10, (solver, k)
    y = host(hb.hub_apply_fields(hub, hl, dev(phis), dev(b), dag=True))
    for k in range(6):
        assert rel_max(y[k], oracle.apply_Mdag(ol, phis[k // 2], b[k])) <= 1e-13
