"""CG iterates and the mixed solver's iteration structure against the oracle.

The solver kernels advance the solution every second CG iteration and complete a
pending step when a CG stops at an odd count; a final solve would hide a missing
step (the FP64 CG restarts from the true residual, FGMRES takes any preconditioner),
so these tests look at the iterates themselves:

* the FP64 CG stopped by its iteration cap after k steps returns the k-th
  Hestenes-Stiefel iterate of the oracle's textbook CG (k = 1 .. 7: both parities,
  one and several tiles, odd L2);
* the mixed FGMRES solve takes the same number of restart cycles as the method
  oracle of Algorithm A.1 (complex64 spCG emulated in numpy) and within two
  iterations per inner solve of its inner-iteration total (the two sides round the
  complex64 arithmetic differently, so a stop can move by an iteration).
"""
import numpy as np
import pytest

import oracle
from oracle.operator import NormalOperator
from oracle.solve import cg as oracle_cg
from paper_1804_07195_amd import binding as hb
from tests.gpu_helpers import dev, host, lattices, rel2

pytestmark = pytest.mark.gpu

SHAPES = [(6, 6, 8, 0.3), (12, 12, 16, 0.25), (5, 7, 6, 0.3)]


@pytest.fixture(scope="module")
def hub():
    ctx = hb.Context(0)
    yield ctx
    ctx.close()


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{a}x{b}x{c}" for a, b, c, _ in SHAPES])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7])
def test_fp64_cg_iterate_after_k_steps(hub, shape, k):
    hl, ol = lattices(*shape)
    rng = np.random.default_rng(40 + k)
    phi = rng.normal(0.0, 0.8, size=ol.shape)
    b = rng.standard_normal(ol.shape) + 1j * rng.standard_normal(ol.shape)
    mu2 = 0.05
    want, its, _ = oracle_cg(NormalOperator(ol, phi, mu2), b.ravel(), tol=0.0, maxiter=k)
    assert its == k
    x, info, st = hb.hub_solve(hub, hl, dev(phi), [mu2], dev(b[None]),
                               opts=hb.default_opts(solver="cg", max_iter=k), allow_noconv=True)
    assert st == hb.HUB_ERR_NOCONV and info[0]["inner_iters"] == k
    assert rel2(host(x)[0].ravel(), want) <= 1e-12


@pytest.mark.parametrize("mu2", [0.0, 0.05])
@pytest.mark.parametrize("shape", [(12, 12, 32, 0.25), (9, 9, 16, 0.375)], ids=["12x12x32", "9x9x16"])
def test_fgmres_structure_matches_method_oracle(hub, shape, mu2):
    hl, ol = lattices(*shape)
    rng = np.random.default_rng(11)
    phi = rng.normal(0.0, np.sqrt(0.75), size=ol.shape)
    eta = rng.standard_normal(ol.shape) + 1j * rng.standard_normal(ol.shape)
    chi = oracle.apply_Mdag(ol, phi, eta)
    _, ref = oracle.fgmres_alg_a1(ol, phi, mu2, chi, TOL=1e-10)
    x, info, st = hb.hub_solve(hub, hl, dev(phi), [mu2], dev(chi[None]), opts=hb.default_opts(solver="fgmres"))
    assert st == hb.HUB_OK
    assert oracle.true_rel_residual(ol, phi, mu2, chi, host(x)[0]) <= 1e-10
    assert info[0]["outer_iters"] == ref["outer"]
    assert abs(info[0]["inner_iters"] - ref["inner_iters"]) <= 2 * ref["inner_solves"]
