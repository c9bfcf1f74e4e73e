"""CG iterates and the mixed solver's iteration structure against the oracle.

The tiled solver kernels advance the solution every second CG iteration and complete
a pending step when a CG stops at an odd count; the single-workgroup kernel of small
systems advances it every iteration.  A final solve would hide a missing step (the
FP64 CG restarts from the true residual, FGMRES takes any preconditioner), so these
tests look at the iterates themselves:

* the FP64 CG stopped by its iteration cap after k steps returns the k-th
  Hestenes-Stiefel iterate of the oracle's textbook CG (k = 1 .. 7: both parities;
  single-workgroup systems, the 512-site tile class with one and several tiles and
  odd L2, and the 2048-site tile class);
* the mixed FGMRES solve takes exactly as many restart cycles as the method oracle
  of Algorithm A.1 (complex64 spCG emulated in numpy) and stays within two
  iterations per inner solve of its inner-iteration total (the two sides round the
  complex64 arithmetic differently, so a stop can move by an iteration).

Algorithm A.1 decides per Arnoldi step whether to run an inner solve by comparing
TOL a |b| / ERR with 1, and ERR depends on the error an inner solve left at its
stopping tolerance, which two complex64 implementations reproduce to a few percent
only.  The cases below are fields on which every decision of the oracle lies at
least 8% from 1, which the test checks; on them a change of branch or of the cycle
count means a real difference.  ERR is the least-squares residual of the cycle's
Arnoldi relation on both sides.
"""
import numpy as np
import pytest

import oracle
from oracle.operator import NormalOperator
from oracle.solve import cg as oracle_cg
from paper_1804_07195_amd import binding as hb
from tests.gpu_helpers import dev, host, lattices, rel2

pytestmark = pytest.mark.gpu

# single-workgroup CG (<= 20480 sites), then the 512-site tile class (several tiles, odd L2)
SHAPES = [(6, 6, 8, 0.3), (12, 12, 16, 0.25), (5, 7, 6, 0.3), (24, 24, 20, 0.25), (17, 33, 20, 0.3)]


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


STRUCT = [  # (L1, L2, N_t, kappa~, seed, mu^2)
    (9, 9, 16, 0.375, 11, 0.05),    # odd L2
    (7, 9, 16, 0.3, 15, 0.05),      # L1 != L2
    (10, 10, 16, 0.375, 12, 0.05),
    (12, 12, 16, 0.3, 17, 0.05),
    (12, 12, 32, 0.25, 17, 0.0),    # two cycles (the printed ERR product took 13 here)
    (24, 24, 20, 0.3, 31, 0.05),    # tiled kernels, even L2: complex64 site-pair path
    (17, 33, 20, 0.3, 33, 0.05),    # tiled kernels, odd L2: generic complex64 path
    (24, 24, 20, 0.25, 34, 0.0),    # tiled kernels, two cycles
]


@pytest.mark.parametrize("case", STRUCT, ids=[f"{a}x{b}x{c}-s{e}-mu{f}" for a, b, c, d, e, f in STRUCT])
def test_fgmres_structure_matches_method_oracle(hub, case):
    L1, L2, Nt, kt, seed, mu2 = case
    hl, ol = lattices(L1, L2, Nt, kt)
    rng = np.random.default_rng(seed)
    phi = rng.normal(0.0, np.sqrt(0.75), size=ol.shape)
    eta = rng.standard_normal(ol.shape) + 1j * rng.standard_normal(ol.shape)
    chi = oracle.apply_Mdag(ol, phi, eta)
    cycles = []
    _, ref = oracle.fgmres_alg_a1(ol, phi, mu2, chi, TOL=1e-10, record=cycles)
    ratios = np.array([r for c in cycles for r in c["ratio"] if r > 0])
    assert np.abs(np.log(ratios)).min() >= 0.08, "the case has a decision too close to the threshold"
    x, info, st = hb.hub_solve(hub, hl, dev(phi), [mu2], dev(chi[None]), opts=hb.default_opts(solver="fgmres"))
    assert st == hb.HUB_OK
    assert oracle.true_rel_residual(ol, phi, mu2, chi, host(x)[0]) <= 1e-10
    assert info[0]["outer_iters"] == ref["outer"], (info[0], ref)
    assert abs(info[0]["inner_iters"] - ref["inner_iters"]) <= 2 * ref["inner_solves"], (info[0], ref)


@pytest.mark.parametrize("k", [1, 2, 5, 6])
def test_fp64_cg_iterate_large_tiles(hub, k):
    """The same iterate check on a system of the 2048-site tile class (80x80x48 =
    614,400 sites, 300 tiles)."""
    hl, ol = lattices(80, 80, 48, 0.25)
    rng = np.random.default_rng(90)
    phi = rng.normal(0.0, 0.8, size=ol.shape)
    b = rng.standard_normal(ol.shape) + 1j * rng.standard_normal(ol.shape)
    mu2 = 0.05
    want, its, _ = oracle_cg(NormalOperator(ol, phi, mu2), b.ravel(), tol=0.0, maxiter=k)
    assert its == k
    x, info, st = hb.hub_solve(hub, hl, dev(phi), [mu2], dev(b[None]),
                               opts=hb.default_opts(solver="cg", max_iter=k), allow_noconv=True)
    assert st == hb.HUB_ERR_NOCONV and info[0]["inner_iters"] == k
    assert rel2(host(x)[0].ravel(), want) <= 1e-12
