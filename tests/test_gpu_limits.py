"""The C ABI at its limits, against the oracle (GPU).

* HUB_MAX_BATCH systems in one call: M, M^dagger and M M^dagger + mu^2 applies, the
  force, and solves with both solvers (a different shift per system) match the
  oracle system by system; one system more is refused with HUB_ERR_ARG;
* the restart lengths m = 1 and m = HUB_MAX_RESTART still reach the tolerance;
* degenerate lattices (one unit cell, one or two time slices: the bonds and the two
  temporal hops of a site coincide) solve to the tolerance with both solvers and
  give the oracle's solution;
* mixed solves at the single-workgroup inner CG's size limit (10,200 sites, even and
  odd L2), one size past it, and on the smallest even-L2 lattices reach the tolerance;
* a batch of zero systems and a zero lattice extent are refused by the C ABI, and a
  zero right-hand side gives x = 0 without iterating;
* two host threads solving on one context, each on its own stream, get the results
  of the same solves made alone, bit for bit.

Bars as in the other parity tests: applies and force <= 1e-13 relative to
max(1, max|y|); solves: the oracle's recomputed true residual <= 1e-10 and the
solution within 1e-6 of the oracle's dense LU solution.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle.operator import NormalOperator, build_M
from paper_1804_07195_amd import binding as hb
from tests.gpu_helpers import dev, host, lattices, rel2, rel_max

pytestmark = pytest.mark.gpu

MAXB = 64  # HUB_MAX_BATCH of include/hub.h


@pytest.fixture(scope="module")
def hub():
    ctx = hb.Context(0)
    yield ctx
    ctx.close()


def _inputs(ol, batch, seed, scale=0.8):
    rng = np.random.default_rng(seed)
    phi = rng.normal(0.0, scale, size=ol.shape)
    x = rng.standard_normal((batch,) + ol.shape) + 1j * rng.standard_normal((batch,) + ol.shape)
    return phi, x


def test_applies_and_force_at_the_batch_limit(hub):
    hl, ol = lattices(12, 12, 16, 0.25, 0.05)
    phi, x = _inputs(ol, MAXB, 1)
    M = build_M(ol, phi)
    pd, xd = dev(phi), dev(x)
    mu2 = [0.01 * k for k in range(MAXB)]
    y = host(hb.hub_apply_M(hub, hl, pd, xd))
    yd = host(hb.hub_apply_Mdag(hub, hl, pd, xd))
    yn = host(hb.hub_apply_normal(hub, hl, pd, mu2, xd))
    F = host(hb.hub_force(hub, hl, pd, xd))
    for b in range(MAXB):
        assert rel_max(y[b], oracle.apply_M(ol, phi, x[b], M=M)) <= 1e-13
        assert rel_max(yd[b], oracle.apply_Mdag(ol, phi, x[b], M=M)) <= 1e-13
        want_n = NormalOperator(ol, phi, mu2[b], M=M)(x[b].ravel()).reshape(ol.shape)
        assert rel_max(yn[b], want_n) <= 1e-13
        assert rel_max(F[b], oracle.force(ol, phi, x[b])) <= 1e-13


def test_one_system_beyond_the_batch_limit_is_refused(hub):
    hl, ol = lattices(3, 3, 8, 0.5)
    phi = dev(np.zeros(ol.shape))
    x = dev(np.ones((MAXB + 1,) + ol.shape, complex))
    with pytest.raises(hb.HubError):
        hb.hub_apply_M(hub, hl, phi, x)
    with pytest.raises(hb.HubError):
        hb.hub_solve(hub, hl, phi, [0.1] * (MAXB + 1), x)
    with pytest.raises(hb.HubError):
        hb.hub_force(hub, hl, phi, x)


@pytest.mark.parametrize("solver", ["cg", "fgmres"])
def test_solve_at_the_batch_limit(hub, solver):
    hl, ol = lattices(6, 6, 8, 0.5)
    phi, eta = _inputs(ol, MAXB, 2, scale=1.0)
    pd = dev(phi)
    chi = hb.hub_apply_Mdag(hub, hl, pd, dev(eta))
    ch = host(chi)
    mu2 = [0.0 if b % 8 == 0 else 0.005 * b for b in range(MAXB)]
    x, info, st = hb.hub_solve(hub, hl, pd, mu2, chi, opts=hb.default_opts(solver=solver))
    assert st == hb.HUB_OK
    xs = host(x)
    M = build_M(ol, phi)
    for b in range(MAXB):
        A = NormalOperator(ol, phi, mu2[b], M=M)
        assert info[b]["converged"] == 1
        assert oracle.true_rel_residual(ol, phi, mu2[b], ch[b], xs[b], A=A) <= 1e-10
        want = np.linalg.solve(A.dense(), ch[b].ravel())
        assert rel2(xs[b].ravel(), want) <= 1e-6


@pytest.mark.parametrize("m", [1, 20])
def test_restart_length_limits(hub, m):
    hl, ol = lattices(12, 12, 16, 0.25)
    phi, eta = _inputs(ol, 2, 3, scale=0.9)
    pd = dev(phi)
    chi = hb.hub_apply_Mdag(hub, hl, pd, dev(eta))
    ch = host(chi)
    mu2 = [0.0, 0.05]
    x, info, st = hb.hub_solve(hub, hl, pd, mu2, chi, opts=hb.default_opts(solver="fgmres", restart_m=m))
    assert st == hb.HUB_OK
    xs = host(x)
    for b in range(2):
        assert oracle.true_rel_residual(ol, phi, mu2[b], ch[b], xs[b]) <= 1e-10
    with pytest.raises(hb.HubError):
        hb.hub_solve(hub, hl, pd, mu2, chi, opts=hb.default_opts(solver="fgmres", restart_m=21))


DEGENERATE = [(1, 1, 1, 0.4, 0.0), (1, 1, 2, 0.4, 0.1), (1, 1, 3, 0.3, 0.0), (2, 1, 1, 0.5, 0.0), (1, 3, 2, 0.2, 0.05)]


@pytest.mark.parametrize("shape", DEGENERATE, ids=[f"{a}x{b}x{c}" for a, b, c, _, _ in DEGENERATE])
@pytest.mark.parametrize("solver", ["cg", "fgmres"])
def test_degenerate_lattices_solve(hub, shape, solver):
    hl, ol = lattices(*shape)
    phi, eta = _inputs(ol, 3, 4, scale=0.7)
    pd = dev(phi)
    chi = hb.hub_apply_Mdag(hub, hl, pd, dev(eta))
    ch = host(chi)
    mu2 = [0.1, 0.5, 1.0]
    x, info, st = hb.hub_solve(hub, hl, pd, mu2, chi, opts=hb.default_opts(solver=solver))
    assert st == hb.HUB_OK
    xs = host(x)
    for b in range(3):
        A = NormalOperator(ol, phi, mu2[b])
        assert np.all(np.isfinite(xs[b]))
        assert oracle.true_rel_residual(ol, phi, mu2[b], ch[b], xs[b], A=A) <= 1e-10
        want = np.linalg.solve(A.dense(), ch[b].ravel())
        assert rel2(xs[b].ravel(), want) <= 1e-6


# The complex64 inner CG of a mixed solve runs on one workgroup for systems of at most
# 10,200 sites: site pairs for even L2, single sites for odd L2; larger systems take the
# tiled kernels.  Both forms at the limit, the first size past it, and the smallest
# even-L2 lattices (L2 = 2: every j-bond wraps).
WG_EDGE = [(10, 10, 51, 0.25, 0.05), (12, 17, 25, 0.25, 0.05), (10, 10, 52, 0.25, 0.05),
           (1, 2, 3, 0.4, 0.1), (3, 2, 5, 0.3, 0.0)]


@pytest.mark.parametrize("shape", WG_EDGE, ids=[f"{a}x{b}x{c}" for a, b, c, _, _ in WG_EDGE])
def test_single_workgroup_size_edges(hub, shape):
    hl, ol = lattices(*shape)
    phi, eta = _inputs(ol, 2, 9, scale=0.7)
    pd = dev(phi)
    chi = hb.hub_apply_Mdag(hub, hl, pd, dev(eta))
    ch = host(chi)
    mu2 = [0.05, 0.0]
    x, info, st = hb.hub_solve(hub, hl, pd, mu2, chi, opts=hb.default_opts(solver="fgmres"))
    assert st == hb.HUB_OK
    xs = host(x)
    for b in range(2):
        assert info[b]["converged"] == 1 and info[b]["inner_iters"] > 0
        assert np.all(np.isfinite(xs[b]))
        assert oracle.true_rel_residual(ol, phi, mu2[b], ch[b], xs[b]) <= 1e-10
        if ol.n <= 64:
            A = NormalOperator(ol, phi, mu2[b])
            assert rel2(xs[b].ravel(), np.linalg.solve(A.dense(), ch[b].ravel())) <= 1e-6


def test_empty_and_zero_inputs(hub):
    """A batch of zero systems and a lattice with a zero extent are refused by the C ABI
    itself (HUB_ERR_ARG) before anything is enqueued; an all-zero right-hand side solves
    to x = 0 without iterating."""
    import ctypes
    lib = hb.load()
    hl, ol = lattices(3, 3, 8, 0.5)
    phi = dev(np.zeros(ol.shape))
    x = dev(np.ones((1,) + ol.shape, complex))
    y = torch.empty_like(x)
    for batch in (0, -1):
        assert lib.hub_apply_M(hub.handle, ctypes.byref(hl), phi.data_ptr(), x.data_ptr(), y.data_ptr(), batch,
                               None) == hb.HUB_ERR_ARG
        o = hb.default_opts()
        info = (hb.HubSolveInfo * 1)()
        mu = (ctypes.c_double * 1)(0.1)
        assert lib.hub_solve(hub.handle, ctypes.byref(hl), phi.data_ptr(), mu, batch, x.data_ptr(), y.data_ptr(),
                             ctypes.byref(o), info, None) == hb.HUB_ERR_ARG
    flat = hb.lattice(3, 3, 8, 0.5)
    flat.Nt = 0
    assert lib.hub_apply_M(hub.handle, ctypes.byref(flat), phi.data_ptr(), x.data_ptr(), y.data_ptr(), 1,
                           None) == hb.HUB_ERR_ARG
    for solver in ("cg", "fgmres"):
        z = dev(np.zeros((2,) + ol.shape, complex))
        xs, infos, st = hb.hub_solve(hub, hl, dev(np.random.default_rng(1).normal(size=ol.shape)), [0.0, 0.3], z,
                                     opts=hb.default_opts(solver=solver))
        assert st == hb.HUB_OK and torch.count_nonzero(xs) == 0
        assert all(i["converged"] == 1 and i["inner_iters"] == 0 for i in infos)


def test_concurrent_host_threads_on_one_context(hub):
    """Two host threads solving on one context, each on its own stream (the context
    serialises its synchronous calls): every result is bit-identical to the same solve
    made alone."""
    import threading
    hl, ol = lattices(12, 12, 16, 0.25)
    jobs = []
    for seed in range(4):
        phi, eta = _inputs(ol, 2, 50 + seed, scale=0.9)
        pd = dev(phi)
        jobs.append((pd, hb.hub_apply_Mdag(hub, hl, pd, dev(eta)), "cg" if seed % 2 else "fgmres"))
    alone = [host(hb.hub_solve(hub, hl, pd, [0.0, 0.1], chi, opts=hb.default_opts(solver=sv))[0])
             for pd, chi, sv in jobs]
    got, errors = {}, []

    def work(k0):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for k in range(k0, len(jobs), 2):
                    pd, chi, sv = jobs[k]
                    x, _, _ = hb.hub_solve(hub, hl, pd, [0.0, 0.1], chi, opts=hb.default_opts(solver=sv), stream=s)
                    s.synchronize()
                    got[k] = x.cpu().numpy()
        except Exception as e:  # reported below
            errors.append(e)

    ts = [threading.Thread(target=work, args=(k0,)) for k0 in (0, 1)]
    for t in ts:
        t.start()
    for t in ts:
        t.join(timeout=120)
    assert not errors and len(got) == len(jobs)
    for k in range(len(jobs)):
        assert np.array_equal(got[k], alone[k]), k
