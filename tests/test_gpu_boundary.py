"""Boundary behaviour of the C ABI on the GPU.

* output buffers that overlap an input (the same start or a partial offset) are
  refused with HUB_ERR_ARG before anything runs, for the applies, the solve, the
  force and a served request;
* a non-finite value in phi, the right-hand side or the initial guess ends a solve
  with HUB_ERR_ARG and converged = 0, for both solvers, in a batch whose other
  systems still converge; a served request with such a phi finishes with that status;
* max_iter of the mixed solver limits the restart cycles exactly;
* hub_force_sum: sum_b scale_b dS_b/dphi against the oracle's forces (kernel parity
  on the same eta, <= 1e-13 relative to the largest entry) and, added to an existing
  field, against hub_force of each system.
"""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_1804_07195_amd import binding as hb
from tests.gpu_helpers import dev, host, lattices, rel_max

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hub():
    ctx = hb.Context(0)
    yield ctx
    ctx.close()


def _system(L=6, Nt=8, kt=0.3, seed=5, batch=2):
    hl, ol = lattices(L, L, Nt, kt)
    rng = np.random.default_rng(seed)
    phi = rng.normal(0.0, 0.8, size=ol.shape)
    eta = rng.standard_normal((batch,) + ol.shape) + 1j * rng.standard_normal((batch,) + ol.shape)
    chi = np.stack([oracle.apply_Mdag(ol, phi, eta[b]) for b in range(batch)])
    return hl, ol, phi, chi


def _raw_solve(hub, hl, phi_t, mu2, b_ptr, x_ptr, batch, opts):
    L = hb.load()
    mu = (hb.ctypes.c_double * batch)(*mu2)
    info = (hb.HubSolveInfo * batch)()
    st = L.hub_solve(hub.handle, hb.ctypes.byref(hl), phi_t.data_ptr(), mu, batch, b_ptr, x_ptr,
                     hb.ctypes.byref(opts), info, hb._stream(None))
    return st, [i.as_dict() for i in info]


def test_overlapping_outputs_are_refused(hub):
    hl, ol, phi, chi = _system()
    n = 2 * hl.L1 * hl.L2 * hl.Nt
    pd = dev(phi)
    buf = dev(np.concatenate([chi.reshape(-1), chi.reshape(-1)]))  # room for an offset overlap
    L = hb.load()
    s = hb._stream(None)
    base = buf.data_ptr()
    # applies: y == x, and y starting inside x
    for f in (L.hub_apply_M, L.hub_apply_Mdag):
        assert f(hub.handle, hb.ctypes.byref(hl), pd.data_ptr(), base, base, 1, s) == hb.HUB_ERR_ARG
        assert f(hub.handle, hb.ctypes.byref(hl), pd.data_ptr(), base, base + 16 * (n // 2), 1, s) == hb.HUB_ERR_ARG
    # solve: x == b, and x starting inside the second right-hand side
    for solver in ("cg", "fgmres"):
        o = hb.default_opts(solver=solver)
        st, _ = _raw_solve(hub, hl, pd, [0.0, 0.1], base, base, 2, o)
        assert st == hb.HUB_ERR_ARG
        st, _ = _raw_solve(hub, hl, pd, [0.0, 0.1], base, base + 16 * (n + 7), 2, o)
        assert st == hb.HUB_ERR_ARG
    assert "overlap" in L.hub_last_error().decode()
    # force: the output over eta
    assert L.hub_force(hub.handle, hb.ctypes.byref(hl), pd.data_ptr(), base, None, 1.0, 0, base, 1, s) == \
        hb.HUB_ERR_ARG
    # a served request whose x_out is its chi
    c1 = dev(chi[:1])
    with pytest.raises(hb.HubError) as e:
        hb.hub_submit(hub, hl, 0.0, pd, c1, x_out=c1)
    assert e.value.status == hb.HUB_ERR_ARG
    # the right-hand sides were not touched
    assert np.array_equal(host(buf)[:n], chi.reshape(-1)[:n])


@pytest.mark.parametrize("solver", ["cg", "fgmres"])
@pytest.mark.parametrize("where", ["phi", "b", "x0"])
def test_non_finite_input_is_an_argument_error(hub, solver, where):
    hl, ol, phi, chi = _system(seed=9)
    o = hb.default_opts(solver=solver)
    b = chi.copy()
    p = phi.copy()
    x0 = np.zeros_like(chi)
    if where == "phi":
        p[3, 1, 2, 4] = np.nan
    elif where == "b":
        b[0, 5, 0, 1, 1] = np.inf
    else:
        o.use_x0 = 1
        x0[1, 2, 1, 0, 3] = np.nan
    x = dev(x0)
    L = hb.load()
    bd = dev(b)
    st, info = _raw_solve(hub, hl, dev(p), [0.0, 0.05], bd.data_ptr(), x.data_ptr(), 2, o)
    assert st == hb.HUB_ERR_ARG, hb.STATUS_NAMES.get(st)
    assert "non-finite" in L.hub_last_error().decode()
    bad = [0, 1] if where == "phi" else [0] if where == "b" else [1]
    for k in range(2):
        if k in bad:
            assert info[k]["converged"] == 0, (k, info[k])
        else:
            # the other system of the batch is unaffected
            assert info[k]["converged"] == 1, (k, info[k])
            res = oracle.true_rel_residual(ol, p, [0.0, 0.05][k], b[k], host(x)[k])
            assert res <= 1e-10


def test_served_request_with_non_finite_phi(hub):
    hl, ol, phi, chi = _system(seed=13, batch=1)
    p = phi.copy()
    p[0, 0, 0, 0] = np.nan
    req = hb.hub_submit(hub, hl, 0.0, dev(p), dev(chi), opts=hb.default_opts(solver="fgmres"))
    good = hb.hub_submit(hub, hl, 0.0, dev(phi), dev(chi), opts=hb.default_opts(solver="fgmres"))
    t0 = time.time()
    res = {}
    while len(res) < 2:
        for name, r in (("bad", req), ("good", good)):
            if name not in res:
                done, info = hb.hub_poll(hub, r)
                if done:
                    res[name] = info
        assert time.time() - t0 < 60
        time.sleep(0.001)
    assert res["bad"]["status"] == hb.HUB_ERR_ARG and res["bad"]["converged"] == 0
    assert res["good"]["status"] == hb.HUB_OK and res["good"]["converged"] == 1


def test_fgmres_cycle_limit_is_exact(hub):
    hl, ol, phi, chi = _system(L=12, Nt=32, kt=0.25, seed=2, batch=1)
    # a loose inner floor makes the solve need several restart cycles
    o = hb.default_opts(solver="fgmres", inner_floor=0.1, restart_m=1)
    _, info_full, st = hb.hub_solve(hub, hl, dev(phi), [0.0], dev(chi), opts=o)
    assert st == hb.HUB_OK and info_full[0]["outer_iters"] > 2
    for cap in (1, 2):
        o.max_iter = cap
        _, info, st = hb.hub_solve(hub, hl, dev(phi), [0.0], dev(chi), opts=o, allow_noconv=True)
        assert st == hb.HUB_ERR_NOCONV and info[0]["outer_iters"] == cap and info[0]["converged"] == 0


@pytest.mark.parametrize("shape", [(6, 6, 8, 0.3), (5, 7, 3, 0.4), (48, 48, 16, 0.25)])
def test_force_sum_matches_oracle(hub, shape):
    hl, ol = lattices(*shape)
    rng = np.random.default_rng(21)
    batch = 3
    phi = rng.normal(0.0, 0.9, size=ol.shape)
    eta = rng.standard_normal((batch,) + ol.shape) + 1j * rng.standard_normal((batch,) + ol.shape)
    scale = [0.7, -1.3, 2.0]
    want = sum(scale[b] * oracle.force(ol, phi, eta[b]) for b in range(batch))
    got = host(hb.hub_force_sum(hub, hl, dev(phi), dev(eta), scale))
    assert rel_max(got, want) <= 1e-13
    # accumulate onto an existing field, with xi given
    pd, ed = dev(phi), dev(eta)
    xi = hb.hub_apply_Mdag(hub, hl, pd, ed)
    base = rng.standard_normal(ol.shape)
    out = dev(base)
    hb.hub_force_sum(hub, hl, pd, ed, scale, xi=xi, accumulate=True, out=out)
    per = [host(hb.hub_force(hub, hl, pd, ed[b:b + 1].contiguous(), scale=scale[b])) for b in range(batch)]
    assert rel_max(host(out), base + sum(p.reshape(ol.shape) for p in per)) <= 1e-13
