"""hub_apply_normal_noalloc against hub_apply_normal, through the C ABI, on the GPU.

The no-allocation variant runs the same kernels with M^dagger x in the library's
per-device scratch array instead of context workspace, so its output must equal
hub_apply_normal's bit for bit (and the oracle's within 1e-13 relative to the largest
entry).  Two calls in a row, the second with a smaller input, check that the scratch
left by the first call does not leak into the second; a call over the scratch size is
refused with HUB_ERR_ARG; the calls change neither the device's free memory nor the
context's workspace.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1804_07195_amd import binding as hb
from tests.gpu_helpers import dev, host, lattices, rel_max

pytestmark = pytest.mark.gpu


def _raw(fn, ctx, hl, pd, mu2, x, y):
    nb = len(mu2)
    mu = (ctypes.c_double * nb)(*mu2)
    return fn(ctx.handle, ctypes.byref(hl), pd.data_ptr(), mu, x.data_ptr(), y.data_ptr(), nb, hb._stream(None))


def test_noalloc_normal_matches_the_allocating_call():
    L = hb.load()
    ctx = hb.Context(0)
    try:
        rng = np.random.default_rng(77)
        cases = [((48, 48, 32, 0.25), [0.0, 0.05, 0.5]),   # 2 x 147,456 x 3 x 16 B = 7 MB of scratch
                 ((6, 7, 8, 0.3), [0.1])]                     # then a smaller one
        prepared = []
        for shape, mu2 in cases:
            hl, ol = lattices(*shape)
            phi = rng.normal(0.0, 0.9, size=ol.shape)
            x = rng.standard_normal((len(mu2),) + ol.shape) + 1j * rng.standard_normal((len(mu2),) + ol.shape)
            xd = dev(x)
            prepared.append((hl, ol, phi, x, mu2, dev(phi), xd, torch.full_like(xd, complex("nan"))))
        # a first call loads the kernels' code object (runtime memory, not the call's)
        warm = torch.empty_like(prepared[1][6])
        assert _raw(L.hub_apply_normal_noalloc, ctx, *[prepared[1][k] for k in (0, 5)], prepared[1][4],
                    prepared[1][6], warm) == hb.HUB_OK
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for hl, ol, phi, x, mu2, pd, xd, y in prepared:
            assert _raw(L.hub_apply_normal_noalloc, ctx, hl, pd, mu2, xd, y) == hb.HUB_OK
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0   # nothing was allocated
        for hl, ol, phi, x, mu2, pd, xd, y in prepared:
            got = host(y)
            ref = torch.empty_like(xd)
            assert _raw(L.hub_apply_normal, ctx, hl, pd, mu2, xd, ref) == hb.HUB_OK
            assert np.array_equal(got, host(ref))
            for b in range(len(mu2)):
                assert rel_max(got[b], oracle.normal_apply(ol, phi, mu2[b], x[b])) <= 1e-13
    finally:
        ctx.close()


def test_noalloc_refuses_inputs_beyond_the_scratch():
    L = hb.load()
    ctx = hb.Context(0)
    try:
        hl, ol = lattices(102, 102, 64, 0.1875)          # 1,331,712 sites: 21.3 MB per vector
        pd = torch.zeros(ol.shape, dtype=torch.float64, device="cuda")
        x = torch.zeros((4,) + ol.shape, dtype=torch.complex128, device="cuda")
        y = torch.empty_like(x)
        assert _raw(L.hub_apply_normal_noalloc, ctx, hl, pd, [0.0] * 4, x, y) == hb.HUB_ERR_ARG
        assert "HUB_NOALLOC_SCRATCH_BYTES" in L.hub_last_error().decode()
        # a batch of 3 fits (63.9 MB)
        assert _raw(L.hub_apply_normal_noalloc, ctx, hl, pd, [0.0] * 3, x[:3], y[:3]) == hb.HUB_OK
        torch.cuda.synchronize()
    finally:
        ctx.close()
