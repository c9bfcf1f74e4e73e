"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Bars (floating point, FP64 results):
* operator applies (M, M^dagger, M M^dagger + mu^2): element-wise max error
  <= 1e-13 relative to max(1, max|y|) - only the rounding order differs;
* solves: the oracle's own recomputed true residual ||b - A x|| / ||b|| <= tol
  (tol = 1e-10, the target of the solve), and ||x - x*|| / ||x*|| <= 1e-6 where the
  oracle's x* is available (error <= cond(A) * residual, cond <= ~4.5e3 here);
* force: kernel-only parity on the same eta, xi <= 1e-13; end to end vs the oracle's
  force <= 1e-8 (2-norm relative); central differences of S <= 1e-6 relative.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle.operator import NormalOperator, build_M
from paper_1804_07195_amd import binding as hb
from tests.gpu_helpers import dev, host, lattices, of_workload, rel2, rel_max
from workloads import WORKLOADS, draw_inputs

pytestmark = pytest.mark.gpu

SHAPES = [
    (3, 3, 8, 0.5, 0.0),
    (2, 2, 4, 0.3, 0.0),
    (5, 7, 3, 0.4, 0.15),
    (1, 1, 3, 0.4, 0.1),
    (2, 2, 1, 0.25, 0.0),
    (12, 12, 32, 0.25, 0.0),
    (33, 17, 6, 0.2, 0.05),
]
SID = [f"{a}x{b}x{c}" for a, b, c, _, _ in SHAPES]


@pytest.fixture(scope="module")
def hub():
    ctx = hb.Context(0)
    yield ctx
    ctx.close()


def _rand(rng, lat, batch):
    phi = rng.normal(0, 1.0, size=lat.shape)
    x = rng.standard_normal((batch,) + lat.shape) + 1j * rng.standard_normal((batch,) + lat.shape)
    return phi, x


@pytest.mark.parametrize("shape", SHAPES, ids=SID)
@pytest.mark.parametrize("batch", [1, 3])
def test_apply_M_and_Mdag_match_oracle(hub, shape, batch):
    hl, ol = lattices(*shape)
    rng = np.random.default_rng(100 + batch)
    phi, x = _rand(rng, ol, batch)
    M = build_M(ol, phi)
    y = host(hb.hub_apply_M(hub, hl, dev(phi), dev(x)))
    yd = host(hb.hub_apply_Mdag(hub, hl, dev(phi), dev(x)))
    want = oracle.apply_M(ol, phi, x, M=M)
    wantd = oracle.apply_Mdag(ol, phi, x, M=M)
    assert rel_max(y, want) <= 1e-13
    assert rel_max(yd, wantd) <= 1e-13


@pytest.mark.parametrize("shape", SHAPES, ids=SID)
def test_apply_normal_matches_oracle(hub, shape):
    hl, ol = lattices(*shape)
    rng = np.random.default_rng(7)
    phi, x = _rand(rng, ol, 3)
    mu2 = [0.0, 0.05, 0.5]
    y = host(hb.hub_apply_normal(hub, hl, dev(phi), mu2, dev(x)))
    for b in range(3):
        want = oracle.normal_apply(ol, phi, mu2[b], x[b])
        assert rel_max(y[b], want) <= 1e-13


def test_apply_full_size_against_oracle_and_adjoint(hub):
    w = WORKLOADS["large2"]
    hl, ol = of_workload(w)
    phi, eta = draw_inputs(w)
    M = build_M(ol, phi)
    pd = dev(phi)
    u, v = dev(eta[0]), dev(eta[1])
    Mv = host(hb.hub_apply_M(hub, hl, pd, v))
    Mdu = host(hb.hub_apply_Mdag(hub, hl, pd, u))
    assert rel_max(Mv, oracle.apply_M(ol, phi, eta[1], M=M)) <= 1e-13
    assert rel_max(Mdu, oracle.apply_Mdag(ol, phi, eta[0], M=M)) <= 1e-13
    lhs = np.vdot(eta[0].ravel(), Mv.ravel())
    rhs = np.vdot(Mdu.ravel(), eta[1].ravel())
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs) + 1e-9


def test_free_field_plane_wave_full_size(hub):
    """phi = 0 at 102x102x64: M on a plane wave is the closed-form 2x2 symbol."""
    w = WORKLOADS["large2"]
    hl, ol = of_workload(w)
    n1, n2, n = 17, 34, 5
    th1, th2, om = 2 * math.pi * n1 / w.L1, 2 * math.pi * n2 / w.L2, math.pi * (2 * n + 1) / w.Nt
    t, i, j = np.meshgrid(np.arange(w.Nt), np.arange(w.L1), np.arange(w.L2), indexing="ij")
    ph = np.exp(1j * (th1 * i + th2 * j + om * t))
    uA, uB = 0.3 - 0.7j, 1.1 + 0.2j
    psi = np.zeros(ol.shape, complex)
    psi[:, 0], psi[:, 1] = uA * ph, uB * ph
    a = np.exp(-1j * om) - 1
    f = 1 + np.exp(-1j * th1) + np.exp(-1j * th2)
    k = w.kappa_t
    want = np.zeros_like(psi)
    want[:, 0] = (a * uA - k * f * uB) * ph
    want[:, 1] = (-k * np.conj(f) * uA - np.conj(a) * uB) * ph
    got = host(hb.hub_apply_M(hub, hl, dev(np.zeros(ol.shape)), dev(psi)))
    assert np.abs(got - want).max() <= 1e-12


@pytest.mark.parametrize("solver", ["cg", "fgmres"])
def test_free_field_solve_full_size_closed_form(hub, solver):
    """phi = 0 at 102x102x64: a sum of five plane waves is solved exactly by
    x = sum_k b_k / (|a_k|^2 + kappa~^2 |f_k|^2 + mu^2) (each plane wave spans an
    eigenspace of M M^dagger), for two shifts in one batch; no oracle solve."""
    w = WORKLOADS["large2"]
    hl, ol = of_workload(w)
    t, i, j = np.meshgrid(np.arange(w.Nt), np.arange(w.L1), np.arange(w.L2), indexing="ij")
    rng = np.random.default_rng(77)
    k = w.kappa_t
    b = np.zeros(ol.shape, complex)
    parts = []
    for (n1, n2, n) in ((0, 0, 0), (17, 34, 5), (3, 90, 31), (51, 51, 12), (34, 68, 63)):
        th1, th2, om = 2 * math.pi * n1 / w.L1, 2 * math.pi * n2 / w.L2, math.pi * (2 * n + 1) / w.Nt
        ph = np.exp(1j * (th1 * i + th2 * j + om * t))
        uA, uB = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        psi = np.zeros(ol.shape, complex)
        psi[:, 0], psi[:, 1] = uA * ph, uB * ph
        a = np.exp(-1j * om) - 1
        f = 1 + np.exp(-1j * th1) + np.exp(-1j * th2)
        parts.append((psi, abs(a) ** 2 + k * k * abs(f) ** 2))
        b += psi
    mu2 = [0.0, 0.1]
    x, info, st = hb.hub_solve(hub, hl, dev(np.zeros(ol.shape)), mu2, dev(np.stack([b, b])),
                               opts=hb.default_opts(solver=solver))
    assert st == hb.HUB_OK
    xs = host(x)
    for q, m in enumerate(mu2):
        want = sum(psi / (lam + m) for psi, lam in parts)
        assert rel2(xs[q], want) <= 1e-9, (q, rel2(xs[q], want))


def test_gauge_covariance_full_size(hub):
    """Time-dependent gauge transformation at 102x102x64 (pinned in the oracle):
    phi'_{A,t} = phi_{A,t} + al_t - al_{t-1}, phi'_{B,t} = phi_{B,t} + al_{t+1} - al_t
    gives M[phi'] = D M[phi] D^dagger with D = diag(e^{i al_t}), so chi' = D chi solves
    to x' = D x, with the same action and the same force."""
    w = WORKLOADS["large2"]
    hl, ol = of_workload(w)
    phi, eta = draw_inputs(w, batch=1)
    rng = np.random.default_rng(91)
    al = rng.normal(0.0, 1.5, size=w.Nt)
    phi2 = phi.copy()
    phi2[:, 0] += (al - np.roll(al, 1))[:, None, None]
    phi2[:, 1] += (np.roll(al, -1) - al)[:, None, None]
    d = np.exp(1j * al)[:, None, None, None]
    pd, pd2 = dev(phi), dev(phi2)
    chi = hb.hub_apply_Mdag(hub, hl, pd, dev(eta))
    chi2 = dev(host(chi) * d[None])
    opts = hb.default_opts(solver="fgmres")
    x, _, st = hb.hub_solve(hub, hl, pd, [0.1], chi, opts=opts)
    x2, _, st2 = hb.hub_solve(hub, hl, pd2, [0.1], chi2, opts=opts)
    assert st == st2 == hb.HUB_OK
    assert rel2(host(x2), host(x) * d[None]) <= 1e-8
    S = hb.hub_action(hub, hl, chi, x)[0]
    S2 = hb.hub_action(hub, hl, chi2, x2)[0]
    assert abs(S2 - S) <= 1e-9 * abs(S)
    F = host(hb.hub_force(hub, hl, pd, x))
    F2 = host(hb.hub_force(hub, hl, pd2, x2))
    assert rel2(F2, F) <= 1e-7


@pytest.mark.parametrize("solver", ["cg", "fgmres"])
def test_solve_tiny(hub, solver):
    w = WORKLOADS["tiny"]
    hl, ol = of_workload(w)
    phi, eta = draw_inputs(w)
    chi = oracle.apply_Mdag(ol, phi, eta[0])
    x, info, st = hb.hub_solve(hub, hl, dev(phi), [0.0], dev(chi), opts=hb.default_opts(solver=solver, tol=1e-12))
    x = host(x)
    assert info[0]["converged"] == 1
    assert oracle.true_rel_residual(ol, phi, 0.0, chi, x) <= 1e-12
    xs, _ = oracle.solve(ol, phi, 0.0, chi)
    assert rel2(x, xs) <= 1e-8


@pytest.mark.parametrize("solver", ["cg", "fgmres"])
def test_solve_sixteen_rhs(hub, solver):
    w = WORKLOADS["small16"]
    hl, ol = of_workload(w)
    phi, eta = draw_inputs(w)
    chi = oracle.apply_Mdag(ol, phi, eta)
    x, info, st = hb.hub_solve(hub, hl, dev(phi), [0.0] * 16, dev(chi), opts=hb.default_opts(solver=solver))
    x = host(x)
    A = NormalOperator(ol, phi, 0.0)
    for b in range(16):
        assert info[b]["converged"] == 1
        res = oracle.true_rel_residual(ol, phi, 0.0, chi[b], x[b], A=A)
        assert res <= 1e-10, (b, res)
        assert abs(res - info[b]["true_rel_resid"]) <= 1e-12
    for b in (0, 7, 15):
        xs, _ = oracle.solve(ol, phi, 0.0, chi[b], A=A)
        assert rel2(x[b], xs) <= 1e-6


@pytest.mark.parametrize("solver", ["cg", "fgmres"])
def test_solve_three_shifts_one_launch(hub, solver):
    w = WORKLOADS["medium3"]
    hl, ol = of_workload(w)
    phi, eta = draw_inputs(w)
    chi = oracle.apply_Mdag(ol, phi, eta)
    mu2 = list(w.mu2)
    x, info, st = hb.hub_solve(hub, hl, dev(phi), mu2, dev(chi), opts=hb.default_opts(solver=solver))
    x = host(x)
    for b in range(3):
        assert info[b]["converged"] == 1
        assert oracle.true_rel_residual(ol, phi, mu2[b], chi[b], x[b]) <= 1e-10
    xs, _ = oracle.solve(ol, phi, mu2[0], chi[0])
    assert rel2(x[0], xs) <= 1e-8


@pytest.mark.parametrize("solver", ["cg", "fgmres"])
def test_solve_full_size(hub, solver):
    w = WORKLOADS["large2"]
    hl, ol = of_workload(w)
    phi, eta = draw_inputs(w)
    M = build_M(ol, phi)
    chi = oracle.apply_Mdag(ol, phi, eta, M=M)
    x, info, st = hb.hub_solve(hub, hl, dev(phi), list(w.mu2), dev(chi), opts=hb.default_opts(solver=solver))
    x = host(x)
    for b, mu2 in enumerate(w.mu2):
        assert info[b]["converged"] == 1
        assert oracle.true_rel_residual(ol, phi, mu2, chi[b], x[b], A=NormalOperator(ol, phi, mu2, M=M)) <= 1e-10


def test_heatbath_source_full_size(hub):
    """chi = M rho, mu^2 = 0: M^dagger (M M^dagger)^{-1} M rho = rho exactly."""
    w = WORKLOADS["large2"]
    hl, ol = of_workload(w)
    phi, rho = draw_inputs(w, batch=1)
    pd = dev(phi)
    chi = hb.hub_apply_M(hub, hl, pd, dev(rho[0]))
    x, info, _ = hb.hub_solve(hub, hl, pd, [0.0], chi, opts=hb.default_opts(solver="fgmres"))
    xi = host(hb.hub_apply_Mdag(hub, hl, pd, x))
    assert rel2(xi, rho[0]) <= 1e-6
    S = hb.hub_action(hub, hl, chi, x)[0]
    assert abs(S - np.vdot(rho[0], rho[0]).real) <= 1e-8 * abs(S)


@pytest.mark.parametrize("shape", SHAPES, ids=SID)
def test_force_kernel_parity(hub, shape):
    hl, ol = lattices(*shape)
    rng = np.random.default_rng(3)
    phi, eta = _rand(rng, ol, 2)
    xi = rng.standard_normal(eta.shape) + 1j * rng.standard_normal(eta.shape)
    F = host(hb.hub_force(hub, hl, dev(phi), dev(eta), dev(xi)))
    want = oracle.force(ol, phi, eta, xi)
    assert rel_max(F, want) <= 1e-13
    # xi computed internally, scaled and accumulated
    base = rng.standard_normal(eta.shape)
    F2 = host(hb.hub_force(hub, hl, dev(phi), dev(eta), None, scale=-0.5, accumulate=True, out=dev(base)))
    want2 = base - 0.5 * oracle.force(ol, phi, eta)
    assert rel_max(F2, want2) <= 1e-13


def test_action_matches_oracle(hub):
    w = WORKLOADS["small16"]
    hl, ol = of_workload(w)
    phi, eta = draw_inputs(w)
    rng = np.random.default_rng(4)
    chi = rng.standard_normal(eta.shape) + 1j * rng.standard_normal(eta.shape)
    S = hb.hub_action(hub, hl, dev(chi), dev(eta))
    want = oracle.action(chi, eta)
    np.testing.assert_allclose(S, want, rtol=1e-13)


def test_force_end_to_end_and_autograd(hub):
    """Autograd adjoint at 48x48x64 vs the oracle force with the oracle's own solve."""
    w = WORKLOADS["medium3"]
    hl, ol = of_workload(w)
    phi, eta = draw_inputs(w)
    chi = oracle.apply_Mdag(ol, phi, eta[0])
    mu2 = 0.5
    pd = dev(phi).requires_grad_(True)
    S = hb.PseudofermionAction.apply(pd, dev(chi), [mu2], hub, hl, hb.default_opts(solver="fgmres"))
    S.sum().backward()
    F = host(pd.grad)
    xs, _ = oracle.solve(ol, phi, mu2, chi)
    want = oracle.force(ol, phi, xs)
    assert rel2(F, want) <= 1e-8
    s0 = float(S.detach()[0])
    assert abs(s0 - oracle.action(chi, xs)) <= 1e-9 * abs(s0)


def test_force_central_differences(hub):
    """dS/dphi at 64 random sites of 48x48x64 vs (S(phi+h) - S(phi-h)) / 2h, h = 1e-6, with
    S(+) - S(-) = x+^dagger (A- - A+) x- from GPU solves (free of cancellation)."""
    w = WORKLOADS["medium3"]
    hl, ol = of_workload(w)
    phi, eta = draw_inputs(w)
    mu2 = 0.0
    pd0 = dev(phi)
    chi = hb.hub_apply_Mdag(hub, hl, pd0, dev(eta[0]))
    pd = pd0.clone().requires_grad_(True)
    S = hb.PseudofermionAction.apply(pd, chi, [mu2], hub, hl, hb.default_opts(solver="cg", tol=1e-12))
    S.sum().backward()
    F = host(pd.grad).ravel()
    rng = np.random.default_rng(64)
    h = 1e-6
    opts = hb.default_opts(solver="cg", tol=1e-12)
    errs = []
    for k in rng.choice(ol.n, size=64, replace=False):
        pp = phi.copy().ravel(); pp[k] += h
        pm = phi.copy().ravel(); pm[k] -= h
        pp, pm = dev(pp.reshape(ol.shape)), dev(pm.reshape(ol.shape))
        xp, _, _ = hb.hub_solve(hub, hl, pp, [mu2], chi, opts=opts)
        xm, _, _ = hb.hub_solve(hub, hl, pm, [mu2], chi, opts=opts)
        d = hb.hub_apply_normal(hub, hl, pm, [mu2], xm) - hb.hub_apply_normal(hub, hl, pp, [mu2], xm)
        dS = torch.vdot(xp.ravel(), d.ravel()).real.item()
        errs.append(abs(dS / (2 * h) - F[k]))
    assert max(errs) <= 1e-6 * np.abs(F).max(), max(errs)


def test_batch_invariance_bitwise(hub):
    """A system's result does not depend on the other systems of its launch."""
    w = WORKLOADS["small16"]
    hl, ol = of_workload(w)
    phi, eta = draw_inputs(w)
    pd = dev(phi)
    chi = hb.hub_apply_Mdag(hub, hl, pd, dev(eta))
    for solver in ("cg", "fgmres"):
        o = hb.default_opts(solver=solver)
        xall, _, _ = hb.hub_solve(hub, hl, pd, [0.0] * 4 + [0.3] * 12, chi, opts=o)
        x0, _, _ = hb.hub_solve(hub, hl, pd, [0.0], chi[0].contiguous(), opts=o)
        x5, _, _ = hb.hub_solve(hub, hl, pd, [0.3], chi[5].contiguous(), opts=o)
        assert torch.equal(xall[0], x0)
        assert torch.equal(xall[5], x5)


def test_zero_rhs_and_warm_start(hub):
    w = WORKLOADS["small16"]
    hl, ol = of_workload(w)
    phi, eta = draw_inputs(w, batch=2)
    pd = dev(phi)
    b = torch.zeros((2,) + ol.shape, dtype=torch.complex128, device="cuda")
    for solver in ("cg", "fgmres"):
        x, info, _ = hb.hub_solve(hub, hl, pd, [0.0, 0.1], b, opts=hb.default_opts(solver=solver))
        assert torch.count_nonzero(x).item() == 0
        assert all(i["converged"] == 1 for i in info)
    chi = hb.hub_apply_Mdag(hub, hl, pd, dev(eta))
    for solver in ("cg", "fgmres"):
        x, info, _ = hb.hub_solve(hub, hl, pd, [0.0, 0.1], chi, opts=hb.default_opts(solver=solver))
        x2, info2, _ = hb.hub_solve(hub, hl, pd, [0.0, 0.1], chi, x=x.clone(),
                                    opts=hb.default_opts(solver=solver, use_x0=1))
        for i in info2:
            assert i["converged"] == 1 and i["inner_iters"] <= 2


def test_iteration_limit_reports_noconv(hub):
    w = WORKLOADS["small16"]
    hl, ol = of_workload(w)
    phi, eta = draw_inputs(w, batch=1)
    pd = dev(phi)
    chi = hb.hub_apply_Mdag(hub, hl, pd, dev(eta))
    x, info, st = hb.hub_solve(hub, hl, pd, [0.0], chi, opts=hb.default_opts(max_iter=5), allow_noconv=True)
    assert st == hb.HUB_ERR_NOCONV and info[0]["converged"] == 0
    assert info[0]["inner_iters"] == 5


def test_argument_errors(hub):
    hl, ol = lattices(3, 3, 8, 0.5)
    phi = dev(np.zeros(ol.shape))
    x = dev(np.zeros((1,) + ol.shape, complex))
    with pytest.raises(hb.HubError):
        hb.hub_solve(hub, hl, phi, [-1.0], x)
    with pytest.raises(hb.HubError):
        hb.hub_solve(hub, hl, phi, [0.0], x, opts=hb.default_opts(restart_m=0))
    bad = hb.lattice(0, 3, 8, 0.5)
    with pytest.raises(ValueError):
        hb.hub_apply_M(hub, bad, phi, x)
