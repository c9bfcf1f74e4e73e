"""Benchmark of the fermion-matrix solve on one MI355X.

One step = the whole hot path on one batch of synthetic input at 102x102 cells,
N_t = 64 (N = 1,331,712 complex unknowns per system): two systems sharing one
Hubbard field phi with Hasenbusch shifts mu^2 = 0.1 and 0, right-hand sides
chi = M^dagger eta, solved to relative true residual 1e-10 by the mixed-precision
flexible GMRES(10) (complex64 CG preconditioner, FP64 outer loop), then the action
S = Re chi^dagger x and the force dS/dphi of both systems (summed).

Printed JSON (one line): solves/s over the timed steps, the roofline of the
dominant kernel (HIP events around its launches in the timed region), the M-apply
bandwidth, the FP64 CG comparison, a short serving run and the CPU oracle baseline.

Further legs (not part of the step): the staggered-mass Hasenbusch split at the
same lattice with the paper's tuned two masses (heat-bath, all-terms and per-term
force evaluations), one full HMC trajectory with the paper's nested Omelyan
schedule for that lattice, and the shared-Krylov multi-shift CG with its Lanczos
spectral bounds against batched separate solves, and a short run of the 4-site
benchmark (HMC ensembles in lockstep chains, quasi-particle energies against exact
diagonalisation).

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-serving] [--no-hasenbusch] [--no-hmc]
       [--no-multishift] [--no-four-site]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import multiprocessing as mp
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from workloads import (HASENBUSCH, WORKLOADS, draw_hasenbusch, draw_hmc, draw_inputs,  # noqa: E402
                       serving_stream)

HBM_PEAK_GBPS = 8000.0   # MI355X HBM3E, published
MALL_BYTES = 256 << 20   # infinity cache
# Algorithmic bytes per site and kernel (distinct vectors read and written once).
APPLY_BYTES = 40.0       # x (16) + phi (8) in, y (16) out, FP64


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1, help="GPUs to use (this build runs on one)")
    ap.add_argument("--steps", type=int, default=10, help="timed steps (one step: the two 102x102x64 solves + S + dS/dphi)")
    ap.add_argument("--warmup", type=int, default=2, help="untimed steps before the timed ones")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-stream leg")
    ap.add_argument("--no-hasenbusch", action="store_true", help="skip the Hasenbusch leg")
    ap.add_argument("--no-hmc", action="store_true", help="skip the HMC trajectory leg")
    ap.add_argument("--no-multishift", action="store_true", help="skip the multi-shift leg")
    ap.add_argument("--no-four-site", action="store_true", help="skip the 4-site ensemble leg")
    ap.add_argument("--no-batches", action="store_true",
                    help="skip the 12x12x32 (16 right-hand sides) and 48x48x64 (3 shifts) solver comparison")
    ap.add_argument("--batches-only", action="store_true",
                    help="run only the 12x12x32 and 48x48x64 solver comparison and print it (a profiling target)")
    ap.add_argument("--counter-run", action="store_true",
                    help="target for rocprofv3 --pmc: a plain 256 MiB copy (counter calibration), then one "
                         "step and nothing else")
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="measured requests of the 200 req/s serving stream (after a warm-up of 200)")
    ap.add_argument("--cpu-budget-s", type=float, default=25.0,
                    help="CPU seconds the oracle baseline may spend on its slowest system")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# CPU baseline: the oracle (test infrastructure), run in worker processes.
# ---------------------------------------------------------------------------
def _oracle_worker(args):
    os.environ["OMP_NUM_THREADS"] = "1"
    import oracle
    from oracle.operator import NormalOperator
    wname, k, budget = args
    w = WORKLOADS[wname]
    lat = oracle.Lattice(w.L1, w.L2, w.Nt, w.kappa_t, w.ms_t)
    phi, eta = draw_inputs(w)
    mu2 = w.mu2_list()[k]
    A = NormalOperator(lat, phi, mu2)
    b = (A.Mh @ eta[k].ravel())
    bn = np.linalg.norm(b)
    # textbook CG (the oracle's algorithm), timed, with a wall-clock budget
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = np.vdot(r, r).real
    t0 = time.perf_counter()
    it = 0
    hist = []
    while math.sqrt(rr) > w.tol * bn:
        q = A(p)
        alpha = rr / np.vdot(p, q).real
        x += alpha * p
        r -= alpha * q
        rr_new = np.vdot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
        hist.append(math.log(math.sqrt(rr) / bn))
        if time.perf_counter() - t0 > budget:
            break
    dt = time.perf_counter() - t0
    done = math.sqrt(rr) <= w.tol * bn
    if done:
        need = it
    else:
        # extrapolate the oracle's own geometric convergence over its last half
        h = np.array(hist[len(hist) // 2:])
        slope = (h[-1] - h[0]) / max(len(h) - 1, 1)
        need = it + (math.log(w.tol) - h[-1]) / slope if slope < 0 else float("inf")
    return {"mu2": mu2, "iters_run": it, "converged": bool(done), "iters_needed": need,
            "sec_per_iter": dt / max(it, 1), "seconds": dt}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_cg2_c64_102x102x64.md")
# the kernels, and what decides the mix of launches the per-launch figure averages over
# (the engine, and the solver defaults such as the block length between convergence checks)
TRAFFIC_SOURCES = ["paper_1804_07195_amd/csrc/hub_kernels.hip", "paper_1804_07195_amd/csrc/hub_internal.h",
                   "paper_1804_07195_amd/csrc/hub_engine.hip", "paper_1804_07195_amd/csrc/hub_engine.h",
                   "paper_1804_07195_amd/csrc/hub_api.hip"]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE counter runs,
    or None when the kernel or engine sources changed since they were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    vals = {}
    for line in text.splitlines():
        parts = line.split()
        if len(parts) == 2 and parts[0] == "source_sha256":
            vals["sha"] = parts[1]
        elif len(parts) == 3 and parts[0] == "traffic_bytes_per_launch":
            vals[parts[1]] = float(parts[2])
    if vals.get("sha") != h.hexdigest():
        return None
    return vals.get(kernel)


def cpu_baseline(wname: str, budget: float) -> dict:
    w = WORKLOADS[wname]
    with mp.get_context("spawn").Pool(w.batch) as pool:
        res = pool.map(_oracle_worker, [(wname, k, budget) for k in range(w.batch)])
    t_solves = sum(r["sec_per_iter"] * r["iters_needed"] for r in res)
    value = w.batch / t_solves if t_solves > 0 else 0.0
    parts = "; ".join(
        f"mu2={r['mu2']}: {r['iters_run']} iterations in {r['seconds']:.1f} s"
        + ("" if r["converged"] else f", {r['iters_needed']:.0f} needed (extrapolated from its own convergence)")
        for r in res)
    return {"value": value, "unit": "solves/s", "cores": w.batch, "kind": "oracle",
            "sample": f"oracle CG (complex128, SciPy CSR, 1 thread per system, one process per system, "
                      f"{platform.processor() or platform.machine()}) on the same two systems to 1e-10: {parts}; "
                      f"value = 2 / sum(seconds per iteration x iterations needed)"}


# ---------------------------------------------------------------------------
def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is a design "
              f"note, not built", file=sys.stderr)
        sys.exit(2)

    if args.counter_run or args.batches_only:
        args.steps, args.warmup, args.no_cpu = 1, 0, True
    # The CPU baseline runs first, in worker processes started before this process
    # touches the GPU.
    cpu = None if args.no_cpu else cpu_baseline("large2", args.cpu_budget_s)

    import torch

    from paper_1804_07195_amd import binding as hb

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.counter_run:
        # counter calibration: 256 MiB read + 256 MiB written by a plain copy kernel
        a = torch.ones(16 << 20, dtype=torch.complex128, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.batches_only:
        ctx = hb.Context(0)
        print(json.dumps({"batches": batch_legs(ctx, hb, torch)}), flush=True)
        ctx.close()
        return
    w = WORKLOADS["large2"]
    hl = hb.lattice(w.L1, w.L2, w.Nt, w.kappa_t, w.ms_t)
    ctx = hb.Context(0)
    phi, eta = draw_inputs(w)
    pd = torch.from_numpy(phi).to("cuda")
    ed = torch.from_numpy(eta).to("cuda")
    chi = hb.hub_apply_Mdag(ctx, hl, pd, ed)
    mu2 = w.mu2_list()
    x = torch.empty_like(chi)
    dS = torch.zeros(pd.shape, dtype=torch.float64, device="cuda")
    opts = hb.default_opts(solver="fgmres", tol=w.tol)
    infos = []

    ones = [1.0] * w.batch

    def step(o=opts):
        _, info, _ = hb.hub_solve(ctx, hl, pd, mu2, chi, x=x, opts=o)
        S = hb.hub_action(ctx, hl, chi, x)
        hb.hub_force_sum(ctx, hl, pd, x, ones, out=dS)   # sum_b dS_b/dphi, one launch
        infos.append((info, S))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if args.counter_run:
        # the M-apply and its streaming ceiling with buffers rotated past the infinity cache
        apply_measure(ctx, hb, torch, w, hl, pd, ed, counter_run=True)
        print(json.dumps({"counter_run": True, "ms_per_step": 1e3 * elapsed}), flush=True)
        return
    # Kernel timing pass: the same steps again with every CG-kernel launch bound to
    # HIP start/stop events on the solver's stream (kept out of the timed region
    # above, whose throughput the per-launch events would lower).
    hb.hub_profile_enable(ctx, True)
    prof_steps = max(1, min(args.steps, 3))
    for _ in range(prof_steps):
        step()
    torch.cuda.synchronize()
    prof = hb.hub_profile_read(ctx)
    hb.hub_profile_enable(ctx, False)
    ms_per_step = 1e3 * elapsed / args.steps
    value = w.batch * args.steps / elapsed
    last_info, last_S = infos[-1]
    resid = [i["true_rel_resid"] for i in last_info]
    assert all(i["converged"] == 1 and i["true_rel_resid"] <= w.tol for i in last_info), last_info

    # dominant kernel of the step (largest summed time among the timed CG kernels)
    dom_name, dom = max(prof.items(), key=lambda kv: kv[1]["total_ms"])
    achieved = dom["GBps"]
    traffic = measured_traffic(dom_name)
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": None if traffic is None else round(traffic),
                "avg_launch_us": round(dom["avg_us"], 3), "launches": dom["launches"],
                "timed_over": f"{prof_steps} steps after the timed region, HIP events bound to every launch",
                "alg_bytes_per_launch": round(dom["bytes"] / max(dom["launches"], 1)),
                # what the complex64 CG of the step keeps live per iteration (r, the p pair, u,
                # the solution z_j, the float angle: 44 bytes per site and system) against the
                # infinity cache: the bytes above are algorithmic, and while the working set fits
                # in the cache much of that traffic is served from it rather than from DRAM
                "working_set_bytes": int(44 * w.nsites * w.batch), "infinity_cache_bytes": MALL_BYTES}
    if traffic is not None:
        roofline["traffic_over_alg"] = round(traffic / max(roofline["alg_bytes_per_launch"], 1), 4)

    m_apply = apply_measure(ctx, hb, torch, w, hl, pd, ed)

    # FP64 CG on the same systems, the same step content (solve + S + summed force), the
    # same final accuracy (every system's FP64 true residual <= tol)
    o64 = hb.default_opts(solver="cg", tol=w.tol)
    step(o64)
    torch.cuda.synchronize()
    reps = 5
    t1 = time.perf_counter()
    for _ in range(reps):
        step(o64)
    torch.cuda.synchronize()
    el64 = time.perf_counter() - t1
    info64 = infos[-1][0]
    assert all(i["converged"] == 1 and i["true_rel_resid"] <= w.tol for i in info64), info64
    cg64 = {"solves_per_s": round(w.batch * reps / el64, 3), "ms_per_step": round(1e3 * el64 / reps, 3),
            "iters": [i["inner_iters"] for i in info64], "true_rel_resid": [i["true_rel_resid"] for i in info64],
            "step": "the same as the mixed step: solve + S + summed force"}

    out = {
        "metric": "M-apply HBM GB/s; solves/s at 1e-10 resid (102x102, Nt=64); p50/p99 latency",
        "value": round(value, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64/f64", "data": "synthetic",
        "config": {"workload": "102x102 honeycomb, N_t=64, kappa=1, U=3.8, beta=12; 2 systems (mu2 0.1, 0) "
                               "sharing phi; chi = M^dagger eta; mixed FGMRES(10, a=5) to 1e-10 + S + dS/dphi",
                   "L": w.L1, "Nt": w.Nt, "systems": w.batch, "mu2": mu2, "tol": w.tol,
                   "solver": "fgmres_mixed", "parallelism": "single GPU"},
        "roofline": roofline,
        "m_apply": m_apply,
        "true_rel_resid": resid,
        "inner_iters": [i["inner_iters"] for i in last_info],
        "fp64_cg": cg64,
        "speedup_vs_fp64_cg": round(value / cg64["solves_per_s"], 3),
        "kernels": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in prof.items()},
    }

    if not args.no_batches:
        out["batches"] = batch_legs(ctx, hb, torch)
    if not args.no_hasenbusch:
        out["hasenbusch"] = hasenbusch_run(ctx, hb, torch)
    if not args.no_hmc:
        out["hmc"] = hmc_run(ctx, hb, torch)
    if not args.no_multishift:
        out["multishift"] = multishift_run(ctx, hb, torch)
    if not args.no_four_site:
        out["four_site"] = four_site_run()
    if not args.no_serving:
        out["serving"] = serving_run(ctx, hb, torch, args.serving_requests)
    ctx.close()
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def apply_measure(ctx, hb, torch, w, hl, pd, ed, counter_run: bool = False) -> dict:
    """FP64 M-apply (one system) through the C ABI: resident and with buffers rotated past
    the infinity cache, next to a streaming kernel that moves the same bytes.  With
    counter_run, only a short cold pass of each (the target of the counter runs)."""
    # The launches go back to back through the C ABI with their arguments marshalled once,
    # so that the host stays ahead of the GPU (through the checking Python wrapper a call
    # costs more host time than the kernel, and the loop would time Python); the host time
    # per call is reported next to the GPU time.
    lib = hb.load()
    sh = hb._stream(None)
    latref = ctypes.byref(hl)

    def timed_raw(args, K):
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        bad = 0
        s.record()
        t0 = time.perf_counter()
        for k in range(K):
            p, x, y = args[k % len(args)]
            bad |= lib.hub_apply_M(ctx.handle, latref, p, x, y, 1, sh)
        host_us = (time.perf_counter() - t0) / K * 1e6
        e.record()
        torch.cuda.synchronize()
        if bad:
            raise RuntimeError("hub_apply_M failed: " + lib.hub_last_error().decode())
        return s.elapsed_time(e) / K, host_us

    def timed_stream(args, K, mode):
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        bad = 0
        s.record()
        for k in range(K):
            p, x, y = args[k % len(args)]
            bad |= lib.hub_profile_stream(ctx.handle, p, x, y, w.nsites, mode, sh)
        e.record()
        torch.cuda.synchronize()
        if bad:
            raise RuntimeError("hub_profile_stream failed: " + lib.hub_last_error().decode())
        return s.elapsed_time(e) / K

    nrot = 1 + (2 * MALL_BYTES) // int(w.nsites * APPLY_BYTES)
    xs = [torch.randn_like(ed[0:1]) for _ in range(nrot)]
    ys = [torch.empty_like(ed[0:1]) for _ in range(nrot)]
    ps = [pd.clone() for _ in range(nrot)]
    cold_args = [(ps[k].data_ptr(), xs[k].data_ptr(), ys[k].data_ptr()) for k in range(nrot)]
    if counter_run:
        timed_raw(cold_args, 2 * nrot)
        for mode in (0, 1):
            timed_stream(cold_args, 2 * nrot, mode)
        return {}
    y = torch.empty_like(ed[0:1])
    hot_args = [(pd.data_ptr(), ed[0:1].data_ptr(), y.data_ptr())]
    timed_raw(hot_args, 5)
    hot_ms, hot_host = timed_raw(hot_args, 200)
    timed_raw(cold_args, nrot)
    cold_ms, cold_host = timed_raw(cold_args, 20 * nrot)
    apply_bytes = w.nsites * APPLY_BYTES
    gbps = lambda ms: round(apply_bytes / (ms * 1e-3) / 1e9, 1)
    # the same bytes through a kernel with no stencil: the ceiling of this process, both
    # cache policies (non-temporal stores as the apply; non-temporal loads)
    ceiling = {}
    for mode, tag in ((0, "nt_store"), (1, "nt_load")):
        timed_stream(hot_args, 5, mode)
        h = timed_stream(hot_args, 200, mode)
        timed_stream(cold_args, nrot, mode)
        c = timed_stream(cold_args, 20 * nrot, mode)
        ceiling[tag] = {"hot_us": round(1e3 * h, 3), "hot_GBps": gbps(h), "cold_us": round(1e3 * c, 3),
                        "cold_GBps": gbps(c)}
    best_hot = min(v["hot_us"] for v in ceiling.values())
    best_cold = min(v["cold_us"] for v in ceiling.values())
    m_apply = {"kernel": "k_apply<M>", "alg_bytes": int(apply_bytes),
               "hot_us": round(1e3 * hot_ms, 3), "hot_GBps": gbps(hot_ms),
               "cold_us": round(1e3 * cold_ms, 3), "cold_GBps": gbps(cold_ms),
               "cold_frac_of_peak": round(gbps(cold_ms) / HBM_PEAK_GBPS, 4),
               "cold_buffers": nrot, "host_us_per_call": [round(hot_host, 2), round(cold_host, 2)],
               "stream_ceiling": ceiling,
               "frac_of_ceiling": {"hot": round(best_hot / (1e3 * hot_ms), 3),
                                   "cold": round(best_cold / (1e3 * cold_ms), 3)}}
    del xs, ys, ps
    return m_apply


def batch_legs(ctx, hb, torch, reps: int = 7) -> dict:
    """The two smaller batched workloads, each solved by FP64 CG and by the mixed
    FGMRES to relative true residual 1e-10 on identical inputs: 12x12, N_t = 32 with 16
    right-hand sides sharing phi (mu^2 = 0), and 48x48, N_t = 64 with the three
    Hasenbusch shifts mu^2 in {0.5, 0.05, 0} in one launch.  Milliseconds per batch
    (median over reps), iterations and the largest FP64 true residual of each."""
    res = {}
    for name in ("small16", "medium3"):
        w = WORKLOADS[name]
        hl = hb.lattice(w.L1, w.L2, w.Nt, w.kappa_t, w.ms_t)
        phi, eta = draw_inputs(w)
        pd = torch.from_numpy(phi).to("cuda")
        chi = hb.hub_apply_Mdag(ctx, hl, pd, torch.from_numpy(eta).to("cuda"))
        x = torch.empty_like(chi)
        mu2 = w.mu2_list()
        row = {"workload": f"{w.L1}x{w.L2}x{w.Nt}, kappa={w.kappa}, U={w.U}, beta={w.beta}, {w.batch} systems, "
                           f"mu2={mu2}", "sites_per_system": w.nsites}
        for solver in ("cg", "fgmres"):
            o = hb.default_opts(solver=solver, tol=w.tol)
            hb.hub_solve(ctx, hl, pd, mu2, chi, x=x, opts=o)
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                _, info, _ = hb.hub_solve(ctx, hl, pd, mu2, chi, x=x, opts=o)
                ts.append(time.perf_counter() - t0)
            assert all(i["converged"] == 1 and i["true_rel_resid"] <= w.tol for i in info), info
            ms = 1e3 * sorted(ts)[len(ts) // 2]
            row[solver] = {"ms_per_batch": round(ms, 3), "solves_per_s": round(w.batch / ms * 1e3, 1),
                           "iters": [i["inner_iters"] for i in info],
                           "cycles": [i["outer_iters"] for i in info],
                           "max_true_rel_resid": max(i["true_rel_resid"] for i in info)}
        row["mixed_speedup"] = round(row["cg"]["ms_per_batch"] / row["fgmres"]["ms_per_batch"], 3)
        res[name] = row
    return res


def hasenbusch_run(ctx, hb, torch, reps: int = 5) -> dict:
    """Staggered-mass Hasenbusch split at 102x102, N_t = 64 with the paper's tuned masses
    (mu_0, mu_1) = (0.4054, 1.09624): heat-bath of the three pseudofermions, then the
    actions and summed force of all terms (three batched mixed-precision solves, 1e-10),
    and each term alone; the plain single-term force on the same field for comparison."""
    hw = HASENBUSCH["hb_large"]
    w = hw.base
    hl = hb.lattice(w.L1, w.L2, w.Nt, w.kappa_t, w.ms_t)
    phi, rho = draw_hasenbusch(hw)
    pd = torch.from_numpy(phi).to("cuda")
    rd = torch.from_numpy(rho).to("cuda")
    opts = hb.default_opts(solver="fgmres", tol=1e-10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chi, hinfo, _ = hb.hub_hasenbusch_heatbath(ctx, hl, pd, hw.mts, rd, opts=opts)
    torch.cuda.synchronize()
    heat_ms = 1e3 * (time.perf_counter() - t0)
    eta = torch.zeros_like(chi)
    F = torch.zeros(pd.shape, dtype=torch.float64, device="cuda")

    def run(terms):
        return hb.hub_hasenbusch_force(ctx, hl, pd, hw.mts, chi, terms=terms, eta=eta, out=F, opts=opts)

    S, infos = run(None)[1], run(None)[3]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run(None)
    torch.cuda.synchronize()
    all_ms = 1e3 * (time.perf_counter() - t0) / reps
    per_term = []
    for i in range(hw.nterms):
        run([i])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _, _, _, inf, _ = run([i])
        torch.cuda.synchronize()
        per_term.append({"term": i, "ms": round(1e3 * (time.perf_counter() - t0) / reps, 3),
                         "inner_iters": inf[i]["inner_iters"], "true_rel_resid": inf[i]["true_rel_resid"],
                         "force_norm": round(float(torch.linalg.norm(F)), 4)})
    r2 = [float(np.vdot(rho[i].ravel(), rho[i].ravel()).real) for i in range(hw.nterms)]
    # the plain pseudofermion term (M with m_s = 0) on the same phi for comparison
    chi0 = hb.hub_apply_M(ctx, hl, pd, rd[0:1])
    x0 = torch.empty_like(chi0)
    hb.hub_solve(ctx, hl, pd, [0.0], chi0, x=x0, opts=opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, inf0, _ = hb.hub_solve(ctx, hl, pd, [0.0], chi0, x=x0, opts=opts)
        hb.hub_force(ctx, hl, pd, x0, out=F)
    torch.cuda.synchronize()
    plain_ms = 1e3 * (time.perf_counter() - t0) / reps
    plain_norm = float(torch.linalg.norm(F))
    return {"workload": "102x102 honeycomb, N_t=64, kappa=1, U=3.8, beta=12; staggered masses "
                        f"{list(hw.masses)} (m~ = {[round(m, 6) for m in hw.mts]}); mixed FGMRES to 1e-10",
            "terms": hw.nterms, "heatbath_ms": round(heat_ms, 3),
            "heatbath_inner_iters": [i["inner_iters"] for i in hinfo],
            "all_terms_force_ms": round(all_ms, 3),
            "all_terms_per_s": round(1e3 / all_ms, 3),
            "per_term": per_term,
            "S_minus_rho2_rel": [abs(S[i] - r2[i]) / r2[i] for i in range(hw.nterms)],
            "inner_iters": [infos[i]["inner_iters"] for i in range(hw.nterms)],
            "plain_term_force_ms": round(plain_ms, 3), "plain_term_inner_iters": inf0[0]["inner_iters"],
            "plain_force_norm": round(plain_norm, 4)}


def hmc_run(ctx, hb, torch) -> dict:
    """One HMC update at 102x102, N_t = 64 with the paper's tuned Hasenbusch schedule for
    that lattice (Table tab_nmds: N_MD = 30, N_MD / N_0 = 15, so N_0 = N_1 = 2), trajectory
    length 1, Omelyan zeta = 0.1931833, mixed FGMRES solves to 1e-10 with warm starts."""
    hw = HASENBUSCH["hb_large"]
    w = hw.base
    hl = hb.lattice(w.L1, w.L2, w.Nt, w.kappa_t, w.ms_t)
    phi, pi, rho = draw_hmc(hw)
    pd = torch.from_numpy(phi).to("cuda")
    qd = torch.from_numpy(pi).to("cuda")
    rd = torch.from_numpy(rho).to("cuda")
    p = hb.hmc_params(w.U_t, 30, hw.mts, [2, 2], traj_length=1.0)
    opts = hb.default_opts(solver="fgmres", tol=1e-10)
    opts.use_x0 = 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = hb.hub_hmc_trajectory(ctx, hl, pd, qd, rd, 0.5, p, opts=opts)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    return {"workload": "102x102 honeycomb, N_t=64, kappa=1, U=3.8, beta=12; Hasenbusch masses "
                        f"{list(hw.masses)}; N_MD=30, N_0=N_1=2, t=1, zeta=0.1931833; hot start phi ~ N(0, U~)",
            "seconds_per_trajectory": round(sec, 3), "dH": info["dH"], "accepted_at_u_0.5": info["accepted"],
            "force_evals_per_term": info["force_evals"], "kick_groups": info["kick_groups"],
            "drifts": info["drifts"], "inner_iters": info["inner_iters"]}


def multishift_run(ctx, hb, torch, reps: int = 3) -> dict:
    """One right-hand side, several shifts: the shared-Krylov FP64 multi-shift CG against
    the same shifts solved as a batch of separate FP64 CG and mixed FGMRES systems, at
    48x48x64 (mu2 in {0.5, 0.05, 0}) and 102x102x64 (mu2 in {0.1, 0}); the Lanczos
    bounds of M M^dagger and the two Hasenbusch masses they give by eq. (mu_i_eqn)."""
    res = {}
    for name, shifts in (("medium3", [0.5, 0.05, 0.0]), ("large2", [0.1, 0.0])):
        w = WORKLOADS[name]
        hl = hb.lattice(w.L1, w.L2, w.Nt, w.kappa_t, w.ms_t)
        phi, eta = draw_inputs(w, batch=1)
        pd = torch.from_numpy(phi).to("cuda")
        b = torch.from_numpy(eta[0]).to("cuda")
        bb = b[None].expand(len(shifts), *b.shape).contiguous()
        x = torch.empty_like(bb)
        row = {"shifts": shifts}

        def t_of(fn):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                out = fn()
            torch.cuda.synchronize()
            return 1e3 * (time.perf_counter() - t0) / reps, out

        ms_ms, (_, infos, lam, _) = t_of(lambda: hb.hub_solve_multishift(ctx, hl, pd, shifts, b, x=x))
        cg_ms, (_, icg, _) = t_of(lambda: hb.hub_solve(ctx, hl, pd, shifts, bb, x=x,
                                                        opts=hb.default_opts(solver="cg")))
        fg_ms, (_, ifg, _) = t_of(lambda: hb.hub_solve(ctx, hl, pd, shifts, bb, x=x,
                                                        opts=hb.default_opts(solver="fgmres")))
        row.update({"multishift_ms": round(ms_ms, 3), "shared_iters": infos[0]["outer_iters"],
                    "certify_iters": [i["inner_iters"] for i in infos],
                    "true_rel_resid": [i["true_rel_resid"] for i in infos],
                    "batched_fp64_cg_ms": round(cg_ms, 3), "batched_fp64_cg_iters": [i["inner_iters"] for i in icg],
                    "batched_fgmres_ms": round(fg_ms, 3),
                    "lanczos_lambda_min": lam[0], "lanczos_lambda_max": lam[1],
                    "hasenbusch_masses_eq_mu_i_n2": hb.hub_hasenbusch_masses(lam[0], lam[1], 2)})
        res[f"{w.L1}x{w.L2}x{w.Nt}"] = row
    return res


def four_site_run() -> dict:
    """The 4-site benchmark (2 x 1 cells, U/kappa = 4, beta kappa = 8, N_t = 64): 32 HMC
    chains in lockstep with one Hasenbusch mass (0.5), 20 thermalisation and 60 measured
    trajectories each; the Gamma and M energies against the exact values 3.429 and 1.565
    (Table tab:fit results, the paper's N_t = 64 column: 3.555(16), 1.647(23))."""
    from paper_1804_07195_amd import four_site
    t0 = time.perf_counter()
    r = four_site.run(64, n_chains=32, n_therm=20, n_meas=60, n_md=8, bin_size=10, n_boot=200)
    r["seconds"] = round(time.perf_counter() - t0, 1)
    r["exact"] = {"E_Gamma": 3.429, "E_M": 1.565}
    return r


def _serving_inputs(hb, torch, ctx, stream):
    """Device inputs of each request of a serving stream, drawn on the device by torch's
    seeded generator (the request's own seed): phi ~ N(0, U~) and chi = M^dagger eta with
    eta complex Gaussian (Re, Im ~ N(0, 1/2)); output buffers allocated up front."""
    reqs = []
    g = torch.Generator(device="cuda")
    for r in stream:
        w = r["workload"]
        g.manual_seed(w.seed)
        hl = hb.lattice(w.L1, w.L2, w.Nt, w.kappa_t, w.ms_t)
        pd = torch.randn(w.shape, dtype=torch.float64, device="cuda", generator=g) * math.sqrt(w.U_t)
        er = torch.randn((1,) + w.shape, dtype=torch.float64, device="cuda", generator=g)
        ei = torch.randn((1,) + w.shape, dtype=torch.float64, device="cuda", generator=g)
        eta = torch.complex(er, ei) * math.sqrt(0.5)
        chi = hb.hub_apply_Mdag(ctx, hl, pd, eta)
        del er, ei, eta
        reqs.append({"t": r["t"], "w": w, "hl": hl, "phi": pd, "chi": chi, "x": torch.empty_like(chi),
                     "dS": torch.empty(w.shape, dtype=torch.float64, device="cuda")})
    torch.cuda.synchronize()
    return reqs


def _serve(hb, ctx, reqs, opts, times):
    """Submit reqs[k] at times[k] (seconds from the start; all at once if None) and poll
    until every request is done.  Returns per-request (latency s, status, converged),
    the makespan and the mean number of requests in flight (submitted, not yet done)."""
    pend = {}
    out = [None] * len(reqs)
    t0 = time.perf_counter()
    k = 0
    inflight_area = 0.0
    last = t0
    while k < len(reqs) or pend:
        now = time.perf_counter()
        inflight_area += len(pend) * (now - last)
        last = now
        while k < len(reqs) and (times is None or times[k] <= now - t0):
            r = reqs[k]
            p = hb.hub_submit(ctx, r["hl"], r["w"].mu2[0], r["phi"], r["chi"], x_out=r["x"], dSdphi_out=r["dS"],
                              opts=opts)
            pend[k] = (p, time.perf_counter())
            k += 1
        # poll at most 128 tickets per pass, oldest first (a long backlog would otherwise
        # spend the pass in the poll calls)
        for q in list(pend)[:128]:
            done, info = hb.hub_poll(ctx, pend[q][0])
            if done:
                out[q] = (time.perf_counter() - pend[q][1], info["status"], info["converged"])
                del pend[q]
        time.sleep(0.0001)
    span = time.perf_counter() - t0
    return out, span, inflight_area / span


def _pct(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, int(q * len(v)))]


def serving_run(ctx, hb, torch, nreq: int, warm: int = 200) -> dict:
    """Seeded Poisson stream (mean 200 req/s) of solve + S + force requests of mixed lattice
    size, N_t and shift through hub_submit / hub_poll (continuous batching):
    * latency percentiles over `nreq` requests after a warm-up window of `warm` requests;
    * capacity: a backlog of the same requests submitted at once, drained as fast as the
      engine admits them (sustained solves/s, requests in flight);
    * offered-rate sweep: the stream replayed at 2x, 4x and 8x the rate."""
    stream = serving_stream(warm + nreq, seed=5)
    reqs = _serving_inputs(hb, torch, ctx, stream)
    opts = hb.default_opts(solver="fgmres", tol=1e-10)
    times = [r["t"] for r in reqs]
    res, span, infl = _serve(hb, ctx, reqs, opts, times)
    meas = res[warm:]
    lat = [1e3 * l for l, _, _ in meas]
    t_meas = times[-1] - times[warm]
    ok = sum(1 for _, st, c in meas if st == 0 and c == 1)
    out = {"requests": len(meas), "warmup_requests": warm, "offered_rate_per_s": 200,
           "solves_per_s": round(len(meas) / max(t_meas, 1e-9), 2),
           "p50_ms": round(_pct(lat, 0.50), 3), "p90_ms": round(_pct(lat, 0.90), 3),
           "p99_ms": round(_pct(lat, 0.99), 3), "max_ms": round(max(lat), 3),
           "converged": ok, "mean_in_flight": round(infl, 2),
           "mix": "L in {6,12,24,48,102}, N_t in {16,32,64}, U~U[1,4], beta=N_t/4, mu2 in {0.5,0.1,0.01,0}; "
                  "mixed FGMRES to 1e-10 + S + dS/dphi per request"}
    # per lattice size: where the latency goes
    by_L = {}
    for r, (l, _, _) in zip(reqs[warm:], meas):
        by_L.setdefault(r["w"].L1, []).append(1e3 * l)
    out["p50_ms_by_L"] = {str(L): round(_pct(v, 0.5), 3) for L, v in sorted(by_L.items())}
    # capacity: everything at once
    cap, cspan, cinfl = _serve(hb, ctx, reqs[warm:], opts, None)
    out["capacity"] = {"requests": len(cap), "solves_per_s": round(len(cap) / cspan, 2),
                       "mean_in_flight": round(cinfl, 1),
                       "converged": sum(1 for _, st, c in cap if st == 0 and c == 1)}
    # offered-rate sweep over the first 600 measured requests, arrival times compressed
    sweep = []
    base = reqs[warm:warm + 600]
    tb = [r["t"] - base[0]["t"] for r in base]
    for f in (2, 4, 8):
        rs, sp, fl = _serve(hb, ctx, base, opts, [t / f for t in tb])
        l = [1e3 * v for v, _, _ in rs]
        sweep.append({"offered_per_s": 200 * f, "achieved_per_s": round(len(rs) / sp, 1),
                      "p50_ms": round(_pct(l, 0.5), 3), "p99_ms": round(_pct(l, 0.99), 3),
                      "mean_in_flight": round(fl, 1)})
    out["rate_sweep"] = sweep
    del reqs
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
