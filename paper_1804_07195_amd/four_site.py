"""The 4-site benchmark of Sec. 7.2 on the GPU: HMC ensembles and quasi-particle energies.

The 4-site hexagonal system is the honeycomb of 2 x 1 unit cells (the bond to cell
(i, j-1) wraps onto cell (i, j), so that pair is bonded twice; free energies +-3 kappa
at Gamma and +-kappa at M).  Ensembles are generated with `hub_hmc_trajectory`
(staggered-mass Hasenbusch split with one mass, nested Omelyan integrator); on each
configuration the single-particle correlators

  C_v(tau_k) = -(1/|S|) sum_{t0 in S} s(t0 + k) v^dag [M^{-1}]_{(t0 + k), (t0)} v

(slices mod N_t, s = -1 across the antiperiodic boundary) are measured with the
library's solves, M^{-1} w = M^dag (M M^dag)^{-1} w, for the Gamma channel
v = (1, 1, 1, 1)/2 and the M channel v = (1, -1, 1, -1)/2 over (A0, A1, B0, B1).
Energies come from least-squares exponential fits of the mean correlator in the
paper's windows (tau kappa in [0.2, 1] for Gamma, [0.6, 2] for M), with bootstrap
errors over binned configurations.

Independent Markov chains run in threads, one context and stream each, so their
small launches overlap on the device.
"""
from __future__ import annotations

import threading

import numpy as np
import torch

from . import binding as hb

GAMMA = np.array([1.0, 1.0, 1.0, 1.0]) / 2
M_POINT = np.array([1.0, -1.0, 1.0, -1.0]) / 2
WINDOWS = {"Gamma": (0.2, 1.0), "M": (0.6, 2.0)}


def measure(ctx: hb.Context, lat: hb.HubLattice, phi: torch.Tensor, t0s, opts=None, stream=None) -> dict:
    """Correlators of both channels on one field (device phi [N_t, 2, 2, 1])."""
    Nt = lat.Nt
    ns = 2 * lat.L1 * lat.L2
    chans = {"Gamma": GAMMA, "M": M_POINT}
    src = torch.zeros((len(chans) * len(t0s), Nt, ns), dtype=torch.complex128, device=phi.device)
    k = 0
    for v in chans.values():
        for t0 in t0s:
            src[k, t0] = torch.from_numpy(v.astype(np.complex128))
            k += 1
    src = src.reshape((len(chans) * len(t0s), Nt, 2, lat.L1, lat.L2)).contiguous()
    o = hb.default_opts(solver="cg", tol=1e-10) if opts is None else opts
    y, _, _ = hb.hub_solve(ctx, lat, phi, [0.0] * src.shape[0], src, opts=o, stream=stream)
    col = hb.hub_apply_Mdag(ctx, lat, phi, y, stream=stream).reshape(src.shape[0], Nt, ns).cpu().numpy()
    out = {}
    k = 0
    for name, v in chans.items():
        C = np.zeros(Nt)
        for t0 in t0s:
            g = col[k]
            k += 1
            for kk in range(Nt):
                t = (t0 + kk) % Nt
                sgn = -1.0 if t0 + kk >= Nt else 1.0
                C[kk] += -sgn * float(np.vdot(v, g[t]).real)
        out[name] = C / len(t0s)
    return out


def fit_energy(C, delta: float, window) -> float:
    tau = np.arange(len(C)) * delta
    sel = (tau >= window[0] - 1e-12) & (tau <= window[1] + 1e-12)
    c = np.asarray(C)[sel]
    if np.any(c <= 0):
        return float("nan")
    A = np.vstack([np.ones(sel.sum()), -tau[sel]]).T
    coef, *_ = np.linalg.lstsq(A, np.log(c), rcond=None)
    return float(coef[1])


def _chain(seed, lat, U_t, params, n_therm, n_meas, t0s, opts, out, idx, errors):
    try:
        ctx = hb.Context(0)
        stream = torch.cuda.Stream()
        rng = np.random.default_rng(seed)
        shape = (lat.Nt, 2, lat.L1, lat.L2)
        with torch.cuda.stream(stream):
            phi = torch.from_numpy(rng.normal(0.0, np.sqrt(U_t), size=shape)).to("cuda")
            acc, dH, samples = [], [], {"Gamma": [], "M": []}
            for traj in range(n_therm + n_meas):
                pi = torch.from_numpy(rng.standard_normal(size=shape)).to("cuda")
                rho = (rng.standard_normal((params.n + 1,) + shape) + 1j * rng.standard_normal((params.n + 1,) + shape))
                rho = torch.from_numpy(rho * np.sqrt(0.5)).to("cuda")
                u = float(rng.uniform())
                info = hb.hub_hmc_trajectory(ctx, lat, phi, pi, rho, u, params, opts=opts, stream=stream)
                if traj >= n_therm:
                    acc.append(info["accepted"])
                    dH.append(info["dH"])
                    m = measure(ctx, lat, phi, t0s, stream=stream)
                    for k in samples:
                        samples[k].append(m[k])
        torch.cuda.synchronize()
        ctx.close()
        out[idx] = {"acc": acc, "dH": dH, "C": {k: np.array(v) for k, v in samples.items()}}
    except Exception as e:  # reported by the caller
        errors.append(repr(e))


def run(Nt: int, n_chains: int = 8, n_therm: int = 50, n_meas: int = 200, U: float = 4.0, beta: float = 8.0,
        kappa: float = 1.0, n_md: int = 8, mass: float = 0.5, seed: int = 1, bin_size: int = 10,
        n_boot: int = 200) -> dict:
    """Ensembles at U/kappa, beta kappa on the 4-site lattice; returns energies with bootstrap errors."""
    delta = beta / Nt
    lat = hb.lattice(2, 1, Nt, delta * kappa)
    U_t = delta * U
    params = hb.hmc_params(U_t, n_md, [delta * mass], [2], traj_length=1.0)
    opts = hb.default_opts(solver="cg", tol=1e-10)
    opts.use_x0 = 1
    t0s = list(range(0, Nt, max(1, Nt // 4)))
    out = [None] * n_chains
    errors = []
    th = [threading.Thread(target=_chain, args=(seed * 1000 + c, lat, U_t, params, n_therm, n_meas, t0s, opts,
                                                 out, c, errors)) for c in range(n_chains)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    if errors:
        raise RuntimeError(errors[0])
    res = {"Nt": Nt, "chains": n_chains, "trajectories_per_chain": n_therm + n_meas, "measured": n_chains * n_meas,
           "acceptance": float(np.mean([a for o in out for a in o["acc"]])),
           "mean_exp_minus_dH": float(np.mean([np.exp(-d) for o in out for d in o["dH"]]))}
    rng = np.random.default_rng(seed)
    for name, win in WINDOWS.items():
        # bins of consecutive configurations within each chain
        bins = []
        for o in out:
            C = o["C"][name]
            for b0 in range(0, len(C) - bin_size + 1, bin_size):
                bins.append(C[b0:b0 + bin_size].mean(axis=0))
        bins = np.array(bins)
        E = fit_energy(bins.mean(axis=0), delta, win)
        boot = [fit_energy(bins[rng.integers(len(bins), size=len(bins))].mean(axis=0), delta, win)
                for _ in range(n_boot)]
        res[f"E_{name}"] = E
        res[f"E_{name}_err"] = float(np.nanstd(boot))
    return res
