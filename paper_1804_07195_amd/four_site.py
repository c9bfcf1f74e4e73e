"""The 4-site benchmark of Sec. 7.2 on the GPU: HMC ensembles and quasi-particle energies.

The 4-site hexagonal system is the honeycomb of 2 x 1 unit cells (the bond to cell
(i, j-1) wraps onto cell (i, j), so that pair is bonded twice; free energies +-3 kappa
at Gamma and +-kappa at M).  Ensembles are generated with `hub_hmc_trajectory`
(staggered-mass Hasenbusch split with one mass, nested Omelyan integrator); on each
configuration the single-particle correlators

  C_v(tau_k) = -(1/|S|) sum_{t0 in S} s(t0 + k) v^dag [M^{-1}]_{(t0 + k), (t0)} v

(slices mod N_t, s = -1 across the antiperiodic boundary) are measured with the
library's solves, M^{-1} w = M^dag (M M^dag)^{-1} w, for all chains together, for the Gamma channel
v = (1, 1, 1, 1)/2 and the M channel v = (1, -1, 1, -1)/2 over (A0, A1, B0, B1).
Energies come from least-squares exponential fits of the mean correlator in the
paper's windows (tau kappa in [0.2, 1] for Gamma, [0.6, 2] for M), with bootstrap
errors over binned configurations.

Independent Markov chains advance together through `hub_hmc_trajectories`, whose
kick groups solve the terms of all chains in one batch: a 4-site system alone would
leave the device idle.
"""
from __future__ import annotations

import sys

import numpy as np
import torch

from . import binding as hb

GAMMA = np.array([1.0, 1.0, 1.0, 1.0]) / 2
M_POINT = np.array([1.0, -1.0, 1.0, -1.0]) / 2
WINDOWS = {"Gamma": (0.2, 1.0), "M": (0.6, 2.0)}


def measure_chains(ctx: hb.Context, lat: hb.HubLattice, phi: torch.Tensor, t0s, opts=None, stream=None) -> dict:
    """Correlators of both channels on each of several fields (device phi [n_fields, N_t, 2,
    2, 1]): {channel: array [n_fields, N_t]}.  The sources of all fields are solved
    together, as many fields per call as the batch limit allows (hub_solve_fields), and
    M^dagger is applied to the solutions per field (hub_apply_fields)."""
    Nt = lat.Nt
    ns = 2 * lat.L1 * lat.L2
    nf = phi.numel() // (Nt * ns)
    chans = {"Gamma": GAMMA, "M": M_POINT}
    per = len(chans) * len(t0s)
    src = torch.zeros((per, Nt, ns), dtype=torch.complex128, device=phi.device)
    k = 0
    for v in chans.values():
        for t0 in t0s:
            src[k, t0] = torch.from_numpy(v.astype(np.complex128))
            k += 1
    o = hb.default_opts(solver="cg", tol=1e-10) if opts is None else opts
    fpc = max(1, hb.HUB_MAX_BATCH // per)  # fields per call
    phis = phi.reshape(nf, Nt, 2, lat.L1, lat.L2)
    cols = []
    for f0 in range(0, nf, fpc):
        f1 = min(nf, f0 + fpc)
        b = src.expand(f1 - f0, per, Nt, ns).reshape((f1 - f0) * per, Nt, 2, lat.L1, lat.L2).contiguous()
        ph = phis[f0:f1].contiguous()
        y, _, _ = hb.hub_solve_fields(ctx, lat, ph, [0.0] * b.shape[0], b, opts=o, stream=stream)
        cols.append(hb.hub_apply_fields(ctx, lat, ph, y, dag=True, stream=stream))
    col = torch.cat(cols).reshape(nf, len(chans), len(t0s), Nt, ns).cpu().numpy()
    # C_v(tau_k) = -(1/|S|) sum_{t0} s(t0 + k) v^dag col[t0 + k mod N_t]
    kk = np.arange(Nt)
    t0a = np.asarray(t0s)
    tt = (t0a[:, None] + kk[None, :]) % Nt                      # [len(t0s), N_t]
    sgn = np.where(t0a[:, None] + kk[None, :] >= Nt, -1.0, 1.0)
    out = {}
    for c, (name, v) in enumerate(chans.items()):
        g = col[:, c, np.arange(len(t0s))[:, None], tt, :]      # [nf, len(t0s), N_t, ns]
        proj = np.einsum("s,fiks->fik", v.conj(), g).real
        out[name] = -(sgn[None] * proj).mean(axis=1)
    return out


def measure(ctx: hb.Context, lat: hb.HubLattice, phi: torch.Tensor, t0s, opts=None, stream=None) -> dict:
    """Correlators of both channels on one field (device phi [N_t, 2, 2, 1])."""
    m = measure_chains(ctx, lat, phi.reshape((1,) + tuple(phi.shape)).contiguous(), t0s, opts=opts, stream=stream)
    return {k: v[0] for k, v in m.items()}


def fit_energy(C, delta: float, window) -> float:
    tau = np.arange(len(C)) * delta
    sel = (tau >= window[0] - 1e-12) & (tau <= window[1] + 1e-12)
    c = np.asarray(C)[sel]
    if np.any(c <= 0):
        return float("nan")
    A = np.vstack([np.ones(sel.sum()), -tau[sel]]).T
    coef, *_ = np.linalg.lstsq(A, np.log(c), rcond=None)
    return float(coef[1])


def run(Nt: int, n_chains: int = 32, n_therm: int = 50, n_meas: int = 200, U: float = 4.0, beta: float = 8.0,
        kappa: float = 1.0, n_md: int = 8, mass: float = 0.5, seed: int = 1, bin_size: int = 10,
        n_boot: int = 200, cold: bool = True, progress: int = 0) -> dict:
    """Ensembles at U/kappa, beta kappa on the 4-site lattice: n_chains Markov chains (from
    phi = 0 unless cold is False) updated together by `hub_hmc_trajectories`, measured
    after every trajectory once thermalised; returns energies with bootstrap errors.  With
    progress > 0 a line goes to stderr every `progress` trajectories."""
    delta = beta / Nt
    lat = hb.lattice(2, 1, Nt, delta * kappa)
    U_t = delta * U
    params = hb.hmc_params(U_t, n_md, [delta * mass], [2], traj_length=1.0)
    opts = hb.default_opts(solver="cg", tol=1e-10)
    opts.use_x0 = 1
    t0s = list(range(0, Nt, max(1, Nt // 4)))
    shape = (Nt, 2, lat.L1, lat.L2)
    rng = np.random.default_rng(seed)
    ctx = hb.Context(0)
    try:
        phi0 = np.zeros((n_chains,) + shape) if cold else rng.normal(0.0, np.sqrt(U_t), size=(n_chains,) + shape)
        phi = torch.from_numpy(phi0).to("cuda")
        acc, dH = [], []
        samples = {"Gamma": [[] for _ in range(n_chains)], "M": [[] for _ in range(n_chains)]}
        for traj in range(n_therm + n_meas):
            pi = torch.from_numpy(rng.standard_normal(size=(n_chains,) + shape)).to("cuda")
            rs = (n_chains, params.n + 1) + shape
            rho = torch.from_numpy((rng.standard_normal(rs) + 1j * rng.standard_normal(rs)) * np.sqrt(0.5)).to("cuda")
            u = rng.uniform(size=n_chains)
            infos = hb.hub_hmc_trajectories(ctx, lat, phi, pi, rho, list(u), params, opts=opts)
            if progress and (traj + 1) % progress == 0:
                print(f"N_t={Nt}: trajectory {traj + 1}/{n_therm + n_meas}", file=sys.stderr, flush=True)
            if traj < n_therm:
                continue
            acc += [i["accepted"] for i in infos]
            dH += [i["dH"] for i in infos]
            m = measure_chains(ctx, lat, phi, t0s)
            for k in samples:
                for c in range(n_chains):
                    samples[k][c].append(m[k][c])
    finally:
        ctx.close()
    res = {"Nt": Nt, "n_md": n_md, "chains": n_chains, "trajectories_per_chain": n_therm + n_meas,
           "measured": n_chains * n_meas, "acceptance": float(np.mean(acc)),
           "mean_exp_minus_dH": float(np.mean(np.exp(-np.array(dH))))}
    for name, win in WINDOWS.items():
        # bins of consecutive configurations within each chain
        bins = []
        for c in range(n_chains):
            C = np.array(samples[name][c])
            for b0 in range(0, len(C) - bin_size + 1, bin_size):
                bins.append(C[b0:b0 + bin_size].mean(axis=0))
        bins = np.array(bins)
        res[f"E_{name}"] = fit_energy(bins.mean(axis=0), delta, win)
        boot = [fit_energy(bins[rng.integers(len(bins), size=len(bins))].mean(axis=0), delta, win)
                for _ in range(n_boot)]
        res[f"E_{name}_err"] = float(np.nanstd(boot))
    return res


def continuum(results, name: str):
    """Weighted least-squares fit E(delta) = E_0 + c delta^2 over ensembles at several N_t
    (the Trotter error of the action is O(delta^2)); returns (E_0, error of E_0)."""
    d2 = np.array([(r["beta"] / r["Nt"]) ** 2 for r in results])
    E = np.array([r[f"E_{name}"] for r in results])
    w = 1.0 / np.array([r[f"E_{name}_err"] for r in results]) ** 2
    A = np.vstack([np.ones_like(d2), d2]).T
    cov = np.linalg.inv(A.T @ (A * w[:, None]))
    coef = cov @ (A.T @ (w * E))
    return float(coef[0]), float(np.sqrt(cov[0, 0]))


def main(argv=None) -> None:
    import argparse
    import json
    import time
    ap = argparse.ArgumentParser(description="4-site benchmark of Sec. 7.2: HMC ensembles at several N_t, "
                                             "quasi-particle energies and their delta -> 0 limit")
    ap.add_argument("--nt", type=int, nargs="+", default=[32, 64, 128],
                    help="time slices of each ensemble (beta kappa = 8, so delta = 8 / N_t)")
    ap.add_argument("--chains", type=int, default=32, help="Markov chains advanced in lockstep on the GPU")
    ap.add_argument("--therm", type=int, default=50, help="thermalisation trajectories per chain")
    ap.add_argument("--meas", type=int, default=200, help="measured trajectories per chain")
    ap.add_argument("--seed", type=int, default=1, help="seed of the chains' random numbers")
    args = ap.parse_args(argv)
    results = []
    for nt in args.nt:
        t0 = time.perf_counter()
        # N_MD = N_t / 8 keeps the acceptance near the paper's target 0.66
        r = run(nt, n_chains=args.chains, n_therm=args.therm, n_meas=args.meas, n_md=max(4, nt // 8),
                seed=args.seed + nt, progress=100)
        r["beta"] = 8.0
        r["seconds"] = round(time.perf_counter() - t0, 1)
        results.append(r)
        print(json.dumps(r), flush=True)
    if len(results) >= 2:
        out = {"continuum": {}}
        for name in ("Gamma", "M"):
            e0, de = continuum(results, name)
            out["continuum"][f"E_{name}"] = round(e0, 4)
            out["continuum"][f"E_{name}_err"] = round(de, 4)
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

