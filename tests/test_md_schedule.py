"""The library's molecular-dynamics schedule (host code, no GPU) against the oracle's
literal recursion of the nested Omelyan integrator (Sec. 5.2).

The library merges every run of consecutive kicks into one group (one batched solve
per group on the device) and drops zero kicks; the oracle kicks one level at a time.
Merging the oracle's trace the same way must give the library's schedule.
"""
import ctypes

import pytest

from oracle import hmc as ohmc
from paper_1804_07195_amd import binding as hb

ZETA = 0.1931833275037836


def _oracle_ops(N, n_md, t, zeta):
    n = len(N)
    ops = []

    def kick(level, eps):
        if eps == 0.0:
            return
        if not ops or ops[-1][0] != "kick":
            ops.append(["kick", [0.0] * (n + 1)])
        ops[-1][1][level] += eps

    def drift(eps):
        if ops and ops[-1][0] == "drift":
            ops[-1][1] += eps
        else:
            ops.append(["drift", eps])

    ohmc.Integrator(N, n_md, t, zeta).run(kick, drift)
    return ops


CASES = [
    ([], 10, 1.0, ZETA),
    ([], 7, 0.5, 0.0),            # leapfrog: one force per step
    ([2, 2], 30, 1.0, ZETA),      # the paper's 102x102 two-mass run: N_MD = 30, N_0 = N_1 = 2
    ([3, 1], 9, 1.0, ZETA),       # odd ratios at both levels
    ([6, 3, 1], 12, 0.8, ZETA),
    ([5], 15, 1.2, 0.25),
    ([4, 2], 8, 1.0, 0.0),
]


@pytest.mark.parametrize("N,n_md,t,zeta", CASES)
def test_schedule_matches_oracle_recursion(N, n_md, t, zeta):
    p = hb.hmc_params(0.5, n_md, [0.1] * len(N), N, traj_length=t, zeta=zeta)
    got = hb.hub_md_schedule(p)
    want = _oracle_ops(N, n_md, t, zeta)
    assert len(got) == len(want)
    for (kg, vg), (kw, vw) in zip(got, want):
        assert kg == kw
        if kg == "drift":
            assert abs(vg - vw) <= 1e-15 * abs(vw)
        else:
            assert all(abs(a - b) <= 1e-15 * max(abs(b), 1e-300) for a, b in zip(vg, vw))


@pytest.mark.parametrize("N,n_md,t,zeta", CASES)
def test_schedule_conserves_time(N, n_md, t, zeta):
    # every level's kicks add up to t (sum of c_i, d_i = 1 per step), the drifts to t
    p = hb.hmc_params(0.5, n_md, [0.1] * len(N), N, traj_length=t, zeta=zeta)
    ops = hb.hub_md_schedule(p)
    assert abs(sum(v for k, v in ops if k == "drift") - t) < 1e-13
    for lev in range(len(N) + 1):
        assert abs(sum(v[lev] for k, v in ops if k == "kick") - t) < 1e-13
    # kicks and drifts alternate, and the trajectory is symmetric
    kinds = [k for k, _ in ops]
    assert all(a != b for a, b in zip(kinds, kinds[1:]))
    assert kinds == kinds[::-1]


def test_paper_two_mass_schedule_cost():
    # 102x102, N_t = 64 (Table tab_nmds): N_MD = 30, N_MD / N_0 = 15 outermost steps
    p = hb.hmc_params(0.7, 30, [0.076, 0.2055], [2, 2])
    ops = hb.hub_md_schedule(p)
    kicks = [v for k, v in ops if k == "kick"]
    evals = [sum(1 for v in kicks if v[l] != 0.0) for l in range(3)]
    # outer levels: 2 merged kicks per step + 1; innermost: 2 per inner step + 1
    assert evals == [31, 31, 61]


@pytest.mark.parametrize("bad", [dict(N=[3], n_md=10), dict(N=[2, 3], n_md=6), dict(N=[0], n_md=4),
                                 dict(N=[], n_md=0), dict(N=[], n_md=4, t=-1.0), dict(N=[], n_md=4, zeta=0.7)])
def test_schedule_rejects_bad_parameters(bad):
    p = hb.hmc_params(0.5, bad["n_md"], [0.1] * len(bad["N"]), bad["N"], traj_length=bad.get("t", 1.0),
                      zeta=bad.get("zeta", ZETA))
    cnt = ctypes.c_int32()
    assert hb.load().hub_md_schedule(ctypes.byref(p), None, 0, ctypes.byref(cnt)) == hb.HUB_ERR_ARG
    assert len(hb.load().hub_last_error()) > 0
