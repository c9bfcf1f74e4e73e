"""Shared helpers of the GPU parity tests (marshalling only, no arithmetic of the method)."""
import numpy as np
import torch

import oracle
from paper_1804_07195_amd import binding


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def lattices(L1, L2, Nt, kappa_t, ms_t=0.0):
    return binding.lattice(L1, L2, Nt, kappa_t, ms_t), oracle.Lattice(L1, L2, Nt, kappa_t, ms_t)


def of_workload(w):
    return lattices(w.L1, w.L2, w.Nt, w.kappa_t, w.ms_t)


def rel_max(got, want):
    scale = max(1.0, float(np.abs(want).max()))
    return float(np.abs(got - want).max()) / scale


def rel2(got, want):
    return float(np.linalg.norm((got - want).ravel()) / np.linalg.norm(np.asarray(want).ravel()))
