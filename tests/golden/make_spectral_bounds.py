"""Write tests/golden/lambda_max_large2.txt: the largest eigenvalue of M M^dagger on the
seeded 102x102, N_t = 64 workload field, computed by ARPACK on the oracle's operator.

Calls only `oracle/` and the seeded input generator (about a minute on 8 cores):
    python tests/golden/make_spectral_bounds.py
"""
import os
import sys

import numpy as np
import scipy.sparse.linalg as spla

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.operator import NormalOperator  # noqa: E402
from workloads import WORKLOADS, draw_inputs  # noqa: E402


def main():
    w = WORKLOADS["large2"]
    lat = oracle.Lattice(w.L1, w.L2, w.Nt, w.kappa_t, w.ms_t)
    phi, _ = draw_inputs(w, batch=1)
    A = NormalOperator(lat, phi, 0.0)
    op = spla.LinearOperator((lat.n, lat.n), matvec=A, dtype=np.complex128)
    lmax = float(spla.eigsh(op, k=1, which="LA", return_eigenvectors=False, tol=1e-12)[0])
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lambda_max_large2.txt")
    with open(out, "w") as f:
        f.write("# lambda_max of M M^dagger, workload large2 (102x102, N_t = 64, seed 4), the phi drawn by\n")
        f.write("# workloads.draw_inputs(w, batch=1); ARPACK (eigsh, tol 1e-12) on oracle.NormalOperator.\n")
        f.write("# Written by tests/golden/make_spectral_bounds.py.\n")
        f.write(f"lambda_max {lmax:.15e}\n")
    print(out, lmax)


if __name__ == "__main__":
    main()
