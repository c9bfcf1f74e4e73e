"""CPU oracle for the fermion-matrix solve of Hubbard-model HMC on the honeycomb lattice.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import anything from here.  The product path
(the HIP library and its Python binding) never calls this code, and this code
never calls the product path: the two share no kernels, headers, helpers or
constants.  The seeded input generators live in `workloads`, which holds none of
the method's arithmetic.

Everything here is plain, slow and written from the paper's definitions in
complex128 / float64 with NumPy and SciPy sparse matrices:

* `operator`  - the fermion matrix M[phi] entry by entry from eq. (ferm_op), its
                adjoint and the normal operator M M^dagger + mu^2 (Sec. 2-3);
* `solve`     - the exact solution of (M M^dagger + mu^2) x = b by dense LU or by
                textbook CG certified by an FP64 true residual (Sec. 3), and a
                step-by-step reading of the flexible GMRES of Appendix A
                (Algorithm A.1) as a method oracle for iteration counts;
* `force`     - the pseudofermion action S = chi^dagger (M M^dagger)^{-1} chi of
                eq. (hamiltonian) and its derivative dS/dphi from eqs. (p_dot),
                (eta_xi), contracting the explicit derivative of M;
* `hasenbusch` - the staggered-mass Hasenbusch split of Sec. 5.1: heat-bath of the
                n+1 pseudofermions, the per-term actions and the ratio forces of
                eq. (f_chi_i);
* `hmc`       - the HMC update of Sec. 2 with the nested second-order Omelyan
                integrator of Sec. 5.2 and the Metropolis step;
* `multishift` - several shifts mu^2 of one right-hand side (plain solves and the
                shared-Krylov CG-M), Lanczos extremes of M M^dagger from the CG
                coefficients, and the Hasenbusch masses of eq. (mu_i_eqn);
* `ed`        - exact diagonalisation of the Hubbard Hamiltonian on the 4-site
                (2 x 1 cells) honeycomb of Sec. 7.2: quasi-particle energies and
                thermal correlators;
* `correlators` - single-particle correlators from M^{-1} and the exponential fits
                that extract quasi-particle energies (Sec. 7.2).

Every function is pinned by a test in `tests/test_oracle_pins.py` or
`tests/test_oracle_hasenbusch.py`, `tests/test_oracle_hmc.py` or
`tests/test_oracle_multishift.py`, `tests/test_oracle_ed.py`,
`tests/test_oracle_correlators.py` against a
closed form, an invariance or brute force that does not reuse its code.
"""
from .operator import Lattice, build_M, build_M_dense_loops, apply_M, apply_Mdag, normal_apply, site_index
from .solve import solve, solve_dense, cg, true_rel_residual, fgmres_alg_a1
from .force import action, force, xi_from_eta
from . import correlators, ed, hasenbusch, hmc, multishift

__all__ = [
    "Lattice", "build_M", "build_M_dense_loops", "apply_M", "apply_Mdag", "normal_apply", "site_index",
    "solve", "solve_dense", "cg", "true_rel_residual", "fgmres_alg_a1",
    "action", "force", "xi_from_eta", "hasenbusch", "hmc", "multishift", "ed", "correlators",
]
