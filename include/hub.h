/*
 * hub.h - C ABI of libhub: the fermion-matrix solve of Hybrid Monte Carlo for the
 * Hubbard model on the honeycomb lattice (Krieg, Luu, Ostmeyer, Papaphilippou,
 * Urbach, "Accelerating Hybrid Monte Carlo simulations of the Hubbard model on the
 * hexagonal lattice").
 *
 * Conventions shared by every call
 * --------------------------------
 * Lattice.  L1 x L2 rhombic unit cells with a two-site basis (A = sublattice 0,
 *   B = sublattice 1), periodic along both oblique axes, N_t time slices.  The A
 *   site of cell (i, j) is bonded to the B sites of cells (i, j), (i-1, j) and
 *   (i, j-1), indices mod L1, L2.  There are N = 2*L1*L2*N_t unknowns.
 * Layout.  Every site field is stored site-major with flat index
 *   ((t*2 + s)*L1 + i)*L2 + j, j fastest.  Complex vectors are interleaved
 *   (re, im) float64 pairs; batched vectors are [batch][N].  phi is real float64 [N].
 * Memory.  Every pointer marked "device" is device memory owned by the caller on
 *   the context's device; "host" pointers are ordinary host memory.  No call frees
 *   or retains a caller buffer beyond its return, except hub_submit (see there).
 * Streams.  Calls taking a hipStream_t enqueue their kernels on that stream (0 =
 *   the null stream) and are stream-ordered with the caller's other work.
 *   hub_apply_*, hub_force and hub_force_sum return without synchronising.  The
 *   solvers and hub_action synchronise the stream: the host drives the outer
 *   iteration (Arnoldi steps, restarts, the true-residual tests) and reads a few
 *   scalars back between kernels, so these calls return once their results are in.
 * Errors.  Every call returns a hub_status; HUB_OK is 0.  On failure
 *   hub_last_error() returns a message for the calling thread.  No call throws.
 *   Argument errors (null pointers, non-positive sizes, batch beyond
 *   HUB_MAX_BATCH, non-finite couplings or tolerances, an output buffer that
 *   overlaps an input or another output) return HUB_ERR_ARG before anything is
 *   enqueued.  The solvers also check the device data they are given: a
 *   non-finite value in phi, the right-hand side or the initial guess shows in the
 *   first reduction of the solve and ends that system with HUB_ERR_ARG
 *   (converged = 0, the solution undefined).  The other calls do not inspect
 *   device data: non-finite input gives non-finite output.
 */
#ifndef HUB_H
#define HUB_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HUB_MAX_BATCH 64     /* systems per hub_apply_* / hub_solve / hub_force call */
#define HUB_MAX_RESTART 20   /* largest FGMRES restart length m                      */
#define HUB_MAX_HB_MASSES 16 /* staggered Hasenbusch masses per hub_hasenbusch_* call */
#define HUB_MAX_SHIFTS 17    /* shifts per hub_solve_multishift call                 */

typedef struct { double re, im; } hub_c128;

/* The lattice and the step-size-weighted couplings of eq. (ferm_op):
 * kappa_t = delta*kappa (hopping entry of M^{AB}), ms_t = delta*m_s (staggered
 * mass on the temporal hop), delta = beta/N_t (Sec. 2). */
typedef struct {
  int32_t L1, L2;    /* unit cells along the two oblique axes, >= 1 */
  int32_t Nt;        /* time slices, >= 1                           */
  int32_t reserved;  /* must be 0                                   */
  double kappa_t;
  double ms_t;
} hub_lattice;

typedef enum {
  HUB_OK = 0,
  HUB_ERR_ARG = 1,       /* invalid argument; nothing was enqueued                  */
  HUB_ERR_OOM = 2,       /* workspace beyond the context's HBM budget               */
  HUB_ERR_NOCONV = 3,    /* iteration limit reached; x holds the last iterate       */
  HUB_ERR_HIP = 4,       /* a HIP runtime call failed                               */
  HUB_ERR_BUSY = 5,      /* request can never fit the serving budget                */
  HUB_ERR_NOTFOUND = 6   /* unknown ticket                                          */
} hub_status;

typedef struct hub_ctx hub_ctx;

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the workspace
 * the library allocates for solves and the serving queue (0 = 75% of the device
 * memory free at creation).  The context owns a workspace pool and, once
 * hub_submit is first called, a serving thread. */
hub_status hub_create(hub_ctx **ctx, int device, size_t hbm_budget_bytes);
/* Wait for outstanding served requests, stop the serving thread, free all workspace. */
hub_status hub_destroy(hub_ctx *ctx);
/* Message describing the last failure on the calling thread ("" if none). */
const char *hub_last_error(void);

/* y_b = M[phi] x_b (eq. (ferm_op)) for b < batch, phi shared by the batch.
 *   A rows: y_A(t) = -x_A(t) + s(t) (e^{i phi_A(t)} - ms_t) x_A(t-1) - kappa_t sum_bonds x_B(t)
 *   B rows: y_B(t) = +x_B(t) - s(t) (e^{-i phi_B(t)} - ms_t) x_B(t+1) - kappa_t sum_bonds x_A(t)
 * s = -1 on the hop that wraps the antiperiodic temporal boundary, else +1.
 * phi: device float64 [N]; x, y: device [batch][N]; x and y must not overlap. */
hub_status hub_apply_M(hub_ctx *ctx, const hub_lattice *lat, const double *phi,
                       const hub_c128 *x, hub_c128 *y, int32_t batch, hipStream_t stream);

/* y_b = M[phi]^dagger x_b, the conjugate transpose of hub_apply_M (used for
 * xi = M^dagger eta, eq. (eta_xi), and chi = M^dagger eta sources).  Same layout. */
hub_status hub_apply_Mdag(hub_ctx *ctx, const hub_lattice *lat, const double *phi,
                          const hub_c128 *x, hub_c128 *y, int32_t batch, hipStream_t stream);

/* y_b = (M M^dagger + mu2[b]) x_b: the Hermitian positive-definite normal operator
 * of Sec. 3 with the Hasenbusch shift of Sec. 5.1.  mu2: host float64 [batch], each
 * finite and >= 0.  Uses library workspace for M^dagger x (HUB_ERR_OOM if over budget). */
hub_status hub_apply_normal(hub_ctx *ctx, const hub_lattice *lat, const double *phi, const double *mu2,
                            const hub_c128 *x, hub_c128 *y, int32_t batch, hipStream_t stream);

/* Bytes of the scratch array behind hub_apply_normal_noalloc (64 MiB per device). */
#define HUB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* hub_apply_normal for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops that must not call hipMalloc): the same kernels and
 * results, with the intermediate M^dagger x in a scratch array that the library holds
 * on each device from the first hub_create on that device until the process ends,
 * instead of context workspace.  Allocates nothing.  batch * N * 16 bytes must not
 * exceed HUB_NOALLOC_SCRATCH_BYTES (else HUB_ERR_ARG; at 102x102x64 that is a batch
 * of up to 3).  Every call on one device uses the same array: calls that overlap in
 * time on one device (other streams, threads or contexts) race, and the caller must
 * order them (one stream, or events).  Returns without synchronising. */
hub_status hub_apply_normal_noalloc(hub_ctx *ctx, const hub_lattice *lat, const double *phi, const double *mu2,
                                    const hub_c128 *x, hub_c128 *y, int32_t batch, hipStream_t stream);

typedef enum {
  HUB_CG_FP64 = 0,        /* double-precision CG (Sec. 3)                                 */
  HUB_FGMRES_MIXED = 1    /* FP64 flexible GMRES(m) with complex64 CG preconditioner (App. A) */
} hub_solver;

typedef struct {
  int32_t solver;          /* hub_solver                                                    */
  int32_t max_iter;        /* CG: iteration limit; FGMRES: limit on restart cycles (exact)  */
  int32_t restart_m;       /* FGMRES restart length m (1..HUB_MAX_RESTART), paper: 10       */
  int32_t inner_max_iter;  /* iteration cap of each single-precision CG                     */
  double tol;              /* relative true-residual target ||b - A x|| / ||b||             */
  double inner_a;          /* factor a of the inner tolerance TOL*a*|b|/ERR, paper: 5       */
  double inner_floor;      /* smallest inner relative tolerance requested in complex64      */
  int32_t use_x0;          /* 1: x holds an initial guess on entry; 0: start from zero      */
  int32_t check_every;     /* iterations enqueued between convergence checks (>= 1)         */
} hub_solve_opts;

/* tol 1e-10, FP64 CG, max_iter 20000, m 10, a 5, inner_floor 1e-5, inner_max_iter 4000,
 * use_x0 0, check_every 8. */
void hub_default_opts(hub_solve_opts *opts);

typedef struct {
  int32_t converged;       /* 1 iff the recomputed FP64 true residual met tol             */
  int32_t outer_iters;     /* CG: restarts after a failed true-residual check; FGMRES: cycles */
  int32_t inner_iters;     /* CG iterations (FP64 CG) or complex64 CG iterations (FGMRES) */
  int32_t applies;         /* FP64 applications of M M^dagger + mu2 outside CG iterations */
  double true_rel_resid;   /* ||b - (M M^dagger + mu2) x|| / ||b||, FP64                   */
} hub_solve_info;

/* Solve (M M^dagger + mu2[b]) x_b = b_b for every b < batch with one shared phi
 * (Sec. 3: the system (M M^dagger) eta = chi; Sec. 5.1: shifted systems; App. A:
 * flexible GMRES).  Systems converge independently.  b, x: device [batch][N]; x is
 * read as initial guess iff opts->use_x0.  mu2: host [batch].  info: host [batch],
 * filled on return.  opts may be NULL (defaults).  Synchronises `stream`.
 * Returns HUB_ERR_NOCONV if any system missed tol (x holds its last iterate). */
hub_status hub_solve(hub_ctx *ctx, const hub_lattice *lat, const double *phi, const double *mu2,
                     int32_t batch, const hub_c128 *b, hub_c128 *x, const hub_solve_opts *opts,
                     hub_solve_info *info, hipStream_t stream);

/* hub_solve for systems on several fields: system k < batch uses the field
 * phi + (k / per_field) * N, so phi holds batch / per_field fields [batch / per_field][N]
 * (device float64), each shared by per_field consecutive systems (several right-hand
 * sides or shifts per field, several fields in one call: independent Markov chains
 * measured together).  batch must be a positive multiple of per_field.  Otherwise as
 * hub_solve (Sec. 3, App. A); all systems share opts and converge independently. */
hub_status hub_solve_fields(hub_ctx *ctx, const hub_lattice *lat, const double *phi, int32_t per_field,
                            const double *mu2, int32_t batch, const hub_c128 *b, hub_c128 *x,
                            const hub_solve_opts *opts, hub_solve_info *info, hipStream_t stream);

/* y_k = M[phi_f] x_k (dag = 0) or M[phi_f]^dagger x_k (dag = 1) with f = k / per_field
 * and the fields phi [batch / per_field][N] as in hub_solve_fields (eq. (ferm_op)).
 * x, y: device [batch][N], not overlapping.  Returns without synchronising. */
hub_status hub_apply_fields(hub_ctx *ctx, const hub_lattice *lat, const double *phi, int32_t per_field,
                            int32_t dag, const hub_c128 *x, hub_c128 *y, int32_t batch, hipStream_t stream);

/* dSdphi_b (+)= scale * dS/dphi for S = Re chi^dagger (M M^dagger + mu2)^{-1} chi,
 * given eta_b = (M M^dagger + mu2)^{-1} chi_b (eqs. (p_dot), (eta_xi)):
 *   dS/dphi_{A,x,t} = 2 Im[ conj(eta_A(t)) s(t) e^{ i phi_A(t)} xi_A(t-1) ]
 *   dS/dphi_{B,x,t} = 2 Im[ conj(eta_B(t)) s(t) e^{-i phi_B(t)} xi_B(t+1) ]
 * with xi = M^dagger eta.  This is minus the molecular-dynamics force of eq. (p_dot).
 * xi: device [batch][N] or NULL (then computed into library workspace).
 * accumulate = 0 overwrites dSdphi, 1 adds to it.  dSdphi: device float64 [batch][N]. */
hub_status hub_force(hub_ctx *ctx, const hub_lattice *lat, const double *phi, const hub_c128 *eta,
                     const hub_c128 *xi, double scale, int32_t accumulate, double *dSdphi,
                     int32_t batch, hipStream_t stream);

/* dSdphi (+)= sum_b scale[b] * dS_b/dphi: the forces of a batch of pseudofermion terms
 * on one phi (eqs. (p_dot), (eta_xi)), contracted as in hub_force and summed into one
 * field, with phi, its phase and the temporal neighbour of each site evaluated once per
 * site for the whole batch (molecular-dynamics kicks and the gradient of a sum of
 * actions need only the sum).  eta: device [batch][N]; xi: device [batch][N] or NULL
 * (then M^dagger eta is computed into library workspace); scale: host float64 [batch],
 * finite; accumulate = 0 overwrites dSdphi, 1 adds to it.  dSdphi: device float64 [N],
 * not overlapping phi, eta or xi. */
hub_status hub_force_sum(hub_ctx *ctx, const hub_lattice *lat, const double *phi, const hub_c128 *eta,
                         const hub_c128 *xi, const double *scale, int32_t accumulate, double *dSdphi,
                         int32_t batch, hipStream_t stream);

/* S_b = Re chi_b^dagger eta_b, the pseudofermion action of eq. (hamiltonian) given
 * eta = (M M^dagger + mu2)^{-1} chi.  FP64 reduction with a fixed summation order.
 * chi, eta: device [batch][N]; S: host float64 [batch].  Synchronises `stream`. */
hub_status hub_action(hub_ctx *ctx, const hub_lattice *lat, const hub_c128 *chi, const hub_c128 *eta,
                      int32_t batch, double *S, hipStream_t stream);

/* Several shifts of one right-hand side: x_s = (M M^dagger + mu2[s])^{-1} b for
 * s < nshift, from one shared Krylov space (Sec. 5.1 shifts; the paper names
 * multi-shift solvers without giving one: this is CG for shifted systems).  One FP64
 * CG runs on the smallest shift; the other systems follow through scalar
 * recurrences and stop updating once their own residual meets tol.  Every x_s is
 * then certified by its FP64 true residual (a warm-started CG that returns at once
 * when the tolerance is met, else finishes the solve).  b: device [N]; x: device
 * [nshift][N]; mu2: host [nshift]; info: host [nshift] (outer_iters = shared Krylov
 * iterations, inner_iters = iterations of the certifying CG).  opts: tol, max_iter,
 * check_every (solver and use_x0 are ignored).  lambda: host [2] or NULL; receives
 * the extreme eigenvalues of the Lanczos matrix of the shared CG (its coefficients
 * alpha_k, beta_k), shifted back to M M^dagger: estimates of lambda_min and
 * lambda_max of eq. (solver_time_eqn).  Synchronises `stream`. */
hub_status hub_solve_multishift(hub_ctx *ctx, const hub_lattice *lat, const double *phi, const double *mu2,
                                int32_t nshift, const hub_c128 *b, hub_c128 *x, const hub_solve_opts *opts,
                                hub_solve_info *info, double *lambda, hipStream_t stream);

/* Host only: n Hasenbusch masses spaced geometrically between the spectral bounds,
 * mu_i = lambda_min (lambda_max / lambda_min)^((i+1)/(n+1)), i < n (eq. (mu_i_eqn)).
 * mu: host [n]; needs 0 < lambda_min < lambda_max and 1 <= n <= HUB_MAX_HB_MASSES. */
hub_status hub_hasenbusch_masses(double lambda_min, double lambda_max, int32_t n, double *mu);

/* Staggered-mass Hasenbusch split (Sec. 5.1).  The pseudofermion term is replaced by
 * n+1 terms built from M_i = M(m_s = mu_i), i = 0..n-1, with M_{-1} = M(lat->ms_t)
 * (the paper's M, m_s = 0).  mt: host [n], the staggered masses as m~_i = delta*mu_i
 * (the convention of hub_lattice.ms_t), 0 <= n <= HUB_MAX_HB_MASSES (n = 0: the one
 * plain pseudofermion term of eq. (hamiltonian); mt may then be NULL).  Term i of
 * pseudofermion chi_i (device [n+1][N], term order 0..n):
 *   term n   : S_n = chi_n^dag (M_{n-1} M_{n-1}^dag)^{-1} chi_n
 *   term i<n : S_i = (M_i chi_i)^dag (M_{i-1} M_{i-1}^dag)^{-1} (M_i chi_i)
 *
 * Heat-bath: chi_n = M_{n-1} rho_n and chi_i = M_i^{-1} M_{i-1} rho_i
 * = M_i^dag (M_i M_i^dag)^{-1} M_{i-1} rho_i for i < n, so that S_i = rho_i^dag rho_i.
 * rho: device [n+1][N], drawn by the caller with density e^{-rho^dag rho}.  The n
 * solves run as one batch.  info: host [n] (solve i; may be NULL if n = 0).  opts may be NULL; use_x0 is
 * ignored.  Synchronises `stream`.  HUB_ERR_NOCONV if a solve missed tol (chi is
 * still written from its last iterate). */
hub_status hub_hasenbusch_heatbath(hub_ctx *ctx, const hub_lattice *lat, const double *phi, const double *mt,
                                   int32_t n, const hub_c128 *rho, hub_c128 *chi, const hub_solve_opts *opts,
                                   hub_solve_info *info, hipStream_t stream);

/* Actions and summed force of the terms selected by term_mask (bit i = term i, at
 * least one bit, none above bit n), for multi-time-scale integration where terms
 * are evaluated at different rates (Sec. 5.2).  For each selected term the solve
 *   (M_d M_d^dag) eta_i = rhs_i,  d = n-1 for term n and i-1 for i < n,
 *   rhs_n = chi_n, rhs_i = M_i chi_i,
 * runs in one batch with the others; then xi_i = M_d^dag eta_i (eq. (def_xi_i)),
 * S_i = Re rhs_i^dag eta_i, and
 *   dSdphi (+)= scale * sum_i dS_i/dphi,
 *   dS_n/dphi = -2 Re(eta_n^dag dM/dphi xi_n),
 *   dS_i/dphi = -2 Re(eta_i^dag dM/dphi (xi_i - chi_i))   (minus eq. (f_chi_i)),
 * the same contraction as hub_force.  eta: device [n+1][N], in/out: the selected
 * terms' solutions are written there (and read as initial guesses iff
 * opts->use_x0); other terms are untouched.  S: host [n+1] or NULL; info: host
 * [n+1]; only selected entries are written.  accumulate = 0 overwrites dSdphi
 * (device float64 [N]), 1 adds to it.  Synchronises `stream`.  HUB_ERR_NOCONV if a
 * solve missed tol (the outputs are still computed from its last iterate). */
hub_status hub_hasenbusch_force(hub_ctx *ctx, const hub_lattice *lat, const double *phi, const double *mt,
                                int32_t n, const hub_c128 *chi, uint32_t term_mask, double scale,
                                int32_t accumulate, double *dSdphi, double *S, hub_c128 *eta,
                                const hub_solve_opts *opts, hub_solve_info *info, hipStream_t stream);

/* Hybrid Monte Carlo update (Sec. 2) with the nested second-order Omelyan
 * integrator of Sec. 5.2 on the Hamiltonian of eq. (hamiltonian),
 *   H = phi^T phi / (2 U_t) + sum_{i=0..n} S_i(phi) + pi^T pi / 2,
 * S_i the terms of the staggered-mass split above (n = 0: one plain term).
 * Molecular dynamics: T(h) = T_F(zeta h) T_pi(h/2) T_F((1-2 zeta) h) T_pi(h/2) T_F(zeta h)
 * with T_F(e): pi -= e dS/dphi and T_pi(e): phi += e pi.  Level k < n kicks with the
 * force of term k and takes steps of n_scale[k] innermost steps; level n kicks with
 * the gauge force phi/U_t plus term n and drifts phi, n_md steps of traj_length/n_md.
 * n_scale[k+1] must divide n_scale[k] and n_scale[0] must divide n_md (the paper's
 * N_i); an odd ratio cuts the inner step next to the middle kick in half as the
 * paper prescribes.  zeta = 0 is the leapfrog.  The paper uses zeta = 0.193. */
typedef struct {
  double traj_length;                  /* trajectory length t > 0                        */
  double zeta;                         /* Omelyan parameter in [0, 0.5]                  */
  double U_t;                          /* delta*U > 0: variance of phi in the gauge term */
  int32_t n_md;                        /* innermost steps per trajectory, >= 1           */
  int32_t n;                           /* Hasenbusch masses, 0..HUB_MAX_HB_MASSES        */
  double mt[HUB_MAX_HB_MASSES];        /* m~_i = delta*mu_i, i < n                       */
  int32_t n_scale[HUB_MAX_HB_MASSES];  /* N_i, i < n                                     */
  int32_t flags;                       /* 0 or HUB_HMC_CHI_GIVEN                         */
  int32_t pad;
} hub_hmc_params;

/* hub_hmc_params.flags: the rho argument of hub_hmc_trajectory holds the
 * pseudofermions chi_0..chi_n themselves and the heat-bath is skipped. */
#define HUB_HMC_CHI_GIVEN 1

/* One operation of the molecular-dynamics schedule: kind 0 moves phi += eps * pi;
 * kind 1 is a group of momentum kicks at one phi, pi -= sum_l coef[l] dS_l/dphi
 * (level l: term l, plus the gauge force for l = n).  Consecutive kicks are merged
 * into one group (their solves run as one batch); zero kicks are dropped. */
typedef struct {
  int32_t kind;
  int32_t reserved;
  double eps;
  double coef[HUB_MAX_HB_MASSES + 1];
} hub_md_op;

typedef struct {
  double dH;                                /* H(end) - H(start), FP64                  */
  double H0, H1;                            /* the Hamiltonian at both ends             */
  int32_t accepted;                         /* u < exp(-dH)                              */
  int32_t kick_groups;                      /* momentum-update groups executed          */
  int32_t drifts;                           /* phi updates executed                      */
  int32_t reserved;
  int64_t inner_iters;                      /* CG iterations over all solves (inner for FGMRES) */
  int32_t force_evals[HUB_MAX_HB_MASSES + 1];  /* solves per term                        */
  int32_t pad;
} hub_hmc_info;

/* Host only (no device call): the schedule of one trajectory.  ops: host array of
 * max_ops entries or NULL (then only *count is set). */
hub_status hub_md_schedule(const hub_hmc_params *params, hub_md_op *ops, int32_t max_ops, int32_t *count);

/* One HMC update.  phi: device [N] float64, in/out: the accepted field (the start
 * field again on rejection).  pi: device [N], in: the momenta drawn by the caller
 * with density e^{-pi^2/2}; out: the momenta at the end of the trajectory (whether
 * or not it is accepted).  rho: device [n+1][N], the heat-bath vectors (density
 * e^{-rho^dag rho}); the pseudofermions are chi = heat-bath(rho) as in
 * hub_hasenbusch_heatbath (with HUB_HMC_CHI_GIVEN: rho holds chi itself).
 * u: the uniform random number of the Metropolis step,
 * in [0, 1]; the trajectory is accepted iff u < exp(-dH).  Solves use opts (NULL =
 * defaults); with opts->use_x0 = 1 each solve after the first of its term starts
 * from the term's previous solution.  info: host.  Synchronises `stream`.  Returns
 * HUB_ERR_NOCONV if a solve missed its tolerance; on any failure phi is restored
 * to the start field and pi is left undefined. */
hub_status hub_hmc_trajectory(hub_ctx *ctx, const hub_lattice *lat, double *phi, double *pi, const hub_c128 *rho,
                              double u, const hub_hmc_params *params, const hub_solve_opts *opts,
                              hub_hmc_info *info, hipStream_t stream);

/* One HMC update of each of nchain independent Markov chains on the same lattice,
 * advanced through the same molecular-dynamics schedule in lockstep: every kick
 * group solves the selected terms of all chains in one batch (small lattices, such
 * as the 4-site benchmark of Sec. 7.2, fill the device only this way).  Each chain
 * is updated exactly as by hub_hmc_trajectory with its own phi, pi, rho and u.
 * phi, pi: device [nchain][N]; rho: device [nchain][n+1][N]; u, info: host
 * [nchain].  Needs nchain * (n + 1) <= HUB_MAX_BATCH. */
hub_status hub_hmc_trajectories(hub_ctx *ctx, const hub_lattice *lat, int32_t nchain, double *phi, double *pi,
                                const hub_c128 *rho, const double *u, const hub_hmc_params *params,
                                const hub_solve_opts *opts, hub_hmc_info *info, hipStream_t stream);

/* Serving: one request = solve (M M^dagger + mu2) x = chi, then S = Re chi^dagger x and
 * dS/dphi, for its own lattice, phi and shift.  Requests are admitted by workspace
 * footprint against the budget as earlier ones retire and run batched with every
 * other request in flight, whatever their lattice sizes (continuous batching).  The
 * result of a request does not depend on which others share its launches.
 * phi, chi, x_out, dSdphi_out: device memory that must stay valid and untouched
 * until hub_poll reports done.  S_out: host, written before done is reported.
 * dSdphi_out may be NULL (no force). */
typedef struct {
  hub_lattice lat;
  double mu2;
  const double *phi;
  const hub_c128 *chi;
  hub_c128 *x_out;
  double *S_out;
  double *dSdphi_out;
  hub_solve_opts opts;
} hub_request;

/* Queue a request; returns at once with a ticket.  HUB_ERR_BUSY if the request alone
 * exceeds the serving budget, HUB_ERR_ARG for invalid fields (x_out and dSdphi_out
 * must not overlap each other, chi or phi). */
hub_status hub_submit(hub_ctx *ctx, const hub_request *req, uint64_t *ticket);
/* Never blocks.  *done = 0 and HUB_OK while the request runs.  Once it is finished,
 * *done = 1, info (if not NULL) is filled, the ticket is released and the return
 * value is the request's own final status: HUB_OK; HUB_ERR_NOCONV if it missed its
 * tolerance (x_out, S and the force then come from its last iterate); HUB_ERR_ARG if
 * phi or chi held a non-finite value; HUB_ERR_HIP if a HIP call failed while it ran.
 * Unknown tickets: HUB_ERR_NOTFOUND with *done = 0. */
hub_status hub_poll(hub_ctx *ctx, uint64_t ticket, int32_t *done, hub_solve_info *info);

/* Measurement: time every launch of the solver's CG-iteration kernels with HIP
 * events on the solve's stream.  Stats are per kernel: "cg1_f64", "cg2_f64" (the
 * two kernels of an FP64 CG iteration of a tiled system), "cg1_c64", "cg2_c64" (the
 * same for the complex64 inner CG), and "cgwg_f64", "cgwg_c64" (the single-workgroup
 * kernel that runs a whole block of CG iterations of each system of at most 20480
 * sites in one launch; its bytes are not counted: it is latency-bound).  bytes accumulates the algorithmic bytes of every timed
 * launch: per site the distinct vector reads and writes and the phase source
 * (FP64: a 16-byte (cos, sin) pair, 80 bytes in stage 1, 80 or 128 in stage 2, the
 * larger at the odd iterations that also update the solution; complex64: a 4-byte
 * angle, 36 bytes in stage 1, 36 or 60 in stage 2), times the sites of the systems
 * that iterated in that launch.  Timing adds an event record around each launch; it
 * is off by default.
 * hub_profile_enable resets the stats; enable = 0 turns timing off. */
typedef struct {
  char name[16];
  int64_t launches;
  double total_ms;
  double bytes;
} hub_kernel_stat;

hub_status hub_profile_enable(hub_ctx *ctx, int32_t enable);
/* Copy up to `max` stats (synchronous solves on every stream of the context) into
 * out (host); *count receives the number written. */
hub_status hub_profile_read(hub_ctx *ctx, hub_kernel_stat *out, int32_t max, int32_t *count);

/* Measurement: a streaming kernel that moves exactly the bytes of one FP64 apply of n
 * sites and does nothing else (per site: x and phi read, y = (Re x * phi, Im x + phi)
 * written; no stencil, no phase; the apply's grid, tile and workgroup order).  It is
 * the bandwidth ceiling hub_apply_M is compared with in the same process.  mode 0:
 * plain loads and non-temporal stores (the store policy of hub_apply_M); 1:
 * non-temporal loads and plain stores; 2: plain loads and stores.  phi: device
 * float64 [n]; x, y: device [n], y not overlapping x or phi.  Returns without
 * synchronising. */
hub_status hub_profile_stream(hub_ctx *ctx, const double *phi, const hub_c128 *x, hub_c128 *y, int64_t n,
                              int32_t mode, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HUB_H */
