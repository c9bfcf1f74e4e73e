"""ctypes binding of libhub (include/hub.h), argument marshalling only.

Torch tensors provide device memory and the current HIP stream; every step of
the computation runs in the library's HIP kernels.  Site fields use the layout
[batch][N_t][2][L1][L2] (complex128) or [N_t][2][L1][L2] (float64 phi).

Importing this module never loads the library; the first call does, and raises
RuntimeError if libhub.so is missing (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhub.so")

HUB_OK, HUB_ERR_ARG, HUB_ERR_OOM, HUB_ERR_NOCONV, HUB_ERR_HIP, HUB_ERR_BUSY, HUB_ERR_NOTFOUND = range(7)
HUB_CG_FP64, HUB_FGMRES_MIXED = 0, 1
HUB_MAX_BATCH = 64
HUB_MAX_RESTART = 20
HUB_MAX_HB_MASSES = 16
HUB_MAX_SHIFTS = 17
HUB_NOALLOC_SCRATCH_BYTES = 64 << 20
STATUS_NAMES = {0: "HUB_OK", 1: "HUB_ERR_ARG", 2: "HUB_ERR_OOM", 3: "HUB_ERR_NOCONV", 4: "HUB_ERR_HIP",
                5: "HUB_ERR_BUSY", 6: "HUB_ERR_NOTFOUND"}

SYMBOLS = ["hub_create", "hub_destroy", "hub_last_error", "hub_apply_M", "hub_apply_Mdag", "hub_apply_normal",
           "hub_default_opts", "hub_solve", "hub_force", "hub_force_sum", "hub_action", "hub_submit", "hub_poll",
           "hub_profile_enable", "hub_profile_read", "hub_hasenbusch_heatbath", "hub_hasenbusch_force",
           "hub_md_schedule", "hub_hmc_trajectory", "hub_hmc_trajectories", "hub_solve_multishift",
           "hub_hasenbusch_masses", "hub_profile_stream", "hub_apply_normal_noalloc", "hub_solve_fields",
           "hub_apply_fields"]


class HubLattice(ctypes.Structure):
    _fields_ = [("L1", ctypes.c_int32), ("L2", ctypes.c_int32), ("Nt", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("kappa_t", ctypes.c_double), ("ms_t", ctypes.c_double)]


class HubSolveOpts(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("restart_m", ctypes.c_int32),
                ("inner_max_iter", ctypes.c_int32), ("tol", ctypes.c_double), ("inner_a", ctypes.c_double),
                ("inner_floor", ctypes.c_double), ("use_x0", ctypes.c_int32), ("check_every", ctypes.c_int32)]


class HubSolveInfo(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int32), ("outer_iters", ctypes.c_int32), ("inner_iters", ctypes.c_int32),
                ("applies", ctypes.c_int32), ("true_rel_resid", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class HubRequest(ctypes.Structure):
    _fields_ = [("lat", HubLattice), ("mu2", ctypes.c_double), ("phi", ctypes.c_void_p), ("chi", ctypes.c_void_p),
                ("x_out", ctypes.c_void_p), ("S_out", ctypes.POINTER(ctypes.c_double)),
                ("dSdphi_out", ctypes.c_void_p), ("opts", HubSolveOpts)]


class HubKernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 16), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


MAXM = 16  # HUB_MAX_HB_MASSES


class HubHmcParams(ctypes.Structure):
    _fields_ = [("traj_length", ctypes.c_double), ("zeta", ctypes.c_double), ("U_t", ctypes.c_double),
                ("n_md", ctypes.c_int32), ("n", ctypes.c_int32), ("mt", ctypes.c_double * MAXM),
                ("n_scale", ctypes.c_int32 * MAXM), ("flags", ctypes.c_int32), ("pad", ctypes.c_int32)]


HUB_HMC_CHI_GIVEN = 1


class HubMdOp(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("eps", ctypes.c_double),
                ("coef", ctypes.c_double * (MAXM + 1))]


class HubHmcInfo(ctypes.Structure):
    _fields_ = [("dH", ctypes.c_double), ("H0", ctypes.c_double), ("H1", ctypes.c_double),
                ("accepted", ctypes.c_int32), ("kick_groups", ctypes.c_int32), ("drifts", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("inner_iters", ctypes.c_int64),
                ("force_evals", ctypes.c_int32 * (MAXM + 1)), ("pad", ctypes.c_int32)]

    def as_dict(self, n: int) -> dict:
        return {"dH": self.dH, "H0": self.H0, "H1": self.H1, "accepted": bool(self.accepted),
                "kick_groups": self.kick_groups, "drifts": self.drifts, "inner_iters": self.inner_iters,
                "force_evals": [self.force_evals[i] for i in range(n + 1)]}


class HubError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load libhub.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1804_07195_amd.build_lib.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    L.hub_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_size_t]
    L.hub_destroy.argtypes = [vp]
    L.hub_last_error.restype = ctypes.c_char_p
    L.hub_last_error.argtypes = []
    for f in (L.hub_apply_M, L.hub_apply_Mdag):
        f.argtypes = [vp, ctypes.POINTER(HubLattice), vp, vp, vp, i32, vp]
    L.hub_apply_normal.argtypes = [vp, ctypes.POINTER(HubLattice), vp, ctypes.POINTER(dbl), vp, vp, i32, vp]
    L.hub_apply_normal_noalloc.argtypes = [vp, ctypes.POINTER(HubLattice), vp, ctypes.POINTER(dbl), vp, vp, i32, vp]
    L.hub_default_opts.argtypes = [ctypes.POINTER(HubSolveOpts)]
    L.hub_default_opts.restype = None
    L.hub_solve.argtypes = [vp, ctypes.POINTER(HubLattice), vp, ctypes.POINTER(dbl), i32, vp, vp,
                            ctypes.POINTER(HubSolveOpts), ctypes.POINTER(HubSolveInfo), vp]
    L.hub_solve_fields.argtypes = [vp, ctypes.POINTER(HubLattice), vp, i32, ctypes.POINTER(dbl), i32, vp, vp,
                                   ctypes.POINTER(HubSolveOpts), ctypes.POINTER(HubSolveInfo), vp]
    L.hub_apply_fields.argtypes = [vp, ctypes.POINTER(HubLattice), vp, i32, i32, vp, vp, i32, vp]
    L.hub_force.argtypes = [vp, ctypes.POINTER(HubLattice), vp, vp, vp, dbl, i32, vp, i32, vp]
    L.hub_force_sum.argtypes = [vp, ctypes.POINTER(HubLattice), vp, vp, vp, ctypes.POINTER(dbl), i32, vp, i32, vp]
    L.hub_action.argtypes = [vp, ctypes.POINTER(HubLattice), vp, vp, i32, ctypes.POINTER(dbl), vp]
    L.hub_submit.argtypes = [vp, ctypes.POINTER(HubRequest), ctypes.POINTER(ctypes.c_uint64)]
    L.hub_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i32), ctypes.POINTER(HubSolveInfo)]
    L.hub_hasenbusch_heatbath.argtypes = [vp, ctypes.POINTER(HubLattice), vp, ctypes.POINTER(dbl), i32, vp, vp,
                                          ctypes.POINTER(HubSolveOpts), ctypes.POINTER(HubSolveInfo), vp]
    L.hub_hasenbusch_force.argtypes = [vp, ctypes.POINTER(HubLattice), vp, ctypes.POINTER(dbl), i32, vp,
                                       ctypes.c_uint32, dbl, i32, vp, ctypes.POINTER(dbl), vp,
                                       ctypes.POINTER(HubSolveOpts), ctypes.POINTER(HubSolveInfo), vp]
    L.hub_md_schedule.argtypes = [ctypes.POINTER(HubHmcParams), ctypes.POINTER(HubMdOp), i32, ctypes.POINTER(i32)]
    L.hub_hmc_trajectory.argtypes = [vp, ctypes.POINTER(HubLattice), vp, vp, vp, dbl, ctypes.POINTER(HubHmcParams),
                                     ctypes.POINTER(HubSolveOpts), ctypes.POINTER(HubHmcInfo), vp]
    L.hub_hmc_trajectories.argtypes = [vp, ctypes.POINTER(HubLattice), i32, vp, vp, vp, ctypes.POINTER(dbl),
                                       ctypes.POINTER(HubHmcParams), ctypes.POINTER(HubSolveOpts),
                                       ctypes.POINTER(HubHmcInfo), vp]
    L.hub_solve_multishift.argtypes = [vp, ctypes.POINTER(HubLattice), vp, ctypes.POINTER(dbl), i32, vp, vp,
                                       ctypes.POINTER(HubSolveOpts), ctypes.POINTER(HubSolveInfo),
                                       ctypes.POINTER(dbl), vp]
    L.hub_hasenbusch_masses.argtypes = [dbl, dbl, i32, ctypes.POINTER(dbl)]
    L.hub_profile_enable.argtypes = [vp, i32]
    L.hub_profile_read.argtypes = [vp, ctypes.POINTER(HubKernelStat), i32, ctypes.POINTER(i32)]
    L.hub_profile_stream.argtypes = [vp, vp, vp, vp, ctypes.c_int64, i32, vp]
    for name in SYMBOLS:
        fn = getattr(L, name)
        if name not in ("hub_last_error", "hub_default_opts"):
            fn.restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int, allow=()) -> int:
    if status != HUB_OK and status not in allow:
        raise HubError(status, load().hub_last_error().decode())
    return status


def lattice(L1: int, L2: int, Nt: int, kappa_t: float, ms_t: float = 0.0) -> HubLattice:
    return HubLattice(int(L1), int(L2), int(Nt), 0, float(kappa_t), float(ms_t))


def default_opts(**kw) -> HubSolveOpts:
    o = HubSolveOpts()
    load().hub_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "solver" and isinstance(v, str):
            v = {"cg": HUB_CG_FP64, "fgmres": HUB_FGMRES_MIXED}[v]
        setattr(o, k, v)
    return o


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _nsites(lat: HubLattice) -> int:
    return 2 * lat.L1 * lat.L2 * lat.Nt


def _vec(t: torch.Tensor, lat: HubLattice, what: str) -> int:
    """Batch size of a complex128 device vector [batch?, N_t, 2, L1, L2] (or flat)."""
    if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous complex128 CUDA tensor")
    n = _nsites(lat)
    if t.numel() % n != 0 or t.numel() == 0:
        raise ValueError(f"{what} has {t.numel()} entries, not a multiple of N = {n}")
    return t.numel() // n


def _phi(t: torch.Tensor, lat: HubLattice) -> None:
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != _nsites(lat):
        raise ValueError("phi must be a contiguous float64 CUDA tensor with N entries")


class Context:
    """A libhub context on one device (hub_create / hub_destroy)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        L = load()
        h = ctypes.c_void_p()
        _check(L.hub_create(ctypes.byref(h), int(device), int(hbm_budget_bytes)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            load().hub_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hub_apply_M(ctx: Context, lat: HubLattice, phi, x, y=None, stream=None):
    """y = M[phi] x (batched over the leading dimension)."""
    _phi(phi, lat)
    nb = _vec(x, lat, "x")
    y = torch.empty_like(x) if y is None else y
    _vec(y, lat, "y")
    _check(load().hub_apply_M(ctx.handle, ctypes.byref(lat), phi.data_ptr(), x.data_ptr(), y.data_ptr(), nb,
                              _stream(stream)))
    return y


def hub_apply_Mdag(ctx: Context, lat: HubLattice, phi, x, y=None, stream=None):
    """y = M[phi]^dagger x."""
    _phi(phi, lat)
    nb = _vec(x, lat, "x")
    y = torch.empty_like(x) if y is None else y
    _vec(y, lat, "y")
    _check(load().hub_apply_Mdag(ctx.handle, ctypes.byref(lat), phi.data_ptr(), x.data_ptr(), y.data_ptr(), nb,
                                 _stream(stream)))
    return y


def hub_apply_normal(ctx: Context, lat: HubLattice, phi, mu2, x, y=None, stream=None):
    """y = (M M^dagger + mu2[b]) x_b."""
    _phi(phi, lat)
    nb = _vec(x, lat, "x")
    mu = (ctypes.c_double * nb)(*[float(m) for m in (mu2 if hasattr(mu2, "__len__") else [mu2] * nb)])
    y = torch.empty_like(x) if y is None else y
    _check(load().hub_apply_normal(ctx.handle, ctypes.byref(lat), phi.data_ptr(), mu, x.data_ptr(), y.data_ptr(),
                                   nb, _stream(stream)))
    return y


def hub_apply_normal_noalloc(ctx: Context, lat: HubLattice, phi, mu2, x, y, stream=None):
    """y = (M M^dagger + mu2[b]) x_b into the caller's y, without any allocation (the
    library's per-device scratch holds M^dagger x)."""
    _phi(phi, lat)
    nb = _vec(x, lat, "x")
    if _vec(y, lat, "y") != nb:
        raise ValueError("y must match x")
    mu = (ctypes.c_double * nb)(*[float(m) for m in (mu2 if hasattr(mu2, "__len__") else [mu2] * nb)])
    _check(load().hub_apply_normal_noalloc(ctx.handle, ctypes.byref(lat), phi.data_ptr(), mu, x.data_ptr(),
                                           y.data_ptr(), nb, _stream(stream)))
    return y


def hub_solve(ctx: Context, lat: HubLattice, phi, mu2, b, x=None, opts: HubSolveOpts | None = None,
              stream=None, allow_noconv: bool = False):
    """Solve (M M^dagger + mu2[k]) x_k = b_k.  Returns (x, [info dicts], status)."""
    _phi(phi, lat)
    nb = _vec(b, lat, "b")
    mu2 = list(mu2) if hasattr(mu2, "__len__") else [mu2] * nb
    if len(mu2) != nb:
        raise ValueError("one shift per system")
    mu = (ctypes.c_double * nb)(*[float(m) for m in mu2])
    if x is None:
        x = torch.empty_like(b)
    _vec(x, lat, "x")
    o = default_opts() if opts is None else opts
    info = (HubSolveInfo * nb)()
    st = load().hub_solve(ctx.handle, ctypes.byref(lat), phi.data_ptr(), mu, nb, b.data_ptr(), x.data_ptr(),
                          ctypes.byref(o), info, _stream(stream))
    _check(st, allow=(HUB_ERR_NOCONV,) if allow_noconv else ())
    return x, [i.as_dict() for i in info], st


def _fields(phi: torch.Tensor, lat: HubLattice, what: str = "phi") -> int:
    """Number of fields in a contiguous float64 CUDA tensor [nfield, N_t, 2, L1, L2] (or flat)."""
    n = _nsites(lat)
    if phi.dtype != torch.float64 or not phi.is_cuda or not phi.is_contiguous() or phi.numel() % n or not phi.numel():
        raise ValueError(f"{what} must be a contiguous float64 CUDA tensor of whole fields")
    return phi.numel() // n


def hub_solve_fields(ctx: Context, lat: HubLattice, phi, mu2, b, x=None, opts: HubSolveOpts | None = None,
                     stream=None, allow_noconv: bool = False):
    """Systems on several fields: b [nfield * per, ...], phi [nfield, ...]; system k uses
    field k // per.  Returns (x, [info dicts], status)."""
    nf = _fields(phi, lat)
    nb = _vec(b, lat, "b")
    if nb % nf:
        raise ValueError("the systems must split evenly over the fields")
    per = nb // nf
    mu2 = list(mu2) if hasattr(mu2, "__len__") else [mu2] * nb
    if len(mu2) != nb:
        raise ValueError("one shift per system")
    mu = (ctypes.c_double * nb)(*[float(m) for m in mu2])
    if x is None:
        x = torch.empty_like(b)
    _vec(x, lat, "x")
    o = default_opts() if opts is None else opts
    info = (HubSolveInfo * nb)()
    st = load().hub_solve_fields(ctx.handle, ctypes.byref(lat), phi.data_ptr(), per, mu, nb, b.data_ptr(),
                                 x.data_ptr(), ctypes.byref(o), info, _stream(stream))
    _check(st, allow=(HUB_ERR_NOCONV,) if allow_noconv else ())
    return x, [i.as_dict() for i in info], st


def hub_apply_fields(ctx: Context, lat: HubLattice, phi, x, dag: bool, y=None, stream=None):
    """y_k = M[phi_{k // per}] x_k, or M^dagger with dag, for x [nfield * per, ...], phi [nfield, ...]."""
    nf = _fields(phi, lat)
    nb = _vec(x, lat, "x")
    if nb % nf:
        raise ValueError("the vectors must split evenly over the fields")
    y = torch.empty_like(x) if y is None else y
    _vec(y, lat, "y")
    _check(load().hub_apply_fields(ctx.handle, ctypes.byref(lat), phi.data_ptr(), nb // nf, 1 if dag else 0,
                                   x.data_ptr(), y.data_ptr(), nb, _stream(stream)))
    return y


def hub_force(ctx: Context, lat: HubLattice, phi, eta, xi=None, scale: float = 1.0, accumulate: bool = False,
              out=None, stream=None):
    """dS/dphi (float64 [batch?, N_t, 2, L1, L2]) given eta = A^{-1} chi (and optionally xi = M^dagger eta)."""
    _phi(phi, lat)
    nb = _vec(eta, lat, "eta")
    if xi is not None:
        _vec(xi, lat, "xi")
    if out is None:
        out = torch.zeros(eta.shape, dtype=torch.float64, device=eta.device)
    if out.dtype != torch.float64 or not out.is_contiguous() or out.numel() != eta.numel():
        raise ValueError("out must be a contiguous float64 tensor shaped like eta")
    _check(load().hub_force(ctx.handle, ctypes.byref(lat), phi.data_ptr(), eta.data_ptr(),
                            None if xi is None else xi.data_ptr(), float(scale), 1 if accumulate else 0,
                            out.data_ptr(), nb, _stream(stream)))
    return out


def hub_force_sum(ctx: Context, lat: HubLattice, phi, eta, scale, xi=None, accumulate: bool = False, out=None,
                  stream=None):
    """sum_b scale[b] dS_b/dphi (float64 [N_t, 2, L1, L2]) for the batch eta_b = A_b^{-1} chi_b."""
    _phi(phi, lat)
    nb = _vec(eta, lat, "eta")
    if xi is not None and _vec(xi, lat, "xi") != nb:
        raise ValueError("xi must match eta")
    sc = list(scale) if hasattr(scale, "__len__") else [scale] * nb
    if len(sc) != nb:
        raise ValueError("one scale per system")
    sca = (ctypes.c_double * nb)(*[float(v) for v in sc])
    if out is None:
        out = torch.zeros(phi.shape, dtype=torch.float64, device=phi.device)
    if out.dtype != torch.float64 or not out.is_contiguous() or out.numel() != phi.numel():
        raise ValueError("out must be a contiguous float64 tensor shaped like phi")
    _check(load().hub_force_sum(ctx.handle, ctypes.byref(lat), phi.data_ptr(), eta.data_ptr(),
                                None if xi is None else xi.data_ptr(), sca, 1 if accumulate else 0,
                                out.data_ptr(), nb, _stream(stream)))
    return out


def hub_action(ctx: Context, lat: HubLattice, chi, eta, stream=None):
    """[Re chi_b^dagger eta_b] as a Python list (synchronises the stream)."""
    nb = _vec(chi, lat, "chi")
    _vec(eta, lat, "eta")
    S = (ctypes.c_double * nb)()
    _check(load().hub_action(ctx.handle, ctypes.byref(lat), chi.data_ptr(), eta.data_ptr(), nb, S,
                             _stream(stream)))
    return list(S)


def hub_hasenbusch_heatbath(ctx: Context, lat: HubLattice, phi, mts, rho, chi=None,
                            opts: HubSolveOpts | None = None, stream=None, allow_noconv: bool = False):
    """Pseudofermions chi_0..chi_n of the staggered-mass Hasenbusch split from rho_0..rho_n
    (device complex128 [n+1, N_t, 2, L1, L2]); mts = [m~_0, ..., m~_{n-1}].
    Returns (chi, [info dicts of the n solves], status)."""
    _phi(phi, lat)
    n = len(mts)
    if _vec(rho, lat, "rho") != n + 1:
        raise ValueError("rho must hold n+1 vectors")
    if chi is None:
        chi = torch.empty_like(rho)
    if _vec(chi, lat, "chi") != n + 1:
        raise ValueError("chi must hold n+1 vectors")
    m = (ctypes.c_double * n)(*[float(v) for v in mts])
    o = default_opts() if opts is None else opts
    info = (HubSolveInfo * n)()
    st = load().hub_hasenbusch_heatbath(ctx.handle, ctypes.byref(lat), phi.data_ptr(), m, n, rho.data_ptr(),
                                        chi.data_ptr(), ctypes.byref(o), info, _stream(stream))
    _check(st, allow=(HUB_ERR_NOCONV,) if allow_noconv else ())
    return chi, [i.as_dict() for i in info], st


def hub_hasenbusch_force(ctx: Context, lat: HubLattice, phi, mts, chi, terms=None, eta=None, scale: float = 1.0,
                         accumulate: bool = False, out=None, opts: HubSolveOpts | None = None, stream=None,
                         allow_noconv: bool = False):
    """Summed dS_i/dphi over `terms` (default all n+1) of the staggered-mass Hasenbusch split.
    Returns (dSdphi [N_t, 2, L1, L2], S list [n+1] (None for terms not evaluated),
    eta [n+1, ...], info list, status)."""
    _phi(phi, lat)
    n = len(mts)
    if _vec(chi, lat, "chi") != n + 1:
        raise ValueError("chi must hold n+1 vectors")
    terms = list(range(n + 1)) if terms is None else sorted(set(int(t) for t in terms))
    mask = 0
    for t in terms:
        mask |= 1 << t
    if eta is None:
        eta = torch.zeros_like(chi)
    if _vec(eta, lat, "eta") != n + 1:
        raise ValueError("eta must hold n+1 vectors")
    if out is None:
        out = torch.zeros(chi.shape[1:], dtype=torch.float64, device=chi.device)
    if out.dtype != torch.float64 or not out.is_contiguous() or out.numel() != _nsites(lat):
        raise ValueError("out must be a contiguous float64 tensor with N entries")
    m = (ctypes.c_double * n)(*[float(v) for v in mts])
    S = (ctypes.c_double * (n + 1))(*([float("nan")] * (n + 1)))
    o = default_opts() if opts is None else opts
    info = (HubSolveInfo * (n + 1))()
    st = load().hub_hasenbusch_force(ctx.handle, ctypes.byref(lat), phi.data_ptr(), m, n, chi.data_ptr(),
                                     ctypes.c_uint32(mask), float(scale), 1 if accumulate else 0, out.data_ptr(),
                                     S, eta.data_ptr(), ctypes.byref(o), info, _stream(stream))
    _check(st, allow=(HUB_ERR_NOCONV,) if allow_noconv else ())
    Sl = [S[i] if i in terms else None for i in range(n + 1)]
    il = [info[i].as_dict() if i in terms else None for i in range(n + 1)]
    return out, Sl, eta, il, st


def hub_hmc_trajectories(ctx: Context, lat: HubLattice, phi, pi, rho, u, params: HubHmcParams,
                         opts: HubSolveOpts | None = None, stream=None) -> list:
    """One HMC update of each of nchain chains in lockstep: phi, pi float64 [nchain, ...],
    rho complex128 [nchain, n+1, ...] (device), u a list of nchain uniforms.  Returns the
    info dicts."""
    n = _nsites(lat)
    nc = len(u)
    for t, what in ((phi, "phi"), (pi, "pi")):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != nc * n:
            raise ValueError(f"{what} must be a contiguous float64 CUDA tensor with nchain * N entries")
    if _vec(rho, lat, "rho") != nc * (params.n + 1):
        raise ValueError("rho must hold nchain * (n+1) vectors")
    uu = (ctypes.c_double * nc)(*[float(v) for v in u])
    o = default_opts() if opts is None else opts
    info = (HubHmcInfo * nc)()
    _check(load().hub_hmc_trajectories(ctx.handle, ctypes.byref(lat), nc, phi.data_ptr(), pi.data_ptr(),
                                       rho.data_ptr(), uu, ctypes.byref(params), ctypes.byref(o), info,
                                       _stream(stream)))
    return [i.as_dict(params.n) for i in info]


def hub_solve_multishift(ctx: Context, lat: HubLattice, phi, mu2, b, x=None, opts: HubSolveOpts | None = None,
                         stream=None, allow_noconv: bool = False):
    """x_s = (M M^dagger + mu2[s])^{-1} b for every shift from one Krylov space.
    b: device complex128 with N entries.  Returns (x [nshift, ...], [info dicts],
    (lambda_min, lambda_max) of M M^dagger from the Lanczos coefficients, status)."""
    _phi(phi, lat)
    if _vec(b, lat, "b") != 1:
        raise ValueError("one right-hand side")
    ns = len(mu2)
    if x is None:
        x = torch.empty((ns,) + tuple(b.shape[-4:]), dtype=torch.complex128, device=b.device)
    if _vec(x, lat, "x") != ns:
        raise ValueError("x must hold one vector per shift")
    mu = (ctypes.c_double * ns)(*[float(m) for m in mu2])
    lam = (ctypes.c_double * 2)()
    o = default_opts() if opts is None else opts
    info = (HubSolveInfo * ns)()
    st = load().hub_solve_multishift(ctx.handle, ctypes.byref(lat), phi.data_ptr(), mu, ns, b.data_ptr(),
                                     x.data_ptr(), ctypes.byref(o), info, lam, _stream(stream))
    _check(st, allow=(HUB_ERR_NOCONV,) if allow_noconv else ())
    return x, [i.as_dict() for i in info], (lam[0], lam[1]), st


def hub_hasenbusch_masses(lambda_min: float, lambda_max: float, n: int) -> list:
    """eq. (mu_i_eqn): n masses geometric between the spectral bounds (host only)."""
    mu = (ctypes.c_double * n)()
    _check(load().hub_hasenbusch_masses(float(lambda_min), float(lambda_max), int(n), mu))
    return list(mu)


def hmc_params(U_t: float, n_md: int, mts=(), n_scale=(), traj_length: float = 1.0,
               zeta: float = 0.1931833275037836, chi_given: bool = False) -> HubHmcParams:
    """Parameters of one HMC trajectory (see hub_hmc_params in include/hub.h)."""
    if len(mts) != len(n_scale) or len(mts) > MAXM:
        raise ValueError("one time-scale factor per Hasenbusch mass, at most 16")
    p = HubHmcParams()
    p.traj_length, p.zeta, p.U_t, p.n_md, p.n = float(traj_length), float(zeta), float(U_t), int(n_md), len(mts)
    p.flags = HUB_HMC_CHI_GIVEN if chi_given else 0
    for i, (m, k) in enumerate(zip(mts, n_scale)):
        p.mt[i] = float(m)
        p.n_scale[i] = int(k)
    return p


def hub_md_schedule(params: HubHmcParams) -> list:
    """The merged operation list of one trajectory: ("drift", eps) or ("kick", [coef per level])."""
    L = load()
    cnt = ctypes.c_int32()
    _check(L.hub_md_schedule(ctypes.byref(params), None, 0, ctypes.byref(cnt)))
    ops = (HubMdOp * max(cnt.value, 1))()
    _check(L.hub_md_schedule(ctypes.byref(params), ops, cnt.value, ctypes.byref(cnt)))
    out = []
    for k in range(cnt.value):
        o = ops[k]
        out.append(("drift", o.eps) if o.kind == 0 else ("kick", [o.coef[i] for i in range(params.n + 1)]))
    return out


def hub_hmc_trajectory(ctx: Context, lat: HubLattice, phi, pi, rho, u: float, params: HubHmcParams,
                       opts: HubSolveOpts | None = None, stream=None) -> dict:
    """One HMC update in place: phi (accepted field), pi (momenta at the trajectory's end).
    rho: device complex128 [n+1, ...] heat-bath vectors (the pseudofermions themselves if
    the params were made with chi_given=True).  Returns the info dict."""
    _phi(phi, lat)
    _phi(pi, lat)
    if _vec(rho, lat, "rho") != params.n + 1:
        raise ValueError("rho must hold n+1 vectors")
    o = default_opts() if opts is None else opts
    info = HubHmcInfo()
    _check(load().hub_hmc_trajectory(ctx.handle, ctypes.byref(lat), phi.data_ptr(), pi.data_ptr(), rho.data_ptr(),
                                     float(u), ctypes.byref(params), ctypes.byref(o), ctypes.byref(info),
                                     _stream(stream)))
    return info.as_dict(params.n)


class Pending:
    """Buffers of one served request; they must stay alive until it is done."""

    def __init__(self, ticket, lat, phi, chi, x, dS, S):
        self.ticket, self.lat, self.phi, self.chi, self.x, self.dS, self._S = ticket, lat, phi, chi, x, dS, S

    @property
    def S(self) -> float:
        return self._S.value


def hub_submit(ctx: Context, lat: HubLattice, mu2: float, phi, chi, x_out=None, dSdphi_out=None, force=True,
               opts: HubSolveOpts | None = None) -> Pending:
    """Queue solve + S + dS/dphi for one system; returns a Pending holding the ticket."""
    _phi(phi, lat)
    if _vec(chi, lat, "chi") != 1:
        raise ValueError("one system per request")
    x_out = torch.empty_like(chi) if x_out is None else x_out
    if force and dSdphi_out is None:
        dSdphi_out = torch.empty(phi.shape, dtype=torch.float64, device=phi.device)
    S = ctypes.c_double(0.0)
    req = HubRequest(lat, float(mu2), phi.data_ptr(), chi.data_ptr(), x_out.data_ptr(), ctypes.pointer(S),
                     dSdphi_out.data_ptr() if force else None, default_opts() if opts is None else opts)
    t = ctypes.c_uint64()
    _check(load().hub_submit(ctx.handle, ctypes.byref(req), ctypes.byref(t)))
    return Pending(t.value, lat, phi, chi, x_out, dSdphi_out, S)


def hub_poll(ctx: Context, pending) -> tuple:
    """(done, info dict or None); never blocks.  A finished request's info carries its
    final status under "status" (HUB_OK, HUB_ERR_NOCONV, HUB_ERR_ARG or HUB_ERR_HIP);
    a failure of the call itself (unknown ticket) raises."""
    ticket = pending.ticket if isinstance(pending, Pending) else int(pending)
    done = ctypes.c_int32(0)
    info = HubSolveInfo()
    st = load().hub_poll(ctx.handle, ctypes.c_uint64(ticket), ctypes.byref(done), ctypes.byref(info))
    if not done.value:
        _check(st)
        return False, None
    d = info.as_dict()
    d["status"] = st
    return True, d


def hub_profile_enable(ctx: Context, enable: bool = True) -> None:
    """Time every CG-iteration kernel launch of later solves with HIP events (resets the stats)."""
    _check(load().hub_profile_enable(ctx.handle, 1 if enable else 0))


def hub_profile_read(ctx: Context) -> dict:
    """{kernel: {launches, total_ms, bytes, avg_us, GBps}} of the timed launches."""
    out = (HubKernelStat * 8)()
    n = ctypes.c_int32()
    _check(load().hub_profile_read(ctx.handle, out, 8, ctypes.byref(n)))
    res = {}
    for k in out[: n.value]:
        d = {"launches": k.launches, "total_ms": k.total_ms, "bytes": k.bytes}
        d["avg_us"] = 1e3 * k.total_ms / k.launches if k.launches else 0.0
        d["GBps"] = k.bytes / (k.total_ms * 1e-3) / 1e9 if k.total_ms > 0 else 0.0
        res[k.name.decode()] = d
    return res


class PseudofermionAction(torch.autograd.Function):
    """phi -> S_b = Re chi_b^dagger (M M^dagger + mu2_b)^{-1} chi_b (eq. (hamiltonian)).

    forward: hub_solve + hub_action; backward: grad_phi = sum_b grad_S[b] dS_b/dphi
    by one hub_force_sum over the batch (xi = M^dagger eta computed inside)."""

    @staticmethod
    def forward(ctx_, phi, chi, mu2, hub_ctx: Context, lat: HubLattice, opts=None):
        x, info, _ = hub_solve(hub_ctx, lat, phi, mu2, chi, opts=opts)
        S = hub_action(hub_ctx, lat, chi, x)
        ctx_.save_for_backward(phi, x)
        ctx_.hub = (hub_ctx, lat)
        ctx_.info = info
        return torch.tensor(S, dtype=torch.float64, device=phi.device)

    @staticmethod
    def backward(ctx_, grad_S):
        phi, x = ctx_.saved_tensors
        hub_ctx, lat = ctx_.hub
        g = grad_S.detach().to("cpu", torch.float64).reshape(-1).tolist()
        # one launch for the batch: sum_b grad_S[b] dS_b/dphi
        out = hub_force_sum(hub_ctx, lat, phi, x, g)
        return out, None, None, None, None, None
