"""ctypes binding of libmdpnop (include/mdpnop.h): argument marshalling only.

Fields are torch tensors on the GPU (float32, contiguous, shape (ny, nx) or
(nx,)); every step of the solve runs in the library's HIP kernels.  The
library must be built (``python -m paper_2509_01416_amd.build``); there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MDPNOP_LIB points the binding at another build of the library (the
# host-sanitizer build of tests/sanitize_build.py); it must exist like the
# default one
LIB_PATH = os.environ.get("MDPNOP_LIB") or os.path.join(_HERE, "libmdpnop.so")

TR_OK = 0
TR_NOT_CONVERGED = 1
TR_RECAST_DIVERGED = 2
TR_ERR_INVALID_ARG = -1
TR_ERR_HIP = -2
TR_ERR_OOM = -3
TR_ERR_NONFINITE = -4
NO_EIGEN_SP = 0
TR_STOP_CHANGE = 0
TR_STOP_ERROR_BOUND = 1
NO_EIGEN_CP = 1

EXPORTS = ("tr_context_create", "tr_context_destroy", "tr_last_error",
           "tr_sweep", "tr_solve", "tr_solve_noalloc", "tr_eigen", "tr_eigen_mg", "no_recast_guess", "no_eigen",
           "no_model_create", "no_model_create_deeponet",
           "no_model_destroy", "no_model_param_count", "no_model_get_params",
           "no_model_set_params", "no_model_get_state", "no_model_set_state",
           "no_model_set_fp32", "no_forward",
           "no_train_step",
           "tr_check_args", "tr_autotune", "tr_set_sweep_config", "tr_set_sweep_kernel",
           "tr_set_stop_rule", "tr_set_sync_checks", "tr_set_persistent", "tr_get_sweep_plan",
           "tr_profile_enable", "tr_profile_read", "tr_profile_read_ex")


class TrProblem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("lx", ctypes.c_double),
                ("ly", ctypes.c_double), ("sigma_t", ctypes.c_void_p),
                ("sigma_s", ctypes.c_void_p), ("source", ctypes.c_void_p),
                ("bc", ctypes.c_int32 * 4), ("sigma_s1", ctypes.c_void_p)]


class TrQuadrature(ctypes.Structure):
    _fields_ = [("n_dir", ctypes.c_int32), ("mu", ctypes.c_void_p),
                ("eta", ctypes.c_void_p), ("w", ctypes.c_void_p)]


class TrStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("residual", ctypes.c_double), ("balance_rel", ctypes.c_double),
                ("seconds", ctypes.c_double)]


class TrEigenStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("inner", ctypes.c_int32), ("k", ctypes.c_double),
                ("dk", ctypes.c_double), ("dphi", ctypes.c_double),
                ("balance_rel", ctypes.c_double), ("seconds", ctypes.c_double)]


class TrMultigroup(ctypes.Structure):
    _fields_ = [("n_groups", ctypes.c_int32), ("sigma_t", ctypes.c_void_p),
                ("sigma_s", ctypes.c_void_p), ("nu_sigma_f", ctypes.c_void_p),
                ("chi", ctypes.c_void_p)]


class MdpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} missing: build it with "
                           "`python -m paper_2509_01416_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    lib.tr_context_create.argtypes = [P(vp), vp]
    lib.tr_context_destroy.argtypes = [vp]
    lib.tr_context_destroy.restype = None
    lib.tr_last_error.argtypes = [vp]
    lib.tr_last_error.restype = ctypes.c_char_p
    lib.tr_sweep.argtypes = [vp, i32, P(TrProblem), P(TrQuadrature), P(vp), P(vp)]
    lib.tr_solve.argtypes = [vp, i32, P(TrProblem), P(TrQuadrature), P(vp), P(vp),
                             d, i32, P(TrStats)]
    lib.tr_solve_noalloc.argtypes = lib.tr_solve.argtypes
    lib.no_recast_guess.argtypes = [vp, vp, i32, P(TrProblem), d, d, d, i32, P(vp),
                                    P(TrStats)]
    lib.no_eigen.argtypes = [vp, vp, i32, P(TrProblem), P(vp), P(TrQuadrature), d, d, i32,
                             P(vp), P(vp), P(d), d, d, i32, P(TrEigenStats)]
    lib.tr_eigen_mg.argtypes = [vp, i32, P(TrProblem), P(TrMultigroup), P(TrQuadrature),
                                P(vp), P(vp), P(d), d, d, d, i32, i32, P(TrEigenStats)]
    lib.tr_eigen.argtypes = [vp, i32, P(TrProblem), P(vp), P(TrQuadrature), P(vp), P(vp),
                             P(d), d, d, d, i32, i32, P(TrEigenStats)]
    lib.no_model_create.argtypes = [vp, P(vp), i32, i32, i32, i32, vp]
    lib.no_model_create_deeponet.argtypes = [vp, P(vp), i32, i32, i32, vp]
    lib.no_model_destroy.argtypes = [vp]
    lib.no_model_destroy.restype = None
    lib.no_model_param_count.argtypes = [vp]
    lib.no_model_param_count.restype = i64
    lib.no_model_get_params.argtypes = [vp, vp, vp]
    lib.no_model_set_params.argtypes = [vp, vp, vp]
    lib.no_model_get_state.argtypes = [vp, vp, vp, vp, vp, P(i64)]
    lib.no_model_set_state.argtypes = [vp, vp, vp, vp, vp, i64]
    lib.no_model_set_fp32.argtypes = [vp, i32]
    lib.no_forward.argtypes = [vp, vp, i32, vp, vp]
    lib.no_train_step.argtypes = [vp, vp, i32, vp, vp, d, P(d), vp]
    lib.tr_check_args.argtypes = [i32, P(TrProblem), P(TrQuadrature), d, i32,
                                  ctypes.c_char_p, i32]
    lib.tr_set_sweep_config.argtypes = [vp, i32, i32, i32, i32]
    lib.tr_set_sweep_kernel.argtypes = [vp, i32]
    lib.tr_set_stop_rule.argtypes = [vp, i32]
    lib.tr_set_sync_checks.argtypes = [vp, i32]
    lib.tr_autotune.argtypes = [vp, i32, P(TrProblem), P(TrQuadrature), i32, P(i32), P(d)]
    lib.tr_get_sweep_plan.argtypes = [vp, i32, P(TrProblem), P(TrQuadrature), P(i32)]
    lib.tr_profile_enable.argtypes = [vp, i32]
    lib.tr_profile_read.argtypes = [vp, P(d)]
    lib.tr_profile_read_ex.argtypes = [vp, P(d)]
    lib.tr_set_persistent.argtypes = [vp, i32, i32]
    for name in EXPORTS:
        f = getattr(lib, name)
        if f.restype is ctypes.c_int:       # default: tr_status
            f.restype = ctypes.c_int32
    _lib = lib
    return lib


# ---------------------------------------------------------------- problems

@dataclass
class Problem:
    """One instance: device tensors sigma_t, sigma_s, source (float32), and
    optionally sigma_s1 (linearly anisotropic scattering)."""
    sigma_t: object
    sigma_s: object
    source: object
    lx: float = 10.0
    ly: float = 10.0
    bc: tuple = (0, 0, 0, 0)
    sigma_s1: object = None

    @property
    def dim(self) -> int:
        return 1 if self.sigma_t.dim() == 1 else 2

    @property
    def nx(self) -> int:
        return int(self.sigma_t.shape[-1])

    @property
    def ny(self) -> int:
        return 1 if self.dim == 1 else int(self.sigma_t.shape[0])


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def make_problems(problems: Sequence[Problem]):
    arr = (TrProblem * len(problems))()
    for i, p in enumerate(problems):
        for t in (p.sigma_t, p.sigma_s, p.source, p.sigma_s1):
            if t is not None and (str(t.dtype) != "torch.float32"
                                  or t.device.type != "cuda"):
                raise ValueError("fields must be float32 GPU tensors")
        if p.sigma_s1 is not None and p.sigma_s1.numel() != p.nx * p.ny:
            raise ValueError(f"problem {i}: sigma_s1 must have {p.nx * p.ny} cells")
        arr[i].dim = p.dim
        arr[i].nx = p.nx
        arr[i].ny = p.ny
        arr[i].lx = float(p.lx)
        arr[i].ly = float(p.ly)
        arr[i].sigma_t = _ptr(p.sigma_t)
        arr[i].sigma_s = _ptr(p.sigma_s)
        arr[i].source = _ptr(p.source)
        arr[i].sigma_s1 = _ptr(p.sigma_s1)
        for f in range(4):
            arr[i].bc[f] = int(p.bc[f]) if f < len(p.bc) else 0
    return arr


class Quad:
    """Host quadrature arrays kept alive for the duration of calls."""

    def __init__(self, mu, eta, w):
        self.mu = np.ascontiguousarray(mu, dtype=np.float64)
        self.eta = None if eta is None else np.ascontiguousarray(eta, dtype=np.float64)
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        self.struct = TrQuadrature(
            len(self.w), self.mu.ctypes.data,
            None if self.eta is None else self.eta.ctypes.data, self.w.ctypes.data)

    @classmethod
    def from_inputs(cls, q):
        return cls(q.mu, q.eta, q.w)


def _ptr_array(ts) -> ctypes.Array:
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = _ptr(t)
    return arr


# ---------------------------------------------------------------- context

class Context:
    """tr_context bound to a torch stream (default: the current stream)."""

    def __init__(self, stream=None):
        import torch
        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        rc = self.lib.tr_context_create(ctypes.byref(h),
                                        ctypes.c_void_p(stream.cuda_stream))
        if rc != TR_OK:
            raise MdpError(rc, "tr_context_create failed")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.tr_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return self.lib.tr_last_error(self.handle).decode()

    def check(self, rc: int, allow=(TR_OK, TR_NOT_CONVERGED, TR_RECAST_DIVERGED)):
        if rc not in allow:
            raise MdpError(rc, self.last_error())
        return rc

    # -------------------------------------------------------------- calls
    def set_sweep_config(self, D=0, W=0, S=0, R=0):
        self.check(self.lib.tr_set_sweep_config(self.handle, D, W, S, R), allow=(TR_OK,))

    def set_sweep_kernel(self, generic: bool):
        self.check(self.lib.tr_set_sweep_kernel(self.handle, int(generic)), allow=(TR_OK,))

    def set_stop_rule(self, rule: str):
        """tr_solve's stopping rule on this context: "change" (the change norm
        below tol) or "bound" (the fixed-point error bound r rho / (1 - rho)
        below tol)."""
        codes = {"change": TR_STOP_CHANGE, "bound": TR_STOP_ERROR_BOUND}
        if rule not in codes:
            raise ValueError(f"unknown stopping rule {rule!r}")
        self.check(self.lib.tr_set_stop_rule(self.handle, codes[rule]), allow=(TR_OK,))

    def set_sync_checks(self, enable: bool = True):
        """Debugging: synchronise and check for errors after every HIP step."""
        self.check(self.lib.tr_set_sync_checks(self.handle, int(enable)), allow=(TR_OK,))

    def set_persistent(self, enable: bool = True, spin_limit: int = 0):
        """Persistent iteration (several source iterations per cooperative
        launch) where the launch shape allows it; spin_limit > 0 bounds the
        polls of its barrier waits (0: the library default)."""
        self.check(self.lib.tr_set_persistent(self.handle, int(enable), int(spin_limit)),
                   allow=(TR_OK,))

    def profile(self, enable: bool = True):
        self.check(self.lib.tr_profile_enable(self.handle, int(enable)), allow=(TR_OK,))

    def profile_read(self) -> dict:
        out = (ctypes.c_double * 6)()
        self.check(self.lib.tr_profile_read_ex(self.handle, out), allow=(TR_OK,))
        return dict(sweep_ms=out[0], sweep_launches=int(out[1]),
                    combine_ms=out[2], combine_launches=int(out[3]),
                    persistent_ms=out[4], persistent_launches=int(out[5]))

    def autotune(self, problems, quad: Quad, reps: int = 3) -> dict:
        """Time the feasible launch shapes on these problems (each sweep with
        its partial-plane sum) and keep the fastest on this context; returns
        its plan and time per sweep."""
        out = (ctypes.c_int32 * 6)()
        ms = ctypes.c_double()
        self.check(self.lib.tr_autotune(self.handle, len(problems), make_problems(problems),
                                        ctypes.byref(quad.struct), int(reps), out,
                                        ctypes.byref(ms)), allow=(TR_OK,))
        return dict(D=out[0], W=out[1], S=out[2], R=out[3], KB=out[4], specialised=out[5],
                    ms=ms.value)

    def sweep_plan(self, problems, quad: Quad):
        return sweep_plan(make_problems(problems), len(problems), quad, self.handle)


def tr_sweep(ctx: Context, problems: Sequence[Problem], quad: Quad,
             emission: Sequence, phi_out: Sequence) -> int:
    arr = make_problems(problems)
    rc = ctx.lib.tr_sweep(ctx.handle, len(problems), arr, ctypes.byref(quad.struct),
                          _ptr_array(emission), _ptr_array(phi_out))
    return ctx.check(rc, allow=(TR_OK,))


def tr_solve(ctx: Context, problems: Sequence[Problem], quad: Quad,
             phi_init: Optional[Sequence], phi_out: Sequence, tol: float,
             max_iter: int, raise_on_error: bool = True, noalloc: bool = False):
    """Returns (status, list of per-instance stats dicts).  noalloc: call
    tr_solve_noalloc (workspaces in the library's fixed device scratch)."""
    n = len(problems)
    arr = make_problems(problems)
    stats = (TrStats * n)()
    init = None if phi_init is None else _ptr_array(phi_init)
    fn = ctx.lib.tr_solve_noalloc if noalloc else ctx.lib.tr_solve
    rc = fn(ctx.handle, n, arr, ctypes.byref(quad.struct), init,
            _ptr_array(phi_out), float(tol), int(max_iter), stats)
    if raise_on_error:
        ctx.check(rc)
    return rc, [dict(status=s.status, iterations=s.iterations,
                     residual=s.residual, balance_rel=s.balance_rel,
                     seconds=s.seconds) for s in stats]


def _check_eigen_fields(problems, nu_sigma_f, phi_init, phi_out):
    n = len(problems)
    if len(nu_sigma_f) != n or len(phi_out) != n or (phi_init is not None
                                                     and len(phi_init) != n):
        raise ValueError("one nu_sigma_f, phi_out (and phi_init) per problem")
    for i, p in enumerate(problems):
        for t in [nu_sigma_f[i], phi_out[i]] + ([] if phi_init is None or phi_init[i] is None
                                                else [phi_init[i]]):
            if (str(t.dtype) != "torch.float32" or t.device.type != "cuda"
                    or t.numel() != p.nx * p.ny):
                raise ValueError(f"problem {i}: nu_sigma_f, phi_init and phi_out must be "
                                 f"float32 GPU tensors of {p.nx * p.ny} cells")


def tr_eigen(ctx: Context, problems: Sequence[Problem], nu_sigma_f: Sequence,
             quad: Quad, phi_init: Optional[Sequence], phi_out: Sequence,
             k_init: Optional[Sequence[float]] = None, tol_k: float = 1e-6,
             tol_phi: float = 1e-5, tol_inner: float = 1e-6, max_outer: int = 1000,
             max_inner: int = 10000, raise_on_error: bool = True):
    """k-eigenvalue power iteration; the problems' source fields are not
    read.  Returns (status, list of per-instance stats dicts)."""
    n = len(problems)
    arr = make_problems(problems)
    stats = (TrEigenStats * n)()
    _check_eigen_fields(problems, nu_sigma_f, phi_init, phi_out)
    init = None if phi_init is None else _ptr_array(phi_init)
    kin = None if k_init is None else (ctypes.c_double * n)(*[float(k) for k in k_init])
    rc = ctx.lib.tr_eigen(ctx.handle, n, arr, _ptr_array(nu_sigma_f),
                          ctypes.byref(quad.struct), init, _ptr_array(phi_out), kin,
                          float(tol_k), float(tol_phi), float(tol_inner), int(max_outer),
                          int(max_inner), stats)
    if raise_on_error:
        ctx.check(rc)
    return rc, _eigen_stats(stats)


def tr_eigen_mg(ctx: Context, problems: Sequence[Problem], groups: Sequence[dict],
                quad: Quad, phi_init: Optional[Sequence[Sequence]], phi_out: Sequence[Sequence],
                k_init: Optional[Sequence[float]] = None, tol_k: float = 1e-6,
                tol_phi: float = 1e-5, tol_inner: float = 1e-6, max_outer: int = 1000,
                max_inner: int = 10000, raise_on_error: bool = True):
    """Multigroup k-eigenvalue.  problems[i] gives the geometry (its sigma_t
    only fixes the grid); groups[i] = dict(sigma_t=[G], sigma_s=[[G x G],
    None = zero], nu_sigma_f=[G], chi=[G floats]); phi_out[i][g] (and
    phi_init[i][g]) are device fields.  Returns (status, stats dicts)."""
    n = len(problems)
    if n < 1 or len(groups) != n or len(phi_out) != n:
        raise ValueError("one group table and one phi_out list per problem")
    if phi_init is not None and len(phi_init) != n:
        raise ValueError("one phi_init list per problem")
    G = len(groups[0]["sigma_t"])
    if not 1 <= G <= 8:
        raise ValueError("1 to 8 groups")
    # every list the library indexes by group must hold G entries: the
    # pointer arrays built below are exactly that long
    for i, gd in enumerate(groups):
        ss_rows = gd["sigma_s"]
        if (len(gd["sigma_t"]) != G or len(gd["nu_sigma_f"]) != G or len(gd["chi"]) != G
                or len(phi_out[i]) != G or len(ss_rows) != G
                or any(len(row) != G for row in ss_rows)
                or (phi_init is not None and len(phi_init[i]) != G)):
            raise ValueError(f"problem {i}: sigma_t, nu_sigma_f, chi, phi_out (and "
                             f"phi_init) need {G} entries and sigma_s {G} x {G}")
    arr = make_problems(problems)
    keep = []
    mg = (TrMultigroup * n)()
    for i, (p, gd) in enumerate(zip(problems, groups)):
        cells = p.nx * p.ny
        fields = list(gd["sigma_t"]) + list(gd["nu_sigma_f"]) + list(phi_out[i]) + [
            t for row in gd["sigma_s"] for t in row if t is not None]
        if phi_init is not None:
            fields += [t for t in phi_init[i] if t is not None]
        for t in fields:
            if (str(t.dtype) != "torch.float32" or t.device.type != "cuda"
                    or t.numel() != cells):
                raise ValueError(f"problem {i}: group fields must be float32 GPU tensors "
                                 f"of {cells} cells")
        st = _ptr_array(gd["sigma_t"])
        nsf = _ptr_array(gd["nu_sigma_f"])
        ss = (ctypes.c_void_p * (G * G))()
        for g in range(G):
            for h in range(G):
                t = gd["sigma_s"][g][h]
                ss[g * G + h] = None if t is None else _ptr(t)
        chi = (ctypes.c_double * G)(*[float(x) for x in gd["chi"]])
        keep += [st, nsf, ss, chi]
        mg[i].n_groups = G
        mg[i].sigma_t = ctypes.cast(st, ctypes.c_void_p)
        mg[i].sigma_s = ctypes.cast(ss, ctypes.c_void_p)
        mg[i].nu_sigma_f = ctypes.cast(nsf, ctypes.c_void_p)
        mg[i].chi = ctypes.cast(chi, ctypes.c_void_p)
    out = _ptr_array([t for row in phi_out for t in row])
    init = None if phi_init is None else _ptr_array([t for row in phi_init for t in row])
    kin = None if k_init is None else (ctypes.c_double * n)(*[float(k) for k in k_init])
    stats = (TrEigenStats * n)()
    rc = ctx.lib.tr_eigen_mg(ctx.handle, n, arr, mg, ctypes.byref(quad.struct), init, out, kin,
                             float(tol_k), float(tol_phi), float(tol_inner), int(max_outer),
                             int(max_inner), stats)
    del keep
    if raise_on_error:
        ctx.check(rc)
    return rc, _eigen_stats(stats)


def _eigen_stats(stats):
    return [dict(status=s.status, outer=s.outer, inner=s.inner, k=s.k, dk=s.dk,
                 dphi=s.dphi, balance_rel=s.balance_rel, seconds=s.seconds) for s in stats]


def no_eigen(ctx: Context, model: "Model", problems: Sequence[Problem], nu_sigma_f: Sequence,
             quad: Quad, sigma_t_star: float, sigma_s_star: float, variant: int,
             phi_init: Optional[Sequence], phi_out: Sequence,
             k_init: Optional[Sequence[float]] = None, tol_k: float = 1e-4,
             tol_phi: float = 1e-4, max_outer: int = 500, raise_on_error: bool = True):
    """Neural-operator outer loop of the eigenvalue problem (NO_EIGEN_SP or
    NO_EIGEN_CP).  Returns (status, list of per-instance stats dicts)."""
    n = len(problems)
    arr = make_problems(problems)
    _check_eigen_fields(problems, nu_sigma_f, phi_init, phi_out)
    stats = (TrEigenStats * n)()
    init = None if phi_init is None else _ptr_array(phi_init)
    kin = None if k_init is None else (ctypes.c_double * n)(*[float(k) for k in k_init])
    rc = ctx.lib.no_eigen(ctx.handle, model.handle, n, arr, _ptr_array(nu_sigma_f),
                          ctypes.byref(quad.struct), float(sigma_t_star), float(sigma_s_star),
                          int(variant), init, _ptr_array(phi_out), kin, float(tol_k),
                          float(tol_phi), int(max_outer), stats)
    if raise_on_error:
        ctx.check(rc)
    return rc, _eigen_stats(stats)


def eigen_preconditioned(ctx: Context, model: "Model", problems: Sequence[Problem],
                         nu_sigma_f: Sequence, quad: Quad, sigma_t_star: float,
                         sigma_s_star: float, variant: int, phi_out: Sequence,
                         tol_k: float = 1e-4, tol_phi: float = 1e-4, tol_inner: float = 1e-4,
                         max_outer: int = 500, max_inner: int = 10000,
                         no_tol_k: float = 1e-3, no_tol_phi: float = 1e-3,
                         no_max_outer: int = 30):
    """SP or CP (Appendix A2): the network loop (its own tolerances: it only
    preconditions, and a BF16 network settles near 1e-3), then the
    model-based eigenvalue solve started from its pair (Eq. A6).  phi_out
    receives the refined eigenfunction.  Returns (status of the refinement,
    network-loop stats, refined stats)."""
    _, st1 = no_eigen(ctx, model, problems, nu_sigma_f, quad, sigma_t_star, sigma_s_star,
                      variant, None, phi_out, None, no_tol_k, no_tol_phi, no_max_outer)
    rc2, st2 = tr_eigen(ctx, problems, nu_sigma_f, quad, phi_out, phi_out,
                        [s["k"] for s in st1], tol_k, tol_phi, tol_inner, max_outer, max_inner)
    return rc2, st1, st2


def tr_check_args(problems_struct, n: int, quad: Quad, tol: float,
                  max_iter: int):
    """Host-only argument check on a prepared TrProblem array."""
    lib = load()
    buf = ctypes.create_string_buffer(512)
    rc = lib.tr_check_args(n, problems_struct, ctypes.byref(quad.struct),
                           float(tol), int(max_iter), buf, 512)
    return rc, buf.value.decode()


def sweep_plan(problems_struct, n: int, quad: Quad, handle=None) -> dict:
    """Launch shape of the 2-D sweep for prepared problems (host-only when
    handle is None)."""
    lib = load()
    out = (ctypes.c_int32 * 6)()
    rc = lib.tr_get_sweep_plan(handle, n, problems_struct, ctypes.byref(quad.struct), out)
    if rc != TR_OK:
        raise MdpError(rc, "tr_get_sweep_plan failed")
    return dict(D=out[0], W=out[1], S=out[2], R=out[3], KB=out[4], specialised=out[5])


# ---------------------------------------------------------------- network

class Model:
    """no_model handle: the 2-D FNO (arch "fno": width 32, modes 12, 4
    layers, 64 x 64) or the DeepONet (arch "deeponet": 64 x 64 sensors,
    hidden 200, basis 100)."""

    def __init__(self, ctx: Context, params: Optional[np.ndarray] = None,
                 width: int = 32, modes: int = 12, layers: int = 4, grid: int = 64,
                 arch: str = "fno"):
        self.ctx = ctx
        self.lib = ctx.lib
        self.grid = grid
        self.arch = arch
        h = ctypes.c_void_p()
        buf = None
        if params is not None:
            buf = np.ascontiguousarray(params, dtype=np.float32)
        ptr = None if buf is None else buf.ctypes.data
        if arch == "fno":
            rc = self.lib.no_model_create(ctx.handle, ctypes.byref(h), width, modes,
                                          layers, grid, ptr)
        elif arch == "deeponet":
            rc = self.lib.no_model_create_deeponet(ctx.handle, ctypes.byref(h), grid, 200, 100,
                                                   ptr)
        else:
            raise ValueError(f"unknown network {arch!r}")
        ctx.check(rc, allow=(TR_OK,))
        self.handle = h
        self.n_params = int(self.lib.no_model_param_count(h))
        if buf is not None and buf.size != self.n_params:
            self.close()
            raise ValueError(f"expected {self.n_params} parameters, got {buf.size}")

    def close(self):
        if getattr(self, "handle", None):
            self.lib.no_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_fp32(self, enable: bool = True):
        self.ctx.check(self.lib.no_model_set_fp32(self.handle, int(enable)), allow=(TR_OK,))

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        self.ctx.check(self.lib.no_model_get_params(self.ctx.handle, self.handle,
                                                    out.ctypes.data), allow=(TR_OK,))
        return out

    def set_params(self, params: np.ndarray):
        buf = np.ascontiguousarray(params, dtype=np.float32)
        if buf.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {buf.size}")
        self.ctx.check(self.lib.no_model_set_params(self.ctx.handle, self.handle,
                                                    buf.ctypes.data), allow=(TR_OK,))

    def get_state(self) -> dict:
        """Training checkpoint: FP32 parameters, Adam moments, step count."""
        p, m, v = (np.empty(self.n_params, dtype=np.float32) for _ in range(3))
        step = ctypes.c_int64()
        self.ctx.check(self.lib.no_model_get_state(self.ctx.handle, self.handle, p.ctypes.data,
                                                   m.ctypes.data, v.ctypes.data,
                                                   ctypes.byref(step)), allow=(TR_OK,))
        return dict(params=p, adam_m=m, adam_v=v, step=int(step.value))

    def set_state(self, state: dict):
        bufs = [np.ascontiguousarray(state[k], dtype=np.float32)
                for k in ("params", "adam_m", "adam_v")]
        if any(b.size != self.n_params for b in bufs):
            raise ValueError(f"expected {self.n_params} values per array")
        self.ctx.check(self.lib.no_model_set_state(self.ctx.handle, self.handle,
                                                   *[b.ctypes.data for b in bufs],
                                                   int(state["step"])), allow=(TR_OK,))

    def forward(self, inp, out=None):
        """inp: float32 GPU tensor (B, grid, grid) -> output tensor (B, grid, grid)."""
        import torch
        if out is None:
            out = torch.empty_like(inp)
        B = int(inp.shape[0])
        self.ctx.check(self.lib.no_forward(self.ctx.handle, self.handle, B,
                                           _ptr(inp), _ptr(out)), allow=(TR_OK,))
        return out

    def train_step(self, inp, target, lr: float, grad_out=None) -> float:
        loss = ctypes.c_double()
        B = int(inp.shape[0])
        self.ctx.check(self.lib.no_train_step(self.ctx.handle, self.handle, B, _ptr(inp),
                                              _ptr(target), float(lr), ctypes.byref(loss),
                                              _ptr(grad_out)), allow=(TR_OK,))
        return loss.value


def no_recast_guess(ctx: Context, model: Model, problems: Sequence[Problem],
                    sigma_t_star: float, sigma_s_star: float, tol: float,
                    max_iter: int, phi_guess: Sequence, raise_on_error: bool = True):
    """Returns (status, list of per-instance stats dicts)."""
    n = len(problems)
    arr = make_problems(problems)
    stats = (TrStats * n)()
    rc = ctx.lib.no_recast_guess(ctx.handle, model.handle, n, arr, float(sigma_t_star),
                                 float(sigma_s_star), float(tol), int(max_iter),
                                 _ptr_array(phi_guess), stats)
    if raise_on_error:
        ctx.check(rc)
    return rc, [dict(status=s.status, iterations=s.iterations, residual=s.residual,
                     seconds=s.seconds) for s in stats]
