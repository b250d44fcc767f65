"""FP64 oracle for the S_N source-iteration path and the operator network.

TEST INFRASTRUCTURE ONLY: this package is imported by the test suite, the
smoke check and the benchmark's CPU-baseline leg, never by the library.  It
shares no code with the HIP path.

Contents
  * ``si_oracle.c`` (loaded here through ctypes): diamond-difference sweeps and
    source iteration in 1-D and 2-D, FP64 (section 5.1, Eq. 12; the iteration
    M of Eq. 3a/4b);
  * ``recast``: the equation-recast loop of Eq. 24 with a caller-given inner
    solution operator (the exact transport operator at p* for the closed-form
    check, or a network);
  * ``fno``: FP64 forward/backward of the Fourier neural operator and Adam;
  * ``deeponet``: FP64 forward/backward of the deep operator network
    (section 4.1 Eq. 11, Appendix A1);
  * ``eigen``: the k-eigenvalue power iteration (one group: section 5.2
    Eq. 26, Appendix A2 Eq. A1-A4, with the SP/CP variants; three groups
    with downscatter: section 5.3 Eq. 27-29) around the source iteration.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "si_oracle.c")
# ORACLE_LIB: another build of si_oracle.c (the sanitizer build)
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "libsi_oracle.so")
_lib = None
_lock = threading.Lock()

OK = 0
NOT_CONVERGED = 1


def build(force: bool = True) -> str:
    """Compile si_oracle.c with gcc into oracle/libsi_oracle.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build(force=True)
            lib = ctypes.CDLL(_LIB_PATH)
            D = ctypes.POINTER(ctypes.c_double)
            I = ctypes.POINTER(ctypes.c_int)
            i, d = ctypes.c_int, ctypes.c_double
            lib.or_sweep2d.argtypes = [i, i, d, d, i, D, D, D, D, D, D, D, I, D, D, D,
                                       D, D, D]
            lib.or_si2d.argtypes = [i, i, d, d, i, D, D, D, D, D, D, D, I, D, d, i,
                                    i, i, D, D, D]
            lib.or_sweep1d.argtypes = [i, d, i, D, D, D, D, D, I, D, D, D, D, D]
            lib.or_si1d.argtypes = [i, d, i, D, D, D, D, D, D, I, D, d, i, i, i, D, D, D]
            for f in (lib.or_sweep2d, lib.or_si2d, lib.or_sweep1d, lib.or_si1d):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.cast(None, ctypes.POINTER(ctypes.c_double))
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _bc(bc) -> ctypes.Array:
    return (ctypes.c_int * 4)(*[int(b) for b in (list(bc) + [0, 0, 0, 0])[:4]])


def _norm_kind(norm: str) -> int:
    """Stopping rule of si1d/si2d: "l2" relative L2 change < tol, "max"
    max relative change < tol, "bound" the fixed-point error bound
    r rho / (1 - rho) < tol with rho = r_l / r_(l-1) (r the relative L2
    change); with stride K > 1 the bound is tested every K iterations on
    the change over those K iterations (rho = r_l / r_(l-K))."""
    kinds = {"l2": 0, "max": 1, "bound": 2}
    if norm not in kinds:
        raise ValueError(f"unknown stopping rule {norm!r}")
    return kinds[norm]


class SolveResult:
    def __init__(self, phi, status, iterations, residual, leak, dscatter,
                 hist):
        self.phi = phi
        self.status = status
        self.iterations = iterations
        self.residual = residual
        self.leakage = leak
        self.dscatter = dscatter
        self.history = hist


def sweep2d(nx, ny, lx, ly, mu, eta, w, sigma_t, emission, bc=(0, 0, 0, 0),
            face_prev=None, return_faces=False, ex=None, ey=None,
            return_current=False):
    """One 2-D DD sweep of every direction for the isotropic emission
    density Q, plus mu_m ex + eta_m ey per direction when the anisotropic
    fields are given (P1: ex, ey = 3 sigma_s1 J).

    Returns phi (ny, nx) [and the face array (4, max(nx,ny), M), leakage]
    [and the current (jx, jy) when return_current]."""
    lib = _load()
    mu, eta, w = _f64(mu), _f64(eta), _f64(w)
    M = mu.shape[0]
    nf = max(nx, ny)
    st = _f64(sigma_t).reshape(-1)
    Q = _f64(emission).reshape(-1)
    phi = np.zeros(nx * ny)
    fo = np.zeros(4 * nf * M)
    fp = None if face_prev is None else _f64(face_prev).reshape(-1)
    exa = None if ex is None else _f64(ex).reshape(-1)
    eya = None if ey is None else _f64(ey).reshape(-1)
    jx = np.zeros(nx * ny) if return_current else None
    jy = np.zeros(nx * ny) if return_current else None
    leak = ctypes.c_double(0.0)
    rc = lib.or_sweep2d(nx, ny, lx, ly, M, _dp(mu), _dp(eta), _dp(w), _dp(st),
                        _dp(Q), _dp(exa), _dp(eya), _bc(bc), _dp(fp), _dp(fo), _dp(phi),
                        _dp(jx), _dp(jy), ctypes.byref(leak))
    if rc != OK:
        raise ValueError(f"or_sweep2d failed ({rc})")
    phi = phi.reshape(ny, nx)
    out = (phi,)
    if return_faces:
        out += (fo.reshape(4, nf, M), leak.value)
    if return_current:
        out += ((jx.reshape(ny, nx), jy.reshape(ny, nx)),)
    return out[0] if len(out) == 1 else out


def si2d(nx, ny, lx, ly, mu, eta, w, sigma_t, sigma_s, q, bc=(0, 0, 0, 0),
         phi0=None, tol=1e-6, max_iter=100000, norm="l2", stride=1,
         sigma_s1=None) -> SolveResult:
    """2-D source iteration to tolerance (zero start unless phi0 is given);
    sigma_s1: first Legendre moment of scattering (P1, Eq. 25), or None."""
    lib = _load()
    mu, eta, w = _f64(mu), _f64(eta), _f64(w)
    M = mu.shape[0]
    st = _f64(sigma_t).reshape(-1)
    ss = _f64(sigma_s).reshape(-1)
    s1 = None if sigma_s1 is None else _f64(sigma_s1).reshape(-1)
    qq = _f64(q).reshape(-1)
    p0 = None if phi0 is None else _f64(phi0).reshape(-1)
    phi = np.zeros(nx * ny)
    stats = np.zeros(4)
    hist = np.zeros(max_iter)
    rc = lib.or_si2d(nx, ny, lx, ly, M, _dp(mu), _dp(eta), _dp(w), _dp(st),
                     _dp(ss), _dp(s1), _dp(qq), _bc(bc), _dp(p0), float(tol),
                     int(max_iter), _norm_kind(norm), int(stride), _dp(phi),
                     _dp(stats), _dp(hist))
    if rc < 0:
        raise ValueError(f"or_si2d failed ({rc})")
    it = int(stats[0])
    return SolveResult(phi.reshape(ny, nx), rc, it, stats[1], stats[2],
                       stats[3], hist[:it].copy())


def sweep1d(nx, lx, mu, w, sigma_t, emission, bc=(0, 0), face_prev=None,
            return_faces=False, ex=None, return_current=False):
    """One 1-D DD sweep for the isotropic emission Q plus mu_m ex per
    direction (P1: ex = 3 sigma_s1 J).  Returns phi [faces, leakage]
    [current]."""
    lib = _load()
    mu, w = _f64(mu), _f64(w)
    M = mu.shape[0]
    st = _f64(sigma_t).reshape(-1)
    Q = _f64(emission).reshape(-1)
    phi = np.zeros(nx)
    fo = np.zeros(2 * M)
    fp = None if face_prev is None else _f64(face_prev).reshape(-1)
    exa = None if ex is None else _f64(ex).reshape(-1)
    jx = np.zeros(nx) if return_current else None
    leak = ctypes.c_double(0.0)
    rc = lib.or_sweep1d(nx, lx, M, _dp(mu), _dp(w), _dp(st), _dp(Q), _dp(exa), _bc(bc),
                        _dp(fp), _dp(fo), _dp(phi), _dp(jx), ctypes.byref(leak))
    if rc != OK:
        raise ValueError(f"or_sweep1d failed ({rc})")
    out = (phi,)
    if return_faces:
        out += (fo.reshape(2, M), leak.value)
    if return_current:
        out += (jx,)
    return out[0] if len(out) == 1 else out


def si1d(nx, lx, mu, w, sigma_t, sigma_s, q, bc=(0, 0), phi0=None, tol=1e-8,
         max_iter=100000, norm="max", stride=1, sigma_s1=None) -> SolveResult:
    lib = _load()
    mu, w = _f64(mu), _f64(w)
    M = mu.shape[0]
    st = _f64(sigma_t).reshape(-1)
    ss = _f64(sigma_s).reshape(-1)
    s1 = None if sigma_s1 is None else _f64(sigma_s1).reshape(-1)
    qq = _f64(q).reshape(-1)
    p0 = None if phi0 is None else _f64(phi0).reshape(-1)
    phi = np.zeros(nx)
    stats = np.zeros(4)
    hist = np.zeros(max_iter)
    rc = lib.or_si1d(nx, lx, M, _dp(mu), _dp(w), _dp(st), _dp(ss), _dp(s1), _dp(qq),
                     _bc(bc), _dp(p0), float(tol), int(max_iter),
                     _norm_kind(norm), int(stride), _dp(phi), _dp(stats),
                     _dp(hist))
    if rc < 0:
        raise ValueError(f"or_si1d failed ({rc})")
    it = int(stats[0])
    return SolveResult(phi, rc, it, stats[1], stats[2], stats[3],
                       hist[:it].copy())


def f32_rounded(a) -> np.ndarray:
    """A field as the FP32 library receives it, widened back to FP64 (the
    oracle then solves exactly the problem the library is given)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def solve_instance(inst, quad, tol, phi0=None, max_iter=100000, norm=None,
                   f32_inputs=False, stride=1):
    """Solve one inputs.Instance with the oracle (dim from the instance).
    f32_inputs: round sigma_t, sigma_s and the source to FP32 first."""
    if f32_inputs:
        import copy
        inst = copy.copy(inst)
        inst.sigma_t = f32_rounded(inst.sigma_t)
        inst.sigma_s = f32_rounded(inst.sigma_s)
        inst.source = f32_rounded(inst.source)
        if getattr(inst, "sigma_s1", None) is not None:
            inst.sigma_s1 = f32_rounded(inst.sigma_s1)
    if inst.dim == 1:
        return si1d(inst.nx, inst.lx, quad.mu, quad.w, inst.sigma_t,
                    inst.sigma_s, inst.source, bc=inst.bc[:2], phi0=phi0,
                    tol=tol, max_iter=max_iter, norm=norm or "max", stride=stride,
                    sigma_s1=getattr(inst, "sigma_s1", None))
    return si2d(inst.nx, inst.ny, inst.lx, inst.ly, quad.mu, quad.eta, quad.w,
                inst.sigma_t, inst.sigma_s, inst.source, bc=inst.bc,
                phi0=phi0, tol=tol, max_iter=max_iter, norm=norm or "l2", stride=stride,
                sigma_s1=getattr(inst, "sigma_s1", None))


def solve_many(insts: Sequence, quad, tol, phi0s=None, threads: int = 1,
               max_iter=100000, norm=None, f32_inputs=False, stride=1):
    """Solve several instances, one per worker thread (the C call releases
    the interpreter lock).  Returns a list of SolveResult."""
    phi0s = phi0s if phi0s is not None else [None] * len(insts)
    kw = dict(norm=norm, f32_inputs=f32_inputs, stride=stride)
    if threads <= 1:
        return [solve_instance(i, quad, tol, p, max_iter, **kw)
                for i, p in zip(insts, phi0s)]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        futs = [ex.submit(solve_instance, i, quad, tol, p, max_iter, **kw)
                for i, p in zip(insts, phi0s)]
        return [f.result() for f in futs]
