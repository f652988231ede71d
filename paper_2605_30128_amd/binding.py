"""Thin Python binding of the C ABI in include/chfsi.h (argument marshalling
only: every step runs in the HIP library).  PyTorch provides device memory
and streams; tensors are passed as raw device pointers.

The library must be built (paper_2605_30128_amd/build.py); importing this
module on a machine without it raises, so no path silently falls back to
anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# CHFSI_LIBRARY selects another build of the same library (e.g. a host-sanitizer build)
LIB_PATH = os.environ.get("CHFSI_LIBRARY") or os.path.join(HERE, "libchfsi.so")

FP64, FP32, BF16 = 0, 1, 2
PREC = {"fp64": FP64, "fp32": FP32, "bf16": BF16, FP64: FP64, FP32: FP32, BF16: BF16}

OK, NOT_CONVERGED = 0, 1
E_ARG, E_DEVICE, E_NOT_SPD, E_BOUNDS, E_NONFINITE, E_DIVERGED, E_WORKSPACE = -1, -2, -3, -4, -5, -6, -7


class ChfsiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"chfsi error {code}: {msg}")
        self.code = code


class _Mesh(C.Structure):
    _fields_ = [("ncell", C.c_int64 * 3), ("h", C.c_double * 3), ("degree", C.c_int), ("nq1d", C.c_int)]


class _Proj(C.Structure):
    _fields_ = [("natoms", C.c_int64), ("nbeta", C.c_int), ("pair_ptr", C.c_void_p),
                ("pair_cell", C.c_void_p), ("phi", C.c_void_p), ("delta", C.c_void_p)]


class SolveOpts(C.Structure):
    _fields_ = [("prec", C.c_int), ("degree", C.c_int), ("tol", C.c_double), ("max_iter", C.c_int),
                ("lanczos_steps", C.c_int), ("lambda_max", C.c_double), ("fixed_iters", C.c_int),
                ("rr_mode", C.c_int), ("resume", C.c_int), ("block", C.c_int64), ("profile", C.c_int)]


class PlanOpts(C.Structure):
    _fields_ = [("max_nvec", C.c_int64), ("filter_block", C.c_int64), ("filter_prec", C.c_int)]


class Report(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("max_res", C.c_double),
                ("lambda_bounds", C.c_double * 3), ("t_filter", C.c_double), ("t_rr", C.c_double),
                ("t_total", C.c_double), ("t_iter_median", C.c_double), ("t_filter_cell", C.c_double),
                ("filter_cell_launches", C.c_int64)]


class PcgOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("cheb_degree", C.c_int),
                ("lanczos_steps", C.c_int), ("lambda_max", C.c_double), ("range", C.c_double)]


class PcgReport(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("res_norm", C.c_double),
                ("lambda_min", C.c_double), ("lambda_max", C.c_double), ("t_lanczos", C.c_double),
                ("t_total", C.c_double)]


SYMBOLS = [
    "chfsi_plan", "chfsi_setup", "chfsi_plan_ex", "chfsi_setup_ex", "chfsi_set_fields", "chfsi_apply_H", "chfsi_apply_M",
    "chfsi_apply_H_adjoint", "chfsi_estimate_bounds", "chfsi_filter", "chfsi_orthonormalize",
    "chfsi_rayleigh_ritz", "chfsi_rayleigh_ritz_general", "chfsi_residual", "chfsi_residual_noalloc", "chfsi_solve_workspace", "chfsi_solve", "chfsi_info",
    "chfsi_mass_diag", "chfsi_profile_apply_H", "chfsi_bfp_bytes", "chfsi_bfp_encode", "chfsi_bfp_decode",
    "chfsi_apply_K", "chfsi_poisson_precond", "chfsi_poisson_solve",
    "chfsi_last_error", "chfsi_destroy",
]

_lib = None


def load(path: str = LIB_PATH):
    """Loads libchfsi.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2605_30128_amd.build")
    L = C.CDLL(path)
    vp, i64, i = C.c_void_p, C.c_int64, C.c_int
    L.chfsi_plan.argtypes = [vp, vp, i64, vp, vp]
    L.chfsi_setup.argtypes = [vp, vp, vp, vp, i64, vp, C.c_size_t, vp, C.c_size_t, vp, vp]
    L.chfsi_plan_ex.argtypes = [vp, vp, vp, vp, vp]
    L.chfsi_setup_ex.argtypes = [vp, vp, vp, vp, vp, vp, C.c_size_t, vp, C.c_size_t, vp, vp]
    L.chfsi_set_fields.argtypes = [vp, vp, vp, vp]
    L.chfsi_apply_H.argtypes = [vp, i, vp, vp, i64, i64, vp]
    L.chfsi_apply_M.argtypes = [vp, vp, vp, i64, i64, vp]
    L.chfsi_apply_H_adjoint.argtypes = [vp, i, vp, vp, i64, i64, vp, vp, vp, vp]
    L.chfsi_estimate_bounds.argtypes = [vp, i, vp, vp, vp]
    L.chfsi_filter.argtypes = [vp, i, i, vp, vp, vp, vp, vp, i64, i64, vp]
    L.chfsi_orthonormalize.argtypes = [vp, vp, vp, vp, i64, i64, vp]
    L.chfsi_rayleigh_ritz.argtypes = [vp, vp, vp, vp, i64, i64, vp, vp, vp, vp]
    L.chfsi_rayleigh_ritz_general.argtypes = [vp, vp, vp, vp, i64, i64, vp, vp, vp, vp]
    L.chfsi_residual.argtypes = [vp, vp, vp, vp, vp, vp, i64, i64, vp]
    L.chfsi_residual_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, i64, i64, vp]
    L.chfsi_solve_workspace.argtypes = [vp, i64, i64, vp]
    L.chfsi_solve.argtypes = [vp, i64, vp, vp, i64, i64, vp, vp, vp, vp, vp, C.c_size_t, vp]
    L.chfsi_info.argtypes = [vp, vp, vp, vp, vp]
    L.chfsi_mass_diag.argtypes = [vp, vp, vp]
    L.chfsi_profile_apply_H.argtypes = [vp, i, vp, vp, i64, i64, vp, vp, vp]
    L.chfsi_bfp_bytes.argtypes = [i, i64, vp]
    L.chfsi_bfp_encode.argtypes = [i, vp, i64, vp, vp]
    L.chfsi_bfp_decode.argtypes = [i, vp, i64, vp, vp]
    L.chfsi_apply_K.argtypes = [vp, vp, vp, vp]
    L.chfsi_poisson_precond.argtypes = [vp, i, C.c_double, C.c_double, vp, vp, vp]
    L.chfsi_poisson_solve.argtypes = [vp, vp, vp, vp, vp, vp]
    L.chfsi_last_error.argtypes = [vp]
    L.chfsi_last_error.restype = C.c_char_p
    L.chfsi_destroy.argtypes = [vp]
    for name in SYMBOLS:
        if name not in ("chfsi_last_error", "chfsi_destroy"):
            getattr(L, name).restype = C.c_int
    L.chfsi_destroy.restype = None
    _lib = L
    return L


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def cplx_dtype(prec) -> torch.dtype:
    return torch.complex128 if PREC[prec] == FP64 else torch.complex64


def _check_global(rc):
    if rc < 0:
        raise ChfsiError(rc, load().chfsi_last_error(None).decode())
    return rc


def bfp_bytes(nbits: int, n: int) -> int:
    """Size in bytes of the block floating-point stream of n values."""
    out = C.c_int64()
    _check_global(load().chfsi_bfp_bytes(int(nbits), int(n), C.byref(out)))
    return out.value


def bfp_encode(x, nbits: int, out=None):
    """Encodes a contiguous float32 device tensor (numel a multiple of 4)
    into a uint8 device tensor (chfsi_bfp_encode)."""
    if x.dtype != torch.float32 or not x.is_contiguous():
        raise ValueError("x must be a contiguous float32 tensor")
    n = x.numel()
    if out is None:
        out = torch.empty(bfp_bytes(nbits, n), dtype=torch.uint8, device=x.device)
    _check_global(load().chfsi_bfp_encode(int(nbits), _ptr(x), n, _ptr(out), _stream()))
    return out


def bfp_decode(stream, n: int, nbits: int, out=None):
    """Decodes n float32 values from a uint8 device stream (chfsi_bfp_decode)."""
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=stream.device)
    _check_global(load().chfsi_bfp_decode(int(nbits), _ptr(stream), int(n), _ptr(out), _stream()))
    return out


@dataclass
class ProblemArrays:
    ncell: tuple
    h: tuple
    degree: int
    nq1: int
    V: np.ndarray
    B: np.ndarray
    nbeta: int
    pair_ptr: np.ndarray
    pair_cell: np.ndarray
    phi: np.ndarray
    delta: np.ndarray


class Chfsi:
    """One operator (mesh, fields, projectors) on the current CUDA device."""

    def __init__(self, prob, max_nvec: int, device="cuda", filter_block: int = 0, filter_prec="fp64"):
        """filter_block, filter_prec: scratch sizing of the filter's two
        recurrence blocks (chfsi_plan_ex); the defaults hold max_nvec
        complex128 columns."""
        L = load()
        self.L = L
        self.prob = prob
        self.max_nvec = int(max_nvec)
        self._popts = PlanOpts(self.max_nvec, int(filter_block), PREC[filter_prec])
        self.device = torch.device(device)
        self._mesh = _Mesh((C.c_int64 * 3)(*prob.ncell), (C.c_double * 3)(*prob.h), int(prob.degree),
                           int(prob.nq1))
        natoms = int(prob.pair_ptr.size - 1) if prob.pair_cell.size else 0
        self._keep = [np.ascontiguousarray(prob.pair_ptr, np.int64),
                      np.ascontiguousarray(prob.pair_cell, np.int64),
                      np.ascontiguousarray(prob.phi, np.complex128),
                      np.ascontiguousarray(prob.delta, np.complex128)]
        k = self._keep
        self._proj = _Proj(natoms, int(prob.nbeta), k[0].ctypes.data, k[1].ctypes.data,
                           k[2].ctypes.data, k[3].ctypes.data)
        pb, sb = C.c_size_t(), C.c_size_t()
        self._check(L.chfsi_plan_ex(C.byref(self._mesh), C.byref(self._proj), C.byref(self._popts),
                                    C.byref(pb), C.byref(sb)), None)
        self.persistent = torch.empty(pb.value, dtype=torch.uint8, device=self.device)
        self.scratch = torch.empty(sb.value, dtype=torch.uint8, device=self.device)
        self.V = torch.as_tensor(np.ascontiguousarray(prob.V, np.float64), device=self.device)
        self.B = torch.as_tensor(np.ascontiguousarray(prob.B, np.float64), device=self.device)
        ctx = C.c_void_p()
        self._check(L.chfsi_setup_ex(C.byref(self._mesh), _ptr(self.V), _ptr(self.B), C.byref(self._proj),
                                     C.byref(self._popts), _ptr(self.persistent), pb.value, _ptr(self.scratch),
                                     sb.value, _stream(), C.byref(ctx)), None)
        self.ctx = ctx
        nn, nc, n, nq = C.c_int64(), C.c_int64(), C.c_int(), C.c_int()
        L.chfsi_info(ctx, C.byref(nn), C.byref(nc), C.byref(n), C.byref(nq))
        self.nnodes, self.ncells, self.n, self.nq = nn.value, nc.value, n.value, nq.value
        self.ndof = 2 * self.nnodes

    def __del__(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            try:
                torch.cuda.synchronize()
            except Exception:
                pass
            self.L.chfsi_destroy(self.ctx)
            self.ctx = None

    def _check(self, rc, ctx="self"):
        if rc < 0:
            c = self.ctx if ctx == "self" else None
            msg = self.L.chfsi_last_error(c)
            raise ChfsiError(rc, msg.decode() if msg else "")
        return rc

    # ------------------------------------------------------------------ ops
    def _block(self, X, dtype, name):
        if X.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {X.dtype}")
        if X.device.type != "cuda" or not X.is_contiguous() or X.dim() != 2 or X.shape[0] != self.ndof:
            raise ValueError(f"{name} must be a contiguous cuda tensor of shape (2M={self.ndof}, ld)")
        return X.shape[1]

    def apply_H(self, X, prec="fp64", nvec=None, Y=None):
        p = PREC[prec]
        ld = self._block(X, cplx_dtype(p), "X")
        nvec = ld if nvec is None else nvec
        Y = torch.empty_like(X) if Y is None else Y
        self._check(self.L.chfsi_apply_H(self.ctx, p, _ptr(X), _ptr(Y), nvec, ld, _stream()))
        return Y

    def apply_M(self, X, nvec=None, Y=None):
        ld = self._block(X, torch.complex128, "X")
        nvec = ld if nvec is None else nvec
        Y = torch.empty_like(X) if Y is None else Y
        self._check(self.L.chfsi_apply_M(self.ctx, _ptr(X), _ptr(Y), nvec, ld, _stream()))
        return Y

    def adjoint(self, X, G, prec="fp64", want_dX=True):
        p = PREC[prec]
        ld = self._block(X, cplx_dtype(p), "X")
        self._block(G, cplx_dtype(p), "G")
        dX = torch.empty_like(X) if want_dX else None
        dV = torch.empty((self.ncells, self.nq), dtype=torch.float64, device=X.device)
        dB = torch.empty((self.ncells, self.nq, 3), dtype=torch.float64, device=X.device)
        self._check(self.L.chfsi_apply_H_adjoint(self.ctx, p, _ptr(X), _ptr(G), ld, ld, _ptr(dX),
                                                 _ptr(dV), _ptr(dB), _stream()))
        return dX, dV, dB

    def set_fields(self, V, B):
        self.V = V.to(self.device, torch.float64).contiguous()
        self.B = B.to(self.device, torch.float64).contiguous()
        self._check(self.L.chfsi_set_fields(self.ctx, _ptr(self.V), _ptr(self.B), _stream()))

    def estimate_bounds(self, v0, steps=20):
        v0 = v0.to(self.device, torch.complex128).contiguous()
        out = C.c_double()
        self._check(self.L.chfsi_estimate_bounds(self.ctx, steps, _ptr(v0), C.byref(out), _stream()))
        return out.value

    def filter(self, X, ritz, R, degree, bounds, prec="fp64", Y=None, nvec=None):
        ld = self._block(X, torch.complex128, "X")
        self._block(R, torch.complex128, "R")
        nvec = ld if nvec is None else nvec
        Y = torch.empty_like(X) if Y is None else Y
        b = (C.c_double * 3)(*[float(v) for v in bounds])
        ritz = ritz.to(self.device, torch.float64).contiguous()
        self._check(self.L.chfsi_filter(self.ctx, PREC[prec], int(degree), b, _ptr(X), _ptr(ritz), _ptr(R),
                                        _ptr(Y), nvec, ld, _stream()))
        return Y

    def orthonormalize(self, Y, HY, MY):
        ld = self._block(Y, torch.complex128, "Y")
        self._check(self.L.chfsi_orthonormalize(self.ctx, _ptr(Y), _ptr(HY), _ptr(MY), ld, ld, _stream()))
        return Y, HY, MY

    def rayleigh_ritz(self, Y, HY, MY, want_residual=True, general=False):
        """general=False: Y must be M-orthonormal; True: generalized subspace problem."""
        ld = self._block(Y, torch.complex128, "Y")
        ritz = torch.empty(ld, dtype=torch.float64, device=Y.device)
        R = torch.empty_like(Y) if want_residual else None
        res = torch.empty(ld, dtype=torch.float64, device=Y.device) if want_residual else None
        fn = self.L.chfsi_rayleigh_ritz_general if general else self.L.chfsi_rayleigh_ritz
        self._check(fn(self.ctx, _ptr(Y), _ptr(HY), _ptr(MY), ld, ld, _ptr(ritz), _ptr(R), _ptr(res),
                       _stream()))
        return ritz, R, res

    def residual(self, HX, MX, ritz, nvec=None, R=None, res=None, noalloc=False):
        """R = HX - MX diag(ritz) and its column norms (chfsi_residual, or
        chfsi_residual_noalloc with noalloc=True: static scratch)."""
        ld = self._block(HX, torch.complex128, "HX")
        nvec = ld if nvec is None else nvec
        R = torch.empty_like(HX) if R is None else R
        res = torch.empty(nvec, dtype=torch.float64, device=HX.device) if res is None else res
        fn = self.L.chfsi_residual_noalloc if noalloc else self.L.chfsi_residual
        self._check(fn(self.ctx, _ptr(HX), _ptr(MX), _ptr(ritz.contiguous()), _ptr(R), _ptr(res), nvec, ld,
                       _stream()))
        return R, res

    # ------------------------------------------------------------ Poisson
    def _vec(self, x, name):
        if x.dtype != torch.float64 or x.device.type != "cuda" or not x.is_contiguous() or x.numel() != self.nnodes:
            raise ValueError(f"{name} must be a contiguous float64 cuda tensor of {self.nnodes} entries")

    def apply_K(self, x, y=None):
        """y = K x, the Poisson stiffness (chfsi_apply_K)."""
        self._vec(x, "x")
        y = torch.empty_like(x) if y is None else y
        self._vec(y, "y")
        self._check(self.L.chfsi_apply_K(self.ctx, _ptr(x), _ptr(y), _stream()))
        return y

    def poisson_precond(self, r, degree, lmin, lmax, z=None):
        """z = P^{-1} r, the Chebyshev-Jacobi preconditioner (chfsi_poisson_precond)."""
        self._vec(r, "r")
        z = torch.empty_like(r) if z is None else z
        self._vec(z, "z")
        self._check(self.L.chfsi_poisson_precond(self.ctx, int(degree), float(lmin), float(lmax), _ptr(r),
                                                 _ptr(z), _stream()))
        return z

    def poisson_solve(self, f, x=None, tol=1e-10, max_iter=5000, cheb_degree=5, lanczos_steps=20,
                      lambda_max=0.0, range_=300.0):
        """PCG solve of K x = f - mean(f) (chfsi_poisson_solve); x is the initial
        guess (zero if None) and is overwritten.  The preconditioner interval is
        [lambda_max / range_, lambda_max]; the default 300 measured best on the
        p = 7 slab (wider intervals gave fewer iterations up to about 300).
        Returns (x, report dict, status)."""
        self._vec(f, "f")
        x = torch.zeros_like(f) if x is None else x
        self._vec(x, "x")
        o = PcgOpts(float(tol), int(max_iter), int(cheb_degree), int(lanczos_steps), float(lambda_max),
                    float(range_))
        rep = PcgReport()
        rc = self._check(self.L.chfsi_poisson_solve(self.ctx, C.byref(o), _ptr(f), _ptr(x), C.byref(rep),
                                                    _stream()))
        out = {k: getattr(rep, k) for k, _ in PcgReport._fields_}
        return x, out, rc

    def mass_diag(self):
        D = torch.empty(self.nnodes, dtype=torch.float64, device=self.device)
        self._check(self.L.chfsi_mass_diag(self.ctx, _ptr(D), _stream()))
        return D

    def profile_apply_H(self, X, prec="fp64", Y=None):
        """One H X with device-event timings: (ms_cell, ms_coeff, ms_total, launches)."""
        p = PREC[prec]
        ld = self._block(X, cplx_dtype(p), "X")
        Y = torch.empty_like(X) if Y is None else Y
        ms = (C.c_double * 3)()
        nl = C.c_int()
        self._check(self.L.chfsi_profile_apply_H(self.ctx, p, _ptr(X), _ptr(Y), ld, ld, ms, C.byref(nl),
                                                 _stream()))
        return ms[0], ms[1], ms[2], nl.value

    def solve(self, X, n_wanted, degree, prec="fp64", tol=1e-8, max_iter=100, v0=None,
              lanczos_steps=20, lambda_max=0.0, fixed_iters=False, resume=False, work=None, rr_mode=1,
              block=0, profile=False):
        """Algorithm RChFSI from the start block X (overwritten with Ritz vectors).
        resume=True continues from the state a previous call left in X and
        `work` (returned as out['work']); lambda_max must then be given.
        profile=True also times the filter steps' cell-operator launches
        (out['t_filter_cell'] seconds over out['filter_cell_launches'])."""
        ld = self._block(X, torch.complex128, "X")
        nsub = ld
        ws = C.c_size_t()
        self._check(self.L.chfsi_solve_workspace(self.ctx, nsub, ld, C.byref(ws)))
        if work is None:
            if resume:
                raise ValueError("resume needs the workspace of the previous call")
            work = torch.empty(ws.value, dtype=torch.uint8, device=X.device)
        opts = SolveOpts(PREC[prec], int(degree), float(tol), int(max_iter),
                         int(lanczos_steps if v0 is not None else 0), float(lambda_max), int(fixed_iters),
                         int(rr_mode), int(resume), int(block), int(bool(profile)))
        eig = np.zeros(n_wanted)
        hist = np.zeros(max_iter + 2)
        rep = Report()
        if v0 is not None:
            v0 = v0.to(self.device, torch.complex128).contiguous()
        rc = self.L.chfsi_solve(self.ctx, n_wanted, C.byref(opts), _ptr(X), nsub, ld, _ptr(v0),
                                eig.ctypes.data_as(C.c_void_p), hist.ctypes.data_as(C.c_void_p),
                                C.byref(rep), _ptr(work), ws.value, _stream())
        self._check(rc)
        return dict(status=rc, eigvals=eig, iters=rep.iters, converged=bool(rep.converged),
                    max_res=rep.max_res, hist_res=hist[:rep.iters + 1], bounds=list(rep.lambda_bounds),
                    t_filter=rep.t_filter, t_rr=rep.t_rr, t_total=rep.t_total,
                    t_iter_median=rep.t_iter_median, t_filter_cell=rep.t_filter_cell,
                    filter_cell_launches=rep.filter_cell_launches, work=work)
