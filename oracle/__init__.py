"""CPU oracle (TEST INFRASTRUCTURE ONLY).

A plain double-precision C implementation of the R-ChFSI eigenproblem and of
every step of its hot path, written from the paper's definitions.  Only the
tests, the smoke check and the CPU baseline leg of the benchmark may import
this package; the product path never does.  It shares no code with the GPU
library: the only common module is the seeded input generator, which holds
none of the method's arithmetic.

Parity pins of each routine live in the CPU test-suite (tests/test_oracle_*).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

KIN, POT, MAG, NLOC, ALL = 1, 2, 4, 8, 15


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        vp, dp, ip, i64, i64p = C.c_void_p, C.c_void_p, C.c_int, C.c_int64, C.c_void_p
        L.orc_create.restype = vp
        L.orc_create.argtypes = [vp, vp, ip, ip, dp, dp, ip, ip, i64p, i64p, dp, dp]
        L.orc_destroy.argtypes = [vp]
        L.orc_gll.argtypes = [ip, dp, dp]
        L.orc_gauss.argtypes = [ip, dp, dp]
        L.orc_lagrange.argtypes = [ip, dp, C.c_double, dp, dp]
        L.orc_mass_diag.argtypes = [vp, dp]
        L.orc_tables.argtypes = [vp, dp, dp, dp]
        L.orc_apply_H.argtypes = [vp, dp, i64, i64, dp, i64, ip]
        L.orc_apply_M.argtypes = [vp, dp, i64, i64, dp, i64]
        L.orc_apply_H_sampled.argtypes = [vp, dp, i64, i64p, i64, i64p, i64, dp]
        L.orc_adjoint_fields.argtypes = [vp, dp, dp, i64, i64, dp, dp]
        L.orc_cholesky.restype = ip
        L.orc_cholesky.argtypes = [ip, dp, dp]
        L.orc_jacobi.restype = ip
        L.orc_jacobi.argtypes = [ip, dp, dp, dp]
        L.orc_dense_geig.restype = ip
        L.orc_dense_geig.argtypes = [ip, dp, dp, dp, dp]
        L.orc_dense.argtypes = [vp, dp, dp, ip]
        L.orc_orthonormalize.restype = ip
        L.orc_orthonormalize.argtypes = [vp, dp, dp, dp, i64, ip]
        L.orc_rayleigh_ritz.argtypes = [vp, dp, dp, dp, i64, ip, dp]
        L.orc_residual.argtypes = [i64, ip, dp, dp, i64, dp, dp, dp]
        L.orc_filter.restype = ip
        L.orc_filter.argtypes = [vp, ip, dp, dp, dp, dp, i64, ip, dp, ip]
        L.orc_chebyshev_plain.restype = ip
        L.orc_chebyshev_plain.argtypes = [vp, ip, dp, dp, i64, ip, dp, ip]
        L.orc_lanczos.restype = C.c_double
        L.orc_lanczos.argtypes = [vp, ip, dp]
        L.orc_chfsi.restype = ip
        L.orc_chfsi.argtypes = [vp, ip, ip, ip, ip, C.c_double, C.c_double, ip, dp, i64, dp, dp, dp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


def set_threads(n: int) -> None:
    os.environ["OMP_NUM_THREADS"] = str(n)


# ---------------------------------------------------------------- 1D tables

def gll(p: int):
    x = np.zeros(p + 1); w = np.zeros(p + 1)
    lib().orc_gll(p, _p(x), _p(w))
    return x, w


def gauss(n: int):
    x = np.zeros(n); w = np.zeros(n)
    lib().orc_gauss(n, _p(x), _p(w))
    return x, w


def lagrange(nodes, x: float):
    nodes = _c(nodes, np.float64)
    l = np.zeros(nodes.size); dl = np.zeros(nodes.size)
    lib().orc_lagrange(nodes.size, _p(nodes), float(x), _p(l), _p(dl))
    return l, dl


# ---------------------------------------------------------------- dense algebra

def cholesky(A):
    A = _c(A, np.complex128)
    L = np.zeros_like(A)
    rc = lib().orc_cholesky(A.shape[0], _p(A), _p(L))
    if rc:
        raise np.linalg.LinAlgError("not positive definite")
    return L


def jacobi(A):
    A = _c(A, np.complex128)
    n = A.shape[0]
    w = np.zeros(n); V = np.zeros((n, n), np.complex128)
    lib().orc_jacobi(n, _p(A), _p(w), _p(V))
    return w, V


def dense_geig(H, M):
    H = _c(H, np.complex128); M = _c(M, np.complex128)
    n = H.shape[0]
    w = np.zeros(n); V = np.zeros((n, n), np.complex128)
    if lib().orc_dense_geig(n, _p(H), _p(M), _p(w), _p(V)):
        raise np.linalg.LinAlgError("M not positive definite")
    return w, V


def residual(HX, MX, ritz):
    HX = _c(HX, np.complex128); MX = _c(MX, np.complex128); ritz = _c(ritz, np.float64)
    rows, ld = HX.shape
    k = ritz.size
    R = np.zeros_like(HX); norms = np.zeros(k)
    lib().orc_residual(rows, k, _p(HX), _p(MX), ld, _p(ritz), _p(R), _p(norms))
    return R, norms


# ---------------------------------------------------------------- problem

class Oracle:
    """The oracle bound to one synthetic problem (synth.Problem)."""

    def __init__(self, prob):
        self.prob = prob
        self._keep = dict(
            ncell=_c(prob.ncell, np.int32), h=_c(prob.h, np.float64),
            V=_c(prob.V, np.float64), B=_c(prob.B, np.float64),
            pair_ptr=_c(prob.pair_ptr, np.int64),
            pair_cell=_c(prob.pair_cell if prob.npairs else np.zeros(1), np.int64),
            phi=_c(prob.phi if prob.npairs else np.zeros(1), np.complex128),
            delta=_c(prob.delta if prob.natoms else np.zeros(1), np.complex128),
        )
        k = self._keep
        self.h = lib().orc_create(_p(k["ncell"]), _p(k["h"]), prob.degree, prob.nq1,
                                  _p(k["V"]), _p(k["B"]), prob.natoms, prob.nbeta,
                                  _p(k["pair_ptr"]), _p(k["pair_cell"]), _p(k["phi"]), _p(k["delta"]))
        self.M = prob.nnodes
        self.ndof = 2 * self.M

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    # tables -----------------------------------------------------------
    def mass_diag(self):
        D = np.zeros(self.M)
        lib().orc_mass_diag(self.h, _p(D))
        return D

    def tables(self):
        n = (self.prob.degree + 1) ** 3
        nq = self.prob.nq
        Nq = np.zeros((nq, n)); dNq = np.zeros((nq, n, 3)); wJ = np.zeros(nq)
        lib().orc_tables(self.h, _p(Nq), _p(dNq), _p(wJ))
        return Nq, dNq, wJ

    # operators --------------------------------------------------------
    def apply_H(self, X, flags=ALL):
        X = _c(X, np.complex128)
        rows, ld = X.shape
        assert rows == self.ndof
        Y = np.zeros_like(X)
        lib().orc_apply_H(self.h, _p(X), ld, ld, _p(Y), ld, flags)
        return Y

    def apply_M(self, X):
        X = _c(X, np.complex128)
        rows, ld = X.shape
        Y = np.zeros_like(X)
        lib().orc_apply_M(self.h, _p(X), ld, ld, _p(Y), ld)
        return Y

    def apply_H_sampled(self, X, nodes, cols):
        X = _c(X, np.complex128)
        nodes = _c(nodes, np.int64); cols = _c(cols, np.int64)
        out = np.zeros((nodes.size, 2, cols.size), np.complex128)
        lib().orc_apply_H_sampled(self.h, _p(X), X.shape[1], _p(nodes), nodes.size,
                                  _p(cols), cols.size, _p(out))
        return out

    def adjoint_fields(self, X, G):
        X = _c(X, np.complex128); G = _c(G, np.complex128)
        p = self.prob
        dV = np.zeros((p.ncells, p.nq)); dB = np.zeros((p.ncells, p.nq, 3))
        lib().orc_adjoint_fields(self.h, _p(X), _p(G), X.shape[1], X.shape[1], _p(dV), _p(dB))
        return dV, dB

    def dense(self, flags=ALL):
        N = self.ndof
        H = np.zeros((N, N), np.complex128); M = np.zeros((N, N), np.complex128)
        lib().orc_dense(self.h, _p(H), _p(M), flags)
        return H, M

    # subspace steps ---------------------------------------------------
    def orthonormalize(self, Y, HY, MY):
        Y = _c(Y, np.complex128).copy(); HY = _c(HY, np.complex128).copy(); MY = _c(MY, np.complex128).copy()
        if lib().orc_orthonormalize(self.h, _p(Y), _p(HY), _p(MY), Y.shape[1], Y.shape[1]):
            raise np.linalg.LinAlgError("Cholesky-QR breakdown")
        return Y, HY, MY

    def rayleigh_ritz(self, Y, HY, MY):
        Y = _c(Y, np.complex128).copy(); HY = _c(HY, np.complex128).copy(); MY = _c(MY, np.complex128).copy()
        k = Y.shape[1]
        ritz = np.zeros(k)
        lib().orc_rayleigh_ritz(self.h, _p(Y), _p(HY), _p(MY), k, k, _p(ritz))
        return Y, HY, MY, ritz

    def filter(self, degree, bounds, X, ritz, R, exactM=False):
        X = _c(X, np.complex128); R = _c(R, np.complex128)
        ritz = _c(ritz, np.float64); bounds = _c(bounds, np.float64)
        Y = np.zeros_like(X)
        rc = lib().orc_filter(self.h, degree, _p(bounds), _p(X), _p(ritz), _p(R), X.shape[1],
                              X.shape[1], _p(Y), int(exactM))
        if rc:
            raise RuntimeError("filter failed")
        return Y

    def filter_sampled(self, degree, bounds, X, ritz, R, nodes):
        """The R-ChFSI filter (eq. rChFSIrecurrence with D^-1, recovery of
        Algorithm RChFSI) at sampled nodes only: Y_q = D^-1 Z_q + X Lambda_q
        on rows (2 node, 2 node + 1) of each node, as [node][spin][column].
        Z_0 = 0, Z_1 = s_1 R / e; the products H D^-1 Z_k of steps
        k < q - 1 are full ones, the last one (step q - 1) is evaluated at
        the sampled nodes only, so a large mesh costs q - 2 full products
        (the filter acts column by column: pass only the columns wanted)."""
        X = _c(X, np.complex128); R = _c(R, np.complex128)
        ritz = _c(ritz, np.float64); nodes = _c(nodes, np.int64)
        lmin, lT, lmax = (float(b) for b in bounds)
        c, e = 0.5 * (lmax + lT), 0.5 * (lmax - lT)
        s1 = e / (lmin - c)
        D = np.repeat(self.mass_diag(), 2)[:, None]          # one value per spinor row
        rows = np.stack([2 * nodes, 2 * nodes + 1], axis=1)  # [node][spin]

        Lkm, Lk = np.ones_like(ritz), s1 * (ritz - c) / e   # C_0, C_1 at the Ritz values
        Zkm, Zk = np.zeros_like(R), s1 * R / e
        sk = s1
        for step in range(1, degree):
            sn = 1.0 / (2.0 / s1 - sk)
            a = 2.0 * sn / e
            if step < degree - 1:
                HW = self.apply_H(Zk / D)
                Zn = a * (HW - c * Zk) - sk * sn * Zkm + a * R * Lk[None, :]
            else:
                HW = self.apply_H_sampled(Zk / D, nodes, np.arange(X.shape[1]))
                Zn = (a * (HW - c * Zk[rows]) - sk * sn * Zkm[rows] + a * R[rows] * Lk[None, None, :])
            Lkm, Lk = Lk, a * (ritz - c) * Lk - sk * sn * Lkm
            Zkm, Zk = Zk, Zn
            sk = sn
        if degree == 1:
            Zk = Zk[rows]
        return Zk / D[rows] + X[rows] * Lk[None, None, :]

    def chebyshev_plain(self, degree, bounds, X, exactM=False):
        X = _c(X, np.complex128); bounds = _c(bounds, np.float64)
        Y = np.zeros_like(X)
        rc = lib().orc_chebyshev_plain(self.h, degree, _p(bounds), _p(X), X.shape[1], X.shape[1],
                                       _p(Y), int(exactM))
        if rc:
            raise RuntimeError("filter failed")
        return Y

    def lanczos(self, ksteps, v0):
        v0 = _c(v0, np.complex128).ravel()
        assert v0.size == self.ndof
        return lib().orc_lanczos(self.h, ksteps, _p(v0))

    def chfsi(self, X0, n_wanted, degree, lmax, tol=1e-8, max_iter=100, variant=0):
        """variant 0: R-ChFSI; 1: ChFSI with D^-1; 2: ChFSI with exact M^-1."""
        X = _c(X0, np.complex128).copy()
        k = X.shape[1]
        ritz = np.zeros(k)
        hres = np.zeros(max_iter + 1)
        hritz = np.zeros((max_iter + 1, k))
        it = lib().orc_chfsi(self.h, variant, k, n_wanted, degree, float(lmax), float(tol), max_iter,
                             _p(X), k, _p(ritz), _p(hres), _p(hritz))
        if it < 0:
            raise RuntimeError("R-ChFSI breakdown")
        return dict(X=X, ritz=ritz, iters=it, hist_res=hres[:it + 1], hist_ritz=hritz[:it + 1])
