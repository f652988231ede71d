"""Pins of the oracle's eigensolver pieces: dense algebra against library
routines, the Chebyshev identities of the residual recurrence (eq.
rChFSIrecurrence vs eq. ChFSIrecurrence), and Algorithm RChFSI against a
dense generalized eigensolve on tiny meshes."""
import math

import numpy as np
import pytest
import scipy.linalg as sl

from paper_2605_30128_amd import synth


def _tiny(**kw):
    base = dict(ncell=(2, 2, 2), box=(4.0, 4.0, 4.0), degree=2, nwells=2, natoms=2, nbeta=4, seed=11)
    base.update(kw)
    return synth.make_problem(**base)


def _herm(n, seed):
    g = np.random.default_rng(seed)
    A = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    return A + A.conj().T


def test_jacobi_matches_library(oracle_lib):
    for n, seed in ((1, 1), (2, 2), (7, 3), (40, 4)):
        A = _herm(n, seed)
        w, V = oracle_lib.jacobi(A)
        assert np.allclose(w, np.linalg.eigvalsh(A), atol=1e-12 * max(1, np.abs(A).max()))
        assert np.abs(V.conj().T @ V - np.eye(n)).max() < 1e-13
        assert np.abs(A @ V - V * w).max() < 1e-12 * max(1, np.abs(A).max())
    # degenerate spectrum (Kramers-like pairs)
    Q, _ = np.linalg.qr(np.random.default_rng(7).standard_normal((6, 6)) + 0j)
    A = Q @ np.diag([1, 1, 2, 2, 5, 5.0]) @ Q.conj().T
    w, _ = oracle_lib.jacobi(A)
    assert np.allclose(w, [1, 1, 2, 2, 5, 5], atol=1e-13)


def test_cholesky_matches_library(oracle_lib):
    A = _herm(12, 8) + 30 * np.eye(12)
    L = oracle_lib.cholesky(A)
    assert np.allclose(L, np.linalg.cholesky(A), atol=1e-13)
    with pytest.raises(np.linalg.LinAlgError):
        oracle_lib.cholesky(-np.eye(3) + 0j)


def test_dense_geig_matches_library(oracle_lib):
    H = _herm(30, 9)
    g = np.random.default_rng(10).standard_normal((30, 30))
    M = g @ g.T + 30 * np.eye(30)
    w, V = oracle_lib.dense_geig(H, M)
    assert np.allclose(w, sl.eigh(H, M, eigvals_only=True), atol=1e-12)
    assert np.abs(V.conj().T @ M @ V - np.eye(30)).max() < 1e-12


def _cq(x, q, lmin, lT, lmax):
    """C_q(x) = T_q((x-c)/e) / T_q((lmin-c)/e) via numpy's Chebyshev series."""
    c, e = 0.5 * (lmax + lT), 0.5 * (lmax - lT)
    T = np.polynomial.chebyshev.Chebyshev.basis(q)
    return T((x - c) / e) / T((lmin - c) / e)


def test_filter_identities_exact_eigenpairs(oracle_lib):
    p = _tiny()
    o = oracle_lib.Oracle(p)
    H, M = o.dense()
    w, V = oracle_lib.dense_geig(H, M)
    k = 4
    X = V[:, :k].copy()
    ritz = w[:k].copy()
    R, norms = oracle_lib.residual(H @ X, M @ X, ritz)
    assert norms.max() < 1e-10
    R[:] = 0  # exact eigenpairs: R = 0
    lmax = w[-1] * 1.01
    bounds = [w[0], w[20], lmax]
    q = 12
    Y = o.filter(q, bounds, X, ritz, R)
    cq = _cq(ritz, q, *bounds)
    assert np.abs(Y - X * cq).max() < 1e-13 * np.abs(X).max() * max(1, np.abs(cq).max())
    # C_q(lmin) = 1: the first column is unchanged
    assert abs(cq[0] - 1) < 1e-14
    assert np.abs(Y[:, 0] - X[:, 0]).max() < 1e-13 * np.abs(X[:, 0]).max()


def test_rchfsi_with_exact_mass_equals_chfsi(oracle_lib):
    """With D = M the residual recurrence reproduces plain ChFSI on M^-1 H,
    for any block and Ritz values."""
    p = _tiny()
    o = oracle_lib.Oracle(p)
    X = synth.random_block(p.ndof, 5, 61)
    ritz = np.array([-0.5, -0.2, 0.1, 0.3, 0.6])
    HX = o.apply_H(X); MX = o.apply_M(X)
    R = HX - MX * ritz
    bounds = [-0.6, 1.0, 60.0]
    q = 9
    Yr = o.filter(q, bounds, X, ritz, R, exactM=True)
    Yc = o.chebyshev_plain(q, bounds, X, exactM=True)
    assert np.abs(Yr - Yc).max() <= 1e-12 * np.abs(Yc).max()
    # with the diagonal D it is a different (approximate) filter
    Yd = o.filter(q, bounds, X, ritz, R, exactM=False)
    assert np.abs(Yd - Yc).max() > 1e-6 * np.abs(Yc).max()


@pytest.mark.parametrize("q", [1, 2, 3, 5])
def test_filter_sampled_matches_full_filter(oracle_lib, q):
    """The sampled filter (a Python restatement of the recurrence whose last
    product is evaluated at sampled nodes only) agrees with the C filter on
    those nodes, on a random block with a random residual (two independent
    codings of eq. rChFSIrecurrence and the recovery).  A sign or index slip
    in either (a dropped Z_{k-1} term, R Lambda_k taken at the wrong step,
    D in place of D^-1) shows up at q >= 3."""
    p = _tiny(degree=3, ncell=(2, 2, 2))
    o = oracle_lib.Oracle(p)
    X = synth.random_block(p.ndof, 6, 71)
    R = synth.random_block(p.ndof, 6, 72)
    ritz = np.array([-0.4, -0.1, 0.2, 0.5, 0.9, 1.4])
    bounds = [-0.5, 1.5, 80.0]
    nodes = np.array([0, 1, 7, 30, p.nnodes // 2, p.nnodes - 1])
    full = o.filter(q, bounds, X, ritz, R)
    ref = np.stack([full[2 * nodes], full[2 * nodes + 1]], axis=1)
    got = o.filter_sampled(q, bounds, X, ritz, R, nodes)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # the residual terms matter: without R the result is X C_q(Lambda) alone
    zero = o.filter_sampled(q, bounds, X, ritz, np.zeros_like(R), nodes)
    assert np.abs(zero - ref).max() > 1e-3 * np.abs(ref).max()
    assert np.abs(zero - np.stack([X[2 * nodes], X[2 * nodes + 1]], axis=1) * _cq(ritz, q, *bounds)).max() \
        <= 1e-12 * np.abs(zero).max()


def test_lanczos_upper_bound(oracle_lib):
    p = _tiny(degree=3)
    o = oracle_lib.Oracle(p)
    H, _ = o.dense()
    D = np.repeat(o.mass_diag(), 2)
    A = H / np.sqrt(D)[:, None] / np.sqrt(D)[None, :]
    lam = np.linalg.eigvalsh(A).max()
    est = o.lanczos(20, synth.random_block(p.ndof, 1, 71)[:, 0])
    assert est >= lam * (1 - 1e-9)
    assert est <= lam * 1.2


def test_orthonormalize_and_rr(oracle_lib):
    p = _tiny()
    o = oracle_lib.Oracle(p)
    Y = synth.random_block(p.ndof, 10, 81)
    Y[:, 3] *= 1e6  # badly scaled column
    HY, MY = o.apply_H(Y), o.apply_M(Y)
    Q, HQ, MQ = o.orthonormalize(Y, HY, MY)
    assert np.abs(Q.conj().T @ o.apply_M(Q) - np.eye(10)).max() < 1e-13
    assert np.abs(HQ - o.apply_H(Q)).max() < 1e-12 * np.abs(HQ).max()
    X, HX, MX, ritz = o.rayleigh_ritz(Q, HQ, MQ)
    assert np.all(np.diff(ritz) >= 0)
    assert np.abs(X.conj().T @ HX - np.diag(ritz)).max() < 1e-11 * np.abs(ritz).max()
    # Ritz values interlace above the true eigenvalues (Cauchy / min-max)
    H, M = o.dense()
    w = sl.eigh(H, M.real, eigvals_only=True)
    assert np.all(ritz >= w[:10] - 1e-10)


@pytest.mark.parametrize("deg,nsub,nw", [(2, 16, 12), (3, 24, 20)])
def test_rchfsi_matches_dense(oracle_lib, deg, nsub, nw):
    p = _tiny(degree=deg, nbeta=8)
    o = oracle_lib.Oracle(p)
    H, M = o.dense()
    w, _ = oracle_lib.dense_geig(H, M)
    lmax = o.lanczos(20, synth.random_block(p.ndof, 1, 91)[:, 0])
    X0 = synth.random_block(p.ndof, nsub, 92)
    out = o.chfsi(X0, nw, degree=12, lmax=lmax, tol=1e-10, max_iter=200)
    assert out["hist_res"][-1] < 1e-10
    assert np.abs(out["ritz"][:nw] - w[:nw]).max() < 1e-10
    # the residual falls over the iterations
    assert out["hist_res"][-1] < 1e-6 * out["hist_res"][0]
