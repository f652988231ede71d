"""CPU oracle of the Poisson solve (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the CPU baseline leg of the benchmark may
import this module; the product path never does.  It shares no code with the
GPU library: the basis tables come from the C oracle (oracle.Oracle.tables,
pinned by the basis tests), everything else is written here from the paper.

* K (Sec. III-A, the discrete Laplacian of K V_el = f): the stiffness matrix
  K_IJ = sum_e int_e grad N_I . grad N_J, applied cell by cell straight from
  the quadrature of the bilinear form -- per cell the physical gradients at
  every Gauss point G_e = dN x_e, then K_e x_e = G^T (w |J|) G x_e -- and
  assembled by summing into the global nodes.  No sum factorisation.
* diag(K): the same quadrature of |grad N_I|^2, summed over the cells of I.
* Chebyshev-Jacobi preconditioner (Sec. III-B1; Sec. III-C1, preconditioner paragraph):
  P^{-1} = chi(D^{-1} K) D^{-1}, D = diag(K), chi of degree m approximating
  1/lambda on [lmin, lmax], applied as m steps of the Chebyshev iteration for
  D^{-1} K z = D^{-1} r from z = 0 (Saad, Iterative Methods for Sparse
  Linear Systems, Chebyshev acceleration).
* Spectral bound: Lanczos on D^{-1/2} K D^{-1/2}, theta_max + |beta_k|, from
  the splitmix64 start vector (Steele, Lea and Flood 2014).
* PCG: Algorithm pcg_fusion (Sec. III-C1) in its order (w = K p, eta, alpha, the x and r
  update, z = P^{-1} r, delta_new and gamma, beta, the new p, the test
  sqrt(gamma) < tol), on f' = f - mean(f), returning the zero-mean solution.

Readings where the paper leaves a choice (each also in the design notes):
the preconditioner degree m counts Chebyshev steps (m - 1 products with K,
matching the paper's m - 1 extra ghost exchanges); lmin = lmax / range; the
Lanczos bound is the same theta_max + |beta_k| used for the eigensolver's
filter; the periodic problem is solved on the range of K (mean of f
removed) and the solution is reported with zero mean.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1


def cell_nodes(prob) -> np.ndarray:
    """Global node index of local node I = i + n1 (j + n1 k) of every cell, [ncells][n]."""
    p = prob.degree
    n1 = p + 1
    ncx, ncy, ncz = prob.ncell
    Nx, Ny, Nz = ncx * p, ncy * p, ncz * p
    e = np.arange(ncx * ncy * ncz)
    ex, ey, ez = e % ncx, (e // ncx) % ncy, e // (ncx * ncy)
    I = np.arange(n1 ** 3)
    i, j, k = I % n1, (I // n1) % n1, I // (n1 * n1)
    gx = (ex[:, None] * p + i[None, :]) % Nx
    gy = (ey[:, None] * p + j[None, :]) % Ny
    gz = (ez[:, None] * p + k[None, :]) % Nz
    return gx + Nx * (gy + Ny * gz)


class Stiffness:
    """K of one mesh, from the C oracle's basis tables at the Gauss points."""

    def __init__(self, orc):
        self.prob = orc.prob
        self.M = orc.M
        _, dNq, wJ = orc.tables()          # dNq[q][I][d] physical gradients, wJ[q] = w_q |J|
        nq, n, _ = dNq.shape
        self.G = np.ascontiguousarray(dNq.transpose(1, 0, 2).reshape(n, nq * 3))  # [I][(q, d)]
        self.w = np.repeat(wJ, 3)           # weight of entry (q, d)
        self.gidx = cell_nodes(self.prob)

    def apply(self, x: np.ndarray) -> np.ndarray:
        """y = K x (x real, length M)."""
        xe = x[self.gidx]                   # [ncells][n]
        grad = xe @ self.G                  # grad u at every Gauss point, [ncells][(q, d)]
        ye = (grad * self.w) @ self.G.T     # int grad N_I . grad u
        return np.bincount(self.gidx.ravel(), weights=ye.ravel(), minlength=self.M)

    def diag(self) -> np.ndarray:
        """diag(K)_I = sum over the cells of I of int |grad N_I|^2."""
        de = (self.G * self.G) @ self.w     # [n], the same for every cell of a uniform mesh
        return np.bincount(self.gidx.ravel(), weights=np.tile(de, self.gidx.shape[0]), minlength=self.M)

    def dense(self) -> np.ndarray:
        """Assembled K (tiny meshes only)."""
        Ke = (self.G * self.w) @ self.G.T
        K = np.zeros((self.M, self.M))
        for g in self.gidx:
            K[np.ix_(g, g)] += Ke
        return K


def splitmix(n: int, seed: int = 0) -> np.ndarray:
    """splitmix64 of the states seed + (i + 1) 0x9E3779B97F4A7C15, i < n, as
    uniform doubles (top 53 bits) in [-0.5, 0.5)."""
    out = np.empty(n)
    for i in range(n):
        z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & MASK64
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        z ^= z >> 31
        out[i] = (z >> 11) * 2.0 ** -53 - 0.5
    return out


def chebyshev_precond(K: Stiffness, r: np.ndarray, degree: int, lmin: float, lmax: float,
                      dinv: np.ndarray = None) -> np.ndarray:
    """z = chi(D^{-1} K) D^{-1} r: `degree` steps of the Chebyshev iteration
    for D^{-1} K z = D^{-1} r on [lmin, lmax] from z = 0."""
    dinv = 1.0 / K.diag() if dinv is None else dinv
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    z = np.zeros_like(r)
    res = dinv * r                      # residual of D^{-1} K z = D^{-1} r at z = 0
    d = res / theta
    for k in range(degree):
        z = z + d
        if k == degree - 1:
            break
        res = dinv * (r - K.apply(z))
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * res
        rho = rho_new
    return z


def lanczos_bound(K: Stiffness, steps: int, v0: np.ndarray = None, dinv: np.ndarray = None,
                  parts: bool = False):
    """theta_max + |beta_k| of `steps` Lanczos steps on D^{-1/2} K D^{-1/2}
    (with parts: the pair (theta_max, |beta_k|))."""
    dinv = 1.0 / K.diag() if dinv is None else dinv
    s = np.sqrt(dinv)
    v = splitmix(K.M) if v0 is None else np.array(v0, float)
    v = v / np.sqrt(v @ v)
    vprev = np.zeros_like(v)
    alpha, beta = [], [0.0]
    for j in range(steps):
        w = s * K.apply(s * v) - beta[j] * vprev
        a = v @ w
        alpha.append(a)
        w = w - a * v
        b = np.sqrt(w @ w)
        beta.append(b)
        if b == 0:
            break
        vprev, v = v, w / b
    m = len(alpha)
    T = np.diag(alpha) + np.diag(beta[1:m], 1) + np.diag(beta[1:m], -1)
    theta = float(np.linalg.eigvalsh(T)[-1])
    return (theta, abs(beta[m])) if parts else theta + abs(beta[m])


def pcg(K: Stiffness, f: np.ndarray, x0: np.ndarray, tol: float, max_iter: int, degree: int,
        lmin: float, lmax: float):
    """Algorithm pcg_fusion on K x = f - mean(f).  Returns (x with zero mean,
    iterations, converged, sqrt(gamma) per iteration)."""
    dinv = 1.0 / K.diag()
    fp = f - f.mean()
    x = np.array(x0, float)
    r = K.apply(x) - fp
    z = chebyshev_precond(K, r, degree, lmin, lmax, dinv)
    delta = r @ z
    gamma = r @ r
    p = -z
    hist = [np.sqrt(gamma)]
    it = 0
    conv = np.sqrt(gamma) < tol
    while not conv and it < max_iter:
        w = K.apply(p)
        eta = p @ w
        alpha = delta / eta
        x = x + alpha * p
        r = r + alpha * w
        z = chebyshev_precond(K, r, degree, lmin, lmax, dinv)
        delta_new, gamma = r @ z, r @ r
        beta = delta_new / delta
        delta = delta_new
        p = -z + beta * p
        it += 1
        hist.append(np.sqrt(gamma))
        conv = np.sqrt(gamma) < tol
    return x - x.mean(), it, conv, np.array(hist)
