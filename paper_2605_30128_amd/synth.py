"""Seeded synthetic inputs for the R-ChFSI eigenproblem.

This module only *draws* inputs: fields sampled at the quadrature points of a
uniform periodic hexahedral mesh, atom positions, spin-orbit projector samples
and their coupling matrices, random start blocks and cotangents.  It performs
none of the method's arithmetic (no basis functions, no integrals, no operator
products), so that the CPU oracle and the GPU path can both consume it without
sharing any code of the method.

Conventions (shared by every consumer; they are data layout, not arithmetic):

* Cells ``e = ex + ncx*(ey + ncy*ez)``; cell ``e`` spans ``[ex*hx, (ex+1)*hx]``
  and likewise in y, z.  The box is periodic with side ``L_d = ncell_d*h_d``.
* Quadrature point ``q = a + n1q*(b + n1q*c)``; its reference coordinate is
  the a-th ascending Gauss-Legendre abscissa on [-1, 1] (NumPy ``leggauss``)
  in x, b-th in y, c-th in z.  Physical position ``ex*hx + (xi_a+1)*hx/2``.
* ``V[e, q]`` (Ha), ``B[e, q, 0:3]`` (Ha, Cartesian x,y,z).
* Projectors: atom ``a`` has ``nbeta`` complex two-component functions
  ``beta_j(r) = g_l(|r|) * Omega_{l,j,m}(r_hat)`` (spinor spherical harmonics,
  s_{1/2}, p_{1/2}, then p_{3/2}), sampled at the quadrature points of every
  cell in its support: ``phi[pair, q, spin, j]``.  Pairs are stored
  atom-major in CSR form (``pair_ptr`` over atoms, ``pair_cell``).
  ``delta[a]`` is the Hermitian coupling matrix (here real diagonal by
  (l, j) channel), so that the nonlocal operator is sum_a P_a Delta_a P_a^H.

Workload recipes follow the paper's setting (complex spinors, FE degree up to
7, SOC projectors per atom): Gaussian wells of width 0.8 bohr and depth
U[1,3] Ha, a B field of magnitude U[0,0.1] Ha with a smooth random direction,
projector radial functions r^l exp(-r^2/(2*0.6^2)) cut at 3.6 bohr.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

WELL_WIDTH = 0.8
PROJ_WIDTH = 0.6
PROJ_CUTOFF = 3.6


@dataclass
class Problem:
    ncell: tuple
    h: tuple
    degree: int
    nq1: int
    V: np.ndarray            # float64 [ncells, nq]
    B: np.ndarray            # float64 [ncells, nq, 3]
    atoms: np.ndarray        # float64 [natoms, 3]
    nbeta: int
    pair_ptr: np.ndarray     # int64 [natoms+1]
    pair_cell: np.ndarray    # int64 [npairs]
    phi: np.ndarray          # complex128 [npairs, nq, 2, nbeta]
    delta: np.ndarray        # complex128 [natoms, nbeta, nbeta]
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def ncells(self) -> int:
        return int(np.prod(self.ncell))

    @property
    def nq(self) -> int:
        return self.nq1 ** 3

    @property
    def nnodes(self) -> int:
        return int(np.prod([c * self.degree for c in self.ncell]))

    @property
    def ndof(self) -> int:
        return 2 * self.nnodes

    @property
    def natoms(self) -> int:
        return int(self.atoms.shape[0])

    @property
    def npairs(self) -> int:
        return int(self.pair_cell.shape[0])

    @property
    def box(self) -> np.ndarray:
        return np.array([c * hh for c, hh in zip(self.ncell, self.h)])


# ----------------------------------------------------------------------------
# sample positions
# ----------------------------------------------------------------------------

def quad_abscissae(nq1: int) -> np.ndarray:
    """Ascending Gauss-Legendre abscissae on [-1,1] from NumPy (sample sites)."""
    x, _ = np.polynomial.legendre.leggauss(nq1)
    return np.sort(x)


def gll_abscissae(p: int) -> np.ndarray:
    """Ascending Gauss-Lobatto-Legendre nodes on [-1,1] (the FE nodes of a
    cell, +-1 and the roots of P_p') from NumPy (sample sites)."""
    inner = np.polynomial.legendre.Legendre.basis(p).deriv().roots() if p > 1 else np.zeros(0)
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


def node_coords(ncell, h, p: int) -> np.ndarray:
    """Physical coordinates [M][3] of the global nodes g = gx + Nx (gy + Ny gz)
    of the periodic mesh (node gx lies in cell gx // p at GLL node gx % p)."""
    xi = gll_abscissae(p)
    axes = []
    for d in range(3):
        g = np.arange(int(ncell[d]) * p)
        axes.append((g // p) * h[d] + 0.5 * (xi[g % p] + 1.0) * h[d])
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def neutral_charge(X: np.ndarray, box, ncentres: int, seed: int, charge=4.0, width=WELL_WIDTH) -> np.ndarray:
    """A neutral charge density sampled at the points X: `ncentres` normalised
    Gaussians of `charge` electrons each (random centres, minimum image) minus
    the uniform background of the same total charge."""
    box = np.asarray(box, float)
    centres = np.random.default_rng([seed, 6]).uniform(0.0, 1.0, size=(ncentres, 3)) * box
    rho = np.zeros(X.shape[0])
    norm = charge / (2 * math.pi * width ** 2) ** 1.5
    for c in centres:
        d = min_image(X - c, box)
        rho += norm * np.exp(-(d * d).sum(axis=1) / (2 * width ** 2))
    return rho - ncentres * charge / float(np.prod(box))


def cell_quad_points(ncell, h, nq1, cells: Optional[np.ndarray] = None) -> np.ndarray:
    """Physical positions [len(cells), nq, 3] of the sample sites of the cells."""
    ncx, ncy, ncz = ncell
    if cells is None:
        cells = np.arange(ncx * ncy * ncz)
    cells = np.asarray(cells, dtype=np.int64)
    ex = cells % ncx
    ey = (cells // ncx) % ncy
    ez = cells // (ncx * ncy)
    xi = quad_abscissae(nq1)
    a = np.arange(nq1 ** 3) % nq1
    b = (np.arange(nq1 ** 3) // nq1) % nq1
    c = np.arange(nq1 ** 3) // (nq1 * nq1)
    out = np.empty((cells.size, nq1 ** 3, 3))
    out[:, :, 0] = ex[:, None] * h[0] + (xi[a][None, :] + 1.0) * 0.5 * h[0]
    out[:, :, 1] = ey[:, None] * h[1] + (xi[b][None, :] + 1.0) * 0.5 * h[1]
    out[:, :, 2] = ez[:, None] * h[2] + (xi[c][None, :] + 1.0) * 0.5 * h[2]
    return out


def min_image(d: np.ndarray, box: np.ndarray) -> np.ndarray:
    return d - box * np.round(d / box)


# ----------------------------------------------------------------------------
# fields
# ----------------------------------------------------------------------------

def well_potential(ncell, h, nq1: int, centres: np.ndarray, depths: np.ndarray, box: np.ndarray,
                   width: float = WELL_WIDTH) -> np.ndarray:
    """V[cell, site] = -sum_w d_w exp(-|r - c_w - L s|^2/(2 width^2)) over the
    periodic images L s of each well that lie within 10 widths of the site.
    Only the cells that can hold such a site are visited for each well (of
    the 27 nearest images, an image shifted along a direction whose half box
    exceeds 10 widths never comes that close and is skipped)."""
    ncell = tuple(int(c) for c in ncell)
    ncells = int(np.prod(ncell))
    V = np.zeros((ncells, nq1 ** 3))
    reach = 10.0 * width
    shifts = [np.array([i, j, k], float) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)]
    shifts = [s for s in shifts if all(s[d] == 0 or 0.5 * box[d] <= reach for d in range(3))]
    for c, d in zip(centres, depths):
        idx = []
        for k in range(3):
            lo = int(math.floor((c[k] - reach) / h[k]))
            hi = int(math.floor((c[k] + reach) / h[k]))
            idx.append(np.unique(np.mod(np.arange(lo, hi + 1), ncell[k])))
        cand = (idx[0][:, None, None] + ncell[0] * (idx[1][None, :, None] + ncell[1] * idx[2][None, None, :])).ravel()
        base = min_image(cell_quad_points(ncell, h, nq1, cand) - c, box)
        for s in shifts:
            r2 = np.sum((base + s * box) ** 2, axis=-1)
            e = np.where(r2 <= reach * reach, np.exp(-r2 / (2.0 * width * width)), 0.0)
            V[cand] -= d * e
    return V


def smooth_direction(pts: np.ndarray, box: np.ndarray, rng: np.random.Generator,
                     nmodes: int = 6) -> np.ndarray:
    """Unit vector field from a random sum of low Fourier modes (|m| <= 2)."""
    ms = []
    while len(ms) < nmodes:
        m = rng.integers(-1, 2, size=3)
        if np.any(m != 0) and np.sum(m * m) <= 4:
            ms.append(m)
    n = np.zeros(pts.shape)
    n += rng.normal(size=3) * 0.5
    for m in ms:
        k = 2.0 * np.pi * np.asarray(m) / box
        ph = pts @ k
        a = rng.normal(size=3)
        b = rng.normal(size=3)
        n += np.cos(ph)[..., None] * a + np.sin(ph)[..., None] * b
    nrm = np.linalg.norm(n, axis=-1, keepdims=True)
    nrm[nrm < 1e-12] = 1.0
    return n / nrm


# ----------------------------------------------------------------------------
# spin-orbit projectors (spinor spherical harmonics in the j-basis)
# ----------------------------------------------------------------------------

def _ylm(l: int, m: int, u: np.ndarray) -> np.ndarray:
    """Complex spherical harmonics Y_lm for l <= 1 at unit vectors u[..., 3]."""
    x, y, z = u[..., 0], u[..., 1], u[..., 2]
    if l == 0:
        return np.full(x.shape, 0.5 / math.sqrt(math.pi), dtype=complex)
    c = math.sqrt(3.0 / (4.0 * math.pi))
    if m == 0:
        return (c * z).astype(complex)
    if m == 1:
        return -c * (x + 1j * y) / math.sqrt(2.0)
    if m == -1:
        return c * (x - 1j * y) / math.sqrt(2.0)
    return np.zeros(x.shape, dtype=complex)


def _spinor_harmonic(l: int, j2: int, m2: int, u: np.ndarray) -> np.ndarray:
    """Omega_{l, j, m}(u) as [..., 2] complex (spin up, spin down).

    j2 = 2j, m2 = 2m (odd integers).  Standard Clebsch-Gordan coupling of
    Y_{l, m-1/2} chi_up and Y_{l, m+1/2} chi_down.
    """
    m = m2 / 2.0
    out = np.zeros(u.shape[:-1] + (2,), dtype=complex)
    mu = int(round(m - 0.5))
    md = int(round(m + 0.5))
    yu = _ylm(l, mu, u) if abs(mu) <= l else np.zeros(u.shape[:-1], complex)
    yd = _ylm(l, md, u) if abs(md) <= l else np.zeros(u.shape[:-1], complex)
    if j2 == 2 * l + 1:
        cu = math.sqrt((l + m + 0.5) / (2 * l + 1))
        cd = math.sqrt((l - m + 0.5) / (2 * l + 1))
    else:
        cu = -math.sqrt((l - m + 0.5) / (2 * l + 1))
        cd = math.sqrt((l + m + 0.5) / (2 * l + 1))
    out[..., 0] = cu * yu
    out[..., 1] = cd * yd
    return out


def projector_channels(nbeta: int):
    """(l, 2j, 2m) of each projector: s1/2 x2, p1/2 x2, then p3/2 x4."""
    ch = [(0, 1, -1), (0, 1, 1), (1, 1, -1), (1, 1, 1)]
    if nbeta == 8:
        ch += [(1, 3, -3), (1, 3, -1), (1, 3, 1), (1, 3, 3)]
    elif nbeta != 4:
        raise ValueError("nbeta must be 4 or 8")
    return ch


def _radial(l: int, r: np.ndarray, width=PROJ_WIDTH, rc=PROJ_CUTOFF) -> np.ndarray:
    norm = math.sqrt(2.0 / (math.gamma(l + 1.5) * width ** (2 * l + 3)))
    g = norm * r ** l * np.exp(-r * r / (2.0 * width * width))
    return np.where(r <= rc, g, 0.0)


def projector_samples(disp: np.ndarray, nbeta: int, spin_rot: Optional[np.ndarray] = None) -> np.ndarray:
    """beta_j at displacements disp[..., 3] -> complex [..., 2, nbeta]."""
    r = np.linalg.norm(disp, axis=-1)
    u = disp / np.where(r > 1e-14, r, 1.0)[..., None]
    u = np.where((r > 1e-14)[..., None], u, np.array([0.0, 0.0, 1.0]))
    out = np.zeros(disp.shape[:-1] + (2, nbeta), dtype=complex)
    for j, (l, j2, m2) in enumerate(projector_channels(nbeta)):
        out[..., :, j] = _radial(l, r)[..., None] * _spinor_harmonic(l, j2, m2, u)
    if spin_rot is not None:
        out = np.einsum("ab,...bj->...aj", spin_rot, out)
    return out


def su2_from_rotation(axis, angle) -> np.ndarray:
    """SU(2) matrix exp(-i angle/2 n.sigma) of the rotation by `angle` about `axis`."""
    n = np.asarray(axis, float)
    n = n / np.linalg.norm(n)
    c, s = math.cos(angle / 2), math.sin(angle / 2)
    return np.array([[c - 1j * s * n[2], -1j * s * n[0] - s * n[1]],
                     [-1j * s * n[0] + s * n[1], c + 1j * s * n[2]]])


def rotation_matrix(axis, angle) -> np.ndarray:
    n = np.asarray(axis, float)
    n = n / np.linalg.norm(n)
    K = np.array([[0, -n[2], n[1]], [n[2], 0, -n[0]], [-n[1], n[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * K @ K


# ----------------------------------------------------------------------------
# problem assembly
# ----------------------------------------------------------------------------

def make_problem(ncell=(4, 4, 4), box=(8.0, 8.0, 8.0), degree=4, nq1=None,
                 nwells=4, natoms=None, nbeta=4, seed=1000,
                 bfield="random", bmag=0.1, b_const=None, v_const=None,
                 soc=True, spin_rot_axis=None, spin_rot_angle=0.0) -> Problem:
    """Draw one synthetic problem.

    bfield: "random" (|B| ~ U[0,bmag] per point, smooth random direction),
            "zero", or "const" (B = b_const everywhere).
    v_const: if given, V is this constant instead of Gaussian wells.
    soc: include projectors (atoms at the first `natoms` well centres).
    spin_rot_axis/angle: rotate B by R and the projector spinors by U(R).
    """
    ncell = tuple(int(c) for c in ncell)
    box = np.asarray(box, float)
    h = tuple(float(b / c) for b, c in zip(box, ncell))
    nq1 = degree + 1 if nq1 is None else int(nq1)
    natoms = nwells if natoms is None else int(natoms)
    rng = np.random.default_rng(seed)
    r_wells = np.random.default_rng([seed, 1])
    r_bdir = np.random.default_rng([seed, 2])
    r_bmag = np.random.default_rng([seed, 3])
    r_proj = np.random.default_rng([seed, 4])

    ncells = int(np.prod(ncell))
    nq = nq1 ** 3
    centres = r_wells.uniform(0.0, 1.0, size=(max(nwells, natoms), 3)) * box
    depths = r_wells.uniform(1.0, 3.0, size=max(nwells, natoms))

    if v_const is not None:
        V = np.full((ncells, nq), float(v_const))
    else:
        V = well_potential(ncell, h, nq1, centres[:nwells], depths[:nwells], box)
    B = np.zeros((ncells, nq, 3))
    chunk = max(1, 200000 // nq)
    dirs_seed = int(r_bdir.integers(0, 2**31))
    for c0 in range(0, ncells, chunk):
        cells = np.arange(c0, min(ncells, c0 + chunk))
        pts = cell_quad_points(ncell, h, nq1, cells)
        if bfield == "random":
            dirs = smooth_direction(pts, box, np.random.default_rng(dirs_seed))
            mag = np.random.default_rng([seed, 3, c0]).uniform(0.0, bmag, size=pts.shape[:-1])
            B[cells] = dirs * mag[..., None]
        elif bfield == "const":
            B[cells] = np.asarray(b_const, float)
        elif bfield != "zero":
            raise ValueError(bfield)
    Rm = None
    U = None
    if spin_rot_axis is not None:
        Rm = rotation_matrix(spin_rot_axis, spin_rot_angle)
        U = su2_from_rotation(spin_rot_axis, spin_rot_angle)
        B = B @ Rm.T

    atoms = centres[:natoms].copy() if soc else np.zeros((0, 3))
    pair_ptr = [0]
    pair_cell = []
    phis = []
    deltas = []
    if soc:
        ncx, ncy, ncz = ncell
        reach = PROJ_CUTOFF + 1e-9
        for a in range(natoms):
            R = atoms[a]
            rng_cells = []
            for d in range(3):
                lo = int(math.floor((R[d] - reach) / h[d]))
                hi = int(math.floor((R[d] + reach) / h[d]))
                idx = np.unique(np.mod(np.arange(lo, hi + 1), ncell[d]))
                rng_cells.append(idx)
            cand = (rng_cells[0][:, None, None] + ncx * (rng_cells[1][None, :, None]
                    + ncy * rng_cells[2][None, None, :])).ravel()
            cand = np.sort(cand)
            pts = cell_quad_points(ncell, h, nq1, cand)
            disp = min_image(pts - R, box)
            r = np.linalg.norm(disp, axis=-1)
            keep = np.any(r <= PROJ_CUTOFF, axis=1)
            cells_a = cand[keep]
            pair_cell.extend(cells_a.tolist())
            pair_ptr.append(len(pair_cell))
            phis.append(projector_samples(disp[keep], nbeta, U))
            # channel couplings D_{l,j}: s1/2, p1/2, p3/2 with a visible SO split
            Ds = r_proj.uniform(-1.0, 1.0)
            Dp12 = r_proj.uniform(-1.0, 1.0)
            while True:
                Dp32 = r_proj.uniform(-1.0, 1.0)
                if abs(Dp32 - Dp12) >= 0.1:
                    break
            diag = [Ds, Ds, Dp12, Dp12] + ([Dp32] * 4 if nbeta == 8 else [])
            deltas.append(np.diag(np.asarray(diag, complex)))
        phi = np.concatenate(phis, axis=0) if phis else np.zeros((0, nq, 2, nbeta), complex)
        delta = np.stack(deltas)
    else:
        phi = np.zeros((0, nq, 2, nbeta), complex)
        delta = np.zeros((0, nbeta, nbeta), complex)
        pair_ptr = [0]
    return Problem(ncell=ncell, h=h, degree=int(degree), nq1=nq1, V=V, B=B,
                   atoms=atoms, nbeta=int(nbeta),
                   pair_ptr=np.asarray(pair_ptr, np.int64),
                   pair_cell=np.asarray(pair_cell, np.int64),
                   phi=np.ascontiguousarray(phi), delta=np.ascontiguousarray(delta),
                   seed=seed,
                   meta=dict(centres=centres, depths=depths, rotation=Rm, su2=U))


def random_block(nrows: int, ncols: int, seed: int, ld: Optional[int] = None) -> np.ndarray:
    """Complex normal block [nrows, ld] (columns >= ncols are zero)."""
    ld = ncols if ld is None else ld
    g = np.random.default_rng([seed, 7])
    out = np.zeros((nrows, ld), complex)
    out[:, :ncols] = (g.standard_normal((nrows, ncols)) + 1j * g.standard_normal((nrows, ncols))) / math.sqrt(2.0)
    return out


def device_block(nrows: int, ncols: int, seed: int, dtype=None, device="cuda", chunk_rows: int = 1 << 20):
    """Complex normal block [nrows, ncols] drawn on the device with torch's
    seeded generator (real and imaginary parts of variance 1/2, like
    random_block), in row chunks so that no temporary exceeds one chunk.
    For blocks too large to draw on the host (the slab's 256 columns are
    69 GB in complex128)."""
    import torch
    dtype = torch.complex128 if dtype is None else dtype
    g = torch.Generator(device=device).manual_seed(int(seed))
    out = torch.empty((nrows, ncols), dtype=dtype, device=device)
    for r0 in range(0, nrows, chunk_rows):
        r1 = min(nrows, r0 + chunk_rows)
        out[r0:r1] = torch.randn((r1 - r0, ncols), generator=g, dtype=torch.complex128, device=device).to(dtype)
    return out


def random_real(shape, seed: int) -> np.ndarray:
    return np.random.default_rng([seed, 9]).standard_normal(shape)


# Workloads of the paper's shape (Hartree atomic units).
CONFIGS = {
    "tiny": dict(ncell=(4, 4, 4), box=(8.0, 8.0, 8.0), degree=4, nwells=4, natoms=4, nbeta=4,
                 seed=1000, n_wanted=32, nsub=40, cheb_degree=20, iters=10, nvec_hx=32),
    "medium": dict(ncell=(16, 16, 16), box=(24.0, 24.0, 24.0), degree=6, nwells=64, natoms=64,
                   nbeta=8, seed=1001, n_wanted=512, nsub=576, cheb_degree=30, iters=None,
                   nvec_hx=512),
    "slab": dict(ncell=(32, 32, 24), box=(48.0, 48.0, 36.0), degree=7, nwells=256, natoms=256,
                 nbeta=8, seed=1004, n_wanted=2048, nsub=2304, cheb_degree=40, iters=None,
                 nvec_hx=256),
}


def make_config(name: str, **over) -> Problem:
    cfg = dict(CONFIGS[name])
    for k in ("n_wanted", "nsub", "cheb_degree", "iters", "nvec_hx"):
        cfg.pop(k)
    cfg.update(over)
    return make_problem(**cfg)
