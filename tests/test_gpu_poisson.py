"""GPU parity of the Poisson path (chfsi_apply_K, chfsi_poisson_precond,
chfsi_poisson_solve) with the CPU oracle: the sum-factorised K x against the
quadrature definition on meshes of every supported (degree, nq1) shape, the
Chebyshev-Jacobi preconditioner, the Lanczos bound, the PCG iterates and
solution, the periodic PDE with a Fourier solution, a full-size K x at the
largest one-GPU shape and a full-size solve on the medium mesh."""
import math

import numpy as np
import pytest

from paper_2605_30128_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    from paper_2605_30128_amd import binding
    binding.load()
    return binding


def _prob(ncell, box, degree, nq1=None):
    return synth.make_problem(ncell=ncell, box=box, degree=degree, nq1=nq1, nwells=1, natoms=0,
                              bfield="zero", soc=False, seed=7)


def _setup(B, prob, oracle_lib):
    from oracle import poisson
    o = oracle_lib.Oracle(prob)
    return B.Chfsi(prob, max_nvec=1), poisson.Stiffness(o), o


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()


SHAPES = [
    ((2, 2, 2), (3.0, 3.0, 3.0), 1, 2),
    ((2, 2, 2), (3.0, 3.0, 3.0), 1, 3),
    ((2, 4, 2), (3.0, 5.0, 4.0), 2, 3),
    ((2, 4, 2), (3.0, 5.0, 4.0), 2, 4),
    ((4, 2, 2), (6.0, 3.0, 4.0), 3, 4),
    ((2, 2, 4), (4.0, 4.0, 7.0), 3, 5),
    ((4, 4, 2), (6.0, 6.0, 3.0), 4, 5),
    ((2, 2, 2), (4.0, 4.0, 4.0), 4, 6),
    ((2, 4, 2), (3.0, 6.0, 3.0), 5, 6),
    ((2, 2, 2), (4.0, 4.0, 4.0), 5, 7),
    ((4, 2, 2), (8.0, 4.0, 4.0), 6, 7),
    ((2, 2, 2), (4.0, 4.0, 4.0), 6, 8),
    ((2, 2, 4), (3.0, 3.0, 6.0), 7, 8),
]


@pytest.mark.parametrize("ncell,box,degree,nq1", SHAPES)
def test_apply_K_parity(B, oracle_lib, ncell, box, degree, nq1):
    print(f"apply_K degree={degree} nq1={nq1} ncell={ncell}", flush=True)
    ctx, K, _ = _setup(B, _prob(ncell, box, degree, nq1), oracle_lib)
    x = np.random.default_rng(degree * 10 + nq1).standard_normal(K.M)
    ref = K.apply(x)
    got = ctx.apply_K(_dev(x)).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # constants are in the null space
    one = ctx.apply_K(torch.ones(K.M, dtype=torch.float64, device="cuda"))
    assert float(one.abs().max()) < 1e-12 * np.abs(ref).max()


def test_unsupported_quadrature_and_argument_errors(B, oracle_lib):
    for nq1 in (3, 7):  # degree 4 needs nq1 = 5 or 6
        ctx = B.Chfsi(_prob((2, 2, 2), (4.0, 4.0, 4.0), 4, nq1), max_nvec=1)
        x = torch.zeros(ctx.nnodes, dtype=torch.float64, device="cuda")
        with pytest.raises(B.ChfsiError):
            ctx.apply_K(x)
    ctx = B.Chfsi(_prob((2, 2, 2), (4.0, 4.0, 4.0), 3), max_nvec=1)
    x = torch.zeros(ctx.nnodes, dtype=torch.float64, device="cuda")
    with pytest.raises(B.ChfsiError):
        ctx.apply_K(x, x)  # y must not overlap x
    with pytest.raises(B.ChfsiError):
        ctx.poisson_precond(x, 0, 0.1, 2.0)
    with pytest.raises(B.ChfsiError):
        ctx.poisson_precond(x, 3, 2.0, 1.0)
    f = torch.ones_like(x)
    with pytest.raises(B.ChfsiError):
        ctx.poisson_solve(f, range_=1.0)
    with pytest.raises(B.ChfsiError):
        ctx.poisson_solve(f, cheb_degree=65)
    with pytest.raises(B.ChfsiError):
        ctx.poisson_solve(f, lambda_max=0.0, lanczos_steps=0)


@pytest.mark.parametrize("degree", [1, 3, 5])
def test_precond_parity(B, oracle_lib, degree):
    from oracle import poisson
    ctx, K, _ = _setup(B, _prob((4, 2, 2), (6.0, 3.0, 4.0), 4), oracle_lib)
    r = np.random.default_rng(degree).standard_normal(K.M)
    lmin, lmax = 0.08, 1.7
    ref = poisson.chebyshev_precond(K, r, degree, lmin, lmax)
    got = ctx.poisson_precond(_dev(r), degree, lmin, lmax).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def test_lanczos_bound_parity(B, oracle_lib):
    from oracle import poisson
    ctx, K, _ = _setup(B, _prob((4, 4, 4), (6.0, 6.0, 6.0), 3), oracle_lib)
    f = _dev(np.random.default_rng(1).standard_normal(K.M))
    _, rep, rc = ctx.poisson_solve(f, max_iter=0, lanczos_steps=20, range_=20.0)
    assert rc == B.NOT_CONVERGED and rep["iters"] == 0
    ref = poisson.lanczos_bound(K, 20)
    assert abs(rep["lambda_max"] - ref) <= 1e-9 * ref
    assert abs(rep["lambda_min"] - rep["lambda_max"] / 20.0) <= 1e-15 * ref


@pytest.mark.parametrize("cheb_degree,rng_", [(1, 20.0), (5, 20.0), (5, 300.0)])
def test_pcg_parity(B, oracle_lib, cheb_degree, rng_):
    """Same interval on both sides: the same iteration count (+-1) and the same
    solution within what the residual tolerance leaves open."""
    from oracle import poisson
    ctx, K, _ = _setup(B, _prob((4, 2, 4), (6.0, 3.0, 6.0), 4), oracle_lib)
    rng = np.random.default_rng(cheb_degree)
    f = rng.standard_normal(K.M) + 0.3
    lmax = poisson.lanczos_bound(K, 20)
    tol = 1e-10 * np.linalg.norm(f)
    xr, itr, convr, hist = poisson.pcg(K, f, np.zeros(K.M), tol, 2000, cheb_degree, lmax / rng_, lmax)
    assert convr
    x, rep, rc = ctx.poisson_solve(_dev(f), tol=tol, max_iter=2000, cheb_degree=cheb_degree, lambda_max=lmax,
                                   range_=rng_)
    assert rc == B.OK and rep["converged"] == 1
    assert abs(rep["iters"] - itr) <= 1
    x = x.cpu().numpy()
    assert abs(x.mean()) < 1e-12 * np.abs(x).max()
    assert np.abs(x - xr).max() <= 1e-7 * np.abs(xr).max()
    # the true residual of the returned solution
    res = K.apply(x) - (f - f.mean())
    assert np.linalg.norm(res) < 10 * tol
    # a warm start at the solution needs no iteration
    x2, rep2, rc2 = ctx.poisson_solve(_dev(f), x=_dev(xr), tol=tol * 100, cheb_degree=cheb_degree, lambda_max=lmax,
                                      range_=rng_)
    assert rc2 == B.OK and rep2["iters"] == 0


def test_periodic_pde_fourier_solution(B, oracle_lib):
    """-Lap u = g, g = |k|^2 cos(k . x): the GPU solve of K u = M g_h gives
    u = cos(k . x) at the nodes (p = 5), with the Lanczos interval."""
    from test_oracle_poisson import node_coords
    box = (6.0, 6.0, 8.0)
    prob = _prob((4, 4, 4), box, 5)
    ctx, K, o = _setup(B, prob, oracle_lib)
    X = node_coords(oracle_lib, prob)
    kv = np.array([2 * math.pi / box[0], 2 * math.pi / box[1], 0.0])
    u = np.cos(X @ kv)
    G = np.zeros((2 * K.M, 1), complex)
    G[0::2, 0] = (kv @ kv) * u
    f = o.apply_M(G)[0::2, 0].real
    x, rep, rc = ctx.poisson_solve(_dev(f), tol=1e-12, max_iter=2000, cheb_degree=5)
    assert rc == B.OK
    assert np.abs(x.cpu().numpy() - (u - u.mean())).max() < 1e-4


def test_apply_K_full_size_slab(B, oracle_lib):
    """K x at the largest one-GPU shape (32x32x24 cells, p = 7, 8.4M nodes),
    all entries against the oracle."""
    print("apply_K slab 32x32x24 p=7", flush=True)
    prob = _prob((32, 32, 24), (48.0, 48.0, 36.0), 7)
    ctx, K, _ = _setup(B, prob, oracle_lib)
    x = np.random.default_rng(3).standard_normal(K.M)
    ref = K.apply(x)
    got = ctx.apply_K(_dev(x)).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_solve_full_size_medium(B, oracle_lib):
    """PCG with a degree-5 Chebyshev-Jacobi preconditioner on the medium mesh
    (16^3 cells, p = 6, 884,736 nodes) for a neutral Gaussian charge; the
    returned solution's residual checked with the oracle's K."""
    print("solve medium 16^3 p=6", flush=True)
    from oracle import poisson
    from test_oracle_poisson import node_coords
    prob = _prob((16, 16, 16), (24.0, 24.0, 24.0), 6)
    ctx, K, o = _setup(B, prob, oracle_lib)
    X = node_coords(oracle_lib, prob)
    rho = synth_charge(X, np.array(prob.box))
    G = np.zeros((2 * K.M, 1), complex)
    G[0::2, 0] = 4 * math.pi * rho
    f = o.apply_M(G)[0::2, 0].real
    tol = 1e-10
    x, rep, rc = ctx.poisson_solve(_dev(f), tol=tol, max_iter=5000, cheb_degree=5)
    assert rc == B.OK, rep
    x = x.cpu().numpy()
    res = K.apply(x) - (f - f.mean())
    assert np.linalg.norm(res) < 10 * tol


def synth_charge(X, box):
    """A neutral charge density: eight Gaussian nuclei minus a uniform background."""
    rng = np.random.default_rng(11)
    centres = rng.uniform(0, 1, (8, 3)) * box
    rho = np.zeros(X.shape[0])
    for c in centres:
        d = X - c
        d -= box * np.round(d / box)
        rho += np.exp(-(d * d).sum(1) / (2 * 0.8 ** 2))
    return rho - rho.mean()


def test_pcg_failure_paths(B, oracle_lib):
    """A non-finite right-hand side is reported as CHFSI_E_NONFINITE; an upper
    bound far below the spectrum makes the preconditioner indefinite, which
    ends in a reported breakdown or in CHFSI_NOT_CONVERGED, never a hang."""
    ctx = B.Chfsi(_prob((2, 2, 2), (4.0, 4.0, 4.0), 3), max_nvec=1)
    f = torch.randn(ctx.nnodes, dtype=torch.float64, device="cuda", generator=torch.Generator(device="cuda").manual_seed(3))
    bad = f.clone()
    bad[5] = float("nan")
    with pytest.raises(B.ChfsiError) as ei:
        ctx.poisson_solve(bad, tol=1e-10, max_iter=50, cheb_degree=3)
    assert ei.value.code == B.E_NONFINITE
    try:
        _, rep, rc = ctx.poisson_solve(f, tol=1e-12, max_iter=200, cheb_degree=7, lambda_max=0.05)
        assert rc in (B.OK, B.NOT_CONVERGED)
        assert rep["iters"] <= 200
    except B.ChfsiError as e:
        assert e.code == B.E_NONFINITE
