"""GPU parity of the R-ChFSI stages (filter, Cholesky-QR2, Rayleigh-Ritz,
Lanczos bound) and of the whole eigensolver against the CPU oracle."""
import json
import os

import numpy as np
import pytest

from paper_2605_30128_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden", "tiny_rchfsi.json")


@pytest.fixture(scope="module")
def B():
    from paper_2605_30128_amd import binding
    binding.load()
    return binding


@pytest.fixture(scope="module")
def tiny_state(oracle_lib):
    """Ritz pairs of a random 40-column block of the tiny problem (oracle)."""
    p = synth.make_config("tiny")
    o = oracle_lib.Oracle(p)
    X0 = synth.random_block(p.ndof, 40, 401)
    Y, HY, MY = o.orthonormalize(X0, o.apply_H(X0), o.apply_M(X0))
    X, HX, MX, ritz = o.rayleigh_ritz(Y, HY, MY)
    R, _ = oracle_lib.residual(HX, MX, ritz)
    lmax = o.lanczos(20, synth.random_block(p.ndof, 1, 402)[:, 0])
    return dict(p=p, o=o, X=X, HX=HX, MX=MX, ritz=ritz, R=R, lmax=lmax, X0=X0)


def _dev(X, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda", dtype)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_filter_parity(B, tiny_state, prec, tol):
    s = tiny_state
    o = s["o"]
    bounds = [s["ritz"][0], s["ritz"][-1], s["lmax"]]
    q = 20
    ref = o.filter(q, bounds, s["X"], s["ritz"], s["R"])
    op = B.Chfsi(s["p"], max_nvec=40)
    Y = op.filter(_dev(s["X"]), torch.from_numpy(s["ritz"]), _dev(s["R"]), q, bounds, prec=prec).cpu().numpy()
    assert _rel(Y, ref) < tol, _rel(Y, ref)


def test_filter_degree_one_and_inplace(B, tiny_state):
    s = tiny_state
    o = s["o"]
    bounds = [s["ritz"][0], s["ritz"][-1], s["lmax"]]
    op = B.Chfsi(s["p"], max_nvec=40)
    for q in (1, 2, 5):
        ref = o.filter(q, bounds, s["X"], s["ritz"], s["R"])
        Xd = _dev(s["X"])
        op.filter(Xd, torch.from_numpy(s["ritz"]), _dev(s["R"]), q, bounds, Y=Xd)  # Y aliases X
        assert _rel(Xd.cpu().numpy(), ref) < 1e-12


def test_bad_bounds_rejected(B, tiny_state):
    s = tiny_state
    op = B.Chfsi(s["p"], max_nvec=40)
    with pytest.raises(B.ChfsiError) as ei:
        op.filter(_dev(s["X"]), torch.from_numpy(s["ritz"]), _dev(s["R"]), 5, [1.0, 0.5, 2.0])
    assert ei.value.code == B.E_BOUNDS


def test_orthonormalize_and_rr_parity(B, tiny_state, oracle_lib):
    s = tiny_state
    o = s["o"]
    X0 = s["X0"]
    HX0, MX0 = o.apply_H(X0), o.apply_M(X0)
    Yr, HYr, MYr = o.orthonormalize(X0, HX0, MX0)
    op = B.Chfsi(s["p"], max_nvec=40)
    Y, HY, MY = _dev(X0), _dev(HX0), _dev(MX0)
    op.orthonormalize(Y, HY, MY)
    # same algorithm, same arithmetic up to rounding order
    assert _rel(Y.cpu().numpy(), Yr) < 1e-10
    G = Y.cpu().numpy().conj().T @ o.apply_M(Y.cpu().numpy())
    assert np.abs(G - np.eye(40)).max() < 1e-12
    ritz, R, res = op.rayleigh_ritz(Y, HY, MY)
    _, _, _, ritz_r = o.rayleigh_ritz(Yr, HYr, MYr)
    assert np.abs(ritz.cpu().numpy() - ritz_r).max() < 1e-11 * np.abs(ritz_r).max()
    Xg = Y.cpu().numpy()
    Rr, nr = oracle_lib.residual(o.apply_H(Xg), o.apply_M(Xg), ritz.cpu().numpy())
    assert np.allclose(res.cpu().numpy(), nr, rtol=1e-9, atol=1e-12)


def test_rank_deficient_block_fails(B, tiny_state):
    s = tiny_state
    o = s["o"]
    X0 = s["X0"].copy()
    X0[:, 5] = X0[:, 4]
    op = B.Chfsi(s["p"], max_nvec=40)
    with pytest.raises(B.ChfsiError) as ei:
        op.orthonormalize(_dev(X0), _dev(o.apply_H(X0)), _dev(o.apply_M(X0)))
    assert ei.value.code == B.E_NOT_SPD


def test_lanczos_parity(B, tiny_state):
    s = tiny_state
    op = B.Chfsi(s["p"], max_nvec=40)
    v0 = synth.random_block(s["p"].ndof, 1, 402)[:, 0]
    lm = op.estimate_bounds(torch.from_numpy(v0), 20)
    # same start vector and FP64 arithmetic: only the summation order of the
    # products differs, and the extreme Ritz value of 20 steps is stable
    print("lanczos bound", lm, "oracle", s["lmax"], "rel diff", abs(lm - s["lmax"]) / s["lmax"])
    assert abs(lm - s["lmax"]) < 1e-10 * s["lmax"]


def test_rr_general_parity(B, tiny_state):
    """Generalized Rayleigh-Ritz on a non-orthonormal block gives the Ritz
    values of the same subspace as Cholesky-QR2 + Rayleigh-Ritz (oracle)."""
    s = tiny_state
    o = s["o"]
    X0 = s["X0"].copy()
    X0[:, 7] *= 1e3  # badly scaled column
    HX0, MX0 = o.apply_H(X0), o.apply_M(X0)
    Yr, HYr, MYr = o.orthonormalize(X0, HX0, MX0)
    _, _, _, ritz_r = o.rayleigh_ritz(Yr, HYr, MYr)
    op = B.Chfsi(s["p"], max_nvec=40)
    Y, HY, MY = _dev(X0), _dev(HX0), _dev(MX0)
    ritz, R, res = op.rayleigh_ritz(Y, HY, MY, general=True)
    assert np.abs(ritz.cpu().numpy() - ritz_r).max() < 1e-11 * np.abs(ritz_r).max()
    Yg = Y.cpu().numpy()
    assert np.abs(Yg.conj().T @ o.apply_M(Yg) - np.eye(40)).max() < 1e-10


@pytest.mark.parametrize("rr_mode", [0, 1])
def test_solve_tiny_fp64_matches_golden(B, rr_mode):
    g = json.load(open(GOLD))
    p = synth.make_config("tiny")
    op = B.Chfsi(p, max_nvec=g["nsub"])
    X = _dev(synth.random_block(p.ndof, g["nsub"], g["x0_seed"]))
    v0 = torch.from_numpy(synth.random_block(p.ndof, 1, g["lanczos_seed"])[:, 0])
    out = op.solve(X, g["n_wanted"], g["degree"], prec="fp64", tol=1e-10, max_iter=200, v0=v0, rr_mode=rr_mode)
    assert out["converged"], out
    ref = np.asarray(g["eigenvalues"][:g["n_wanted"]])
    assert np.abs(out["eigvals"] - ref).max() < 1e-10, np.abs(out["eigvals"] - ref).max()


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_solve_mixed_subspace_rotation(B, prec):
    """rr_mode 2 (FP32 off-diagonal blocks of the subspace rotation) with a
    subspace of 144 columns (two full 64-column blocks and a 16-column tail):
    converges to tol and its lowest eigenvalues match the oracle's golden
    values as closely as the FP64 rotation does."""
    g = json.load(open(GOLD))
    p = synth.make_config("tiny")
    op = B.Chfsi(p, max_nvec=144)
    X = _dev(synth.random_block(p.ndof, 144, 2101))
    v0 = torch.from_numpy(synth.random_block(p.ndof, 1, g["lanczos_seed"])[:, 0])
    out = op.solve(X, 128, g["degree"], prec=prec, tol=1e-8, max_iter=300, v0=v0, rr_mode=2)
    print(prec, "iterations", out["iters"], "max residual", out["max_res"])
    assert out["converged"], out
    ref = np.asarray(g["eigenvalues"][:g["n_wanted"]])
    assert np.abs(out["eigvals"][:g["n_wanted"]] - ref).max() < 1e-9


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_solve_tiny_mixed(B, prec):
    g = json.load(open(GOLD))
    p = synth.make_config("tiny")
    op = B.Chfsi(p, max_nvec=g["nsub"])
    X = _dev(synth.random_block(p.ndof, g["nsub"], g["x0_seed"]))
    v0 = torch.from_numpy(synth.random_block(p.ndof, 1, g["lanczos_seed"])[:, 0])
    out = op.solve(X, g["n_wanted"], g["degree"], prec=prec, tol=1e-8, max_iter=200, v0=v0)
    print(prec, "iterations", out["iters"], "max residual", out["max_res"])
    assert out["converged"], out
    ref = np.asarray(g["eigenvalues"][:g["n_wanted"]])
    assert np.abs(out["eigvals"] - ref).max() < 1e-9


def test_solve_max_iter_not_converged(B):
    p = synth.make_config("tiny")
    op = B.Chfsi(p, max_nvec=40)
    X = _dev(synth.random_block(p.ndof, 40, 2001))
    v0 = torch.from_numpy(synth.random_block(p.ndof, 1, 2000)[:, 0])
    out = op.solve(X, 32, 20, prec="fp64", tol=1e-14, max_iter=1, v0=v0)
    assert out["status"] == B.NOT_CONVERGED and out["iters"] == 1
    assert np.all(np.isfinite(out["eigvals"]))


def test_solve_blocked_filter_matches(B):
    """Filtering the subspace in column blocks (blocks of wavefunctions,
    Sec. III-C4) changes no result: the filter is column-wise, so a solve
    with blocks of 16 columns (16 + 16 + 8) reproduces the unblocked solve
    bit for bit."""
    p = synth.make_config("tiny")
    op = B.Chfsi(p, max_nvec=40)
    X0 = synth.random_block(p.ndof, 40, 2201)
    v0 = torch.from_numpy(synth.random_block(p.ndof, 1, 2202)[:, 0])
    outs, Xs = [], []
    for block in (0, 16):
        X = _dev(X0)
        outs.append(op.solve(X, 32, 12, prec="bf16", tol=1e-8, max_iter=6, v0=v0, block=block, rr_mode=2))
        Xs.append(X.cpu().numpy())
    assert outs[0]["iters"] == outs[1]["iters"]
    assert np.array_equal(outs[0]["eigvals"], outs[1]["eigvals"])
    assert np.array_equal(Xs[0], Xs[1])


def test_solve_profile_filter_cell_launches(B):
    """opts.profile times the filter's cell-operator launches with device
    events and changes no result: one (start, end) pair per filter step and
    column block, eight colour launches each on the 4x4x4-cell mesh."""
    p = synth.make_config("tiny")
    op = B.Chfsi(p, max_nvec=40)
    X0 = synth.random_block(p.ndof, 40, 2201)
    v0 = torch.from_numpy(synth.random_block(p.ndof, 1, 2202)[:, 0])
    q, outs, Xs = 12, [], []
    for profile in (False, True):
        X = _dev(X0)
        outs.append(op.solve(X, 32, q, prec="bf16", tol=1e-8, max_iter=4, v0=v0, block=16, rr_mode=2,
                             fixed_iters=True, profile=profile))
        Xs.append(X.cpu().numpy())
    assert np.array_equal(Xs[0], Xs[1]) and np.array_equal(outs[0]["eigvals"], outs[1]["eigvals"])
    assert outs[0]["filter_cell_launches"] == 0 and outs[0]["t_filter_cell"] == 0
    o = outs[1]
    assert o["iters"] == 4
    assert o["filter_cell_launches"] == o["iters"] * (q - 1) * 3 * 8
    assert 0 < o["t_filter_cell"] < o["t_filter"]


def test_plan_for_reduced_precision_filter(B, tiny_state):
    """A scratch planned for complex64 recurrence blocks (filter_prec bf16)
    runs the bfloat16 filter at full width and an FP64 filter up to half of
    it; wider FP64 filters report CHFSI_E_WORKSPACE before any device work.
    Its Rayleigh-Ritz rotations run in row chunks and give the same Ritz
    values as the default plan."""
    s = tiny_state
    o = s["o"]
    bounds = [s["ritz"][0], s["ritz"][-1], s["lmax"]]
    op = B.Chfsi(s["p"], max_nvec=40, filter_prec="bf16")
    ritz = torch.from_numpy(s["ritz"])
    op.filter(_dev(s["X"]), ritz, _dev(s["R"]), 4, bounds, prec="bf16")
    with pytest.raises(B.ChfsiError) as ei:
        op.filter(_dev(s["X"]), ritz, _dev(s["R"]), 4, bounds, prec="fp64")
    assert ei.value.code == B.E_WORKSPACE
    ref = o.filter(4, bounds, s["X"][:, :20], s["ritz"][:20], s["R"][:, :20])
    Y = op.filter(_dev(s["X"][:, :20]), ritz[:20], _dev(s["R"][:, :20]), 4, bounds, prec="fp64").cpu().numpy()
    assert _rel(Y, ref) < 1e-12
    X0 = s["X0"]
    HX0, MX0 = o.apply_H(X0), o.apply_M(X0)
    Yr, HYr, MYr = o.orthonormalize(X0, HX0, MX0)
    _, _, _, ritz_r = o.rayleigh_ritz(Yr, HYr, MYr)
    Yd, HYd, MYd = _dev(X0), _dev(HX0), _dev(MX0)
    rr, _, _ = op.rayleigh_ritz(Yd, HYd, MYd, general=True)
    assert np.abs(rr.cpu().numpy() - ritz_r).max() < 1e-11 * np.abs(ritz_r).max()


def test_solve_with_reduced_precision_plan():
    """The solve under a complex64-sized scratch (the mixed-precision
    subspace rotation then runs in two row chunks) converges to the same
    eigenvalues as under the default plan."""
    from paper_2605_30128_amd import binding as B
    B.load()
    p = synth.make_config("tiny")
    X0 = synth.random_block(p.ndof, 40, 2301)
    v0 = torch.from_numpy(synth.random_block(p.ndof, 1, 2302)[:, 0])
    ev = []
    for fp in ("fp64", "bf16"):
        op = B.Chfsi(p, max_nvec=40, filter_prec=fp)
        out = op.solve(_dev(X0), 32, 20, prec="bf16", tol=1e-9, max_iter=100, v0=v0, rr_mode=2)
        assert out["converged"]
        ev.append(out["eigvals"])
    assert np.abs(ev[0] - ev[1]).max() < 1e-11
