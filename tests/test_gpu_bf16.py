"""GPU parity of the bfloat16 path, term by term.

In CHFSI_BF16 every cell-GEMM and projector-product operand is rounded to
bfloat16 (8 significant bits: unit roundoff 2^-8, an rms relative
error of about 1.7e-3 per rounding for round-to-nearest-even) and accumulated in
float (Sec. III-C2 stages i-iv with the reduced-precision operands).  A
whole-product gate hides the small terms: on the tiny workload the field
term w|J|(V + B.sigma) is about 1.2 % of ||H X||, the magnetic part 0.3 %
and the spin-orbit term 0.2 %.  So each term is isolated here as the
difference of two GPU products whose other terms are bitwise identical
(same rounded operands, same summation order), and compared with the
oracle's own evaluation of that term alone, at 1e-2 of the term's norm:
a term passes through three to four rounded operands (about 3.4e-3 rms
together), so the gate leaves a factor of three.  Each test also checks on the CPU that the gate would
fail if the term were dropped or replaced (the oracle with that term zero).
"""
import dataclasses

import numpy as np
import pytest

from paper_2605_30128_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TERM_TOL = 1e-2      # per-term relative error (about 3x the rms of four bfloat16 roundings)
ROUNDED_FLOOR = 1e-5  # a float (not bfloat16) product would be below this


@pytest.fixture(scope="module")
def B():
    from paper_2605_30128_amd import binding
    binding.load()
    return binding


def _dev(X, dtype=torch.complex64):
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda", dtype)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _no_soc(p):
    return dataclasses.replace(p, atoms=np.zeros((0, 3)), pair_ptr=np.zeros(1, np.int64),
                               pair_cell=np.zeros(0, np.int64), phi=np.zeros((0, p.nq, 2, p.nbeta), complex),
                               delta=np.zeros((0, p.nbeta, p.nbeta), complex))


def _no_fields(p):
    return dataclasses.replace(p, V=np.zeros_like(p.V), B=np.zeros_like(p.B))


def bf16_round(x):
    """Complex64 array with both parts rounded to bfloat16 (nearest even)."""
    f = np.ascontiguousarray(np.asarray(x, np.complex64)).view(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).view(np.complex64)


def test_bf16_round_helper():
    x = np.array([1.0 + 1.00390625j, 1.0 + 1.01171875j, -3.0e-3 + 0j], np.complex64)
    r = bf16_round(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa -> 1
    assert r[0].real == 1.0 and r[0].imag == 1.0
    # 1 + 3 * 2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6: even -> 1 + 2^-6
    assert r[1].imag == np.float32(1.015625)
    assert abs(r[2].real + 3.0e-3) <= 2.0 ** -8 * 3.0e-3
    assert r[2].imag == 0.0


@pytest.fixture(scope="module")
def tiny_nosoc():
    return _no_soc(synth.make_config("tiny"))


@pytest.mark.parametrize("which", ["V+B", "B"])
def test_bf16_field_term(B, oracle_lib, tiny_nosoc, which):
    """Y(V, B) - Y(fields off) against the oracle's potential (and Zeeman)
    term alone; spin-orbit off so that nothing else enters T."""
    o = oracle_lib
    p = tiny_nosoc
    X = synth.random_block(p.ndof, 32, 501)
    op = B.Chfsi(p, max_nvec=32)
    Xd = _dev(X)
    if which == "V+B":
        on_V, on_B = p.V, p.B
        flags = o.POT | o.MAG
    else:
        on_V, on_B = np.zeros_like(p.V), p.B
        flags = o.MAG
    op.set_fields(torch.from_numpy(on_V), torch.from_numpy(on_B))
    Y1 = op.apply_H(Xd, prec="bf16").cpu().numpy()
    op.set_fields(torch.zeros_like(torch.from_numpy(p.V)), torch.zeros_like(torch.from_numpy(p.B)))
    Y0 = op.apply_H(Xd, prec="bf16").cpu().numpy()
    ref = o.Oracle(dataclasses.replace(p, V=on_V, B=on_B)).apply_H(X, flags=flags)
    err = _rel(Y1 - Y0, ref)
    print(f"bf16 {which} term: rel err {err:.3e}, term/HX {np.linalg.norm(ref) / np.linalg.norm(Y1):.3e}")
    assert ROUNDED_FLOOR < err < TERM_TOL, err
    # the gate has power: the term dropped gives error 1, the potential
    # without its magnetic part (or the reverse) is far outside the gate
    other = o.Oracle(dataclasses.replace(p, V=on_V, B=on_B)).apply_H(X, flags=o.POT if which == "V+B" else 0)
    assert _rel(other, ref) > 10 * TERM_TOL


def test_bf16_soc_term(B, oracle_lib):
    """Y(projectors) - Y(no projectors), fields off in both, against the
    oracle's spin-orbit term sum_a P_a Delta_a P_a^H X alone."""
    o = oracle_lib
    p = _no_fields(synth.make_config("tiny"))
    X = synth.random_block(p.ndof, 32, 502)
    Xd = _dev(X)
    Y1 = B.Chfsi(p, max_nvec=32).apply_H(Xd, prec="bf16").cpu().numpy()
    Y0 = B.Chfsi(_no_soc(p), max_nvec=32).apply_H(Xd, prec="bf16").cpu().numpy()
    ref = o.Oracle(p).apply_H(X, flags=o.NLOC)
    err = _rel(Y1 - Y0, ref)
    print(f"bf16 spin-orbit term: rel err {err:.3e}, term/HX {np.linalg.norm(ref) / np.linalg.norm(Y1):.3e}")
    assert ROUNDED_FLOOR < err < TERM_TOL, err
    # power: the same projectors with Delta halved is far outside the gate
    ph = dataclasses.replace(p, delta=0.5 * p.delta)
    assert _rel(o.Oracle(ph).apply_H(X, flags=o.NLOC), ref) > 10 * TERM_TOL


@pytest.mark.parametrize("prec,tol", [("bf16", 6e-3), ("fp32", 2e-6)])
def test_rounded_input_whole_product(B, oracle_lib, prec, tol):
    """With X already representable in bfloat16, the only bfloat16 roundings
    left are those of the tables and of the quadrature-point term: the whole
    product (all terms, spin-orbit on) then sits well inside the 2e-2 gate of
    an unrounded input."""
    p = synth.make_config("tiny")
    X = bf16_round(synth.random_block(p.ndof, 32, 503))
    ref = oracle_lib.Oracle(p).apply_H(X.astype(np.complex128))
    Y = B.Chfsi(p, max_nvec=32).apply_H(_dev(X), prec=prec).cpu().numpy()
    err = _rel(Y, ref)
    print(f"{prec} H X of a bfloat16-representable block: rel err {err:.3e}")
    assert err < tol, err
    if prec == "bf16":
        assert err > ROUNDED_FLOOR


@pytest.mark.parametrize("degree", [6, 7])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_hx_high_degree_soc(B, oracle_lib, prec, degree):
    """p = 6 and p = 7 (343 and 512 nodes per cell, the medium and slab
    workloads' degrees, whose bfloat16 kernels use other wave tilings than
    the tiny one) in the reduced precisions with spin-orbit on: whole
    product and, in bfloat16, the field and spin-orbit terms separately."""
    o = oracle_lib
    p = synth.make_problem(ncell=(2, 2, 2), box=(4.0, 4.0, 4.0), degree=degree, nwells=2, natoms=2, nbeta=8,
                           seed=200 + degree)
    assert p.npairs > 0
    X = synth.random_block(p.ndof, 24, 497 + degree)
    ref = o.Oracle(p).apply_H(X)
    op = B.Chfsi(p, max_nvec=24)
    Y = op.apply_H(_dev(X), prec=prec).cpu().numpy()
    err = _rel(Y, ref)
    print(f"p={degree} {prec} H X rel err {err:.3e}")
    if prec == "fp32":
        assert err < 2e-6, err
        return
    assert ROUNDED_FLOOR < err < 2e-2, err
    # field term: same context, fields on and off
    Xd = _dev(X)
    op.set_fields(torch.zeros_like(op.V), torch.zeros_like(op.B))
    Y0 = op.apply_H(Xd, prec="bf16").cpu().numpy()
    e_f = _rel(Y - Y0, o.Oracle(p).apply_H(X, flags=o.POT | o.MAG))
    # spin-orbit term with the fields off
    pz = _no_fields(p)
    Y0n = B.Chfsi(_no_soc(pz), max_nvec=24).apply_H(Xd, prec="bf16").cpu().numpy()
    e_s = _rel(Y0 - Y0n, o.Oracle(pz).apply_H(X, flags=o.NLOC))
    print(f"p={degree} bf16 terms: field {e_f:.3e}, spin-orbit {e_s:.3e}")
    assert e_s < TERM_TOL, e_s
    # Y - Y0 = Phi^T (bf16(W Phi X + S) - bf16(S)): the spin-orbit part S
    # rounds with the field term, so the gate is on the pair difference
    assert e_f < 2 * TERM_TOL, e_f


@pytest.fixture(scope="module")
def tiny_ritz(oracle_lib):
    p = synth.make_config("tiny")
    o = oracle_lib.Oracle(p)
    X0 = synth.random_block(p.ndof, 40, 401)
    Y, HY, MY = o.orthonormalize(X0, o.apply_H(X0), o.apply_M(X0))
    X, HX, MX, ritz = o.rayleigh_ritz(Y, HY, MY)
    R, _ = oracle_lib.residual(HX, MX, ritz)
    lmax = o.lanczos(20, synth.random_block(p.ndof, 1, 402)[:, 0])
    return dict(p=p, o=o, X=X, ritz=ritz, R=R, lmax=lmax)


@pytest.mark.parametrize("q", [2, 20])
def test_filter_bf16(B, oracle_lib, tiny_ritz, q):
    """The bfloat16 filter (cell kernel with D^-1 gather and accumulation
    into complex64 Z_{k+1}, bfloat16 projector coefficients, spin-orbit on)
    against the oracle's filter.  Y = D^-1 Z_q + X Lambda_q; the X Lambda_q
    part is formed in FP64 from exact inputs, so the comparison is made on
    the filtered-residual part D^-1 Z_q = Y - filter(R = 0).  Each step
    adds one bfloat16 H D^-1 Z_k (about 3e-3 relative error per product, as
    above) scaled by the Chebyshev coefficient; the gate is 1e-2 of the Z
    part at q = 2 and 2e-2 after 20 steps.  At q = 20 the recurrence with the
    fields off (1.5 % of H) lands more than five gates away, so the test
    also fails if the field term is dropped from the filter's products; at
    q = 2 the Z part is still mostly R and the gate cannot see that term."""
    s = tiny_ritz
    o = s["o"]
    bounds = [s["ritz"][0], s["ritz"][-1], s["lmax"]]
    zero = np.zeros_like(s["R"])
    base = o.filter(q, bounds, s["X"], s["ritz"], zero)
    zref = o.filter(q, bounds, s["X"], s["ritz"], s["R"]) - base
    op = B.Chfsi(s["p"], max_nvec=40)
    Y = op.filter(_dev(s["X"], torch.complex128), torch.from_numpy(s["ritz"]), _dev(s["R"], torch.complex128), q,
                  bounds, prec="bf16").cpu().numpy()
    err = _rel(Y - base, zref)
    tol = 1e-2 if q == 2 else 2e-2
    print(f"bf16 filter q={q}: Z-part rel err {err:.3e}")
    assert ROUNDED_FLOOR < err < tol, err
    if q == 20:
        zoff = oracle_lib.Oracle(_no_fields(s["p"])).filter(q, bounds, s["X"], s["ritz"], s["R"]) - base
        e_off = _rel(zoff, zref)
        print(f"fields off: {e_off:.3e}")
        assert e_off > 5 * tol, e_off
