"""Pins of the oracle's operators H and M (Sec. II-A eq. hloc/hnloc, Sec. III-A)
against invariants, closed forms and brute force on tiny meshes."""
import math

import numpy as np
import pytest

from paper_2605_30128_amd import synth


def _tiny(**kw):
    base = dict(ncell=(2, 2, 2), box=(4.0, 4.0, 4.0), degree=2, nwells=2, natoms=2, nbeta=4, seed=11)
    base.update(kw)
    return synth.make_problem(**base)


def _eig(o, flags=None):
    import oracle
    H, M = o.dense(oracle.ALL if flags is None else flags)
    w, V = oracle.dense_geig(H, M)
    return w, V, H, M


def test_mass_spd_total_rowsum(oracle_lib):
    p = _tiny(degree=3)
    o = oracle_lib.Oracle(p)
    _, M = o.dense()
    assert np.abs(M.imag).max() == 0
    Mr = M.real
    assert np.abs(Mr - Mr.T).max() < 1e-15
    assert np.linalg.eigvalsh(Mr).min() > 0
    # sum of all entries = 2 (spins) x box volume
    assert abs(Mr.sum() - 2 * 64.0) < 1e-12
    # spin-diagonal: no coupling between alpha and beta
    assert np.abs(Mr[0::2, 1::2]).max() == 0
    # row sums = D (GLL-integrated diagonal) and D in closed form
    D = o.mass_diag()
    assert np.allclose(Mr.sum(axis=1)[0::2], D, rtol=0, atol=1e-14)
    xg, wg = oracle_lib.gll(3)
    detJ = (2.0 ** 3) / 8
    # the node at the origin is a corner of 8 cells
    assert abs(D[0] - 8 * detJ * wg[0] ** 3) < 1e-14
    # an interior node (1,1,1) of cell 0 belongs only to it
    Nx = 2 * 3
    g = 1 + Nx * (1 + Nx * 1)
    assert abs(D[g] - detJ * wg[1] ** 3) < 1e-14


def test_kinetic_annihilates_constants(oracle_lib):
    p = synth.make_config("tiny")
    o = oracle_lib.Oracle(p)
    X = np.zeros((p.ndof, 2), complex)
    X[0::2, 0] = 1.0
    X[1::2, 1] = 1.0j
    Y = o.apply_H(X, flags=oracle_lib.KIN)
    assert np.abs(Y).max() < 1e-13


def test_hermitian_dot_test(oracle_lib):
    p = synth.make_config("tiny")
    o = oracle_lib.Oracle(p)
    U = synth.random_block(p.ndof, 2, 21)
    X = synth.random_block(p.ndof, 2, 22)
    HU = o.apply_H(U)
    HX = o.apply_H(X)
    a = np.vdot(U, HX)
    b = np.vdot(HU, X)
    assert abs(a - b) / abs(a) < 1e-13
    MU = o.apply_M(U)
    MX = o.apply_M(X)
    assert abs(np.vdot(U, MX) - np.vdot(MU, X)) / abs(np.vdot(U, MX)) < 1e-13


def test_dense_hermitian(oracle_lib):
    o = oracle_lib.Oracle(_tiny())
    _, _, H, M = _eig(o)
    assert np.abs(H - H.conj().T).max() <= 1e-14 * np.abs(H).max()


def test_constant_potential_shift(oracle_lib):
    v0 = 0.37
    o0 = oracle_lib.Oracle(_tiny(v_const=0.0, bfield="zero", soc=False))
    o1 = oracle_lib.Oracle(_tiny(v_const=v0, bfield="zero", soc=False))
    w0 = _eig(o0)[0]
    w1 = _eig(o1)[0]
    assert np.abs(w1 - (w0 + v0)).max() < 1e-12


def test_zeeman_closed_form(oracle_lib):
    b = np.array([0.03, -0.04, 0.05])
    bn = np.linalg.norm(b)
    os_ = oracle_lib.Oracle(_tiny(bfield="zero", soc=False))
    ob = oracle_lib.Oracle(_tiny(bfield="const", b_const=b, soc=False))
    ws = _eig(os_)[0]
    wb = _eig(ob)[0]
    # B = 0: every scalar level appears twice (spin up, spin down)
    assert np.abs(ws[0::2] - ws[1::2]).max() < 1e-12
    scal = ws[0::2]
    expect = np.sort(np.concatenate([scal - bn, scal + bn]))
    assert np.abs(wb - expect).max() < 1e-12


def test_kramers_degeneracy(oracle_lib):
    o = oracle_lib.Oracle(_tiny(bfield="zero", soc=True, nbeta=8, degree=2))
    w = _eig(o)[0]
    assert np.abs(w[0::2] - w[1::2]).max() < 1e-10
    # and the spin-orbit term is really on: with B random, degeneracy lifts
    o2 = oracle_lib.Oracle(_tiny(bfield="random", soc=True, nbeta=8, degree=2))
    w2 = _eig(o2)[0]
    assert np.abs(w2[0::2] - w2[1::2]).max() > 1e-4


def test_soc_term_changes_spectrum(oracle_lib):
    a = _eig(oracle_lib.Oracle(_tiny(bfield="zero", soc=True, nbeta=8)))[0]
    b = _eig(oracle_lib.Oracle(_tiny(bfield="zero", soc=False)))[0]
    assert np.abs(a - b).max() > 1e-3


@pytest.mark.parametrize("soc", [False, True])
def test_spin_rotation_invariance(oracle_lib, soc):
    axis, ang = (1.0, 2.0, -0.5), 0.9
    a = _eig(oracle_lib.Oracle(_tiny(soc=soc, nbeta=8)))[0]
    b = _eig(oracle_lib.Oracle(_tiny(soc=soc, nbeta=8, spin_rot_axis=axis, spin_rot_angle=ang)))[0]
    assert np.abs(a - b).max() < 1e-10
    if soc:
        # rotating B alone (projector spin frame fixed) does change the spectrum
        p = _tiny(soc=True, nbeta=8, spin_rot_axis=axis, spin_rot_angle=ang)
        p0 = _tiny(soc=True, nbeta=8)
        p.phi = p0.phi
        c = _eig(oracle_lib.Oracle(p))[0]
        assert np.abs(a - c).max() > 1e-8


def _free_levels(L, nmax=3):
    ks = []
    for i in range(-nmax, nmax + 1):
        for j in range(-nmax, nmax + 1):
            for k in range(-nmax, nmax + 1):
                ks.append(2 * math.pi ** 2 * (i * i + j * j + k * k) / L ** 2)
    ks = np.sort(np.repeat(ks, 2))  # two spin states
    return ks


def test_free_electron_convergence(oracle_lib):
    L = 4.0
    exact = _free_levels(L)
    errs = []
    for deg in (2, 3):
        o = oracle_lib.Oracle(_tiny(degree=deg, v_const=0.0, bfield="zero", soc=False))
        w = _eig(o)[0]
        nlow = 2 * 7  # k = 0 and the six |n| = 1 modes, two spins each
        assert abs(w[0]) < 1e-12 and abs(w[1]) < 1e-12
        # Galerkin eigenvalues bound the exact ones from above
        assert np.all(w[:nlow] >= exact[:nlow] - 1e-12)
        errs.append(np.max(w[:nlow] - exact[:nlow]))
    assert errs[1] < errs[0] / 4
    # the twelve |n| = 1 states split into the cos-type and sin-type sextets
    # (cubic symmetry times spin) because the mesh is not translation
    # invariant; both sextets lie above the exact level
    o = oracle_lib.Oracle(_tiny(degree=3, v_const=0.0, bfield="zero", soc=False))
    w = _eig(o)[0]
    assert np.abs(w[2:8] - w[2]).max() < 1e-10
    assert np.abs(w[8:14] - w[8]).max() < 1e-10
    assert w[14] - w[13] > 1e-3


def test_adjoint_dot_test_fields(oracle_lib):
    """d/dt Re<G, H(V+t dV, B+t dB) X> = sum dV*adjV + dB*adjB (linear in t)."""
    p = _tiny(degree=2)
    o = oracle_lib.Oracle(p)
    X = synth.random_block(p.ndof, 3, 31)
    G = synth.random_block(p.ndof, 3, 32)
    adjV, adjB = o.adjoint_fields(X, G)
    dV = synth.random_real(p.V.shape, 33)
    dB = synth.random_real(p.B.shape, 34)
    t = 1e-6
    vals = []
    for s in (+1, -1):
        q = _tiny(degree=2)
        q.V = p.V + s * t * dV
        q.B = p.B + s * t * dB
        Y = oracle_lib.Oracle(q).apply_H(X)
        vals.append(np.real(np.vdot(G, Y)))
    fd = (vals[0] - vals[1]) / (2 * t)
    an = np.sum(adjV * dV) + np.sum(adjB * dB)
    assert abs(fd - an) <= 1e-8 * abs(an)


def test_adjoint_x_is_H_G(oracle_lib):
    p = _tiny(degree=2)
    o = oracle_lib.Oracle(p)
    X = synth.random_block(p.ndof, 2, 41)
    G = synth.random_block(p.ndof, 2, 42)
    dX = synth.random_block(p.ndof, 2, 43)
    # Re<G, H dX> = Re<H G, dX>
    assert abs(np.real(np.vdot(G, o.apply_H(dX))) - np.real(np.vdot(o.apply_H(G), dX))) < 1e-12 * np.abs(np.vdot(G, o.apply_H(dX)))


def test_hellmann_feynman_fd(oracle_lib):
    """d(sum of the lowest N eigenvalues)/dV_q = wJ rho(x_q), /dB_q = wJ m(x_q)
    (Sec. II-A densities), by central differences of re-solved spectra."""
    p = _tiny(degree=2, nbeta=8)
    o = oracle_lib.Oracle(p)
    w, V, _, _ = _eig(o)
    N = 6
    assert w[N] - w[N - 1] > 1e-3
    X = V[:, :N]
    adjV, adjB = o.adjoint_fields(X, X)
    rng = np.random.default_rng(5)
    h = 1e-4
    for trial in range(3):
        e = int(rng.integers(p.ncells)); q = int(rng.integers(p.nq))
        for comp in ("V", 0, 2):
            sums = []
            for s in (+1, -1):
                pp = _tiny(degree=2, nbeta=8)
                if comp == "V":
                    pp.V = p.V.copy(); pp.V[e, q] += s * h
                else:
                    pp.B = p.B.copy(); pp.B[e, q, comp] += s * h
                ww = _eig(oracle_lib.Oracle(pp))[0]
                sums.append(ww[:N].sum())
            fd = (sums[0] - sums[1]) / (2 * h)
            an = adjV[e, q] if comp == "V" else adjB[e, q, comp]
            assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-3), (comp, fd, an)


def test_sampled_apply_matches_full(oracle_lib):
    p = synth.make_config("tiny")
    o = oracle_lib.Oracle(p)
    X = synth.random_block(p.ndof, 8, 51)
    Y = o.apply_H(X)
    nodes = np.array([0, 5, 77, 1000, p.nnodes - 1])
    cols = np.array([0, 3, 7])
    S = o.apply_H_sampled(X, nodes, cols)
    ref = np.stack([Y[2 * nodes][:, cols], Y[2 * nodes + 1][:, cols]], axis=1)
    assert np.abs(S - ref).max() < 1e-12 * np.abs(Y).max()
