"""Pins of the oracle's reference element (Sec. III-A: Lagrange polynomials on
GLL nodes, Gauss-Legendre quadrature) against closed forms and library
routines."""
import math

import numpy as np
import pytest


def test_gll_closed_forms(oracle_lib):
    x, w = oracle_lib.gll(2)
    assert np.allclose(x, [-1, 0, 1], atol=1e-15)
    assert np.allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    x, w = oracle_lib.gll(4)
    r = math.sqrt(3 / 7)
    assert np.allclose(x, [-1, -r, 0, r, 1], atol=1e-15)
    assert np.allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_gll_exactness(oracle_lib, p):
    x, w = oracle_lib.gll(p)
    assert abs(w.sum() - 2) < 1e-14
    assert np.all(np.diff(x) > 0)
    # GLL with p+1 points integrates polynomials of degree 2p-1 exactly
    for k in range(2 * p):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 8, 9])
def test_gauss_matches_library_and_is_exact(oracle_lib, n):
    x, w = oracle_lib.gauss(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, xr, atol=1e-15, rtol=0)
    assert np.allclose(w, wr, atol=1e-15, rtol=0)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14


@pytest.mark.parametrize("p", [2, 4, 6, 7])
def test_lagrange_cardinal_partition_derivative(oracle_lib, p):
    nodes, _ = oracle_lib.gll(p)
    for j, xj in enumerate(nodes):
        l, _ = oracle_lib.lagrange(nodes, xj)
        e = np.zeros(p + 1); e[j] = 1
        assert np.allclose(l, e, atol=1e-13)
    for x in np.linspace(-1, 1, 11):
        l, dl = oracle_lib.lagrange(nodes, x)
        assert abs(l.sum() - 1) < 1e-13
        assert abs(dl.sum()) < 1e-11
        # derivative against a central difference
        hh = 1e-6
        lp, _ = oracle_lib.lagrange(nodes, x + hh)
        lm, _ = oracle_lib.lagrange(nodes, x - hh)
        assert np.allclose(dl, (lp - lm) / (2 * hh), atol=1e-6 * max(1, np.abs(dl).max()))
        # reproduces x^k for k <= p (value and derivative)
        for k in range(p + 1):
            assert abs(np.dot(l, nodes ** k) - x ** k) < 1e-12
            if k > 0:
                assert abs(np.dot(dl, nodes ** k) - k * x ** (k - 1)) < 1e-10


def test_cell_tables(oracle_lib):
    from paper_2605_30128_amd import synth
    p = synth.make_problem(ncell=(2, 2, 2), box=(3.0, 4.0, 5.0), degree=3, soc=False)
    o = oracle_lib.Oracle(p)
    Nq, dNq, wJ = o.tables()
    vol = 1.5 * 2.0 * 2.5
    assert abs(wJ.sum() - vol) < 1e-13
    assert np.allclose(Nq.sum(axis=1), 1, atol=1e-13)
    assert np.allclose(dNq.sum(axis=1), 0, atol=1e-11)
    # gradient of the linear field x reproduces 1
    n1 = 4
    xi, _ = oracle_lib.gll(3)
    I = np.arange(n1 ** 3)
    xnode = (xi[I % n1] + 1) * 0.75
    assert np.allclose(dNq[:, :, 0] @ xnode, 1.0, atol=1e-12)
    assert np.allclose(dNq[:, :, 1] @ xnode, 0.0, atol=1e-12)
