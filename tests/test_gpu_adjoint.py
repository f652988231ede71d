"""GPU parity of the adjoint of H X with respect to X and the quadrature
fields V, B (chfsi_apply_H_adjoint) against the oracle, and the
Hellmann-Feynman identity on converged eigenvectors."""
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


def _dev(X, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda", dtype)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("prec,tol,dtype", [("fp64", 1e-12, torch.complex128), ("fp32", 2e-6, torch.complex64)])
def test_adjoint_parity_tiny(B, oracle_lib, prec, tol, dtype):
    p = synth.make_config("tiny")
    o = oracle_lib.Oracle(p)
    X = synth.random_block(p.ndof, 12, 501)
    G = synth.random_block(p.ndof, 12, 502)
    dVr, dBr = o.adjoint_fields(X, G)
    op = B.Chfsi(p, max_nvec=12)
    dX, dV, dB = op.adjoint(_dev(X, dtype), _dev(G, dtype), prec=prec)
    assert _rel(dV.cpu().numpy(), dVr) < tol
    assert _rel(dB.cpu().numpy(), dBr) < tol
    assert _rel(dX.cpu().numpy(), o.apply_H(G)) < max(tol, 1e-12)


def test_adjoint_identity_with_density(B, oracle_lib):
    """G = X gives w|J| rho and w|J| m (Sec. II-A densities) at the
    quadrature points, computed here directly by the oracle."""
    p = synth.make_problem(ncell=(2, 2, 2), box=(4.0, 4.0, 4.0), degree=3, nwells=2, natoms=2, nbeta=8, seed=12)
    o = oracle_lib.Oracle(p)
    X = synth.random_block(p.ndof, 6, 503)
    dVr, dBr = o.adjoint_fields(X, X)
    op = B.Chfsi(p, max_nvec=8)
    _, dV, dB = op.adjoint(_dev(X), _dev(X), want_dX=False)
    assert _rel(dV.cpu().numpy(), dVr) < 1e-12
    assert _rel(dB.cpu().numpy(), dBr) < 1e-12
    assert np.all(dV.cpu().numpy() >= -1e-15)  # a density is non-negative
