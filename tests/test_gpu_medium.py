"""Parity at the medium workload's full size in the launch configuration the
benchmark times (16^3 cells, p = 6, 64 atoms x 8 projectors, 512 vectors):
the GPU product is compared with the oracle on sampled outputs (nodes x
columns) that the oracle computes one by one."""
import numpy as np
import pytest

from paper_2605_30128_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def medium(oracle_lib):
    from paper_2605_30128_amd import binding
    binding.load()
    p = synth.make_config("medium")
    X = synth.random_block(p.ndof, 512, 701)
    op = binding.Chfsi(p, max_nvec=512)
    # sampled nodes: the 8 corners of cell 1000 (shared by 8 cells each), an
    # edge, a face and an interior node of it, and nodes of a far-away cell
    n1, Nx = 7, 96
    ex, ey, ez = 1000 % 16, (1000 // 16) % 16, 1000 // 256
    nodes = []
    for (i, j, k) in [(0, 0, 0), (6, 0, 0), (0, 6, 0), (6, 6, 6), (3, 0, 0), (3, 3, 0), (3, 3, 3), (1, 5, 2)]:
        gx, gy, gz = (ex * 6 + i) % Nx, (ey * 6 + j) % Nx, (ez * 6 + k) % Nx
        nodes.append(gx + Nx * (gy + Nx * gz))
    nodes += [0, p.nnodes - 1]
    cols = np.array([0, 1, 15, 16, 255, 383, 511])
    o = oracle_lib.Oracle(p)
    ref = o.apply_H_sampled(X, np.array(nodes), cols)
    return dict(p=p, X=X, op=op, nodes=np.array(nodes), cols=cols, ref=ref, binding=binding)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 5e-6), ("bf16", 2e-2)])
def test_hx_medium_sampled(medium, prec, tol):
    m = medium
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    Xd = torch.from_numpy(m["X"]).to("cuda", dt)
    Y = m["op"].apply_H(Xd, prec=prec)
    rows = np.stack([2 * m["nodes"], 2 * m["nodes"] + 1], axis=1)  # [node][spin]
    got = Y[torch.from_numpy(rows.ravel()).cuda()][:, torch.from_numpy(m["cols"]).cuda()].cpu().numpy()
    got = got.reshape(len(m["nodes"]), 2, len(m["cols"]))
    err = np.abs(got - m["ref"]).max() / np.abs(m["ref"]).max()
    assert err < tol, err
    del Y, Xd
    torch.cuda.empty_cache()


def test_hx_medium_properties(medium):
    """At full size: the product is deterministic and Hermitian on random
    blocks, <U, H X> = <H U, X> (FP64)."""
    m = medium
    X = torch.from_numpy(m["X"][:, :16].copy()).cuda()
    U = torch.from_numpy(synth.random_block(m["p"].ndof, 16, 702)).cuda()
    HX = m["op"].apply_H(X)
    HU = m["op"].apply_H(U)
    a = torch.sum(torch.conj(U) * HX).item()
    b = torch.sum(torch.conj(HU) * X).item()
    assert abs(a - b) <= 1e-12 * abs(a)
    HX2 = m["op"].apply_H(X)
    assert torch.equal(HX, HX2)
