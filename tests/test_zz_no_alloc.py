"""chfsi_residual_noalloc (static scratch, no allocation) against
chfsi_residual (the context's scratch) through the C ABI: the same kernels
in the same order, so R and the column norms must agree bit for bit.  Two
calls in a row, the second with a smaller block, so that stale partials of
the first call in the shared static array would show; a block wider than
the static array is rejected with CHFSI_E_WORKSPACE before any work."""
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


def _dev(X):
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda", torch.complex128)


def test_residual_noalloc_matches(B):
    p = synth.make_config("tiny")
    op = B.Chfsi(p, max_nvec=48)
    for nvec, ld, seed in ((48, 48, 901), (21, 24, 902)):
        HX = _dev(synth.random_block(p.ndof, nvec, seed, ld=ld))
        MX = _dev(synth.random_block(p.ndof, nvec, seed + 10, ld=ld))
        ritz = torch.linspace(-0.5, 3.0, nvec, dtype=torch.float64, device="cuda")
        R0, n0 = op.residual(HX, MX, ritz, nvec=nvec)
        R1 = torch.full_like(HX, complex(7.0, -7.0))
        n1 = torch.full((nvec,), -1.0, dtype=torch.float64, device="cuda")
        op.residual(HX, MX, ritz, nvec=nvec, R=R1, res=n1, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(R1[:, :nvec], R0[:, :nvec])
        assert torch.equal(n1, n0)
        # columns past nvec are not written
        assert bool((R1[:, nvec:] == complex(7.0, -7.0)).all())
        # and the norms are those of R
        ref = torch.linalg.vector_norm(R0[:, :nvec], dim=0)
        assert torch.allclose(n1, ref, rtol=1e-12, atol=0)


def test_residual_noalloc_rejects_wide_blocks(B):
    p = synth.make_problem(ncell=(2, 2, 2), box=(4.0, 4.0, 4.0), degree=1, nwells=1, soc=False, seed=903)
    op = B.Chfsi(p, max_nvec=4100)
    HX = torch.zeros((p.ndof, 4100), dtype=torch.complex128, device="cuda")
    ritz = torch.zeros(4100, dtype=torch.float64, device="cuda")
    with pytest.raises(B.ChfsiError) as ei:
        op.residual(HX, HX, ritz, noalloc=True)
    assert ei.value.code == B.E_WORKSPACE
    R, n = op.residual(HX, HX, ritz, nvec=4096, noalloc=True)
    torch.cuda.synchronize()
    assert float(n.abs().max()) == 0.0
