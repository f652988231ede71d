"""GPU parity of the block floating-point codec (chfsi_bfp_encode /
chfsi_bfp_decode) with the CPU oracle: the encoded streams are compared byte
for byte and the decoded values bit for bit, for every rate, on blocks that
cover many binades, zero blocks, clamped maxima, ties and subnormal blocks,
with a ragged block count; plus a large stream checked through invariants."""
import numpy as np
import pytest

from oracle import bfp
from paper_2605_30128_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    from paper_2605_30128_amd import binding
    binding.load()
    return binding


def _cases():
    x = synth.random_real(4 * 1237, 4242).astype(np.float32)
    x = (x * np.exp2(np.repeat(np.random.default_rng(5).integers(-40, 40, 1237), 4))).astype(np.float32)
    x[16:20] = 0.0                                                   # all-zero block
    x[20:24] = [np.nextafter(np.float32(4.0), np.float32(0)), -1.0, 0.5, 0.0]  # clamped maximum
    x[24:28] = [1.0, 2.5 / 64, 3.5 / 64, -2.5 / 64]                  # ties at n_bits = 10
    x[28:32] = [1e-40, -2e-40, 0.0, 3e-45]                           # subnormal block
    x[32:36] = [3.0e38, -1.0e38, 1.0, -2.0]                          # largest binade
    return x


@pytest.mark.parametrize("nbits", [16, 12, 10])
def test_bfp_bit_exact(B, nbits):
    x = _cases()
    ref = bfp.encode(x, nbits)
    xd = torch.from_numpy(x).cuda()
    s = B.bfp_encode(xd, nbits)
    got = s.cpu().numpy()
    assert got.size == ref.size == B.bfp_bytes(nbits, x.size)
    assert np.array_equal(got, ref)
    y = B.bfp_decode(s, x.size, nbits).cpu().numpy()
    assert np.array_equal(y.view(np.uint32), bfp.decode(ref, x.size, nbits).view(np.uint32))


@pytest.mark.parametrize("nbits", [16, 12, 10])
def test_bfp_large_stream_invariants(B, nbits):
    """At the size of one complex64 filter block of the medium workload per
    column group (8M values): every block's exponent byte is that of its
    largest magnitude (torch.frexp) and decode(encode(x)) stays within half a
    quantum of x (a whole one where the top value is clamped)."""
    n = 1 << 23
    g = torch.Generator(device="cuda").manual_seed(9)
    x = torch.randn(n, generator=g, device="cuda", dtype=torch.float32)
    s = B.bfp_encode(x, nbits)
    y = B.bfp_decode(s, n, nbits)
    blkmax = x.view(-1, 4).abs().amax(dim=1, keepdim=True)
    _, e = torch.frexp(blkmax)
    assert torch.equal(s.view(-1, nbits // 2)[:, :1].to(torch.int32), (e + 127).to(torch.int32))
    quantum = torch.ldexp(torch.ones_like(blkmax), e - (nbits - 2) + 1)
    assert bool(((y - x).view(-1, 4).abs() <= quantum).all())
    # sampled blocks against the oracle
    idx = np.random.default_rng(1).integers(0, n // 4, 64)
    xs = x.view(-1, 4)[torch.from_numpy(idx).cuda()].cpu().numpy().ravel()
    nb = nbits // 2
    sg = s.view(-1, nb)[torch.from_numpy(idx).cuda()].cpu().numpy().ravel()
    assert np.array_equal(sg, bfp.encode(xs, nbits))


def test_bfp_argument_errors(B):
    x = torch.zeros(8, dtype=torch.float32, device="cuda")
    with pytest.raises(B.ChfsiError):
        B.bfp_encode(x, 11)
    with pytest.raises(B.ChfsiError):
        B.bfp_encode(torch.zeros(6, dtype=torch.float32, device="cuda"), 16)
    with pytest.raises(B.ChfsiError):  # misaligned float buffer
        B.bfp_encode(x.narrow(0, 1, 4), 16)
