"""Pins of the block floating-point codec oracle against what its definition
fixes (Sec. III-C3, compressed communication): the size of the stream, the
zero-block flag, the shared exponent (checked against numpy's frexp), exact
round trips of representable values, the half-quantum error bound, the
upper-bound clamp, ties to even, block locality and subnormal blocks."""
import numpy as np
import pytest

from oracle import bfp

RATES = [16, 12, 10]


def _blocks(rng, nblk):
    """Blocks with magnitudes spread over many binades, signs mixed."""
    mant = rng.uniform(-1.0, 1.0, size=(nblk, 4))
    expo = rng.integers(-30, 30, size=(nblk, 1))
    return (mant * np.exp2(expo)).astype(np.float32).ravel()


@pytest.mark.parametrize("nbits", RATES)
def test_stream_size_and_zero_block(nbits):
    x = np.zeros(12, np.float32)
    s = bfp.encode(x, nbits)
    assert s.size == 3 * nbits // 2 == 12 * nbits // 8
    assert not s.any()  # exponent field 0 flags an all-zero block
    assert np.array_equal(bfp.decode(s, 12, nbits), x)


@pytest.mark.parametrize("nbits", RATES)
def test_shared_exponent_matches_frexp(nbits):
    rng = np.random.default_rng(1)
    x = _blocks(rng, 200)
    s = bfp.encode(x, nbits).reshape(200, nbits // 2)
    for b in range(200):
        _, e = np.frexp(np.abs(x[4 * b:4 * b + 4]).max())  # 2^(e-1) <= max < 2^e
        assert int(s[b, 0]) == e + 127  # low byte of the little-endian block


@pytest.mark.parametrize("nbits", RATES)
def test_representable_values_round_trip_exactly(nbits):
    v = nbits - 2
    rng = np.random.default_rng(2)
    for emax in (-100, -3, 0, 5, 90):
        q = rng.integers(-(1 << (v - 1)) + 1, 1 << (v - 1), size=(64, 4))  # |q| < 2^(v-1): max stays < 2^emax
        q[:, 0] = rng.integers(1 << (v - 2), 1 << (v - 1), size=64)  # max in [2^(emax-1), 2^emax)
        x = (q * np.exp2(emax - v + 1)).astype(np.float32).ravel()
        y = bfp.decode(bfp.encode(x, nbits), x.size, nbits)
        assert np.array_equal(x, y)


@pytest.mark.parametrize("nbits", RATES)
def test_error_bound_half_quantum(nbits):
    v = nbits - 2
    rng = np.random.default_rng(3)
    x = _blocks(rng, 500)
    y = bfp.decode(bfp.encode(x, nbits), x.size, nbits)
    for b in range(500):
        blk = x[4 * b:4 * b + 4].astype(np.float64)
        _, e = np.frexp(np.abs(blk).max())
        quantum = 2.0 ** (e - v + 1)
        err = np.abs(y[4 * b:4 * b + 4] - blk)
        # round to nearest: half a quantum, except a clamped top value (one quantum)
        assert np.all(err <= quantum * 0.5 + 1e-300) or (err.max() <= quantum and np.abs(blk).max() * 2.0 ** (v - 1 - e) > (1 << (v - 1)) - 0.5)


@pytest.mark.parametrize("nbits", RATES)
def test_upper_clamp_and_negative_extreme(nbits):
    v = nbits - 2
    top = np.nextafter(np.float32(8.0), np.float32(0.0))  # just below 2^3: e_max = 3
    x = np.array([top, -top, 0.0, 1.0], np.float32)
    y = bfp.decode(bfp.encode(x, nbits), 4, nbits)
    quantum = 2.0 ** (3 - v + 1)
    assert y[0] == ((1 << (v - 1)) - 1) * quantum  # clamped, not wrapped to negative
    assert y[1] == -8.0  # -2^(v-1) is representable: no clamp below
    assert y[2] == 0.0 and y[3] == 1.0


def test_round_half_to_even():
    # n_bits = 10: v = 8, max 1.0 -> e_max = 1, quantum 2^-6
    q = 2.0 ** -6
    x = np.array([1.0, 2.5 * q, 3.5 * q, -2.5 * q], np.float32)
    y = bfp.decode(bfp.encode(x, 10), 4, 10)
    assert list(y) == [1.0, 2 * q, 4 * q, -2 * q]


@pytest.mark.parametrize("nbits", RATES)
def test_blocks_are_independent(nbits):
    rng = np.random.default_rng(4)
    a, b = _blocks(rng, 7), _blocks(rng, 5)
    whole = bfp.encode(np.concatenate([a, b]), nbits)
    assert np.array_equal(whole, np.concatenate([bfp.encode(a, nbits), bfp.encode(b, nbits)]))


@pytest.mark.parametrize("nbits", RATES)
def test_subnormal_block_uses_smallest_normal_exponent(nbits):
    x = np.array([1e-40, -2e-40, 0.0, 3e-45], np.float32)  # all below 2^-126
    s = bfp.encode(x, nbits)
    assert s[0] == 1  # e_max clamped to -126
    y = bfp.decode(s, 4, nbits)
    assert np.all(np.abs(y - x) <= 2.0 ** (-126 - (nbits - 2)))
