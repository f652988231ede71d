"""CPU oracle of the block floating-point (BFP) codec (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the CPU baseline leg of the benchmark may
import this module; the product path never does.  It shares no code with the
GPU library.

Written from the paper's description of its lightweight BFP compression
(Sec. III-C3, the compressed-communication paragraphs and fig. layout):

* four FP32 values form a block of N_bits = 4 n_bits bits; the low 8 bits
  hold a shared biased exponent, the remaining N_bits - 8 bits four signed
  coefficients of v_bits = n_bits - 2 bits each (n_bits = 16, 12, 10 give
  v_bits = 14, 10, 8);
* the shared exponent e_max satisfies 2^(e_max - 1) <= max_i |x_i| < 2^e_max;
  an all-zero block is flagged by a zero exponent field, otherwise
  e = e_max + 127 is stored;
* q_i = round(x_i 2^(v_bits - 1 - e_max)) in [-2^(v_bits-1), 2^(v_bits-1) - 1],
  only the upper bound needing a clamp; q_i is kept as its low v_bits bits in
  two's complement;
* decoding restores e_max = e - 127, sign-extends q_i and returns
  q_i 2^(e_max - v_bits + 1).

Readings where the text leaves a choice (each also listed in the design
notes): the coefficients follow the exponent in value order (q_0 in the
lowest bits after the exponent), the block's bits are stored little-endian
in N_bits / 8 consecutive bytes, "round" is round-half-to-even, and a block
whose largest magnitude is below 2^-126 (FP32 subnormals only) uses the
smallest normal exponent e_max = -126 so that e stays >= 1.

All arithmetic is exact in float64 (scaling by powers of two, integer
rounding), so the encoded bytes are fixed bit for bit by the definition.
"""
from __future__ import annotations

import numpy as np

RATES = (16, 12, 10)


def vbits(nbits: int) -> int:
    """Coefficient width v_bits = n_bits - 2."""
    if nbits not in RATES:
        raise ValueError(f"n_bits must be one of {RATES}")
    return nbits - 2


def block_bytes(nbits: int) -> int:
    """Bytes per four-value block, N_bits / 8."""
    vbits(nbits)
    return nbits // 2


def shared_exponent(block: np.ndarray) -> int:
    """e_max of one block of four float32 values (None for an all-zero block):
    the integer with 2^(e_max-1) <= max|x| < 2^e_max, at least -126."""
    m = float(np.max(np.abs(block.astype(np.float64))))
    if m == 0.0:
        return None
    _, e = np.frexp(m)  # m = f 2^e with 0.5 <= f < 1
    return max(int(e), -126)


def encode(x: np.ndarray, nbits: int) -> np.ndarray:
    """Encodes float32 values (length a multiple of 4) into a uint8 stream of
    len(x) / 4 * N_bits / 8 bytes."""
    v = vbits(nbits)
    x = np.asarray(x, dtype=np.float32)
    if x.ndim != 1 or x.size % 4:
        raise ValueError("the input must be a 1-D array whose length is a multiple of 4")
    nb = block_bytes(nbits)
    out = np.zeros(x.size // 4 * nb, dtype=np.uint8)
    qmax, qmin = (1 << (v - 1)) - 1, -(1 << (v - 1))
    mask = (1 << v) - 1
    for b in range(x.size // 4):
        blk = x[4 * b:4 * b + 4].astype(np.float64)
        emax = shared_exponent(blk)
        word = 0
        if emax is not None:
            word = emax + 127
            for i in range(4):
                q = int(np.rint(blk[i] * 2.0 ** (v - 1 - emax)))
                q = min(max(q, qmin), qmax)
                word |= (q & mask) << (8 + i * v)
        out[b * nb:(b + 1) * nb] = np.frombuffer(word.to_bytes(nb, "little"), dtype=np.uint8)
    return out


def decode(stream: np.ndarray, n: int, nbits: int) -> np.ndarray:
    """Decodes n float32 values (a multiple of 4) from an encoded stream."""
    v = vbits(nbits)
    nb = block_bytes(nbits)
    stream = np.asarray(stream, dtype=np.uint8)
    if n % 4 or stream.size < n // 4 * nb:
        raise ValueError("n must be a multiple of 4 and the stream long enough")
    out = np.zeros(n, dtype=np.float32)
    mask = (1 << v) - 1
    for b in range(n // 4):
        word = int.from_bytes(stream[b * nb:(b + 1) * nb].tobytes(), "little")
        e = word & 0xFF
        if e == 0:
            continue
        emax = e - 127
        for i in range(4):
            q = (word >> (8 + i * v)) & mask
            if q >> (v - 1):  # restore the dropped copies of the sign bit
                q -= 1 << v
            out[4 * b + i] = np.float32(q * 2.0 ** (emax - v + 1))
    return out
