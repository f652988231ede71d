// Block floating-point codec (paper Sec. III-C3, compressed communication,
// fig. layout): four FP32 values share an 8-bit biased exponent stored in
// the low bits of an N_bits = 4 n_bits block, followed by four signed
// v_bits = n_bits - 2 coefficients (q_0 lowest), rounded to nearest (ties
// to even) with only the upper bound clamped.  The exponent is that of the
// largest magnitude (2^(e_max-1) <= max|x| < 2^e_max, at least -126); an
// all-zero block stores exponent field 0.  Blocks are little-endian and
// back to back (N_bits / 8 bytes each), one thread per block: n_bits = 16
// is one 8-byte store, 12 three 2-byte stores, 10 five 1-byte stores, so no
// storage word is shared by two blocks and no atomics are needed.
#include "internal.h"

namespace chfsi {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int NBITS>
__device__ __forceinline__ void store_block(uint8_t *out, int64_t b, uint64_t w) {
    if constexpr (NBITS == 16) {
        reinterpret_cast<uint64_t *>(out)[b] = w;
    } else if constexpr (NBITS == 12) {
        uint16_t *o = reinterpret_cast<uint16_t *>(out) + 3 * b;
        o[0] = (uint16_t)w;
        o[1] = (uint16_t)(w >> 16);
        o[2] = (uint16_t)(w >> 32);
    } else {
        uint8_t *o = out + 5 * b;
#pragma unroll
        for (int i = 0; i < 5; ++i) o[i] = (uint8_t)(w >> (8 * i));
    }
}

template <int NBITS>
__device__ __forceinline__ uint64_t load_block(const uint8_t *in, int64_t b) {
    if constexpr (NBITS == 16) {
        return reinterpret_cast<const uint64_t *>(in)[b];
    } else if constexpr (NBITS == 12) {
        const uint16_t *p = reinterpret_cast<const uint16_t *>(in) + 3 * b;
        return (uint64_t)p[0] | ((uint64_t)p[1] << 16) | ((uint64_t)p[2] << 32);
    } else {
        const uint8_t *p = in + 5 * b;
        uint64_t w = 0;
#pragma unroll
        for (int i = 0; i < 5; ++i) w |= (uint64_t)p[i] << (8 * i);
        return w;
    }
}

template <int NBITS>
__global__ void bfp_encode_kernel(const float *x, int64_t nblk, uint8_t *out) {
    constexpr int V = NBITS - 2;
    constexpr int QMAX = (1 << (V - 1)) - 1, QMIN = -(1 << (V - 1));
    constexpr uint64_t MASK = (1ull << V) - 1;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblk) return;
    const f4 v = reinterpret_cast<const f4 *>(x)[b];
    const float m = fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])));
    uint64_t w = 0;
    if (m != 0.0f) {
        int emax;
        frexpf(m, &emax);  // m = f 2^emax, 0.5 <= f < 1
        emax = emax < -126 ? -126 : emax;
        w = (uint64_t)(emax + 127);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int q = (int)rintf(ldexpf(v[i], V - 1 - emax));
            q = q > QMAX ? QMAX : (q < QMIN ? QMIN : q);
            w |= ((uint64_t)(int64_t)q & MASK) << (8 + i * V);
        }
    }
    store_block<NBITS>(out, b, w);
}

template <int NBITS>
__global__ void bfp_decode_kernel(const uint8_t *in, int64_t nblk, float *x) {
    constexpr int V = NBITS - 2;
    constexpr uint64_t MASK = (1ull << V) - 1;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblk) return;
    const uint64_t w = load_block<NBITS>(in, b);
    const int e = (int)(w & 0xFF);
    f4 r = f4{0.f, 0.f, 0.f, 0.f};
    if (e != 0) {
        const int sh = e - 127 - V + 1;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int q = (int)((w >> (8 + i * V)) & MASK);
            q -= (q >> (V - 1)) << V;  // sign extension from V bits
            r[i] = ldexpf((float)q, sh);
        }
    }
    reinterpret_cast<f4 *>(x)[b] = r;
}

hipError_t launch_bfp(bool enc, int nbits, const void *src, int64_t n, void *dst, hipStream_t s) {
    const int64_t nblk = n / 4;
    if (nblk == 0) return hipSuccess;
    const dim3 g((unsigned)((nblk + 255) / 256)), t(256);
    switch (nbits) {
    case 16:
        if (enc) hipLaunchKernelGGL(bfp_encode_kernel<16>, g, t, 0, s, (const float *)src, nblk, (uint8_t *)dst);
        else hipLaunchKernelGGL(bfp_decode_kernel<16>, g, t, 0, s, (const uint8_t *)src, nblk, (float *)dst);
        break;
    case 12:
        if (enc) hipLaunchKernelGGL(bfp_encode_kernel<12>, g, t, 0, s, (const float *)src, nblk, (uint8_t *)dst);
        else hipLaunchKernelGGL(bfp_decode_kernel<12>, g, t, 0, s, (const uint8_t *)src, nblk, (float *)dst);
        break;
    case 10:
        if (enc) hipLaunchKernelGGL(bfp_encode_kernel<10>, g, t, 0, s, (const float *)src, nblk, (uint8_t *)dst);
        else hipLaunchKernelGGL(bfp_decode_kernel<10>, g, t, 0, s, (const uint8_t *)src, nblk, (float *)dst);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace chfsi
