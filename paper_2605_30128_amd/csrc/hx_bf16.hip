// Cell operator with bfloat16 MFMA operands and float accumulation (the
// CHFSI_BF16 precision of the filter's products).  Same factored local
// operator and assembly as the float/double kernels; differences:
//   * v_mfma_f32_16x16x32_bf16: each lane supplies 8 consecutive k of its
//     A row and 8 consecutive k of its B column, so the LDS block is stored
//     [real column][node] (k contiguous, padded rows) and the shared tables
//     are read in [column][k] order (K is symmetric; Phi serves the first
//     contraction, Phi^T the second).
//   * the vector block is rounded to bfloat16 (nearest even) once, after the
//     D^{-1} scaling; Phi X is accumulated in float, the 2x2 spin term is
//     applied in float and the result rounded to bfloat16 for Phi^T (.).
//   * four waves split the tile as 2 (row halves) x 2 (column halves), so
//     each B fragment fetched from L2 feeds two MFMAs.
#include "cell_common.h"

namespace chfsi {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

template <int NP, int NTW, int KS>
__device__ __forceinline__ void panel_bf16(f4 (*acc)[NTW], const __bf16 *xs, const __bf16 *B, int mh,
                                           int nt0, int lane) {
    const int cn = lane & 15, kq = 8 * (lane >> 4);
    const __bf16 *a0p = xs + (32 * mh + cn) * KS + kq;
    const __bf16 *a1p = a0p + 16 * KS;
    const __bf16 *bp = B + (size_t)(nt0 * 16 + cn) * NP + kq;
    bf8 bc[NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) bc[t] = *reinterpret_cast<const bf8 *>(bp + (size_t)t * 16 * NP);
    for (int kk = 0; kk < NP; kk += 32) {
        const int kn = kk + 32 < NP ? kk + 32 : kk;  // B fragments of the next k-step
        bf8 bn[NTW];
#pragma unroll
        for (int t = 0; t < NTW; ++t) bn[t] = *reinterpret_cast<const bf8 *>(bp + (size_t)t * 16 * NP + kn);
        bf8 a0 = *reinterpret_cast<const bf8 *>(a0p + kk);
        bf8 a1 = *reinterpret_cast<const bf8 *>(a1p + kk);
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            acc[0][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bc[t], acc[0][t], 0, 0, 0);
            acc[1][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bc[t], acc[1][t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < NTW; ++t) bc[t] = bn[t];
    }
}

template <int NP>
__global__ __launch_bounds__(kThreads) void cell_kernel_bf16(CellParams a) {
    constexpr int CB = 64, VB = 16;
    constexpr int KS = NP + 8;  // padded row (16 B multiple; rotates LDS banks)
    constexpr int NT = NP / 16, NTW = NT / 2;
    static_assert(NP % 32 == 0, "k steps of 32");
    __shared__ __attribute__((aligned(16))) __bf16 xs[CB * KS];
    __shared__ int ijk[NP];

    const int64_t nvb = (a.nvec + VB - 1) / VB;
    const int64_t t_log = xcd_remap(blockIdx.x, a.ncl * nvb);
    const int64_t ci = t_log / nvb, vb = t_log - ci * nvb;
    const int64_t e = a.cells[ci];
    const int64_t ex = e % a.ncx, ey = (e / a.ncx) % a.ncy, ez = e / (a.ncx * a.ncy);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int mh = wave & 1, nt0 = (wave >> 1) * NTW;

    for (int I = tid; I < NP; I += kThreads) {
        int i = I % a.n1, j = (I / a.n1) % a.n1, k = I / (a.n1 * a.n1);
        ijk[I] = i | (j << 8) | (k << 16);
    }
    __syncthreads();
    {
        const cf *X = reinterpret_cast<const cf *>(a.X);
        const float *dinv = (a.flags & FLAG_DINV) ? reinterpret_cast<const float *>(a.dinv) : nullptr;
        constexpr int TOT = NP * 2 * VB, ITER = (TOT + kThreads - 1) / kThreads;
        // all loads of this thread are issued before the first LDS store
        cf z[ITER];
        float sc[ITER];
#pragma unroll
        for (int u = 0; u < ITER; ++u) {
            const int idx = tid + u * kThreads;
            const int v = idx % VB, s = (idx / VB) & 1, I = idx / (2 * VB);
            const int64_t col = vb * VB + v;
            z[u] = cf{0.f, 0.f};
            sc[u] = 1.0f;
            if (idx < TOT && I < a.n && col < a.nvec) {
                const int64_t g = gnode_of(ijk[I], ex, ey, ez, a.p, a.Nx, a.Ny, a.Nz);
                z[u] = X[(2 * g + s) * a.ld + col];
                if (dinv) sc[u] = dinv[g];
            }
        }
#pragma unroll
        for (int u = 0; u < ITER; ++u) {
            const int idx = tid + u * kThreads;
            const int v = idx % VB, s = (idx / VB) & 1, I = idx / (2 * VB);
            if (idx < TOT) {
                xs[(4 * v + 2 * s) * KS + I] = (__bf16)(z[u].x * sc[u]);
                xs[(4 * v + 2 * s + 1) * KS + I] = (__bf16)(z[u].y * sc[u]);
            }
        }
    }
    __syncthreads();

    f4 y[2][NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) { y[0][t] = f4{0, 0, 0, 0}; y[1][t] = f4{0, 0, 0, 0}; }
    panel_bf16<NP, NTW, KS>(y, xs, reinterpret_cast<const __bf16 *>(a.Bk), mh, nt0, lane);
    {
        f4 tq[2][NTW];
#pragma unroll
        for (int t = 0; t < NTW; ++t) { tq[0][t] = f4{0, 0, 0, 0}; tq[1][t] = f4{0, 0, 0, 0}; }
        panel_bf16<NP, NTW, KS>(tq, xs, reinterpret_cast<const __bf16 *>(a.BphiT), mh, nt0, lane);
        const float *W = reinterpret_cast<const float *>(a.W) + (size_t)e * NP * 4;
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            int q = (nt0 + t) * 16 + (lane & 15);
            float v = W[q * 4 + 0], bx = W[q * 4 + 1], by = W[q * 4 + 2], bz = W[q * 4 + 3];
#pragma unroll
            for (int mm = 0; mm < 2; ++mm) {
                float ur = tq[mm][t][0], ui = tq[mm][t][1], dr = tq[mm][t][2], di = tq[mm][t][3];
                tq[mm][t][0] = (v + bz) * ur + bx * dr + by * di;
                tq[mm][t][1] = (v + bz) * ui + bx * di - by * dr;
                tq[mm][t][2] = bx * ur - by * ui + (v - bz) * dr;
                tq[mm][t][3] = bx * ui + by * ur + (v - bz) * di;
            }
        }
        // spin-orbit apply at the quadrature points, T += w|J| phi_a d_a: one
        // K=32 MFMA step per 8 projectors with k = (j, spin s', re|im part)
        // and A[(v, s, r)][k] = delta_{s s'} (re/im part of d_j(v))
        if ((a.flags & FLAG_NLOC) && a.cell_pair_ptr) {
            const int pb = a.cell_pair_ptr[e], pe = a.cell_pair_ptr[e + 1];
            const int r = lane & 15, vr = r >> 2, comp = r & 3, sA = comp >> 1, rA = comp & 1;
            const int kq = 8 * (lane >> 4);
            for (int pp = pb; pp < pe; ++pp) {
                const int pair = a.cell_pairs[pp];
                const int atom = a.pair_atom[pair];
                const __bf16 *wp = reinterpret_cast<const __bf16 *>(a.P) + (size_t)pair * NP * a.ldw;
                const cf *dc = reinterpret_cast<const cf *>(a.dcoef) + (size_t)atom * a.nbeta * a.ldd;
                for (int ks = 0; ks < a.ldw; ks += 32) {
                    bf8 av[2];
#pragma unroll
                    for (int mm = 0; mm < 2; ++mm) {
                        const int64_t colA = vb * VB + 4 * (2 * mh + mm) + vr;
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int j = (ks + kq) / 4 + h;
                            cf d = {0.f, 0.f};
                            if (j < a.nbeta && colA < a.nvec) d = dc[(size_t)j * a.ldd + colA];
#pragma unroll
                            for (int sp = 0; sp < 2; ++sp) {
                                float re = 0.f, im = 0.f;  // the (part = re, part = im) entries
                                if (sp == sA) {
                                    re = rA == 0 ? d.x : d.y;
                                    im = rA == 0 ? -d.y : d.x;
                                }
                                av[mm][4 * h + 2 * sp] = (__bf16)re;
                                av[mm][4 * h + 2 * sp + 1] = (__bf16)im;
                            }
                        }
                    }
#pragma unroll
                    for (int t = 0; t < NTW; ++t) {
                        const int q = (nt0 + t) * 16 + (lane & 15);
                        bf8 bv = *reinterpret_cast<const bf8 *>(wp + (size_t)q * a.ldw + ks + kq);
                        tq[0][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], bv, tq[0][t], 0, 0, 0);
                        tq[1][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1], bv, tq[1][t], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();  // every wave is done reading the gathered block
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            int q = (nt0 + t) * 16 + (lane & 15);
#pragma unroll
            for (int mm = 0; mm < 2; ++mm) {
                int row = 16 * (2 * mh + mm) + 4 * (lane >> 4);
#pragma unroll
                for (int i = 0; i < 4; ++i) xs[(row + i) * KS + q] = (__bf16)tq[mm][t][i];
            }
        }
        __syncthreads();
    }
    panel_bf16<NP, NTW, KS>(y, xs, reinterpret_cast<const __bf16 *>(a.Bphi), mh, nt0, lane);

    // colour-ordered assembly: all previous values of the lane's nodes are
    // loaded before any is written back
    cf *Y = reinterpret_cast<cf *>(a.Y);
    const float al = (float)a.alpha;
    const bool accum = (a.flags & FLAG_ACCUM) != 0;
    const int64_t col0 = vb * VB + 4 * (2 * mh) + (lane >> 4), col1 = col0 + 4;
    int64_t off[NTW];
    cf o[2][NTW][2];
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        const int J = (nt0 + t) * 16 + (lane & 15);
        off[t] = -1;
#pragma unroll
        for (int mm = 0; mm < 2; ++mm) { o[mm][t][0] = cf{0.f, 0.f}; o[mm][t][1] = cf{0.f, 0.f}; }
        if (J < a.n) {
            const int c = ijk[J];
            off[t] = (2 * gnode_of(c, ex, ey, ez, a.p, a.Nx, a.Ny, a.Nz)) * a.ld;
            if (!first_touch(c, a.p, a.px, a.py, a.pz, accum)) {
                if (col0 < a.nvec) { o[0][t][0] = Y[off[t] + col0]; o[0][t][1] = Y[off[t] + a.ld + col0]; }
                if (col1 < a.nvec) { o[1][t][0] = Y[off[t] + col1]; o[1][t][1] = Y[off[t] + a.ld + col1]; }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        if (off[t] < 0) continue;
#pragma unroll
        for (int mm = 0; mm < 2; ++mm) {
            const int64_t col = mm ? col1 : col0;
            if (col >= a.nvec) continue;
            cf v0, v1;
            v0.x = al * y[mm][t][0] + o[mm][t][0].x; v0.y = al * y[mm][t][1] + o[mm][t][0].y;
            v1.x = al * y[mm][t][2] + o[mm][t][1].x; v1.y = al * y[mm][t][3] + o[mm][t][1].y;
            Y[off[t] + col] = v0;
            Y[off[t] + a.ld + col] = v1;
        }
    }
}

template <int NP>
static hipError_t run_cell_bf16(const chfsi_ctx *c, int flags, double alpha, const void *X, void *Y,
                                int64_t nvec, int64_t ld, hipStream_t s) {
    const Mesh &m = c->m;
    const Layout &L = c->L;
    CellParams a{};
    a.X = X; a.Y = Y; a.ld = ld; a.nvec = nvec;
    a.ncx = m.ncell[0]; a.ncy = m.ncell[1];
    a.Nx = m.Nd[0]; a.Ny = m.Nd[1]; a.Nz = m.Nd[2];
    a.p = m.p; a.n1 = m.n1; a.n = m.n;
    // [column][k] views: K (symmetric), Phi rows for Phi X, Phi^T rows for Phi^T T
    a.Bk = c->P<char>(L.Kb);
    a.BphiT = c->P<char>(L.Phib);
    a.Bphi = c->P<char>(L.PhiTb);
    a.W = c->P<char>(L.W32);
    a.dinv = c->P<char>(L.Dinv32);
    a.alpha = alpha;
    a.mode = MODE_HAM;
    a.flags = flags;
    if ((flags & FLAG_NLOC) && m.npairs > 0) {
        a.cell_pair_ptr = c->P<int>(L.cell_pair_ptr);
        a.cell_pairs = c->P<int>(L.cell_pairs);
        a.pair_atom = c->P<int>(L.pair_atom);
        a.P = c->P<char>(L.WPb);
        a.ldw = L.kpad;
        a.dcoef = c->S<char>(L.dcoef);
        a.nbeta = m.nbeta;
        a.ldd = nvec;
    } else {
        a.flags &= ~FLAG_NLOC;
    }
    const int64_t nvb = (nvec + 15) / 16;
    for (int col = 0; col < 8; ++col) {
        int64_t ncl = c->colour_ptr[col + 1] - c->colour_ptr[col];
        if (ncl == 0) continue;
        a.cells = c->P<int>(L.colour_cells) + c->colour_ptr[col];
        a.ncl = ncl;
        a.px = col & 1; a.py = (col >> 1) & 1; a.pz = (col >> 2) & 1;
        hipLaunchKernelGGL(cell_kernel_bf16<NP>, dim3((unsigned)(ncl * nvb)), dim3(kThreads), 0, s, a);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t launch_cell_op_bf16(const chfsi_ctx *c, int mode, int flags, double alpha, const void *X, void *Y,
                               int64_t nvec, int64_t ld, hipStream_t s) {
    if (mode != MODE_HAM) return hipErrorInvalidValue;
    switch (c->m.npad) {
    case 32: return run_cell_bf16<32>(c, flags, alpha, X, Y, nvec, ld, s);
    case 64: return run_cell_bf16<64>(c, flags, alpha, X, Y, nvec, ld, s);
    case 128: return run_cell_bf16<128>(c, flags, alpha, X, Y, nvec, ld, s);
    case 224: return run_cell_bf16<224>(c, flags, alpha, X, Y, nvec, ld, s);
    case 352: return run_cell_bf16<352>(c, flags, alpha, X, Y, nvec, ld, s);
    case 512: return run_cell_bf16<512>(c, flags, alpha, X, Y, nvec, ld, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace chfsi
