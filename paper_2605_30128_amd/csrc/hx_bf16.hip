// Cell operator with bfloat16 MFMA operands and float accumulation (the
// CHFSI_BF16 precision of the filter's products).  Same factored local
// operator and assembly as the float/double kernels; differences:
//   * v_mfma_f32_16x16x32_bf16: each lane supplies 8 consecutive k of its
//     A row and 8 consecutive k of its B column, so the LDS block is stored
//     [real column][node] (k contiguous, padded rows) and the shared tables
//     are read in [column][k] order (K is symmetric; Phi serves the first
//     contraction, Phi^T the second).
//   * the shared tables are staged through LDS one 32-wide k-slice at a
//     time (double buffered: the next slice is fetched from L2 while the
//     current one feeds the MFMAs), so each table byte crosses L2 once per
//     workgroup and is reused by all four waves.
//   * a workgroup owns one cell and VB = CB/4 vectors (CB = 32 MH rows, MH
//     the largest row-tile count per wave for which both the H X and the
//     Phi X accumulators stay in registers); the four waves split the tile 2
//     (row halves) x 2 (column halves).
//   * the vector block is rounded to bfloat16 (nearest even) once, after the
//     D^{-1} scaling; Phi X is accumulated in float, the 2x2 spin term and
//     the spin-orbit apply are added in float/bfloat16 MFMA, and the result
//     is rounded to bfloat16 for Phi^T (.).
#include "cell_common.h"

namespace chfsi {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int kSlice = 32;       // k per MFMA step
constexpr int kSliceRow = 40;    // padded LDS row of a staged slice (bf16)

template <int NP> struct Bf16Cfg {
    // 16-row tiles per wave: both accumulator sets (2 x MH x NP/32 tiles of
    // 4 floats) must stay in the 512 registers of a lane
    static constexpr int MH = NP <= 128 ? 4 : (NP <= 224 ? 3 : (NP <= 352 ? 2 : 1));
    static constexpr int CB = 32 * MH;                // rows (real columns) per workgroup
    static constexpr int VB = CB / 4;                 // vectors per workgroup
    static constexpr int NTW = NP / 32;               // 16-column tiles per wave
    static constexpr int KS = NP + 8;                 // padded row of the block (bf16)
    static constexpr int CHUNKS = NP * (kSlice / 8);  // 16-byte pieces of one slice
    static constexpr int SITER = (CHUNKS + kThreads - 1) / kThreads;
};

// stage one k-slice [NP columns][32 k] of a [column][k] table into LDS
template <int NP>
__device__ __forceinline__ void slice_load(u4 (&r)[Bf16Cfg<NP>::SITER], const __bf16 *B, int k0) {
    using C = Bf16Cfg<NP>;
#pragma unroll
    for (int u = 0; u < C::SITER; ++u) {
        const int c = threadIdx.x + u * kThreads;
        if (c < C::CHUNKS) r[u] = *reinterpret_cast<const u4 *>(B + (size_t)(c >> 2) * NP + k0 + 8 * (c & 3));
    }
}
template <int NP>
__device__ __forceinline__ void slice_store(const u4 (&r)[Bf16Cfg<NP>::SITER], __bf16 *bs) {
    using C = Bf16Cfg<NP>;
#pragma unroll
    for (int u = 0; u < C::SITER; ++u) {
        const int c = threadIdx.x + u * kThreads;
        if (c < C::CHUNKS) *reinterpret_cast<u4 *>(bs + (c >> 2) * kSliceRow + 8 * (c & 3)) = r[u];
    }
}

// acc[mm][t] += A(rows of tile mh*MH+mm) B(columns of tile nt0+t) over k in [0, NP),
// A = as[row][k] in LDS, B = a [column][k] table staged slice by slice.
// Ends with a barrier; starts assuming the caller's barrier made `as` valid.
template <int NP>
__device__ __forceinline__ void panel_bf16(f4 (*acc)[Bf16Cfg<NP>::NTW], const __bf16 *as, const __bf16 *B,
                                           __bf16 *bs, int mh, int nt0, int lane) {
    using C = Bf16Cfg<NP>;
    constexpr int S = NP / kSlice, MH = C::MH, NTW = C::NTW, KS = C::KS;
    const int cn = lane & 15, kq = 8 * (lane >> 4);
    u4 r[C::SITER];
    slice_load<NP>(r, B, 0);
    slice_store<NP>(r, bs);
    __syncthreads();
#pragma unroll 1
    for (int s = 0; s < S; ++s) {
        __bf16 *cur = bs + (s & 1) * NP * kSliceRow;
        if (s + 1 < S) slice_load<NP>(r, B, (s + 1) * kSlice);
        bf8 a[MH];
#pragma unroll
        for (int mm = 0; mm < MH; ++mm)
            a[mm] = *reinterpret_cast<const bf8 *>(as + (16 * (mh * MH + mm) + cn) * KS + s * kSlice + kq);
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            const bf8 b = *reinterpret_cast<const bf8 *>(cur + (16 * (nt0 + t) + cn) * kSliceRow + kq);
#pragma unroll
            for (int mm = 0; mm < MH; ++mm)
                acc[mm][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mm], b, acc[mm][t], 0, 0, 0);
        }
        if (s + 1 < S) slice_store<NP>(r, bs + ((s + 1) & 1) * NP * kSliceRow);
        __syncthreads();
    }
}

template <int NP>
__global__ __launch_bounds__(kThreads) void cell_kernel_bf16(CellParams a) {
    using C = Bf16Cfg<NP>;
    constexpr int CB = C::CB, VB = C::VB, MH = C::MH, NTW = C::NTW, KS = C::KS;
    static_assert(NP % 32 == 0, "k steps of 32");
    __shared__ __attribute__((aligned(16))) __bf16 xs[CB * KS];
    __shared__ __attribute__((aligned(16))) __bf16 bs[2 * NP * kSliceRow];
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
        // gather in parts of the vector block so that all loads of a part
        // are in flight together
        const cf *X = reinterpret_cast<const cf *>(a.X);
        const float *dinv = (a.flags & FLAG_DINV) ? reinterpret_cast<const float *>(a.dinv) : nullptr;
        constexpr int NH = VB % 4 == 0 ? 4 : 2, HV = VB / NH, TOT = NP * 2 * HV, ITER = (TOT + kThreads - 1) / kThreads;
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            cf z[ITER];
            float sc[ITER];
#pragma unroll
            for (int u = 0; u < ITER; ++u) {
                const int idx = tid + u * kThreads;
                const int v = h * HV + idx % HV, s = (idx / HV) & 1, I = idx / (2 * HV);
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
                const int v = h * HV + idx % HV, s = (idx / HV) & 1, I = idx / (2 * HV);
                if (idx < TOT) {
                    xs[(4 * v + 2 * s) * KS + I] = (__bf16)(z[u].x * sc[u]);
                    xs[(4 * v + 2 * s + 1) * KS + I] = (__bf16)(z[u].y * sc[u]);
                }
            }
        }
    }
    __syncthreads();

    f4 y[MH][NTW], tq[MH][NTW];
#pragma unroll
    for (int mm = 0; mm < MH; ++mm)
#pragma unroll
        for (int t = 0; t < NTW; ++t) { y[mm][t] = f4{0, 0, 0, 0}; tq[mm][t] = f4{0, 0, 0, 0}; }
    panel_bf16<NP>(y, xs, reinterpret_cast<const __bf16 *>(a.Bk), bs, mh, nt0, lane);
    panel_bf16<NP>(tq, xs, reinterpret_cast<const __bf16 *>(a.BphiT), bs, mh, nt0, lane);
    {
        const float *W = reinterpret_cast<const float *>(a.W) + (size_t)e * NP * 4;
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            const int q = (nt0 + t) * 16 + (lane & 15);
            const float v = W[q * 4 + 0], bx = W[q * 4 + 1], by = W[q * 4 + 2], bz = W[q * 4 + 3];
#pragma unroll
            for (int mm = 0; mm < MH; ++mm) {
                const float ur = tq[mm][t][0], ui = tq[mm][t][1], dr = tq[mm][t][2], di = tq[mm][t][3];
                tq[mm][t][0] = (v + bz) * ur + bx * dr + by * di;
                tq[mm][t][1] = (v + bz) * ui + bx * di - by * dr;
                tq[mm][t][2] = bx * ur - by * ui + (v - bz) * dr;
                tq[mm][t][3] = bx * ui + by * ur + (v - bz) * di;
            }
        }
        // spin-orbit apply at the quadrature points, T += w|J| phi_a d_a: K=32
        // MFMA steps over k = (j, spin s', re|im part) with
        // A[(v, s, r)][k] = delta_{s s'} (re/im part of d_j(v))
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
                    bf8 av[MH];
#pragma unroll
                    for (int mm = 0; mm < MH; ++mm) {
                        const int64_t colA = vb * VB + 4 * (mh * MH + mm) + vr;
#pragma unroll
                        for (int hh = 0; hh < 2; ++hh) {
                            const int j = (ks + kq) / 4 + hh;
                            cf d = {0.f, 0.f};
                            if (j < a.nbeta && colA < a.nvec) d = dc[(size_t)j * a.ldd + colA];
#pragma unroll
                            for (int sp = 0; sp < 2; ++sp) {
                                float re = 0.f, im = 0.f;  // the (part = re, part = im) entries
                                if (sp == sA) {
                                    re = rA == 0 ? d.x : d.y;
                                    im = rA == 0 ? -d.y : d.x;
                                }
                                av[mm][4 * hh + 2 * sp] = (__bf16)re;
                                av[mm][4 * hh + 2 * sp + 1] = (__bf16)im;
                            }
                        }
                    }
#pragma unroll
                    for (int t = 0; t < NTW; ++t) {
                        const int q = (nt0 + t) * 16 + (lane & 15);
                        const bf8 bv = *reinterpret_cast<const bf8 *>(wp + (size_t)q * a.ldw + ks + kq);
#pragma unroll
                        for (int mm = 0; mm < MH; ++mm)
                            tq[mm][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mm], bv, tq[mm][t], 0, 0, 0);
                    }
                }
            }
        }
        // the panels ended with a barrier: the gathered block is free
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            const int q = (nt0 + t) * 16 + (lane & 15);
#pragma unroll
            for (int mm = 0; mm < MH; ++mm) {
                const int row = 16 * (mh * MH + mm) + 4 * (lane >> 4);
#pragma unroll
                for (int i = 0; i < 4; ++i) xs[(row + i) * KS + q] = (__bf16)tq[mm][t][i];
            }
        }
        __syncthreads();
    }
    panel_bf16<NP>(y, xs, reinterpret_cast<const __bf16 *>(a.Bphi), bs, mh, nt0, lane);

    // colour-ordered assembly: the previous values of the lane's nodes are
    // loaded (per row tile) before they are written back
    cf *Y = reinterpret_cast<cf *>(a.Y);
    const float al = (float)a.alpha;
    const bool accum = (a.flags & FLAG_ACCUM) != 0, init = (a.flags & FLAG_INIT) != 0;
    int64_t off[NTW], row[NTW];
    bool rd[NTW], it[NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        const int J = (nt0 + t) * 16 + (lane & 15);
        off[t] = -1;
        row[t] = 0;
        rd[t] = false;
        it[t] = false;
        if (J < a.n) {
            const int c = ijk[J];
            row[t] = 2 * gnode_of(c, ex, ey, ez, a.p, a.Nx, a.Ny, a.Nz);
            off[t] = row[t] * a.ld;
            rd[t] = !first_touch(c, a.p, a.px, a.py, a.pz, accum);
            it[t] = init && !rd[t];
        }
    }
#pragma unroll
    for (int mm = 0; mm < MH; ++mm) {
        const int64_t col = vb * VB + 4 * (mh * MH + mm) + (lane >> 4);
        if (col >= a.nvec) continue;
        cf o[NTW][2];
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            o[t][0] = cf{0.f, 0.f};
            o[t][1] = cf{0.f, 0.f};
            if (rd[t]) {
                o[t][0] = Y[off[t] + col];
                o[t][1] = Y[off[t] + a.ld + col];
            } else if (it[t]) {
                o[t][0] = init_terms<cf>(a, row[t], off[t] + col, col);
                o[t][1] = init_terms<cf>(a, row[t] + 1, off[t] + a.ld + col, col);
            }
        }
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            if (off[t] < 0) continue;
            cf v0, v1;
            v0.x = al * y[mm][t][0] + o[t][0].x; v0.y = al * y[mm][t][1] + o[t][0].y;
            v1.x = al * y[mm][t][2] + o[t][1].x; v1.y = al * y[mm][t][3] + o[t][1].y;
            Y[off[t] + col] = v0;
            Y[off[t] + a.ld + col] = v1;
        }
    }
}

template <int NP>
static hipError_t run_cell_bf16(const chfsi_ctx *c, int flags, double alpha, const void *X, void *Y,
                                int64_t nvec, int64_t ld, hipStream_t s, const InitTerms *init) {
    const Mesh &m = c->m;
    const Layout &L = c->L;
    CellParams a{};
    if (flags & FLAG_INIT) {
        if (!init || !init->Zk || !init->R || (flags & FLAG_ACCUM)) return hipErrorInvalidValue;
        set_init(a, *init);
    }
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
    constexpr int VB = Bf16Cfg<NP>::VB;
    const int64_t nvb = (nvec + VB - 1) / VB;
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
                               int64_t nvec, int64_t ld, hipStream_t s, const InitTerms *init) {
    if (mode != MODE_HAM) return hipErrorInvalidValue;
    switch (c->m.npad) {
    case 32: return run_cell_bf16<32>(c, flags, alpha, X, Y, nvec, ld, s, init);
    case 64: return run_cell_bf16<64>(c, flags, alpha, X, Y, nvec, ld, s, init);
    case 128: return run_cell_bf16<128>(c, flags, alpha, X, Y, nvec, ld, s, init);
    case 224: return run_cell_bf16<224>(c, flags, alpha, X, Y, nvec, ld, s, init);
    case 352: return run_cell_bf16<352>(c, flags, alpha, X, Y, nvec, ld, s, init);
    case 512: return run_cell_bf16<512>(c, flags, alpha, X, Y, nvec, ld, s, init);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace chfsi
