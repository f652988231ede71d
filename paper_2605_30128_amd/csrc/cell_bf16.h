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
//   * a workgroup of eight waves owns one cell and VB = CB/4 vectors (CB =
//     64 MH rows, MH the largest row-tile count per wave for which both the
//     H X and the Phi X accumulators stay in the registers of two waves per
//     SIMD); the waves split the tile 4 (row groups) x 2 (column halves), so
//     each staged table slice feeds 32 vectors and each SIMD has a second
//     wave to issue MFMAs while one waits.
//   * the vector block is rounded to bfloat16 (nearest even) once, after the
//     D^{-1} scaling; Phi X is accumulated in float, the 2x2 spin term and
//     the spin-orbit apply are added in float/bfloat16 MFMA, and the result
//     is rounded to bfloat16 for Phi^T (.).
#pragma once

#include "cell_common.h"

namespace chfsi {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int kSlice = 32;       // k per MFMA step
constexpr int kSliceRow = 32;    // LDS row of a staged slice (bf16): one column's 32 k, four 16-byte chunks

// 16-byte chunk q (k = 8q..8q+7) of column col sits at position q ^ ((col >> 2) & 3)
// of the column's row: the 16 lanes of an MFMA B read (16 columns, one chunk)
// and the 16 lanes of a slice store (4 columns x 4 chunks) then fall on
// disjoint LDS banks without padding
__device__ __forceinline__ int slice_pos(int col, int q) { return col * kSliceRow + 8 * (q ^ ((col >> 2) & 3)); }

constexpr int kBfWaves = 8;                  // waves per workgroup: row groups x column groups
constexpr int kBfThreads = 64 * kBfWaves;

template <int NP> struct Bf16Cfg {
    // 16-row tiles per wave: the accumulators (MH x NTW tiles of 4 floats)
    // and the bfloat16 copy of T must fit the 256 registers a lane has with
    // two waves per SIMD
    static constexpr int MH = NP <= 128 ? 4 : (NP <= 224 ? 3 : 2);
    // row groups x column groups of waves: at NP = 512 (p = 7) a wave owns
    // 2 row tiles x 8 column tiles; each table fragment it reads from LDS
    // then feeds two MFMAs (4 row groups of one tile each and 16 column
    // tiles took 1.3x longer per panel); 4 x 2 elsewhere
    static constexpr int RG = NP == 512 ? 2 : 4;
    static constexpr int CG = kBfWaves / RG;          // column groups
    static constexpr int CB = 16 * MH * RG;           // rows (real columns) per workgroup
    static constexpr int VB = CB / 4;                 // vectors per workgroup
    static constexpr int NTW = NP / (16 * CG);        // 16-column tiles per wave
    static_assert(NTW * 16 * CG == NP, "column tiles split evenly");
    static constexpr int KS = NP + 8;                 // padded row of the block (bf16)
    static constexpr int CHUNKS = NP * (kSlice / 8);  // 16-byte pieces of one slice
    static constexpr int SITER = (CHUNKS + kBfThreads - 1) / kBfThreads;
    static constexpr int SCOLS = SITER * kBfThreads / 4;  // columns of an LDS slice buffer (>= NP)
};

// stage one k-slice [NP columns][32 k] of a [column][k] table into LDS.
// The loads are unconditional (a thread past the slice reloads its last
// chunk): without branches around them the compiler can wait for exactly
// the loads a slice needs, so the prefetch two slices ahead stays in flight.
template <int NP>
__device__ __forceinline__ void slice_load(u4 (&r)[Bf16Cfg<NP>::SITER], const __bf16 *B, int k0, int ldb = NP) {
    using C = Bf16Cfg<NP>;
#pragma unroll
    for (int u = 0; u < C::SITER; ++u) {
        const int c = min((int)threadIdx.x + u * kBfThreads, C::CHUNKS - 1);
        r[u] = *reinterpret_cast<const u4 *>(B + (size_t)(c >> 2) * ldb + k0 + 8 * (c & 3));
    }
}
// The LDS slice buffers have SCOLS >= NP columns, so every thread stores all
// its chunks without a branch (chunks past the slice land in the unread
// padding columns).
template <int NP>
__device__ __forceinline__ void slice_store(const u4 (&r)[Bf16Cfg<NP>::SITER], __bf16 *bs) {
    using C = Bf16Cfg<NP>;
#pragma unroll
    for (int u = 0; u < C::SITER; ++u) {
        const int c = threadIdx.x + u * kBfThreads;
        *reinterpret_cast<u4 *>(bs + slice_pos(c >> 2, c & 3)) = r[u];
    }
}

// MFMAs of one staged slice: acc[mm][t] += A(rows of tile mh*MH+mm, k of
// slice s) B(columns of tile nt0+t, same k)
template <int NP>
__device__ __forceinline__ void slice_mfma(f4 (*acc)[Bf16Cfg<NP>::NTW], const __bf16 *as, const __bf16 *cur,
                                           int s, int mh, int nt0, int lane) {
    using C = Bf16Cfg<NP>;
    constexpr int MH = C::MH, NTW = C::NTW, KS = C::KS;
    const int cn = lane & 15, kq = 8 * (lane >> 4);
    bf8 a[MH];
#pragma unroll
    for (int mm = 0; mm < MH; ++mm)
        a[mm] = *reinterpret_cast<const bf8 *>(as + (16 * (mh * MH + mm) + cn) * KS + s * kSlice + kq);
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        const bf8 b = *reinterpret_cast<const bf8 *>(cur + slice_pos(16 * (nt0 + t) + cn, kq >> 3));
#pragma unroll
        for (int mm = 0; mm < MH; ++mm)
            acc[mm][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mm], b, acc[mm][t], 0, 0, 0);
    }
}

// One iteration of the slice pipeline: slice s is in LDS buffer s&1 and
// slice s+1 in registers `nxt`; slice s+2 is fetched into `frees` (free
// since its slice went to LDS one iteration earlier), so every slice has two
// iterations to arrive from L2.
template <int NP, class Hook>
__device__ __forceinline__ void slice_step(f4 (*acc)[Bf16Cfg<NP>::NTW], const __bf16 *as, const __bf16 *B,
                                           __bf16 *bs, int s, u4 (&frees)[Bf16Cfg<NP>::SITER],
                                           const u4 (&nxt)[Bf16Cfg<NP>::SITER], int mh, int nt0, int lane,
                                           Hook &hook) {
    constexpr int S = NP / kSlice;
    if (s + 2 < S) slice_load<NP>(frees, B, (s + 2) * kSlice);
    if (s == (S > 2 ? S - 3 : 0)) hook();
    slice_mfma<NP>(acc, as, bs + (s & 1) * Bf16Cfg<NP>::SCOLS * kSliceRow, s, mh, nt0, lane);
    if (s + 1 < S) slice_store<NP>(nxt, bs + ((s + 1) & 1) * Bf16Cfg<NP>::SCOLS * kSliceRow);
    __syncthreads();
}

struct NoHook {
    __device__ void operator()() const {}
};

// acc[mm][t] += A(rows of tile mh*MH+mm) B(columns of tile nt0+t) over k in [0, NP),
// A = as[row][k] in LDS, B = a [column][k] table staged slice by slice.
// Ends with a barrier; starts assuming the caller's barrier made `as` valid.
// `hook` runs once, right after the last slice's load is issued: loads it
// issues complete in order after every slice, so the panel never waits for them.
template <int NP, class Hook = NoHook>
__device__ __forceinline__ void panel_bf16(f4 (*acc)[Bf16Cfg<NP>::NTW], const __bf16 *as, const __bf16 *B,
                                           __bf16 *bs, int mh, int nt0, int lane, Hook &&hook = Hook{}) {
    using C = Bf16Cfg<NP>;
    constexpr int S = NP / kSlice;
    u4 r0[C::SITER], r1[C::SITER];
    slice_load<NP>(r0, B, 0);
    if (S > 1) slice_load<NP>(r1, B, kSlice);
    slice_store<NP>(r0, bs);
    __syncthreads();
    // fully unrolled: every load and wait of the pipeline is static
#pragma unroll
    for (int s = 0; s < S; s += 2) {
        slice_step<NP>(acc, as, B, bs, s, r0, r1, mh, nt0, lane, hook);
        if (s + 1 < S) slice_step<NP>(acc, as, B, bs, s + 1, r1, r0, mh, nt0, lane, hook);
    }
}

// Rounds of the assembly: the fewest that split the VB vectors into rounds of
// whole row tiles (four vectors each) whose [node][spin][vector] staging fits
// `bytes` of LDS and whose vector count divides the thread count (so a
// thread keeps its spin and columns across its pieces of a round).
constexpr int assembly_rounds(int np, int vb, int bytes) {
    for (int n = 1; n <= vb; ++n) {
        const int vr = vb / n;
        if (vb % n == 0 && vr % 4 == 0 && kBfThreads % vr == 0 && np * (4 * vr + 4) * 4 <= bytes) return n;
    }
    return 0;
}

// Two consecutive complex64 values of a row (one 16-byte load when the row
// start keeps them aligned; the second is zero past the last column).
__device__ __forceinline__ f4 load_pair(const cf *p, bool even_ld, bool two) {
    if (even_ld && two) return *reinterpret_cast<const f4 *>(p);
    const cf z0 = p[0];
    const cf z1 = two ? p[1] : cf{0.f, 0.f};
    return f4{z0.x, z0.y, z1.x, z1.y};
}

template <int NP, bool EPI>
__global__ __launch_bounds__(kBfThreads) void cell_kernel_bf16(CellParams a, EpiArgs ep) {
    using C = Bf16Cfg<NP>;
    constexpr int CB = C::CB, VB = C::VB, MH = C::MH, NTW = C::NTW, KS = C::KS;
    static_assert(NP % 32 == 0, "k steps of 32");
    // the gathered block and the table slices; after the last panel the
    // whole area stages the result for the assembly
    constexpr int XSB = CB * KS * 2, BSB = 2 * C::SCOLS * kSliceRow * 2;
    __shared__ __attribute__((aligned(16))) char smem[XSB + BSB];
    __bf16 *xs = reinterpret_cast<__bf16 *>(smem), *bs = reinterpret_cast<__bf16 *>(smem + XSB);
    __shared__ int ijk[NP];
    __shared__ int grow[NP];     // 2 g: first spinor row of the cell's node I
    __shared__ float gsc[NP];    // D^-1 of node I (1 without FLAG_DINV)
    __shared__ __attribute__((aligned(16))) float ws[NP * 4];  // w|J| (V, Bx, By, Bz) of the cell

    const int64_t nvb = (a.nvec + VB - 1) / VB;
    const int64_t t_log = xcd_remap(blockIdx.x, a.ncl * nvb);
    const int64_t ci = t_log / nvb, vb = t_log - ci * nvb;
    const int64_t e = a.cells[ci];
    const int64_t ex = e % a.ncx, ey = (e / a.ncx) % a.ncy, ez = e / (a.ncx * a.ncy);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int mh = wave % C::RG, nt0 = (wave / C::RG) * NTW;

    // node tables of the cell (arithmetic only); its D^-1 and w|J| (V, B)
    // values are fetched now but stored to LDS only after the gather's loads
    // are issued, so their latency overlaps the gather
    static_assert(NP <= kBfThreads, "one thread per node of the cell");
    float dv = 1.0f;
    f4 wv = f4{0.f, 0.f, 0.f, 0.f};
    if (tid < NP) {
        const int I = tid;
        const int i = I % a.n1, j = (I / a.n1) % a.n1, k = I / (a.n1 * a.n1);
        const int c = i | (j << 8) | (k << 16);
        ijk[I] = c;
        int64_t g = 0;
        if (I < a.n) g = gnode_of(c, ex, ey, ez, a.p, a.Nx, a.Ny, a.Nz);
        grow[I] = (int)(2 * g);
        if ((a.flags & FLAG_DINV) && I < a.n) dv = reinterpret_cast<const float *>(a.dinv)[g];
        wv = reinterpret_cast<const f4 *>(a.W)[(size_t)e * NP + I];
    }
    __syncthreads();
    {
        // gather: a task is (vector v, spin s, eight consecutive nodes): eight
        // 8-byte row loads (the 16 vectors of a lane group read a 128-byte
        // row piece), the loads of a half of the vectors issued at once and
        // without branches (a load past the block or the cell reads element 0
        // and is discarded); the eight real parts and the eight imaginary
        // parts then go to LDS as one 16-byte store each.  With rows KS apart the 16
        // stores of a pass fall on disjoint banks at NP = 352.
        const cf *X = reinterpret_cast<const cf *>(a.X);
        constexpr int NH = VB >= 32 ? 2 : 1, HV = VB / NH, NB8 = NP / 8;
        constexpr int TASKS = HV * 2 * NB8, ITER = (TASKS + kBfThreads - 1) / kBfThreads;
        static_assert(NP % 8 == 0 && (KS * 2) % 16 == 0, "16-byte node pieces");
        // both halves' loads are in flight before the first conversion
        cf z[NH][ITER][8];
#pragma unroll
        for (int h = 0; h < NH; ++h) {
#pragma unroll
            for (int u = 0; u < ITER; ++u) {
                const int idx = tid + u * kBfThreads;
                const int v = h * HV + idx % HV, sp = (idx / HV) & 1, b = min(idx / (2 * HV), NB8 - 1);
                const int64_t col = vb * VB + v;
                const bool ok = idx < TASKS && col < a.nvec;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int I = 8 * b + k;
                    const bool valid = ok && I < a.n;
                    const cf t = X[valid ? (int64_t)(grow[I] + sp) * a.ld + col : 0];
                    z[h][u][k] = valid ? t : cf{0.f, 0.f};
                }
            }
        }
        if (tid < NP) {
            gsc[tid] = dv;
            reinterpret_cast<f4 *>(ws)[tid] = wv;
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < NH; ++h) {
#pragma unroll
            for (int u = 0; u < ITER; ++u) {
                const int idx = tid + u * kBfThreads;
                const int v = h * HV + idx % HV, sp = (idx / HV) & 1, b = idx / (2 * HV);
                if (idx >= TASKS) continue;
                bf8 re, im;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const float sc = gsc[8 * b + k];
                    re[k] = (__bf16)(z[h][u][k].x * sc);
                    im[k] = (__bf16)(z[h][u][k].y * sc);
                }
                *reinterpret_cast<bf8 *>(xs + (4 * v + 2 * sp) * KS + 8 * b) = re;
                *reinterpret_cast<bf8 *>(xs + (4 * v + 2 * sp + 1) * KS + 8 * b) = im;
            }
        }
    }
    __syncthreads();

    // T = (w|J| (V + B.sigma)) Phi X (+ spin-orbit term) is formed first and
    // kept in registers as bfloat16 while K X is accumulated, so only one
    // float accumulator set is live at a time
    bf4 tp[MH][NTW];
    {
        f4 tq[MH][NTW];
#pragma unroll
        for (int mm = 0; mm < MH; ++mm)
#pragma unroll
            for (int t = 0; t < NTW; ++t) tq[mm][t] = f4{0, 0, 0, 0};
        // spin-orbit apply at the quadrature points, T += w|J| phi_a d_a: K=32
        // MFMA steps over k = (j, spin s', re|im part) with
        // A[(v, s, r)][k] = delta_{s s'} (re/im part of d_j(v)); the pair's
        // [q][k] table slice is staged through LDS like the panels' tables.
        // A unit is one 32-wide k slice of one pair; each unit's table slice
        // and coefficients are loaded one unit ahead (the first during the
        // Phi X panel, after its last table slice), so their latency overlaps
        // the previous unit's MFMAs.
        const bool soc = (a.flags & FLAG_NLOC) && a.cell_pair_ptr;
        const int pb = soc ? a.cell_pair_ptr[e] : 0, pe = soc ? a.cell_pair_ptr[e + 1] : 0;
        const int nks = soc ? a.ldw / kSlice : 1, units = (pe - pb) * nks;
        const int vr = (lane & 15) >> 2, comp = lane & 3, sA = comp >> 1, rA = comp & 1;
        const int cn = lane & 15, kq = 8 * (lane >> 4);
        u4 rs[C::SITER];
        cf dd[MH][2];
        auto load_unit = [&](int u) {
            const int pair = a.cell_pairs[pb + u / nks], ks = (u % nks) * kSlice;
            const int atom = a.pair_atom[pair];
            slice_load<NP>(rs, reinterpret_cast<const __bf16 *>(a.P) + (size_t)pair * NP * a.ldw, ks, a.ldw);
            const cf *dc = reinterpret_cast<const cf *>(a.dcoef) + (size_t)atom * a.nbeta * a.ldd;
#pragma unroll
            for (int mm = 0; mm < MH; ++mm) {
                const int64_t colA = vb * VB + 4 * (mh * MH + mm) + vr;
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    const int j = (ks + kq) / 4 + hh;
                    const bool ok = j < a.nbeta && colA < a.nvec;
                    const cf d = dc[ok ? (size_t)j * a.ldd + colA : 0];
                    dd[mm][hh] = ok ? d : cf{0.f, 0.f};
                }
            }
        };
        panel_bf16<NP>(tq, xs, reinterpret_cast<const __bf16 *>(a.BphiT), bs, mh, nt0, lane, [&]() {
            if (units > 0) load_unit(0);
        });
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            const int q = (nt0 + t) * 16 + (lane & 15);
            const f4 w = reinterpret_cast<const f4 *>(ws)[q];
            const float v = w[0], bx = w[1], by = w[2], bz = w[3];
#pragma unroll
            for (int mm = 0; mm < MH; ++mm) {
                const float ur = tq[mm][t][0], ui = tq[mm][t][1], dr = tq[mm][t][2], di = tq[mm][t][3];
                tq[mm][t][0] = (v + bz) * ur + bx * dr + by * di;
                tq[mm][t][1] = (v + bz) * ui + bx * di - by * dr;
                tq[mm][t][2] = bx * ur - by * ui + (v - bz) * dr;
                tq[mm][t][3] = bx * ui + by * ur + (v - bz) * di;
            }
        }
        for (int u = 0; u < units; ++u) {
            bf8 av[MH];
#pragma unroll
            for (int mm = 0; mm < MH; ++mm) {
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    const cf d = dd[mm][hh];
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
            // the previous unit's MFMAs (or panel 1) ended with a barrier: the slice buffer is free
            slice_store<NP>(rs, bs);
            if (u + 1 < units) load_unit(u + 1);
            __syncthreads();
#pragma unroll
            for (int t = 0; t < NTW; ++t) {
                const bf8 bv = *reinterpret_cast<const bf8 *>(bs + slice_pos(16 * (nt0 + t) + cn, kq >> 3));
#pragma unroll
                for (int mm = 0; mm < MH; ++mm)
                    tq[mm][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mm], bv, tq[mm][t], 0, 0, 0);
            }
            __syncthreads();
        }
#pragma unroll
        for (int mm = 0; mm < MH; ++mm)
#pragma unroll
            for (int t = 0; t < NTW; ++t)
                tp[mm][t] = bf4{(__bf16)tq[mm][t][0], (__bf16)tq[mm][t][1], (__bf16)tq[mm][t][2],
                                (__bf16)tq[mm][t][3]};
    }
    f4 y[MH][NTW];
#pragma unroll
    for (int mm = 0; mm < MH; ++mm)
#pragma unroll
        for (int t = 0; t < NTW; ++t) y[mm][t] = f4{0, 0, 0, 0};
    panel_bf16<NP>(y, xs, reinterpret_cast<const __bf16 *>(a.Bk), bs, mh, nt0, lane);
    // the panel ended with a barrier: the gathered block is free for T
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        const int q = (nt0 + t) * 16 + (lane & 15);
#pragma unroll
        for (int mm = 0; mm < MH; ++mm) {
            const int row = 16 * (mh * MH + mm) + 4 * (lane >> 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) xs[(row + i) * KS + q] = tp[mm][t][i];
        }
    }
    __syncthreads();
    // colour-ordered assembly through LDS, in NR rounds of VR vectors: the
    // waves owning the round's row tiles write their results as
    // [node][spin][vector] complex values, then all threads update Y in
    // 16-byte pieces (two vectors of one spinor row), so every read-back and
    // store covers whole rows of the vector block.  A thread's pieces of a
    // round share its spin and its two columns (kBfThreads is a multiple of
    // VR) and differ in the node.
    constexpr int NR = assembly_rounds(NP, VB, XSB + BSB);
    constexpr int VR = VB / NR, TPR = VR / 4;        // vectors and row tiles per round
    constexpr int OS = 4 * VR + 4;                  // floats per node (padded to 16 bytes)
    static_assert(NP * OS * 4 <= XSB + BSB && VR % 2 == 0, "assembly staging fits the LDS area");
    static_assert(kBfThreads % VR == 0, "a thread keeps its columns across pieces");
    constexpr int PIECES = NP * VR, PIT = (PIECES + kBfThreads - 1) / kBfThreads;
    panel_bf16<NP>(y, xs, reinterpret_cast<const __bf16 *>(a.Bphi), bs, mh, nt0, lane);
    cf *Y = reinterpret_cast<cf *>(a.Y);
    const bool accum = (a.flags & FLAG_ACCUM) != 0, even_ld = (a.ld & 1) == 0;
    const int rem = tid % VR, sp = rem / (VR / 2), q = rem - sp * (VR / 2), J0 = tid / VR;
    // read-backs of the pieces of round r (nodes an earlier colour wrote),
    // issued before the round's staging.  (Issued during the last panel they
    // would delay its table-slice waits, which count loads in issue order;
    // issued a round ahead they spill.)
    [[maybe_unused]] f4 rb[EPI ? 1 : PIT];
    [[maybe_unused]] auto readback = [&](int r) {
        const int64_t col = vb * VB + r * VR + 2 * q;
        const bool colok = col < a.nvec, two = col + 1 < a.nvec;
#pragma unroll
        for (int u = 0; u < PIT; ++u) {
            const int J = J0 + u * (kBfThreads / VR);
            rb[u] = f4{0.f, 0.f, 0.f, 0.f};
            if (J < a.n && colok && !first_touch(ijk[J], a.p, a.px, a.py, a.pz, accum))
                rb[u] = load_pair(Y + (int64_t)(grow[J] + sp) * a.ld + col, even_ld, two);
        }
    };
    float *ob = reinterpret_cast<float *>(smem);
    const float al = (float)a.alpha;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        // panel 3 (or the previous round) ended with a barrier
        if constexpr (!EPI) readback(r);
#pragma unroll
        for (int mm = 0; mm < MH; ++mm) {
            const int rt = mh * MH + mm - r * TPR;
            if (rt < 0 || rt >= TPR) continue;
            const int v = 4 * rt + (lane >> 4);
#pragma unroll
            for (int t = 0; t < NTW; ++t) {
                const int J = (nt0 + t) * 16 + (lane & 15);
                float *o = ob + J * OS + 2 * v;
                *reinterpret_cast<float2 *>(o) = float2{y[mm][t][0], y[mm][t][1]};
                *reinterpret_cast<float2 *>(o + 2 * VR) = float2{y[mm][t][2], y[mm][t][3]};
            }
        }
        __syncthreads();
        // with the recurrence terms (EPI) a first-touch piece reads Z_k,
        // Z_{k-1} and R, so the loads go four pieces at a time; otherwise the
        // round's read-backs are already in flight
        constexpr int PG = EPI ? 4 : PIT;
        const int64_t col = vb * VB + r * VR + 2 * q;
        const bool colok = col < a.nvec, two = col + 1 < a.nvec, wide = even_ld && two;
        [[maybe_unused]] double lam2[2] = {0.0, 0.0};
        if constexpr (EPI) {
            if (colok) {
                lam2[0] = ep.lam[col];
                if (two) lam2[1] = ep.lam[col + 1];
            }
        }
#pragma unroll
        for (int u0 = 0; u0 < PIT; u0 += PG) {
            f4 old[PG];
            [[maybe_unused]] f4 zm[EPI ? PG : 1];
            [[maybe_unused]] double rr[EPI ? PG : 1][4];
            [[maybe_unused]] bool ft[EPI ? PG : 1];
#pragma unroll
            for (int uu = 0; uu < PG; ++uu) {
                const int J = J0 + (u0 + uu) * (kBfThreads / VR);
                const bool valid = u0 + uu < PIT && J < a.n && colok;
                if constexpr (!EPI) {
                    old[uu] = rb[u0 + uu];
                } else {
                    old[uu] = f4{0.f, 0.f, 0.f, 0.f};
                    const int64_t o = (int64_t)(grow[valid ? J : 0] + sp) * a.ld + col;
                    zm[uu] = f4{0.f, 0.f, 0.f, 0.f};
                    ft[uu] = valid && first_touch(ijk[J], a.p, a.px, a.py, a.pz, accum);
                    if (valid) {
                        // the read-back, or Z_k (the input block) at a first touch
                        const cf *src = ft[uu] ? reinterpret_cast<const cf *>(a.X) + o : Y + o;
                        old[uu] = load_pair(src, even_ld, two);
                    }
                    if (ft[uu]) {
                        if (ep.Zkm) zm[uu] = load_pair(reinterpret_cast<const cf *>(ep.Zkm) + o, even_ld, two);
                        const cd *R = ep.R + (int64_t)(grow[J] + sp) * ep.ldr + col;
                        const cd r0 = R[0], r1 = two ? R[1] : cd{0.0, 0.0};
                        rr[uu][0] = r0.x; rr[uu][1] = r0.y; rr[uu][2] = r1.x; rr[uu][3] = r1.y;
                    }
                }
            }
            // all of the group's results are formed before its first store:
            // a store's data registers may not be overwritten by an ALU or
            // LDS instruction before the store has completed, so forming the
            // next piece in the registers of the previous one's store would
            // wait for that store's round trip, piece by piece
            f4 nv[PG];
#pragma unroll
            for (int uu = 0; uu < PG; ++uu) {
                const int J = min(J0 + (u0 + uu) * (kBfThreads / VR), NP - 1);
                if constexpr (EPI) {
                    if (ft[uu]) {
                        // beta Z_k + gamma Z_{k-1} + alpha lam R in double, rounded once
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            old[uu][i] = (float)(ep.beta * (double)old[uu][i] + ep.gamma * (double)zm[uu][i] +
                                                 a.alpha * lam2[i >> 1] * rr[uu][i]);
                    }
                }
                const f4 yv = *reinterpret_cast<const f4 *>(ob + J * OS + sp * 2 * VR + 4 * q);
                nv[uu] = f4{al * yv[0] + old[uu][0], al * yv[1] + old[uu][1], al * yv[2] + old[uu][2],
                            al * yv[3] + old[uu][3]};
            }
#pragma unroll
            for (int uu = 0; uu < PG; ++uu) asm volatile("" : "+v"(nv[uu]));
#pragma unroll
            for (int uu = 0; uu < PG; ++uu) {
                const int J = J0 + (u0 + uu) * (kBfThreads / VR);
                if (u0 + uu >= PIT || J >= a.n || !colok) continue;
                cf *dst = Y + (int64_t)(grow[J] + sp) * a.ld + col;
                if (wide) {
                    *reinterpret_cast<f4 *>(dst) = nv[uu];
                } else {
                    dst[0] = cf{nv[uu][0], nv[uu][1]};
                    if (two) dst[1] = cf{nv[uu][2], nv[uu][3]};
                }
            }
        }
        if (r + 1 < NR) __syncthreads();
    }
}

template <int NP, bool EPI>
static hipError_t run_cell_bf16(const chfsi_ctx *c, int flags, double alpha, const void *X, void *Y,
                                int64_t nvec, int64_t ld, hipStream_t s, const EpiArgs *epi) {
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
    if (EPI != ((flags & FLAG_EPI) != 0) || (EPI && !epi)) return hipErrorInvalidValue;
    const EpiArgs ep = EPI ? *epi : EpiArgs{};
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
        hipLaunchKernelGGL((cell_kernel_bf16<NP, EPI>), dim3((unsigned)(ncl * nvb)), dim3(kBfThreads), 0, s, a, ep);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

// one translation unit per EPI value: instantiating both kernels in one unit
// changed the register allocation of both (spills at NP = 352)
template <bool EPI>
hipError_t dispatch_cell_bf16(const chfsi_ctx *c, int flags, double alpha, const void *X, void *Y, int64_t nvec,
                              int64_t ld, hipStream_t s, const EpiArgs *epi) {
    switch (c->m.npad) {
    case 32: return run_cell_bf16<32, EPI>(c, flags, alpha, X, Y, nvec, ld, s, epi);
    case 64: return run_cell_bf16<64, EPI>(c, flags, alpha, X, Y, nvec, ld, s, epi);
    case 128: return run_cell_bf16<128, EPI>(c, flags, alpha, X, Y, nvec, ld, s, epi);
    case 224: return run_cell_bf16<224, EPI>(c, flags, alpha, X, Y, nvec, ld, s, epi);
    case 352: return run_cell_bf16<352, EPI>(c, flags, alpha, X, Y, nvec, ld, s, epi);
    case 512: return run_cell_bf16<512, EPI>(c, flags, alpha, X, Y, nvec, ld, s, epi);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cell_op_bf16_epi(const chfsi_ctx *c, int flags, double alpha, const void *X, void *Y,
                                   int64_t nvec, int64_t ld, hipStream_t s, const EpiArgs *epi);

}  // namespace chfsi
