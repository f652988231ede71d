// Matrix-free cell-level Hamiltonian-times-multivector product for gfx950
// (double and float MFMA; the bfloat16 cell kernel is in hx_bf16.hip), the
// spin-orbit projection kernels of every precision (the bfloat16 one
// included), the per-atom reduction with Delta, and the adjoint.
//
// Stages follow the paper's product (Sec. III-C2, stages i-iv): gather of the
// cell block, dense cell contraction, spin-orbit projector term, assembly.
// The local cell operator of eq. cellHam is applied in factored form:
//     Y^(e) = K X^(e) + Phi^T [ w|J| (V_q I + B_q . sigma) (Phi X^(e)) + w|J| phi d ],
// with K the reference stiffness (1/2 grad N . grad N, identical for every
// cell of the uniform mesh), Phi[q][I] = N_I(x_q), and the last term the
// spin-orbit apply P_a(e) d_a written at the quadrature points
// (P_a(e) = Phi^T diag(w|J|) phi_a, so Phi^T (w|J| phi_a d_a) = P_a(e) d_a).
// This is the 2n x 2n spin-block operator of eq. cellHam (H_scal = K +
// V-mass, H_Bd = B_d-mass) without storing four n x n matrices per cell.
//
// MFMA tiling.  Every cell block is a GEMM with rows = real columns of the
// vector block (re/im x spin x vector) and columns = nodes or quadrature
// points.  One workgroup (4 waves) owns one cell and VB vectors; each wave
// owns one 16-row tile and a slice of the column tiles.  The gathered block
// sits in LDS as [node][real column]; the shared tables (K, Phi, Phi^T) are
// read as MFMA B fragments from L2, one k-step ahead of their use.  The
// 16x16 accumulator layout puts the four real columns (re up, im up, re down,
// im down) of one vector at one quadrature point into one lane, so the 2x2
// spin term is applied in registers.  Assembly is colour-ordered: the eight
// parity classes of cells are launched one after another, so no two
// workgroups of a launch touch the same node and no atomics are needed
// (results are deterministic).
#include <type_traits>

#include "cell_common.h"

namespace chfsi {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct MM;
template <> struct MM<double> {
    using acc = d4;
    static __device__ __forceinline__ acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct MM<float> {
    using acc = f4;
    static __device__ __forceinline__ acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

template <typename T> struct LdsPad { static constexpr int v = 4; };
template <> struct LdsPad<float> { static constexpr int v = 8; };

// Row (GEMM M index) of component `comp` (re up, im up, re down, im down) of
// vector v of the block.  The 16x16 accumulators hold, in lane l and
// register i, row 4*(l/16)+i for the f32 MFMA but row 4*i+l/16 for the f64
// MFMA; the order below puts the four components of vector 4m + l/16 into
// registers 0..3 of lane l in both cases.
template <typename T> __device__ __forceinline__ constexpr int rcol(int v, int comp) {
    return sizeof(T) == 8 ? 16 * (v >> 2) + 4 * comp + (v & 3) : 4 * v + comp;
}
// inverse within a 16-row tile: row r -> (vector in tile, component)
template <typename T> __device__ __forceinline__ void rinv(int r, int &v, int &comp) {
    if (sizeof(T) == 8) { v = r & 3; comp = r >> 2; } else { v = r >> 2; comp = r & 3; }
}

// Gathers the vector block of one cell into LDS as xs[I][rcol(v, 2s + r)]
// (scaled by gsc[I] when gsc is given); grow[I] = 2 g(I) is the node's first
// spinor row.
template <typename T, int VB, int NP, int XS, int TH = kThreads>
__device__ __forceinline__ void gather_block(T *xs, const int *grow, const T *gsc, const void *Xv, int64_t ld,
                                             int64_t nvec, int64_t col0, int n) {
    using TC = typename Cplx<T>::type;
    const TC *X = reinterpret_cast<const TC *>(Xv);
    constexpr int TOT = NP * 2 * VB, ITER = (TOT + TH - 1) / TH;
    // all loads of this thread are issued before the first LDS store
    TC z[ITER];
    T sc[ITER];
#pragma unroll
    for (int u = 0; u < ITER; ++u) {
        const int idx = threadIdx.x + u * TH;
        const int v = idx % VB, s = (idx / VB) & 1, I = idx / (2 * VB);
        const int64_t col = col0 + v;
        z[u] = TC{0, 0};
        sc[u] = T(1);
        if (idx < TOT && I < n && col < nvec) {
            z[u] = X[(int64_t)(grow[I] + s) * ld + col];
            if (gsc) sc[u] = gsc[I];
        }
    }
#pragma unroll
    for (int u = 0; u < ITER; ++u) {
        const int idx = threadIdx.x + u * TH;
        const int v = idx % VB, s = (idx / VB) & 1, I = idx / (2 * VB);
        if (idx < TOT) {
            xs[I * XS + rcol<T>(v, 2 * s)] = z[u].x * sc[u];
            xs[I * XS + rcol<T>(v, 2 * s + 1)] = z[u].y * sc[u];
        }
    }
}

// node tables of cell (ex, ey, ez): packed local indices, first spinor rows
// and (when dinv is given) D^-1 values
template <typename T>
__device__ __forceinline__ void cell_tables(int *ijk, int *grow, T *gsc, const T *dinv, int NP, int n, int n1,
                                            int64_t ex, int64_t ey, int64_t ez, int p, int64_t Nx, int64_t Ny,
                                            int64_t Nz) {
    for (int I = threadIdx.x; I < NP; I += blockDim.x) {
        const int i = I % n1, j = (I / n1) % n1, k = I / (n1 * n1);
        const int c = i | (j << 8) | (k << 16);
        ijk[I] = c;
        int64_t g = 0;
        if (I < n) g = gnode_of(c, ex, ey, ez, p, Nx, Ny, Nz);
        grow[I] = (int)(2 * g);
        if (gsc) gsc[I] = (dinv && I < n) ? dinv[g] : T(1);
    }
}

// acc[t] += A^T(rows 16m.., k) * B(k, cols (nt0+t)*16..) over k in [0, NP):
// A from LDS (as[k][c]), B from global ([k][NP] row-major), the B fragments
// of step k+4 loaded while the MFMAs of step k run.
template <typename T, int NTW, int NP, int XS, bool PREFETCH = true>
__device__ __forceinline__ void mfma_panel(typename MM<T>::acc *acc, const T *as, const T *B, int m,
                                           int nt0, int lane) {
    const int kr = lane >> 4, cn = lane & 15;
    const T *bp = B + (size_t)kr * NP + nt0 * 16 + cn;
    const T *ap = as + kr * XS + 16 * m + cn;
    if (!PREFETCH) {
        for (int kk = 0; kk < NP; kk += 4) {
            T av = ap[kk * XS];
            const T *brow = bp + (size_t)kk * NP;
#pragma unroll
            for (int t = 0; t < NTW; ++t) acc[t] = MM<T>::mma(av, brow[16 * t], acc[t]);
        }
        return;
    }
    // the B fragments of the next PD k-steps are in flight in a register
    // ring; each step's reload is issued after its MFMAs (one step ahead
    // measured fastest: deeper rings and issuing before the MFMAs were slower)
    constexpr int PD = 1, NK = NP / 4;
    static_assert(NK % PD == 0, "k steps per prefetch ring");
    T bq[PD][NTW];
#pragma unroll
    for (int u = 0; u < PD; ++u)
#pragma unroll
        for (int t = 0; t < NTW; ++t) bq[u][t] = bp[(size_t)(4 * u) * NP + 16 * t];
    for (int k0 = 0; k0 < NK; k0 += PD) {
#pragma unroll
        for (int u = 0; u < PD; ++u) {
            const int kk = 4 * (k0 + u);
            const T av = ap[kk * XS];
#pragma unroll
            for (int t = 0; t < NTW; ++t) acc[t] = MM<T>::mma(av, bq[u][t], acc[t]);
            const int kn = k0 + u + PD < NK ? kk + 4 * PD : kk;
#pragma unroll
            for (int t = 0; t < NTW; ++t) bq[u][t] = bp[(size_t)kn * NP + 16 * t];
        }
    }
}

// 32 zero bytes: the source of the assembly's loads that need no data.  In
// the global address space like the blocks (not const, which would place it
// in the constant space and turn the selected loads into flat loads, whose
// completion the LDS counter also waits for); never written.
__device__ double kZeroPiece[4] = {0.0, 0.0, 0.0, 0.0};

// threads of a cell-kernel workgroup: MT row tiles x two column groups of waves
constexpr int cell_threads(int mt) { return 128 * mt; }

// One workgroup per (cell, VB = 4 MT vectors): its waves split the 16 MT
// rows x NP columns of the block MT (16-row tiles) x WN (column groups of
// NTW 16-column tiles).
template <typename T, int MT, int NP>
__global__ __launch_bounds__(cell_threads(MT), MT == 1 || (sizeof(T) == 4 && NP <= 352) ? 2 : 1) void cell_kernel(CellParams a, EpiArgs ep) {
    using TC = typename Cplx<T>::type;
    using acc_t = typename MM<T>::acc;
    constexpr int CB = 16 * MT, VB = 4 * MT;
    constexpr int XS = CB + LdsPad<T>::v;
    constexpr int NT = NP / 16, WN = cell_threads(MT) / 64 / MT, NTW = NT / WN;
    static_assert(NT % WN == 0, "column tiles split evenly over the wave groups");
    __shared__ __attribute__((aligned(16))) T xs[NP * XS];
    __shared__ int ijk[NP], grow[NP];
    __shared__ T gsc[NP];

    const int64_t nvb = (a.nvec + VB - 1) / VB;
    const int64_t t_log = xcd_remap(blockIdx.x, a.ncl * nvb);
    const int64_t ci = t_log / nvb, vb = t_log - ci * nvb;
    const int64_t e = a.cells[ci];
    const int64_t ex = e % a.ncx, ey = (e / a.ncx) % a.ncy, ez = e / (a.ncx * a.ncy);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = wave % MT, nt0 = (wave / MT) * NTW;

    const bool scaled = (a.flags & FLAG_DINV) != 0;
    cell_tables<T>(ijk, grow, gsc, scaled ? reinterpret_cast<const T *>(a.dinv) : nullptr, NP, a.n, a.n1, ex, ey,
                   ez, a.p, a.Nx, a.Ny, a.Nz);
    __syncthreads();
    gather_block<T, VB, NP, XS, cell_threads(MT)>(xs, grow, scaled ? gsc : nullptr, a.X, a.ld, a.nvec, vb * VB, a.n);
    __syncthreads();

    acc_t y[NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) y[t] = acc_t{0, 0, 0, 0};
    mfma_panel<T, NTW, NP, XS>(y, xs, reinterpret_cast<const T *>(a.Bk), m, nt0, lane);

    if (a.mode == MODE_HAM) {
        acc_t tq[NTW];
#pragma unroll
        for (int t = 0; t < NTW; ++t) tq[t] = acc_t{0, 0, 0, 0};
        mfma_panel<T, NTW, NP, XS>(tq, xs, reinterpret_cast<const T *>(a.BphiT), m, nt0, lane);
        // pointwise (V + B.sigma) w|J| on (re up, im up, re down, im down)
        const T *W = reinterpret_cast<const T *>(a.W) + (size_t)e * NP * 4;
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            int q = (nt0 + t) * 16 + (lane & 15);
            T v = W[q * 4 + 0], bx = W[q * 4 + 1], by = W[q * 4 + 2], bz = W[q * 4 + 3];
            T ur = tq[t][0], ui = tq[t][1], dr = tq[t][2], di = tq[t][3];
            tq[t][0] = (v + bz) * ur + bx * dr + by * di;
            tq[t][1] = (v + bz) * ui + bx * di - by * dr;
            tq[t][2] = bx * ur - by * ui + (v - bz) * dr;
            tq[t][3] = bx * ui + by * ur + (v - bz) * di;
        }
        // spin-orbit apply at the quadrature points: T += w|J| phi_a d_a, as
        // an MFMA with k = (projector j, spin s', re|im part) and
        // A[(v, s, r)][(j, s', part)] = delta_{s s'} (re/im part of d_j(v))
        if ((a.flags & FLAG_NLOC) && a.cell_pair_ptr) {
            const int pb = a.cell_pair_ptr[e], pe = a.cell_pair_ptr[e + 1];
            int vr, comp;
            rinv<T>(lane & 15, vr, comp);
            const int sA = comp >> 1, rA = comp & 1, kr = lane >> 4, sB = kr >> 1, part = kr & 1;
            const int64_t colA = vb * VB + 4 * m + vr;
            const bool act = sA == sB && colA < a.nvec;
            for (int pp = pb; pp < pe; ++pp) {
                const int pair = a.cell_pairs[pp];
                const int atom = a.pair_atom[pair];
                const T *wp = reinterpret_cast<const T *>(a.P) + (size_t)pair * 4 * a.nbeta * NP;
                const TC *dc = reinterpret_cast<const TC *>(a.dcoef) + (size_t)atom * a.nbeta * a.ldd;
                for (int j = 0; j < a.nbeta; ++j) {
                    T av = 0;
                    if (act) {
                        TC d = dc[(size_t)j * a.ldd + colA];
                        av = rA == 0 ? (part == 0 ? d.x : -d.y) : (part == 0 ? d.y : d.x);
                    }
                    const T *brow = wp + (size_t)(4 * j + kr) * NP + nt0 * 16 + (lane & 15);
#pragma unroll
                    for (int t = 0; t < NTW; ++t) tq[t] = MM<T>::mma(av, brow[16 * t], tq[t]);
                }
            }
        }
        __syncthreads();  // every wave is done reading the gathered block
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            int q = (nt0 + t) * 16 + (lane & 15);
            const int vl = 4 * m + (lane >> 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) xs[q * XS + rcol<T>(vl, i)] = tq[t][i];
        }
        __syncthreads();
        mfma_panel<T, NTW, NP, XS>(y, xs, reinterpret_cast<const T *>(a.Bphi), m, nt0, lane);
    }

    // colour-ordered assembly.  Each lane owns one column and, per column
    // tile t, one node (both spin rows).  The loads of a group of tiles are
    // all issued before the first is used: a read-back where an earlier
    // colour wrote the node, or (FLAG_EPI, at the node's first touch) Z_k,
    // Z_{k-1} and R, from which beta Z_k + gamma Z_{k-1} + alpha lam R is
    // formed in double (Z_{k-1} may be the output buffer: it is read first).
    // Every register a load writes is zeroed before the loads, so no load
    // waits on another path's write of its register.  The group's results
    // are all formed before its first store, because a store's data
    // registers cannot be rewritten until the store has completed.  Without
    // FLAG_EPI one group covers all tiles; with it, the loads of EPG tiles.
    TC *Y = reinterpret_cast<TC *>(a.Y);
    const int64_t col = vb * VB + 4 * m + (lane >> 4);
    if (col < a.nvec) {
        const T al = (T)a.alpha;
        const bool accum = (a.flags & FLAG_ACCUM) != 0, epi = (a.flags & FLAG_EPI) != 0;
        const TC *Zk = reinterpret_cast<const TC *>(a.X), *Zkm = reinterpret_cast<const TC *>(ep.Zkm);
        constexpr int EPG = sizeof(T) == 8 ? 4 : 6;
        const double dl = epi ? a.alpha * ep.lam[col] : 0.0;
        // pieces that need no load read this zero piece instead (it stays
        // in cache), so every load is unconditional and no loaded register
        // has to be merged with a zero from another path
        const TC *zc = reinterpret_cast<const TC *>(kZeroPiece);
        const cd *zd = reinterpret_cast<const cd *>(kZeroPiece);
        auto group = [&](auto epi_c, auto g_c, int t0) {
            constexpr bool EPI = decltype(epi_c)::value;
            constexpr int G = decltype(g_c)::value;
            TC o0[G], o1[G];
            [[maybe_unused]] TC m0[EPI ? G : 1], m1[EPI ? G : 1];
            [[maybe_unused]] cd r0[EPI ? G : 1], r1[EPI ? G : 1];
            bool ft[G], ok[G];
            int64_t off[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int t = t0 + g;
                const int J = (nt0 + t) * 16 + (lane & 15);
                ok[g] = t < NTW && J < a.n;
                const int Jc = ok[g] ? J : 0;
                const int64_t row = grow[Jc];
                off[g] = row * a.ld + col;
                ft[g] = first_touch(ijk[Jc], a.p, a.px, a.py, a.pz, accum);
                // the read-back, or Z_k at a first touch with FLAG_EPI
                const bool rd = EPI ? ok[g] : ok[g] && !ft[g];
                const TC *src = (EPI && ft[g]) ? Zk : Y;
                o0[g] = *(rd ? src + off[g] : zc);
                o1[g] = *(rd ? src + off[g] + a.ld : zc);
                if constexpr (EPI) {
                    const bool fe = ok[g] && ft[g];
                    m0[g] = *(fe && Zkm ? Zkm + off[g] : zc);
                    m1[g] = *(fe && Zkm ? Zkm + off[g] + a.ld : zc);
                    r0[g] = *(fe ? ep.R + row * ep.ldr + col : zd);
                    r1[g] = *(fe ? ep.R + (row + 1) * ep.ldr + col : zd);
                }
            }
            TC v0[G], v1[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int t = t0 + g < NTW ? t0 + g : NTW - 1;
                if constexpr (EPI) {
                    if (ft[g]) {
                        o0[g] = TC{(T)(dl * r0[g].x + ep.beta * (double)o0[g].x + ep.gamma * (double)m0[g].x),
                                   (T)(dl * r0[g].y + ep.beta * (double)o0[g].y + ep.gamma * (double)m0[g].y)};
                        o1[g] = TC{(T)(dl * r1[g].x + ep.beta * (double)o1[g].x + ep.gamma * (double)m1[g].x),
                                   (T)(dl * r1[g].y + ep.beta * (double)o1[g].y + ep.gamma * (double)m1[g].y)};
                    }
                }
                v0[g] = TC{al * y[t][0] + o0[g].x, al * y[t][1] + o0[g].y};
                v1[g] = TC{al * y[t][2] + o1[g].x, al * y[t][3] + o1[g].y};
            }
#pragma unroll
            for (int g = 0; g < G; ++g) asm volatile("" : "+v"(v0[g].x), "+v"(v0[g].y), "+v"(v1[g].x), "+v"(v1[g].y));
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (ok[g]) {
                    Y[off[g]] = v0[g];
                    Y[off[g] + a.ld] = v1[g];
                }
            }
        };
        if (epi) {
#pragma unroll
            for (int t0 = 0; t0 < NTW; t0 += EPG)
                group(std::true_type{}, std::integral_constant<int, EPG>{}, t0);
        } else {
            group(std::false_type{}, std::integral_constant<int, NTW>{}, 0);
        }
    }
}

// ---------------------------------------------------------------------------
// spin-orbit projection: part[pair][j][col] = sum_{I,s} conj(P[pair][I][s][j]) x[I][s][col]
// (x = D^-1 z when FLAG_DINV).  One 16x16x4 MFMA contracts four nodes of one
// component c = (spin, re|im): rows = 16 vectors, k = node, columns =
// (projector j of an 8-wide tile, re|im of the result), with
//   B_(s,re)[I][(j,re)] = Re P, B_(s,re)[I][(j,im)] = -Im P,
//   B_(s,im)[I][(j,re)] = Im P, B_(s,im)[I][(j,im)] = Re P.
// Both operands come straight from memory into registers: lane (k, m) loads
// x of node 4g+k, vector m (both spins), and the two spin values of
// P[I][.][j] from the table laid out [pair][tile][I][j%8][spin], which is
// zero for padded nodes and projectors.  Nothing is staged in LDS except
// the cell's node numbers and D^-1 values, so occupancy is limited only by
// registers and many waves hide the gather latency.  One wave owns
// (cell, 16 vectors) and walks all nodes for up to four (pair, tile) units
// at once, so no cross-wave reduction is needed.
// ---------------------------------------------------------------------------
struct ProjParams {
    const void *X;
    int64_t ld, nvec;
    const int *cells;  // cells with at least one pair
    int64_t ncl;
    int64_t ncx, ncy, Nx, Ny, Nz;
    int p, n1, n, npad;
    const void *dinv;
    const int *cell_pair_ptr, *cell_pairs;
    const void *P;
    void *part;
    int nbeta, ntile;
    int flags;
};

constexpr int kProjMaxUnits = 4;   // (pair, tile) units per pass over the nodes
constexpr int kProjMaxNodes = 512; // (p+1)^3 for p <= 7

template <typename T, int NB>
__device__ __forceinline__ void proj_pass(const ProjParams &a, const int *gtab, const T *sc, int64_t vb16,
                                          int u0, int pb, int lane) {
    using TC = typename Cplx<T>::type;
    using acc_t = typename MM<T>::acc;
    const int k = lane >> 4, m = lane & 15, jj = m >> 1;
    const bool odd = m & 1;
    const int64_t col = vb16 + m;
    const bool cv = col < a.nvec;
    const TC *X = reinterpret_cast<const TC *>(a.X);
    const TC *Q[NB];
    int pair[NB], tile[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        pair[u] = a.cell_pairs[pb + (u0 + u) / a.ntile];
        tile[u] = (u0 + u) % a.ntile;
        Q[u] = reinterpret_cast<const TC *>(a.P) +
               (((size_t)pair[u] * a.ntile + tile[u]) * a.npad + k) * 16 + 2 * jj;
    }
    acc_t acc[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) acc[u] = acc_t{0, 0, 0, 0};
    const int ngroups = (a.n + 3) >> 2;
#pragma unroll 2
    for (int g = 0; g < ngroups; ++g) {
        const int I = 4 * g + k;
        TC xu{0, 0}, xd{0, 0};
        if (cv && I < a.n) {
            const int64_t r = 2 * (int64_t)gtab[I] * a.ld + col;
            xu = X[r];
            xd = X[r + a.ld];
            const T f = sc[I];
            xu.x *= f; xu.y *= f; xd.x *= f; xd.y *= f;
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const TC pu = Q[u][(size_t)g * 64], pd = Q[u][(size_t)g * 64 + 1];
            acc[u] = MM<T>::mma(xu.x, odd ? -pu.y : pu.x, acc[u]);
            acc[u] = MM<T>::mma(xu.y, odd ? pu.x : pu.y, acc[u]);
            acc[u] = MM<T>::mma(xd.x, odd ? -pd.y : pd.x, acc[u]);
            acc[u] = MM<T>::mma(xd.y, odd ? pd.x : pd.y, acc[u]);
        }
    }
    // accumulator: lane l, register i holds row (vector) 4*(l/16)+i for the
    // f32 MFMA, 4*i+l/16 for the f64 MFMA; column = lane & 15 = (jj, re|im)
    T *part = reinterpret_cast<T *>(a.part);
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int j = 8 * tile[u] + jj;
        if (j >= a.nbeta) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int v = sizeof(T) == 8 ? 4 * i + k : 4 * k + i;
            const int64_t c = vb16 + v;
            if (c < a.nvec) part[(((size_t)pair[u] * a.nbeta + j) * a.nvec + c) * 2 + odd] = acc[u][i];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void proj_kernel(ProjParams a) {
    __shared__ int gtab[kProjMaxNodes];
    __shared__ T sc[kProjMaxNodes];
    const int64_t nvb = (a.nvec + 63) / 64;  // 64 vectors per workgroup, 16 per wave
    const int64_t t_log = xcd_remap(blockIdx.x, a.ncl * nvb);
    const int64_t ci = t_log / nvb, vb = t_log - ci * nvb;
    const int64_t e = a.cells[ci];
    const int64_t ex = e % a.ncx, ey = (e / a.ncx) % a.ncy, ez = e / (a.ncx * a.ncy);
    const T *dinv = (a.flags & FLAG_DINV) ? reinterpret_cast<const T *>(a.dinv) : nullptr;
    for (int I = threadIdx.x; I < a.n; I += kThreads) {
        const int i = I % a.n1, j = (I / a.n1) % a.n1, k = I / (a.n1 * a.n1);
        const int64_t g = gnode_of(i | (j << 8) | (k << 16), ex, ey, ez, a.p, a.Nx, a.Ny, a.Nz);
        gtab[I] = (int)g;
        sc[I] = dinv ? dinv[g] : T(1);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t vb16 = vb * 64 + wave * 16;
    if (vb16 >= a.nvec) return;
    const int pb = a.cell_pair_ptr[e];
    const int nunits = (a.cell_pair_ptr[e + 1] - pb) * a.ntile;
    for (int u0 = 0; u0 < nunits; u0 += kProjMaxUnits) {
        switch (min(kProjMaxUnits, nunits - u0)) {
            case 1: proj_pass<T, 1>(a, gtab, sc, vb16, u0, pb, lane); break;
            case 2: proj_pass<T, 2>(a, gtab, sc, vb16, u0, pb, lane); break;
            case 3: proj_pass<T, 3>(a, gtab, sc, vb16, u0, pb, lane); break;
            default: proj_pass<T, 4>(a, gtab, sc, vb16, u0, pb, lane); break;
        }
    }
}

// Projection with bfloat16 MFMA operands (the CHFSI_BF16 filter): one wave
// owns (cell, 16 vectors) as in proj_kernel, but a v_mfma_f32_16x16x32_bf16
// step takes eight nodes: k = 4 (node in the group) + component (x_up re,
// x_up im, x_dn re, x_dn im), each lane supplying two nodes of its vector
// (A) and the matching 8 k of its column (jj, re|im) of the [k][column]
// table PB (B), built once from the FP32 projector table with the signs of
// the complex conjugate product folded in.  Float accumulation; the partial
// sums have the layout of the FP32 path.
typedef __bf16 pbf8 __attribute__((ext_vector_type(8)));
typedef float pf4 __attribute__((ext_vector_type(4)));

template <int NB>
__device__ __forceinline__ void proj_pass_bf16(const ProjParams &a, const int *gtab, const float *sc, int64_t vb16,
                                               int u0, int pb, int lane) {
    const int m = lane & 15, kq = lane >> 4;
    const int64_t col = vb16 + m;
    const bool cv = col < a.nvec;
    const cf *X = reinterpret_cast<const cf *>(a.X);
    const int ng = a.npad / 8;
    const __bf16 *Q[NB];
    int pair[NB], tile[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        pair[u] = a.cell_pairs[pb + (u0 + u) / a.ntile];
        tile[u] = (u0 + u) % a.ntile;
        Q[u] = reinterpret_cast<const __bf16 *>(a.P) + ((size_t)pair[u] * a.ntile + tile[u]) * ng * 512 + m * 32 + 8 * kq;
    }
    pf4 acc[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) acc[u] = pf4{0, 0, 0, 0};
    const int ngroups = (a.n + 7) >> 3;
    // the x values of node group g+1 are loaded while group g is converted
    // and multiplied; every load is unconditional (a lane past the block or
    // the cell reads element 0, and its values are replaced by zero), so the
    // loads of the next group need not wait for any branch
    cf xn[4];
    float fn[2];
    bool okn[2];
    auto load_group = [&](int g) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int I = 8 * g + 2 * kq + h;
            okn[h] = cv && I < a.n;
            const int64_t r = okn[h] ? 2 * (int64_t)gtab[I] * a.ld + col : 0;
            fn[h] = okn[h] ? sc[I] : 0.f;
            xn[2 * h] = X[r];
            xn[2 * h + 1] = X[okn[h] ? r + a.ld : 0];
        }
    };
    load_group(0);
    for (int g = 0; g < ngroups; ++g) {
        cf xc[4];
        float fc[2];
        bool okc[2];
#pragma unroll
        for (int i = 0; i < 4; ++i) xc[i] = xn[i];
        fc[0] = fn[0];
        fc[1] = fn[1];
        okc[0] = okn[0];
        okc[1] = okn[1];
        if (g + 1 < ngroups) load_group(g + 1);
        pbf8 av;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float f = fc[h];
            const bool ok = okc[h];
            av[4 * h] = (__bf16)(ok ? xc[2 * h].x * f : 0.f);
            av[4 * h + 1] = (__bf16)(ok ? xc[2 * h].y * f : 0.f);
            av[4 * h + 2] = (__bf16)(ok ? xc[2 * h + 1].x * f : 0.f);
            av[4 * h + 3] = (__bf16)(ok ? xc[2 * h + 1].y * f : 0.f);
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const pbf8 bv = *reinterpret_cast<const pbf8 *>(Q[u] + (size_t)g * 512);
            acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[u], 0, 0, 0);
        }
    }
    // accumulator: lane l, register i holds row (vector) 4*(l/16)+i, column l & 15 = (jj, re|im)
    float *part = reinterpret_cast<float *>(a.part);
    const int jj = m >> 1, odd = m & 1;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int j = 8 * tile[u] + jj;
        if (j >= a.nbeta) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t c = vb16 + 4 * kq + i;
            if (c < a.nvec) part[(((size_t)pair[u] * a.nbeta + j) * a.nvec + c) * 2 + odd] = acc[u][i];
        }
    }
}

__global__ __launch_bounds__(kThreads) void proj_kernel_bf16(ProjParams a) {
    __shared__ int gtab[kProjMaxNodes];
    __shared__ float sc[kProjMaxNodes];
    const int64_t nvb = (a.nvec + 63) / 64;  // 64 vectors per workgroup, 16 per wave
    const int64_t t_log = xcd_remap(blockIdx.x, a.ncl * nvb);
    const int64_t ci = t_log / nvb, vb = t_log - ci * nvb;
    const int64_t e = a.cells[ci];
    const int64_t ex = e % a.ncx, ey = (e / a.ncx) % a.ncy, ez = e / (a.ncx * a.ncy);
    const float *dinv = (a.flags & FLAG_DINV) ? reinterpret_cast<const float *>(a.dinv) : nullptr;
    for (int I = threadIdx.x; I < a.n; I += kThreads) {
        const int i = I % a.n1, j = (I / a.n1) % a.n1, k = I / (a.n1 * a.n1);
        const int64_t g = gnode_of(i | (j << 8) | (k << 16), ex, ey, ez, a.p, a.Nx, a.Ny, a.Nz);
        gtab[I] = (int)g;
        sc[I] = dinv ? dinv[g] : 1.0f;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t vb16 = vb * 64 + wave * 16;
    if (vb16 >= a.nvec) return;
    const int pb = a.cell_pair_ptr[e];
    const int nunits = (a.cell_pair_ptr[e + 1] - pb) * a.ntile;
    for (int u0 = 0; u0 < nunits; u0 += kProjMaxUnits) {
        switch (min(kProjMaxUnits, nunits - u0)) {
            case 1: proj_pass_bf16<1>(a, gtab, sc, vb16, u0, pb, lane); break;
            case 2: proj_pass_bf16<2>(a, gtab, sc, vb16, u0, pb, lane); break;
            case 3: proj_pass_bf16<3>(a, gtab, sc, vb16, u0, pb, lane); break;
            default: proj_pass_bf16<4>(a, gtab, sc, vb16, u0, pb, lane); break;
        }
    }
}

// PB[pair][tile][g][c][k] (bfloat16, g = node group of 8, c = (jj, re|im),
// k = 4 (node in group) + component): the coefficient of component k of x in
// the real (c even) or imaginary (c odd) part of conj(P_{I,j}) . x, from the
// FP32 table P32[pair][tile][I][jj][spin]
__global__ void setup_projb_kernel(const cf *P32, __bf16 *PB, int64_t total, int NP) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int k = (int)(idx & 31), c = (int)((idx >> 5) & 15);
    const int64_t rest = idx >> 9;  // (pair * ntile + tile) * (NP / 8) + g
    const int64_t pt = rest / (NP / 8), g = rest - pt * (NP / 8);
    const int I = 8 * (int)g + (k >> 2), comp = k & 3, jj = c >> 1, odd = c & 1;
    const cf pz = P32[(pt * NP + I) * 16 + 2 * jj + (comp >> 1)];
    float v;
    if ((comp & 1) == 0) v = odd ? -pz.y : pz.x;  // coefficient of the real part of x
    else v = odd ? pz.x : pz.y;                    // coefficient of the imaginary part
    PB[idx] = (__bf16)v;
}

// dcoef[atom][i][col] = sum_j Delta[atom][i][j] * sum_{pairs of atom} part[pair][j][col].
// A workgroup owns one atom and 64 columns; thread (j, col) sums projector j
// over the atom's pairs (in pair order, coalesced over the columns), the
// sums meet in LDS, and thread (i, col) applies row i of Delta.
constexpr int kNlCols = 64;

template <typename TC>
__global__ __launch_bounds__(kNlCols * kMaxBeta) void nl_reduce_kernel(const TC *part, const int *atom_pair_ptr,
                                                                       const cd *delta, TC *dcoef, int nbeta,
                                                                       int64_t nvec) {
    __shared__ double sr[kMaxBeta][kNlCols], si[kMaxBeta][kNlCols];
    const int64_t atom = blockIdx.x;
    const int cl = threadIdx.x % kNlCols, j = threadIdx.x / kNlCols;
    const int64_t col = (int64_t)blockIdx.y * kNlCols + cl;
    double ar = 0, ai = 0;
    if (col < nvec)
        for (int pr = atom_pair_ptr[atom]; pr < atom_pair_ptr[atom + 1]; ++pr) {
            const TC v = part[((size_t)pr * nbeta + j) * nvec + col];
            ar += v.x;
            ai += v.y;
        }
    sr[j][cl] = ar;
    si[j][cl] = ai;
    __syncthreads();
    if (col >= nvec) return;
    const int i = j;
    const cd *D = delta + ((size_t)atom * nbeta + i) * nbeta;
    double xr = 0, xi = 0;
    for (int jj = 0; jj < nbeta; ++jj) {
        const cd d = D[jj];
        xr += d.x * sr[jj][cl] - d.y * si[jj][cl];
        xi += d.x * si[jj][cl] + d.y * sr[jj][cl];
    }
    TC o;
    o.x = xr;
    o.y = xi;
    dcoef[((size_t)atom * nbeta + i) * nvec + col] = o;
}

// ---------------------------------------------------------------------------
// adjoint with respect to the quadrature fields
// ---------------------------------------------------------------------------
struct AdjParams {
    const void *X, *G;
    int64_t ld, nvec;
    int64_t ncells, ncx, ncy, Nx, Ny, Nz;
    int p, n1, n, nq;
    const void *BphiT;
    const double *wq;
    double *dV, *dB;
};

template <typename T, int MT, int NP>
__global__ __launch_bounds__(kThreads, sizeof(T) == 4 && NP <= 352 ? 2 : 1) void adjoint_kernel(AdjParams a) {
    using acc_t = typename MM<T>::acc;
    constexpr int VB = 4 * MT, CB = 16 * MT;
    constexpr int XS = CB + LdsPad<T>::v;
    constexpr int NT = NP / 16, WN = 4 / MT, NTW = NT / WN;
    __shared__ __attribute__((aligned(16))) T xs[NP * XS];
    __shared__ int ijk[NP], grow[NP];
    static_assert(NP * XS * sizeof(T) >= 4 * NP * sizeof(double), "reduction buffer");

    const int64_t e = blockIdx.x;
    const int64_t ex = e % a.ncx, ey = (e / a.ncx) % a.ncy, ez = e / (a.ncx * a.ncy);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = wave % MT, nt0 = (wave / MT) * NTW;
    cell_tables<T>(ijk, grow, nullptr, nullptr, NP, a.n, a.n1, ex, ey, ez, a.p, a.Nx, a.Ny, a.Nz);
    double sv[NTW], sx[NTW], sy[NTW], sz[NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) { sv[t] = 0; sx[t] = 0; sy[t] = 0; sz[t] = 0; }
    const T *BphiT = reinterpret_cast<const T *>(a.BphiT);
    const int64_t nvb = (a.nvec + VB - 1) / VB;
    for (int64_t vb = 0; vb < nvb; ++vb) {
        __syncthreads();
        gather_block<T, VB, NP, XS>(xs, grow, nullptr, a.X, a.ld, a.nvec, vb * VB, a.n);
        __syncthreads();
        acc_t tx[NTW], tg[NTW];
#pragma unroll
        for (int t = 0; t < NTW; ++t) { tx[t] = acc_t{0, 0, 0, 0}; tg[t] = acc_t{0, 0, 0, 0}; }
        mfma_panel<T, NTW, NP, XS, (NP <= 352)>(tx, xs, BphiT, m, nt0, lane);
        __syncthreads();
        gather_block<T, VB, NP, XS>(xs, grow, nullptr, a.G, a.ld, a.nvec, vb * VB, a.n);
        __syncthreads();
        mfma_panel<T, NTW, NP, XS, (NP <= 352)>(tg, xs, BphiT, m, nt0, lane);
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            double xur = tx[t][0], xui = tx[t][1], xdr = tx[t][2], xdi = tx[t][3];
            double gur = tg[t][0], gui = tg[t][1], gdr = tg[t][2], gdi = tg[t][3];
            sv[t] += gur * xur + gui * xui + gdr * xdr + gdi * xdi;
            // Re(conj(gu) xd + conj(gd) xu)
            sx[t] += gur * xdr + gui * xdi + gdr * xur + gdi * xui;
            // Im(conj(gu) xd) - Im(conj(gd) xu)
            sy[t] += (gur * xdi - gui * xdr) - (gdr * xui - gdi * xur);
            sz[t] += gur * xur + gui * xui - gdr * xdr - gdi * xdi;
        }
    }
    // reduce over the 4 vector lanes of each quadrature point (lane>>4), then over waves
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        for (int off = 16; off < 64; off <<= 1) {
            sv[t] += __shfl_xor(sv[t], off);
            sx[t] += __shfl_xor(sx[t], off);
            sy[t] += __shfl_xor(sy[t], off);
            sz[t] += __shfl_xor(sz[t], off);
        }
    }
    __syncthreads();  // the block tile is free: reuse it for the reduction
    double *red = reinterpret_cast<double *>(xs);
    for (int i = tid; i < 4 * NP; i += kThreads) red[i] = 0;
    __syncthreads();
    // deterministic order over the MT waves sharing a column slice
    for (int mm = 0; mm < MT; ++mm) {
        if (m == mm && lane < 16) {
#pragma unroll
            for (int t = 0; t < NTW; ++t) {
                int q = (nt0 + t) * 16 + lane;
                red[0 * NP + q] += sv[t];
                red[1 * NP + q] += sx[t];
                red[2 * NP + q] += sy[t];
                red[3 * NP + q] += sz[t];
            }
        }
        __syncthreads();
    }
    for (int q = tid; q < a.nq; q += kThreads) {
        double w = a.wq[q];
        a.dV[e * a.nq + q] = w * red[0 * NP + q];
        a.dB[(e * a.nq + q) * 3 + 0] = w * red[1 * NP + q];
        a.dB[(e * a.nq + q) * 3 + 1] = w * red[2 * NP + q];
        a.dB[(e * a.nq + q) * 3 + 2] = w * red[3 * NP + q];
    }
}

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------
__global__ void setup_fields_kernel(const double *V, const double *B, const double *wq, double *W64,
                                    float *W32, int64_t ncells, int nq, int NP) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ncells * NP) return;
    int64_t e = idx / NP;
    int q = (int)(idx % NP);
    double v = 0, bx = 0, by = 0, bz = 0;
    if (q < nq) {
        double w = wq[q];
        v = w * V[e * nq + q];
        bx = w * B[(e * nq + q) * 3 + 0];
        by = w * B[(e * nq + q) * 3 + 1];
        bz = w * B[(e * nq + q) * 3 + 2];
    }
    double *o = W64 + idx * 4;
    o[0] = v; o[1] = bx; o[2] = by; o[3] = bz;
    float *f = W32 + idx * 4;
    f[0] = (float)v; f[1] = (float)bx; f[2] = (float)by; f[3] = (float)bz;
}

// P[pair][I][s][j] = sum_q wq[q] Phi[q][I] phi[pair][q][s][j]
__global__ void setup_proj_kernel(const cd *phi, const double *Phi, const double *wq, cd *P64,
                                  cf *P32, int64_t npairs, int n, int nq, int NP, int nbeta) {
    // P[pair][tile][I][j % 8][spin] = sum_q w_q Phi_I(q) phi[pair][q][spin][j], zero when
    // I >= n or j >= nbeta
    const int ntile = (nbeta + 7) / 8;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)ntile * NP * 16;
    if (idx >= npairs * per) return;
    const int64_t pair = idx / per;
    int r = (int)(idx % per);
    const int tile = r / (NP * 16);
    r -= tile * NP * 16;
    const int I = r >> 4, j = 8 * tile + ((r >> 1) & 7), sp = r & 1;
    double ar = 0, ai = 0;
    if (I < n && j < nbeta) {
        const cd *ph = phi + (size_t)pair * nq * 2 * nbeta + sp * nbeta + j;
        for (int q = 0; q < nq; ++q) {
            double w = wq[q] * Phi[(size_t)q * NP + I];
            cd z = ph[(size_t)q * 2 * nbeta];
            ar += w * z.x;
            ai += w * z.y;
        }
    }
    P64[idx].x = ar; P64[idx].y = ai;
    P32[idx].x = (float)ar; P32[idx].y = (float)ai;
}

// w|J| phi at the quadrature points, k = (j, spin, re|im):
//   WP[pair][k][q] (double, float) and WPb[pair][q][k] (bfloat16, k padded)
__global__ void setup_wphi_kernel(const cd *phi, const double *wq, double *W64, float *W32, __bf16 *Wb,
                                  int64_t npairs, int nq, int NP, int nbeta, int kpad) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= npairs * NP * kpad) return;
    int64_t pair = idx / ((int64_t)NP * kpad);
    int r = (int)(idx % ((int64_t)NP * kpad));
    int q = r / kpad, k = r % kpad;
    double v = 0;
    if (q < nq && k < 4 * nbeta) {
        int j = k >> 2, s = (k >> 1) & 1, part = k & 1;
        cd z = phi[((size_t)pair * nq + q) * 2 * nbeta + s * nbeta + j];
        v = wq[q] * (part ? z.y : z.x);
    }
    Wb[idx] = (__bf16)(float)v;
    if (k < 4 * nbeta) {
        size_t o = ((size_t)pair * 4 * nbeta + k) * NP + q;
        W64[o] = v;
        W32[o] = (float)v;
    }
}

__global__ void cast_table_kernel(const double *src, float *dst, __bf16 *dstb, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[i] = (float)src[i];
    if (dstb) dstb[i] = (__bf16)(float)src[i];
}

__global__ void dinv_kernel(const double *D, double *d64, float *d32, int64_t M) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    double v = 1.0 / D[i];
    d64[i] = v;
    d32[i] = (float)v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, int MT, int NP>
static hipError_t run_cell(const chfsi_ctx *c, int mode, int flags, double alpha, const void *X,
                           void *Y, int64_t nvec, int64_t ld, hipStream_t s, const EpiArgs *epi) {
    const Mesh &m = c->m;
    const Layout &L = c->L;
    constexpr bool dbl = sizeof(T) == 8;
    CellParams a{};
    a.X = X; a.Y = Y; a.ld = ld; a.nvec = nvec;
    a.ncx = m.ncell[0]; a.ncy = m.ncell[1];
    a.Nx = m.Nd[0]; a.Ny = m.Nd[1]; a.Nz = m.Nd[2];
    a.p = m.p; a.n1 = m.n1; a.n = m.n;
    if (mode == MODE_MASS) a.Bk = c->P<char>(L.M64);
    else a.Bk = dbl ? c->P<char>(L.K64) : c->P<char>(L.K32);
    a.BphiT = dbl ? c->P<char>(L.PhiT64) : c->P<char>(L.PhiT32);
    a.Bphi = dbl ? c->P<char>(L.Phi64) : c->P<char>(L.Phi32);
    a.W = dbl ? c->P<char>(L.W64) : c->P<char>(L.W32);
    a.dinv = dbl ? c->P<char>(L.Dinv64) : c->P<char>(L.Dinv32);
    a.alpha = alpha;
    a.mode = mode;
    a.flags = flags;
    if ((flags & FLAG_EPI) && !epi) return hipErrorInvalidValue;
    const EpiArgs ep = (flags & FLAG_EPI) ? *epi : EpiArgs{};
    if ((flags & FLAG_NLOC) && m.npairs > 0 && mode == MODE_HAM) {
        a.cell_pair_ptr = c->P<int>(L.cell_pair_ptr);
        a.cell_pairs = c->P<int>(L.cell_pairs);
        a.pair_atom = c->P<int>(L.pair_atom);
        a.P = dbl ? c->P<char>(L.WP64) : c->P<char>(L.WP32);
        a.dcoef = c->S<char>(L.dcoef);
        a.nbeta = m.nbeta;
        a.ldd = nvec;
    } else {
        a.flags &= ~FLAG_NLOC;
    }
    constexpr int VB = 4 * MT;
    const int64_t nvb = (nvec + VB - 1) / VB;
    for (int col = 0; col < 8; ++col) {
        int64_t ncl = c->colour_ptr[col + 1] - c->colour_ptr[col];
        if (ncl == 0) continue;
        a.cells = c->P<int>(L.colour_cells) + c->colour_ptr[col];
        a.ncl = ncl;
        a.px = col & 1; a.py = (col >> 1) & 1; a.pz = (col >> 2) & 1;
        hipLaunchKernelGGL((cell_kernel<T, MT, NP>), dim3((unsigned)(ncl * nvb)), dim3(cell_threads(MT)), 0, s, a, ep);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

template <typename T>
static hipError_t run_proj(const chfsi_ctx *c, int flags, const void *X, int64_t nvec, int64_t ld,
                           hipStream_t s, bool bf16 = false) {
    const Mesh &m = c->m;
    const Layout &L = c->L;
    constexpr bool dbl = sizeof(T) == 8;
    if (m.n > kProjMaxNodes) return hipErrorInvalidValue;
    ProjParams a{};
    a.X = X; a.ld = ld; a.nvec = nvec;
    a.cells = c->P<int>(L.nl_cells);
    a.ncl = m.n_nl_cells;
    a.ncx = m.ncell[0]; a.ncy = m.ncell[1];
    a.Nx = m.Nd[0]; a.Ny = m.Nd[1]; a.Nz = m.Nd[2];
    a.p = m.p; a.n1 = m.n1; a.n = m.n; a.npad = m.npad;
    a.dinv = dbl ? c->P<char>(L.Dinv64) : c->P<char>(L.Dinv32);
    a.cell_pair_ptr = c->P<int>(L.cell_pair_ptr);
    a.cell_pairs = c->P<int>(L.cell_pairs);
    a.P = dbl ? c->P<char>(L.P64) : c->P<char>(L.P32);
    a.part = c->S<char>(L.partial);
    a.nbeta = m.nbeta;
    a.ntile = (m.nbeta + 7) / 8;
    a.flags = flags;
    const int64_t nvb = (nvec + 63) / 64;
    if (bf16) {
        a.P = c->P<char>(L.PB);
        hipLaunchKernelGGL(proj_kernel_bf16, dim3((unsigned)(a.ncl * nvb)), dim3(kThreads), 0, s, a);
    } else {
        hipLaunchKernelGGL((proj_kernel<T>), dim3((unsigned)(a.ncl * nvb)), dim3(kThreads), 0, s, a);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const dim3 grd((unsigned)m.natoms, (unsigned)((nvec + kNlCols - 1) / kNlCols));
    if (dbl)
        hipLaunchKernelGGL(nl_reduce_kernel<cd>, grd, dim3(kNlCols * m.nbeta), 0, s, c->S<cd>(L.partial),
                           c->P<int>(L.atom_pair_ptr), c->P<cd>(L.delta64), c->S<cd>(L.dcoef), m.nbeta, nvec);
    else
        hipLaunchKernelGGL(nl_reduce_kernel<cf>, grd, dim3(kNlCols * m.nbeta), 0, s, c->S<cf>(L.partial),
                           c->P<int>(L.atom_pair_ptr), c->P<cd>(L.delta64), c->S<cf>(L.dcoef), m.nbeta, nvec);
    return hipGetLastError();
}

template <typename T, int MT, int NP>
static hipError_t run_adjoint(const chfsi_ctx *c, const void *X, const void *G, int64_t nvec,
                              int64_t ld, double *dV, double *dB, hipStream_t s) {
    const Mesh &m = c->m;
    const Layout &L = c->L;
    constexpr bool dbl = sizeof(T) == 8;
    AdjParams a{};
    a.X = X; a.G = G; a.ld = ld; a.nvec = nvec;
    a.ncells = m.ncells; a.ncx = m.ncell[0]; a.ncy = m.ncell[1];
    a.Nx = m.Nd[0]; a.Ny = m.Nd[1]; a.Nz = m.Nd[2];
    a.p = m.p; a.n1 = m.n1; a.n = m.n; a.nq = m.nq;
    a.BphiT = dbl ? c->P<char>(L.PhiT64) : c->P<char>(L.PhiT32);
    a.wq = c->P<double>(L.Wq);
    a.dV = dV; a.dB = dB;
    hipLaunchKernelGGL((adjoint_kernel<T, MT, NP>), dim3((unsigned)m.ncells), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

// dispatch on the padded table size (one instantiation per FE degree class)
#define CHFSI_DISPATCH_NP(NPV, CALL)          \
    switch (NPV) {                            \
    case 32: { constexpr int NP = 32; CALL; } \
    case 64: { constexpr int NP = 64; CALL; } \
    case 128: { constexpr int NP = 128; CALL; } \
    case 224: { constexpr int NP = 224; CALL; } \
    case 352: { constexpr int NP = 352; CALL; } \
    case 512: { constexpr int NP = 512; CALL; } \
    default: return hipErrorInvalidValue;     \
    }

hipError_t launch_cell_op(const chfsi_ctx *c, chfsi_prec prec, int mode, int flags, double alpha,
                          const void *X, void *Y, int64_t nvec, int64_t ld, hipStream_t s, const EpiArgs *epi) {
    if (prec == CHFSI_FP64) {
        // double: up to p = 6, 4 vectors per workgroup (62 KB of LDS at p = 6),
        // two workgroups per CU, one's gather and assembly beside the other's
        // MFMAs (146.7 against 149.8 ms per H X with 8 vectors and one
        // workgroup per CU); at p = 7 the 8-vector block
        CHFSI_DISPATCH_NP(c->m.npad, return (run_cell<double, NP <= 352 ? 1 : 2, NP>(c, mode, flags, alpha, X, Y,
                                                                                     nvec, ld, s, epi)));
    }
    if (prec == CHFSI_BF16) return launch_cell_op_bf16(c, mode, flags, alpha, X, Y, nvec, ld, s, epi);
    // float: 8 vectors per workgroup (two column groups of tiles per row
    // tile).  Up to p = 6 the block (46 KB of LDS) and at most 256 registers
    // per lane let two workgroups share a CU, so one workgroup's gather and
    // assembly overlap the other's MFMAs (16 vectors per workgroup, one per
    // CU, took 89.5 against 82.7 ms per H X at p = 6)
    CHFSI_DISPATCH_NP(c->m.npad, return (run_cell<float, 2, NP>(c, mode, flags, alpha, X, Y, nvec, ld, s, epi)));
}

// the projection of the bfloat16 path runs in float (complex64 blocks)
hipError_t launch_nonlocal_coeffs(const chfsi_ctx *c, chfsi_prec prec, int flags, const void *X,
                                  int64_t nvec, int64_t ld, hipStream_t s) {
    if (c->m.npairs == 0 || c->m.n_nl_cells == 0) return hipSuccess;
    if (prec == CHFSI_FP64) return run_proj<double>(c, flags, X, nvec, ld, s);
    return run_proj<float>(c, flags, X, nvec, ld, s, prec == CHFSI_BF16);
}

hipError_t launch_adjoint_fields(const chfsi_ctx *c, chfsi_prec prec, const void *X, const void *G,
                                 int64_t nvec, int64_t ld, double *dV, double *dB, hipStream_t s) {
    if (prec == CHFSI_FP64) {
        CHFSI_DISPATCH_NP(c->m.npad, return (run_adjoint<double, 2, NP>(c, X, G, nvec, ld, dV, dB, s)));
    }
    CHFSI_DISPATCH_NP(c->m.npad, return (run_adjoint<float, 2, NP>(c, X, G, nvec, ld, dV, dB, s)));
}

hipError_t launch_setup_fields(const chfsi_ctx *c, const double *V, const double *B, hipStream_t s) {
    const int64_t nthr = c->m.ncells * c->m.npad;
    hipLaunchKernelGGL(setup_fields_kernel, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, V, B,
                       c->P<double>(c->L.Wq), c->P<double>(c->L.W64), c->P<float>(c->L.W32),
                       c->m.ncells, c->m.nq, c->m.npad);
    return hipGetLastError();
}

hipError_t launch_setup_projectors(const chfsi_ctx *c, const cd *phi_dev, hipStream_t s) {
    const Mesh &m = c->m;
    if (m.npairs == 0) return hipSuccess;
    const int64_t nthr = m.npairs * ((m.nbeta + 7) / 8) * m.npad * 16;
    hipLaunchKernelGGL(setup_proj_kernel, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, phi_dev,
                       c->P<double>(c->L.Phi64), c->P<double>(c->L.Wq), c->P<cd>(c->L.P64),
                       c->P<cf>(c->L.P32), m.npairs, m.n, m.nq, m.npad, m.nbeta);
    const int64_t nb = m.npairs * ((m.nbeta + 7) / 8) * m.npad * 64;
    hipLaunchKernelGGL(setup_projb_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, c->P<cf>(c->L.P32),
                       c->P<__bf16>(c->L.PB), nb, m.npad);
    const int64_t nw = m.npairs * m.npad * c->L.kpad;
    hipLaunchKernelGGL(setup_wphi_kernel, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, phi_dev,
                       c->P<double>(c->L.Wq), c->P<double>(c->L.WP64), c->P<float>(c->L.WP32),
                       c->P<__bf16>(c->L.WPb), m.npairs, m.nq, m.npad, m.nbeta, c->L.kpad);
    return hipGetLastError();
}

hipError_t launch_setup_casts(const chfsi_ctx *c, hipStream_t s) {
    const Layout &L = c->L;
    const int64_t nn = (int64_t)c->m.npad * c->m.npad;
    const unsigned g = (unsigned)((nn + 255) / 256);
    hipLaunchKernelGGL(cast_table_kernel, dim3(g), dim3(256), 0, s, c->P<double>(L.K64), c->P<float>(L.K32),
                       c->P<__bf16>(L.Kb), nn);
    hipLaunchKernelGGL(cast_table_kernel, dim3(g), dim3(256), 0, s, c->P<double>(L.Phi64),
                       c->P<float>(L.Phi32), c->P<__bf16>(L.Phib), nn);
    hipLaunchKernelGGL(cast_table_kernel, dim3(g), dim3(256), 0, s, c->P<double>(L.PhiT64),
                       c->P<float>(L.PhiT32), c->P<__bf16>(L.PhiTb), nn);
    const int64_t M = c->m.M;
    hipLaunchKernelGGL(dinv_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, c->P<double>(L.D64),
                       c->P<double>(L.Dinv64), c->P<float>(L.Dinv32), M);
    return hipGetLastError();
}

}  // namespace chfsi
