// Poisson operator, Chebyshev-Jacobi preconditioner and fused PCG vector
// kernels (paper Sec. III-B1 and Sec. III-C1, the GPU matrix-free CG solver
// with Algorithm pcg_fusion), all FP64.
//
// Kx: y = K x with K_IJ = sum_e int_e grad N_I . grad N_J (periodic mesh),
// sum-factorised on the tensor-product cell.  The nodal values of a cell are
// interpolated to the Gauss points by three 1D contractions with
// l_i(x_q) (z, y, x), differentiated along each axis there by the Gauss-point
// collocation derivative Dq (exact: a degree-p polynomial is reproduced by
// its interpolant on nq1 >= p+1 points), scaled by w_q |J| (2/h_d)^2,
// multiplied by Dq^T and taken back to the nodes by the transposed
// contractions: O(d p^(d+1)) work per cell instead of O(p^(2d)).
//
// One wave per cell.  A lane owns one 1D line of the cube in each phase, so
// the three gradient lines and their transposed derivatives stay in
// registers (the paper's register/shared-memory hybrid); only the values at
// the Gauss points and the partial sums pass through one LDS cube, which
// every phase reads into registers and then overwrites.  The
// gather of the first phase goes straight into registers (one z-line per
// lane) and the last contraction is assembled from registers with FP64
// atomic adds, so y is zeroed first.
#include "cell_common.h"

namespace chfsi {

struct KxParams {
    const double *x;
    double *y;
    int64_t ncx, ncy, ncells, Nx, Ny, Nz;
    int p;
    double cx, cy, cz;        // |J| (2/h_d)^2
    double tab[kPoiTab];      // even/odd 1D operators and Gauss weights (KxTab layout)
};

constexpr int cmax3(int a, int b, int c) { return a > b ? (a > c ? a : c) : (b > c ? b : c); }

__device__ __forceinline__ int64_t wrap1(int64_t g, int64_t N) { return g >= N ? g - N : g; }

// Even/odd application of a 1D operator T (NO x NI) whose entries satisfy
// T[NO-1-a][NI-1-b] = S T[a][b] (S = +1 for the interpolation l_i(x_q) and
// its transpose, -1 for the collocation derivative and its transpose: the
// GLL nodes and Gauss points are symmetric about the cell midpoint).  With
// pe_b = v_b + v_{NI-1-b}, me_b = v_b - v_{NI-1-b} (b < NI/2, pe of the
// middle entry = v_mid) and the tables E = (T[a][b] + T[a][NI-1-b]) / 2,
// O = (T[a][b] - T[a][NI-1-b]) / 2 over the first ceil(NO/2) rows,
// e_a = E pe, o_a = O me give out[a] = e_a + o_a and
// out[NO-1-a] = S (e_a - o_a): half the multiplications of T v.
template <int NI, int NO, int S>
__device__ __forceinline__ void eo_apply(const double *E, const double *O, const double (&v)[NI], double (&out)[NO]) {
    constexpr int HI = NI / 2, HIC = (NI + 1) / 2, HO = (NO + 1) / 2;
    double pe[HIC], me[HI > 0 ? HI : 1];
#pragma unroll
    for (int b = 0; b < HI; ++b) {
        pe[b] = v[b] + v[NI - 1 - b];
        me[b] = v[b] - v[NI - 1 - b];
    }
    if constexpr (NI & 1) pe[HI] = v[HI];
#pragma unroll
    for (int a = 0; a < HO; ++a) {
        double e = 0, o = 0;
#pragma unroll
        for (int b = 0; b < HIC; ++b) e += E[a * HIC + b] * pe[b];
#pragma unroll
        for (int b = 0; b < HI; ++b) o += O[a * HI + b] * me[b];
        out[a] = e + o;
        if (NO - 1 - a != a) out[NO - 1 - a] = S > 0 ? e - o : o - e;
    }
}

// offsets of the even/odd tables in KxParams::tab (built by the host in the
// same order): interpolation N (Q1 x N1), its transpose (N1 x Q1), the
// derivative Dq (Q1 x Q1), its transpose, then the 1D Gauss weights
template <int N1, int Q1>
struct KxTab {
    static constexpr int sz(int no, int ni) { return (no + 1) / 2 * ni; }  // E and O together
    static constexpr int NE = 0, NO = NE + (Q1 + 1) / 2 * ((N1 + 1) / 2);
    static constexpr int TE = NE + sz(Q1, N1), TO = TE + (N1 + 1) / 2 * ((Q1 + 1) / 2);
    static constexpr int DE = TE + sz(N1, Q1), DO = DE + (Q1 + 1) / 2 * ((Q1 + 1) / 2);
    static constexpr int XE = DE + sz(Q1, Q1), XO = XE + (Q1 + 1) / 2 * ((Q1 + 1) / 2);
    static constexpr int W = XE + sz(Q1, Q1);
    static constexpr int total = W + Q1;
};

// w[idx] for a lane-dependent idx without indexing the kernel-argument
// table dynamically (which would force a private copy of it)
template <int Q>
__device__ __forceinline__ double pick(const double *w, int idx) {
    double r = 0;
#pragma unroll
    for (int t = 0; t < Q; ++t) r = t == idx ? w[t] : r;
    return r;
}

// The five layouts the kernel's LDS cube takes in turn: plane (qz) stride P
// and row stride R in doubles, for X[qz][row][col] at qz P + row R + col.
// A1 = z-interpolated nodes [qz][j][i], B2 = [qz][qy][i], A3 = Gauss-point
// values [qz][qy][qx] (then the gradient terms), A6 = [qz][qy][i],
// B7 = [qz][j][i].  The
// strides are chosen so that the 64-bit accesses of each phase (lanes
// running over two of the three indices) spread over the 64 LDS banks:
// at most two lanes of a 32-lane pass share a bank (the unpadded cubes
// have up to eight).
template <int N1, int Q1> struct KxLds;
#define KX_LDS(N, Q, PA1, RA1, PB2, RB2, PA3, RA3, PA6, RA6, PB7, RB7)                                          \
    template <> struct KxLds<N, Q> {                                                                            \
        static constexpr int pA1 = PA1, rA1 = RA1, pB2 = PB2, rB2 = RB2, pA3 = PA3, rA3 = RA3, pA6 = PA6,       \
                             rA6 = RA6, pB7 = PB7, rB7 = RB7;                                                   \
        static constexpr int size = Q * cmax3(cmax3(PA1, PA3, PA6), PB2, PB7);                                  \
    };
KX_LDS(2, 2, 4, 2, 4, 2, 4, 2, 4, 2, 4, 2)
KX_LDS(2, 3, 4, 2, 6, 2, 9, 3, 6, 2, 4, 2)
KX_LDS(3, 3, 9, 3, 9, 3, 9, 3, 9, 3, 9, 3)
KX_LDS(3, 4, 9, 3, 12, 3, 19, 4, 12, 3, 9, 3)
KX_LDS(4, 4, 18, 4, 19, 4, 19, 4, 19, 4, 18, 4)
KX_LDS(4, 5, 18, 4, 25, 5, 25, 5, 25, 5, 18, 4)
KX_LDS(5, 5, 26, 5, 37, 7, 25, 5, 37, 7, 26, 5)
KX_LDS(5, 6, 27, 5, 37, 6, 36, 6, 37, 6, 27, 5)
KX_LDS(6, 6, 38, 6, 42, 7, 36, 6, 42, 7, 38, 6)
KX_LDS(6, 7, 38, 6, 70, 7, 51, 7, 70, 7, 38, 6)
KX_LDS(7, 7, 71, 7, 71, 8, 51, 7, 71, 8, 71, 7)
KX_LDS(7, 8, 71, 7, 103, 12, 72, 9, 103, 12, 71, 7)
KX_LDS(8, 8, 72, 8, 72, 9, 72, 9, 72, 9, 72, 8)
#undef KX_LDS

template <int N1, int Q1>
__global__ __launch_bounds__(64) void kx_kernel(const KxParams a) {
    using T = KxTab<N1, Q1>;
    static_assert(T::total <= kPoiTab, "1D tables exceed the kernel-argument area");
    using L = KxLds<N1, Q1>;
    static_assert(L::rA1 >= N1 && L::pA1 >= N1 * L::rA1 && L::rB2 >= N1 && L::pB2 >= Q1 * L::rB2 &&
                      L::rA3 >= Q1 && L::pA3 >= Q1 * L::rA3 && L::rA6 >= N1 && L::pA6 >= Q1 * L::rA6 &&
                      L::rB7 >= N1 && L::pB7 >= N1 * L::rB7,
                  "LDS strides must not overlap rows or planes");
    // one LDS cube, re-laid out by every phase: each phase reads its lines
    // into registers, waits, then writes its results over the cube, so a
    // wave needs a single cube (the barriers of a one-wave workgroup are
    // nearly free) and more waves fit a CU
    __shared__ double C[L::size];
    // the 1D tables are kernel arguments: after unrolling every index is a
    // constant, so they are read through scalar loads into SGPRs
    const double *tw = a.tab + T::W;
    const int lane = threadIdx.x;
    const int64_t e = xcd_remap(blockIdx.x, a.ncells);
    const int64_t ex = e % a.ncx, ey = (e / a.ncx) % a.ncy, ez = e / (a.ncx * a.ncy);
    const int64_t NxNy = a.Nx * a.Ny;
    // z-line of lane (j, i): global offsets of its nodes
    const int li = lane % N1, lj = lane / N1;
    const int64_t base = wrap1(ex * a.p + li, a.Nx) + a.Nx * wrap1(ey * a.p + lj, a.Ny);
    const int64_t gz0 = ez * a.p;

    // 1: gather the z-line into registers and interpolate along z -> C[qz][j][i]
    if (lane < N1 * N1) {
        double xv[N1], o[Q1];
#pragma unroll
        for (int k = 0; k < N1; ++k) xv[k] = a.x[base + NxNy * wrap1(gz0 + k, a.Nz)];
        eo_apply<N1, Q1, 1>(a.tab + T::NE, a.tab + T::NO, xv, o);
#pragma unroll
        for (int qz = 0; qz < Q1; ++qz) C[qz * L::pA1 + lj * L::rA1 + li] = o[qz];
    }
    __syncthreads();
    // 2: along y, lane (qz, i) -> C[qz][qy][i]
    {
        const int qz = lane / N1, i = lane % N1;
        const bool act = lane < Q1 * N1;
        double v[N1], o[Q1];
        if (act) {
#pragma unroll
            for (int j = 0; j < N1; ++j) v[j] = C[qz * L::pA1 + j * L::rA1 + i];
        }
        __syncthreads();
        if (act) {
            eo_apply<N1, Q1, 1>(a.tab + T::NE, a.tab + T::NO, v, o);
#pragma unroll
            for (int qy = 0; qy < Q1; ++qy) C[qz * L::pB2 + qy * L::rB2 + i] = o[qy];
        }
    }
    __syncthreads();
    // 3: along x, lane (qz, qy): values at the Gauss points -> C[qz][qy][qx];
    //    the x-gradient line and its transposed derivative stay in registers
    double ux[Q1];
    {
        const int qz = lane / Q1, qy = lane % Q1;
        const bool act = lane < Q1 * Q1;
        double v[N1], u[Q1], g[Q1];
        if (act) {
#pragma unroll
            for (int i = 0; i < N1; ++i) v[i] = C[qz * L::pB2 + qy * L::rB2 + i];
        }
        __syncthreads();
        if (act) {
            eo_apply<N1, Q1, 1>(a.tab + T::NE, a.tab + T::NO, v, u);
#pragma unroll
            for (int qx = 0; qx < Q1; ++qx) C[qz * L::pA3 + qy * L::rA3 + qx] = u[qx];
            eo_apply<Q1, Q1, -1>(a.tab + T::DE, a.tab + T::DO, u, g);
            const double wzy = pick<Q1>(tw, qz) * pick<Q1>(tw, qy) * a.cx;
#pragma unroll
            for (int t = 0; t < Q1; ++t) g[t] *= wzy * tw[t];
            eo_apply<Q1, Q1, -1>(a.tab + T::XE, a.tab + T::XO, g, ux);
        }
    }
    __syncthreads();
    // 4, 5: lane (b, qx) reads the y-line (qz = b) and the z-line (qy = b) of
    //    the values, then writes Dq^T (W_y dy u) over the cube and adds
    //    Dq^T (W_z dz u) to it
    {
        const int b = lane / Q1, qx = lane % Q1;
        const bool act = lane < Q1 * Q1;
        double uy[Q1], uz[Q1], g[Q1], h[Q1];
        if (act) {
#pragma unroll
            for (int t = 0; t < Q1; ++t) {
                uy[t] = C[b * L::pA3 + t * L::rA3 + qx];
                uz[t] = C[t * L::pA3 + b * L::rA3 + qx];
            }
        }
        __syncthreads();
        const double wb = pick<Q1>(tw, b) * pick<Q1>(tw, qx);
        if (act) {
            eo_apply<Q1, Q1, -1>(a.tab + T::DE, a.tab + T::DO, uy, g);
#pragma unroll
            for (int t = 0; t < Q1; ++t) g[t] *= wb * a.cy * tw[t];
            eo_apply<Q1, Q1, -1>(a.tab + T::XE, a.tab + T::XO, g, h);
#pragma unroll
            for (int qy = 0; qy < Q1; ++qy) C[b * L::pA3 + qy * L::rA3 + qx] = h[qy];
        }
        __syncthreads();
        if (act) {
            eo_apply<Q1, Q1, -1>(a.tab + T::DE, a.tab + T::DO, uz, g);
#pragma unroll
            for (int t = 0; t < Q1; ++t) g[t] *= wb * a.cz * tw[t];
            eo_apply<Q1, Q1, -1>(a.tab + T::XE, a.tab + T::XO, g, h);
#pragma unroll
            for (int qz = 0; qz < Q1; ++qz) C[qz * L::pA3 + b * L::rA3 + qx] += h[qz];
        }
    }
    __syncthreads();
    // 6: lane (qz, qy): total line, back along x -> C[qz][qy][i]
    {
        const int qz = lane / Q1, qy = lane % Q1;
        const bool act = lane < Q1 * Q1;
        double sq[Q1], o[N1];
        if (act) {
#pragma unroll
            for (int qx = 0; qx < Q1; ++qx) sq[qx] = ux[qx] + C[qz * L::pA3 + qy * L::rA3 + qx];
        }
        __syncthreads();
        if (act) {
            eo_apply<Q1, N1, 1>(a.tab + T::TE, a.tab + T::TO, sq, o);
#pragma unroll
            for (int i = 0; i < N1; ++i) C[qz * L::pA6 + qy * L::rA6 + i] = o[i];
        }
    }
    __syncthreads();
    // 7: back along y, lane (qz, i) -> C[qz][j][i]
    {
        const int qz = lane / N1, i = lane % N1;
        const bool act = lane < Q1 * N1;
        double v[Q1], o[N1];
        if (act) {
#pragma unroll
            for (int qy = 0; qy < Q1; ++qy) v[qy] = C[qz * L::pA6 + qy * L::rA6 + i];
        }
        __syncthreads();
        if (act) {
            eo_apply<Q1, N1, 1>(a.tab + T::TE, a.tab + T::TO, v, o);
#pragma unroll
            for (int j = 0; j < N1; ++j) C[qz * L::pB7 + j * L::rB7 + i] = o[j];
        }
    }
    __syncthreads();
    // 8: back along z in registers, assembled with atomic adds
    if (lane < N1 * N1) {
        double v[Q1], o[N1];
#pragma unroll
        for (int qz = 0; qz < Q1; ++qz) v[qz] = C[qz * L::pB7 + lj * L::rB7 + li];
        eo_apply<Q1, N1, 1>(a.tab + T::TE, a.tab + T::TO, v, o);
#pragma unroll
        for (int k = 0; k < N1; ++k) atomicAdd(a.y + base + NxNy * wrap1(gz0 + k, a.Nz), o[k]);
    }
}

// ---------------------------------------------------------------- reductions
// Deterministic two-stage sums: each of kDotBlocks workgroups reduces a
// grid-stride share (wave shuffles, then the four waves in a fixed order)
// and writes its partials; one workgroup adds the partials as a fixed tree.
constexpr int kDotBlocks = 512;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// part[2 b + 0] = sum a.b (b == nullptr: sum a), part[2 b + 1] = sum c.d (c == nullptr: 0)
__global__ __launch_bounds__(256) void dot2_partial_kernel(int64_t n, const double *a, const double *b,
                                                          const double *c, const double *d, double *part) {
    __shared__ double s0[4], s1[4];
    double u = 0, v = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        u += b ? a[i] * b[i] : a[i];
        if (c) v += c[i] * d[i];
    }
    u = wave_sum(u);
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s0[w] = u;
        s1[w] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = (s0[0] + s0[1]) + (s0[2] + s0[3]);
        part[2 * blockIdx.x + 1] = (s1[0] + s1[1]) + (s1[2] + s1[3]);
    }
}

// op PCG_SUMS:  sc[SUM0], sc[SUM1] = the two sums
// op PCG_ETA:   sc[ETA] = sum0
// op PCG_FIRST: sc[DELTA] = sum0, sc[GAMMA] = sum1 (first iteration)
// op PCG_NEXT:  sc[BETA] = sum0 / sc[DELTA], sc[DELTA] = sum0, sc[GAMMA] = sum1
__global__ __launch_bounds__(256) void dot2_finish_kernel(const double *part, int op, double *sc) {
    __shared__ double s0[256], s1[256];
    const int t = threadIdx.x;
    s0[t] = part[2 * t] + part[2 * (t + 256)];
    s1[t] = part[2 * t + 1] + part[2 * (t + 256) + 1];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            s0[t] += s0[t + h];
            s1[t] += s1[t + h];
        }
        __syncthreads();
    }
    if (t != 0) return;
    const double u = s0[0], v = s1[0];
    switch (op) {
    case PCG_SUMS:
        sc[SC_SUM0] = u;
        sc[SC_SUM1] = v;
        break;
    case PCG_ETA:
        sc[SC_ETA] = u;
        break;
    case PCG_FIRST:
        sc[SC_DELTA] = u;
        sc[SC_GAMMA] = v;
        break;
    default:
        sc[SC_BETA] = u / sc[SC_DELTA];
        sc[SC_DELTA] = u;
        sc[SC_GAMMA] = v;
        break;
    }
}

// ---------------------------------------------------------------- PCG vectors
// fused update: alpha = delta / eta, x += alpha p, r += alpha w (one pass)
__global__ void pcg_update_kernel(int64_t n, const double *sc, const double *p, const double *w, double *x,
                                  double *r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double alpha = sc[SC_DELTA] / sc[SC_ETA];
    x[i] += alpha * p[i];
    r[i] += alpha * w[i];
}

// p = -z + beta p (first: p = -z)
__global__ void pcg_dir_kernel(int64_t n, const double *sc, bool first, const double *z, double *p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    p[i] = first ? -z[i] : -z[i] + sc[SC_BETA] * p[i];
}

// r = K x - (f - mean f), mean f = sc[SUM0] / n
__global__ void pcg_init_kernel(int64_t n, const double *sc, const double *Kx, const double *f, double *r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    r[i] = Kx[i] - (f[i] - sc[SC_SUM0] / (double)n);
}

// x -= sc[SUM0] / n (zero-mean representative of the periodic solution)
__global__ void sub_mean_kernel(int64_t n, const double *sc, double *x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    x[i] -= sc[SC_SUM0] / (double)n;
}

// Chebyshev step on D^-1 K z = D^-1 r, D = diag(K), from z_0 = 0:
//   first: d = c2 D^-1 r, z = d
//   else:  d = c1 d + c2 D^-1 (r - K z), z += d
__global__ void cheb_step_kernel(int64_t n, bool first, double c1, double c2, const double *dinv, const double *r,
                                 const double *Kz, double *d, double *z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (first) {
        const double v = c2 * dinv[i] * r[i];
        d[i] = v;
        z[i] = v;
        return;
    }
    const double v = c1 * d[i] + c2 * dinv[i] * (r[i] - Kz[i]);
    d[i] = v;
    z[i] += v;
}

// The last Chebyshev step fused with the PCG's (r.z, r.r) partial sums:
// z += c1 d + c2 D^-1 (r - K z) (first: z = c2 D^-1 r), d is not kept; the
// grid (kDotBlocks x 256, grid-stride) and the reduction are those of
// dot2_partial_kernel, so the partial sums are the same bits as a separate
// pass over r and z would give.
__global__ __launch_bounds__(256) void cheb_last_dot_kernel(int64_t n, bool first, double c1, double c2,
                                                            const double *dinv, const double *r, const double *Kz,
                                                            const double *d, double *z, double *part) {
    __shared__ double s0[4], s1[4];
    double u = 0, v = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double ri = r[i];
        const double zi = first ? c2 * dinv[i] * ri : z[i] + (c1 * d[i] + c2 * dinv[i] * (ri - Kz[i]));
        z[i] = zi;
        u += ri * zi;
        v += ri * ri;
    }
    u = wave_sum(u);
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s0[w] = u;
        s1[w] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = (s0[0] + s0[1]) + (s0[2] + s0[3]);
        part[2 * blockIdx.x + 1] = (s1[0] + s1[1]) + (s1[2] + s1[3]);
    }
}

// y = s (alpha x + beta y); x may be null (y = s beta y), s may be null (no scale)
__global__ void axpby_real_kernel(int64_t n, double alpha, const double *x, double beta, double *y,
                                  const double *s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = beta * y[i] + (x ? alpha * x[i] : 0.0);
    y[i] = s ? s[i] * v : v;
}

// Start vector of the Lanczos run: splitmix64 (Steele, Lea and Flood 2014)
// of the state seed + (i + 1) 0x9E3779B97F4A7C15, top 53 bits as a uniform
// double in [-0.5, 0.5).
__global__ void splitmix_kernel(int64_t n, uint64_t seed, double *v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    v[i] = (double)(z >> 11) * 0x1.0p-53 - 0.5;
}

__global__ void sqrt_kernel(int64_t n, const double *x, double *y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = sqrt(x[i]);
}

static dim3 g1(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

template <int N1, int Q1>
static void kx_go(const KxParams &a, int64_t ncells, hipStream_t s) {
    hipLaunchKernelGGL((kx_kernel<N1, Q1>), dim3((unsigned)ncells), dim3(64), 0, s, a);
}

bool kx_supported(int n1, int q1) { return n1 >= 2 && n1 <= 8 && (q1 == n1 || (q1 == n1 + 1 && q1 <= 8)); }

hipError_t launch_kx(const chfsi_ctx *c, const double *x, double *y, hipStream_t s) {
    const Mesh &m = c->m;
    if (!kx_supported(m.n1, m.nq1)) return hipErrorInvalidValue;
    hipError_t e = hipMemsetAsync(y, 0, (size_t)m.M * sizeof(double), s);
    if (e != hipSuccess) return e;
    KxParams a{};
    a.x = x;
    a.y = y;
    a.ncx = m.ncell[0];
    a.ncy = m.ncell[1];
    a.ncells = m.ncells;
    a.Nx = m.Nd[0];
    a.Ny = m.Nd[1];
    a.Nz = m.Nd[2];
    a.p = m.p;
    for (int i = 0; i < kPoiTab; ++i) a.tab[i] = c->poi_tab[i];
    const double detJ = m.h[0] * m.h[1] * m.h[2] / 8.0;
    a.cx = detJ * 4.0 / (m.h[0] * m.h[0]);
    a.cy = detJ * 4.0 / (m.h[1] * m.h[1]);
    a.cz = detJ * 4.0 / (m.h[2] * m.h[2]);
    switch (m.n1 * 16 + m.nq1) {
#define KX_CASE(N, Q) \
    case N * 16 + Q: kx_go<N, Q>(a, m.ncells, s); break;
        KX_CASE(2, 2) KX_CASE(2, 3) KX_CASE(3, 3) KX_CASE(3, 4) KX_CASE(4, 4) KX_CASE(4, 5) KX_CASE(5, 5)
        KX_CASE(5, 6) KX_CASE(6, 6) KX_CASE(6, 7) KX_CASE(7, 7) KX_CASE(7, 8) KX_CASE(8, 8)
#undef KX_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dot2(int64_t n, const double *a, const double *b, const double *c, const double *d, double *part,
                       int op, double *sc, hipStream_t s) {
    static_assert(kDotBlocks == 512, "the finish kernel folds 512 partials");
    hipLaunchKernelGGL(dot2_partial_kernel, dim3(kDotBlocks), dim3(256), 0, s, n, a, b, c, d, part);
    hipLaunchKernelGGL(dot2_finish_kernel, dim3(1), dim3(256), 0, s, (const double *)part, op, sc);
    return hipGetLastError();
}

hipError_t launch_pcg_update(int64_t n, const double *sc, const double *p, const double *w, double *x, double *r,
                             hipStream_t s) {
    hipLaunchKernelGGL(pcg_update_kernel, g1(n), dim3(256), 0, s, n, sc, p, w, x, r);
    return hipGetLastError();
}

hipError_t launch_pcg_dir(int64_t n, const double *sc, bool first, const double *z, double *p, hipStream_t s) {
    hipLaunchKernelGGL(pcg_dir_kernel, g1(n), dim3(256), 0, s, n, sc, first, z, p);
    return hipGetLastError();
}

hipError_t launch_pcg_init(int64_t n, const double *sc, const double *Kx, const double *f, double *r,
                           hipStream_t s) {
    hipLaunchKernelGGL(pcg_init_kernel, g1(n), dim3(256), 0, s, n, sc, Kx, f, r);
    return hipGetLastError();
}

hipError_t launch_sub_mean(int64_t n, const double *sc, double *x, hipStream_t s) {
    hipLaunchKernelGGL(sub_mean_kernel, g1(n), dim3(256), 0, s, n, sc, x);
    return hipGetLastError();
}

hipError_t launch_cheb_step(int64_t n, bool first, double c1, double c2, const double *dinv, const double *r,
                            const double *Kz, double *d, double *z, hipStream_t s) {
    hipLaunchKernelGGL(cheb_step_kernel, g1(n), dim3(256), 0, s, n, first, c1, c2, dinv, r, Kz, d, z);
    return hipGetLastError();
}

hipError_t launch_cheb_last_dot(int64_t n, bool first, double c1, double c2, const double *dinv, const double *r,
                                const double *Kz, const double *d, double *z, double *part, int op, double *sc,
                                hipStream_t s) {
    hipLaunchKernelGGL(cheb_last_dot_kernel, dim3(kDotBlocks), dim3(256), 0, s, n, first, c1, c2, dinv, r, Kz, d, z,
                       part);
    hipLaunchKernelGGL(dot2_finish_kernel, dim3(1), dim3(256), 0, s, (const double *)part, op, sc);
    return hipGetLastError();
}

hipError_t launch_axpby_real(int64_t n, double alpha, const double *x, double beta, double *y,
                             const double *scale, hipStream_t s) {
    hipLaunchKernelGGL(axpby_real_kernel, g1(n), dim3(256), 0, s, n, alpha, x, beta, y, scale);
    return hipGetLastError();
}

hipError_t launch_splitmix(int64_t n, uint64_t seed, double *v, hipStream_t s) {
    hipLaunchKernelGGL(splitmix_kernel, g1(n), dim3(256), 0, s, n, seed, v);
    return hipGetLastError();
}

hipError_t launch_sqrt(int64_t n, const double *x, double *y, hipStream_t s) {
    hipLaunchKernelGGL(sqrt_kernel, g1(n), dim3(256), 0, s, n, x, y);
    return hipGetLastError();
}

}  // namespace chfsi
