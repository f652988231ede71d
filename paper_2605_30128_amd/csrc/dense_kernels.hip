// Small dense FP64 kernels of the Rayleigh-Ritz stage (matrices of the
// subspace size N, row-major complex128): Hermitian equilibration, Cholesky
// factorisation, the triangular inverse that turns a Cholesky factor into
// the orthonormalizing transform, and the dense Hermitian eigensolve
// (parallel cyclic Jacobi: every round rotates N/2 disjoint index pairs in a
// round-robin order, reading the previous iterate and writing the next one,
// so one launch per round has no intra-launch dependencies).
#include <cmath>
#include <vector>

#include "internal.h"

namespace chfsi {

// ---------------------------------------------------------------------------
// S <- diag(s) (S + S^H)/2 diag(s), s_i = 1 / sqrt(Re S_ii)
// ---------------------------------------------------------------------------
__global__ void equil_scale_kernel(int N, const cd *S, double *scale, int *flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double d = S[(int64_t)i * N + i].x;
    if (!(d > 0.0) || !isfinite(d)) {
        *flag = 1;
        scale[i] = 1.0;
    } else {
        scale[i] = 1.0 / sqrt(d);
    }
}

__global__ void equil_apply_kernel(int N, cd *S, const double *scale) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)N * N) return;
    int i = (int)(idx / N), j = (int)(idx % N);
    if (j > i) return;  // lower thread handles the pair (i, j), (j, i)
    cd a = S[(int64_t)i * N + j], b = S[(int64_t)j * N + i];
    double sc = scale ? scale[i] * scale[j] : 1.0;
    cd h;
    h.x = 0.5 * (a.x + b.x) * sc;
    h.y = 0.5 * (a.y - b.y) * sc;
    S[(int64_t)i * N + j] = h;
    h.y = -h.y;
    if (i == j) h.y = 0;
    S[(int64_t)j * N + i] = h;
}

// out = sum over the nparts partial matrices, in order
__global__ void sum_parts_kernel(int64_t n, int nparts, const cd *parts, cd *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x = 0, y = 0;
    for (int p = 0; p < nparts; ++p) {
        cd v = parts[(int64_t)p * n + i];
        x += v.x;
        y += v.y;
    }
    out[i] = cd{x, y};
}

hipError_t launch_sum_parts(int64_t n, int nparts, const cd *parts, cd *out, hipStream_t s) {
    hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, nparts, parts, out);
    return hipGetLastError();
}

hipError_t launch_herm_equilibrate(int N, cd *S, double *scale, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(equil_scale_kernel, dim3((N + 255) / 256), dim3(256), 0, s, N, S, scale, flag);
    int64_t nn = (int64_t)N * N;
    hipLaunchKernelGGL(equil_apply_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, N, S, scale);
    return hipGetLastError();
}

hipError_t launch_hermitize(int N, cd *S, hipStream_t s) {
    int64_t nn = (int64_t)N * N;
    hipLaunchKernelGGL(equil_apply_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, N, S,
                       (const double *)nullptr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// in-place Cholesky A = L L^H of an n x n diagonal block (row stride lda;
// lower L, the block's strict upper triangle is zeroed).  One workgroup:
// right-looking, column by column.  The matrices factored here are
// equilibrated to a unit diagonal, so a pivot below 64 eps means the block
// is numerically rank deficient: flag = 1.  The blocked factorization of the
// whole matrix (panel solves and trailing updates as BLAS-3 calls) is
// driven from the host.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void cholesky_block_kernel(int n, int lda, cd *A, int *flag) {
    __shared__ double djj;
    __shared__ int bad;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (tid == 0) {
            double d = A[(int64_t)j * lda + j].x;
            if (!(d > 64.0 * 2.220446049250313e-16) || !isfinite(d)) {
                bad = 1;
                d = 1.0;
            }
            djj = sqrt(d);
            A[(int64_t)j * lda + j] = cd{djj, 0.0};
        }
        __syncthreads();
        if (bad) break;
        const double inv = 1.0 / djj;
        for (int i = j + 1 + tid; i < n; i += nt) {
            cd v = A[(int64_t)i * lda + j];
            v.x *= inv;
            v.y *= inv;
            A[(int64_t)i * lda + j] = v;
        }
        __syncthreads();
        const int m = n - j - 1;
        for (int idx = tid; idx < m * m; idx += nt) {
            const int i = j + 1 + idx / m, k = j + 1 + idx % m;
            if (k > i) continue;
            const cd lij = A[(int64_t)i * lda + j], lkj = A[(int64_t)k * lda + j];
            cd v = A[(int64_t)i * lda + k];
            // v -= lij * conj(lkj)
            v.x -= lij.x * lkj.x + lij.y * lkj.y;
            v.y -= lij.y * lkj.x - lij.x * lkj.y;
            A[(int64_t)i * lda + k] = v;
        }
        __syncthreads();
    }
    if (bad) {
        if (tid == 0) *flag = 1;
        return;
    }
    for (int idx = tid; idx < n * n; idx += nt) {
        const int i = idx / n, k = idx % n;
        if (k > i) A[(int64_t)i * lda + k] = cd{0.0, 0.0};
    }
}

hipError_t launch_cholesky_block(int n, int lda, cd *A, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(cholesky_block_kernel, dim3(1), dim3(1024), 0, s, n, lda, A, flag);
    return hipGetLastError();
}

// zero the strict upper triangle of a row-major N x N matrix (the blocks
// right of the diagonal blocks, which the blocked factorization leaves alone)
__global__ void zero_upper_kernel(int N, cd *A) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)N * N) return;
    const int i = (int)(idx / N), k = (int)(idx % N);
    if (k > i) A[idx] = cd{0.0, 0.0};
}

// T = diag(scale) (identity if scale is null), the right-hand side of the
// triangular solve that forms diag(scale) L^{-H}
__global__ void diag_kernel(int N, const double *scale, cd *T) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)N * N) return;
    const int i = (int)(idx / N), k = (int)(idx % N);
    T[idx] = cd{i == k ? (scale ? scale[i] : 1.0) : 0.0, 0.0};
}

// B = A diag(w) for row-major N x N matrices (column j scaled by w[j])
__global__ void scale_cols_kernel(int N, const double *w, const cd *A, cd *B) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)N * N) return;
    const double f = w[idx % N];
    B[idx] = cd{A[idx].x * f, A[idx].y * f};
}

hipError_t launch_scale_cols(int N, const double *w, const cd *A, cd *B, hipStream_t s) {
    const int64_t nn = (int64_t)N * N;
    hipLaunchKernelGGL(scale_cols_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, N, w, A, B);
    return hipGetLastError();
}

// strict lower triangle of a row-major N x N matrix := conjugate of the upper
__global__ void fill_lower_kernel(int N, cd *A) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)N * N) return;
    const int i = (int)(idx / N), k = (int)(idx % N);
    if (i > k) {
        const cd u = A[(int64_t)k * N + i];
        A[idx] = cd{u.x, -u.y};
    }
}

hipError_t launch_fill_lower(int N, cd *A, hipStream_t s) {
    const int64_t nn = (int64_t)N * N;
    hipLaunchKernelGGL(fill_lower_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, N, A);
    return hipGetLastError();
}

// Q32 = complex64 copy of the N x N matrix Q with its diagonal bs x bs blocks zeroed
__global__ void offdiag_cf_kernel(int N, int bs, const cd *Q, cf *Q32) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)N * N) return;
    const int i = (int)(idx / N), k = (int)(idx % N);
    const cd q = Q[idx];
    Q32[idx] = (i / bs == k / bs) ? cf{0.f, 0.f} : cf{(float)q.x, (float)q.y};
}

hipError_t launch_offdiag_cf(int N, int bs, const cd *Q, cf *Q32, hipStream_t s) {
    const int64_t nn = (int64_t)N * N;
    hipLaunchKernelGGL(offdiag_cf_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, N, bs, Q, Q32);
    return hipGetLastError();
}

hipError_t launch_zero_upper(int N, cd *A, hipStream_t s) {
    const int64_t nn = (int64_t)N * N;
    hipLaunchKernelGGL(zero_upper_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, N, A);
    return hipGetLastError();
}

hipError_t launch_diag(int N, const double *scale, cd *T, hipStream_t s) {
    const int64_t nn = (int64_t)N * N;
    hipLaunchKernelGGL(diag_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, N, scale, T);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// parallel cyclic Jacobi
// ---------------------------------------------------------------------------
// round-robin pairing of N2 (even) indices: index 0 fixed, the rest rotate
__device__ __forceinline__ void rr_pair(int i, int r, int N2, int &a, int &b) {
    auto pos = [&](int k) { return k == 0 ? 0 : 1 + (k - 1 + r) % (N2 - 1); };
    a = pos(i);
    b = pos(N2 - 1 - i);
    if (a > b) { int t = a; a = b; b = t; }
}

struct Rot { double c, s; cd ph; bool id; };  // G = diag(1, conj(ph)) [[c, s], [-s, c]]

__device__ __forceinline__ Rot make_rot(const cd *A, int N, int a, int b) {
    Rot R;
    R.c = 1; R.s = 0; R.ph = cd{1, 0}; R.id = true;
    if (b >= N) return R;
    cd apq = A[(int64_t)a * N + b];
    double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
    if (mag == 0.0) return R;
    double app = A[(int64_t)a * N + a].x, aqq = A[(int64_t)b * N + b].x;
    double tau = (aqq - app) / (2.0 * mag);
    double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    R.c = 1.0 / sqrt(1.0 + t * t);
    R.s = t * R.c;
    R.ph = cd{apq.x / mag, apq.y / mag};
    R.id = false;
    return R;
}

// G entries: gaa = c, gab = s, gba = -s conj(ph), gbb = c conj(ph)
__device__ __forceinline__ void rot_entries(const Rot &R, cd &gaa, cd &gab, cd &gba, cd &gbb) {
    gaa = cd{R.c, 0};
    gab = cd{R.s, 0};
    gba = cd{-R.s * R.ph.x, R.s * R.ph.y};
    gbb = cd{R.c * R.ph.x, -R.c * R.ph.y};
}

__device__ __forceinline__ cd cmul(cd a, cd b) { return cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return cd{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd cconj(cd a) { return cd{a.x, -a.y}; }

// one round: A2 = G^H A G, V2 = V G (G block diagonal over the round's pairs)
__global__ void jacobi_round_kernel(int N, int N2, int r, const cd *A, cd *A2, const cd *V, cd *V2) {
    const int H = N2 / 2;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nblk = (int64_t)H * H;
    if (idx < nblk) {
        int bi = (int)(idx / H), bj = (int)(idx % H);
        int a1, b1, a2, b2;
        rr_pair(bi, r, N2, a1, b1);
        rr_pair(bj, r, N2, a2, b2);
        Rot R1 = make_rot(A, N, a1, b1), R2 = make_rot(A, N, a2, b2);
        cd g1[4], g2[4];
        rot_entries(R1, g1[0], g1[1], g1[2], g1[3]);
        rot_entries(R2, g2[0], g2[1], g2[2], g2[3]);
        auto ld = [&](int x, int y) { return (x < N && y < N) ? A[(int64_t)x * N + y] : cd{0, 0}; };
        cd m00 = ld(a1, a2), m01 = ld(a1, b2), m10 = ld(b1, a2), m11 = ld(b1, b2);
        // T = M G2
        cd t00 = cadd(cmul(m00, g2[0]), cmul(m01, g2[2]));
        cd t01 = cadd(cmul(m00, g2[1]), cmul(m01, g2[3]));
        cd t10 = cadd(cmul(m10, g2[0]), cmul(m11, g2[2]));
        cd t11 = cadd(cmul(m10, g2[1]), cmul(m11, g2[3]));
        // G1^H T
        cd n00 = cadd(cmul(cconj(g1[0]), t00), cmul(cconj(g1[2]), t10));
        cd n01 = cadd(cmul(cconj(g1[0]), t01), cmul(cconj(g1[2]), t11));
        cd n10 = cadd(cmul(cconj(g1[1]), t00), cmul(cconj(g1[3]), t10));
        cd n11 = cadd(cmul(cconj(g1[1]), t01), cmul(cconj(g1[3]), t11));
        if (bi == bj && !R1.id) {  // the annihilated pivot block
            n01 = cd{0, 0};
            n10 = cd{0, 0};
            n00.y = 0;
            n11.y = 0;
        }
        if (a1 < N && a2 < N) A2[(int64_t)a1 * N + a2] = n00;
        if (a1 < N && b2 < N) A2[(int64_t)a1 * N + b2] = n01;
        if (b1 < N && a2 < N) A2[(int64_t)b1 * N + a2] = n10;
        if (b1 < N && b2 < N) A2[(int64_t)b1 * N + b2] = n11;
        return;
    }
    idx -= nblk;
    if (idx >= (int64_t)N * H) return;
    int x = (int)(idx / H), bj = (int)(idx % H);
    int a2, b2;
    rr_pair(bj, r, N2, a2, b2);
    Rot R2 = make_rot(A, N, a2, b2);
    cd g[4];
    rot_entries(R2, g[0], g[1], g[2], g[3]);
    cd va = a2 < N ? V[(int64_t)x * N + a2] : cd{0, 0};
    cd vb = b2 < N ? V[(int64_t)x * N + b2] : cd{0, 0};
    if (a2 < N) V2[(int64_t)x * N + a2] = cadd(cmul(va, g[0]), cmul(vb, g[2]));
    if (b2 < N) V2[(int64_t)x * N + b2] = cadd(cmul(va, g[1]), cmul(vb, g[3]));
}

__global__ void identity_kernel(int N, cd *V) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)N * N) return;
    int i = (int)(idx / N), j = (int)(idx % N);
    V[idx] = cd{i == j ? 1.0 : 0.0, 0.0};
}

// red[0] = sum_{i != j} |A_ij|^2, red[1] = sum_i |A_ii|^2 (one workgroup, fixed order)
__global__ void offnorm_kernel(int N, const cd *A, double *out) {
    __shared__ double so[256], sd[256];
    double o = 0, d = 0;
    for (int64_t idx = threadIdx.x; idx < (int64_t)N * N; idx += blockDim.x) {
        int i = (int)(idx / N), j = (int)(idx % N);
        cd v = A[idx];
        double m2 = v.x * v.x + v.y * v.y;
        if (i == j) d += m2; else o += m2;
    }
    so[threadIdx.x] = o;
    sd[threadIdx.x] = d;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            so[threadIdx.x] += so[threadIdx.x + w];
            sd[threadIdx.x] += sd[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = so[0]; out[1] = sd[0]; }
}

// w = Re diag(A) sorted ascending (ties by index), columns of V permuted alike
__global__ void sort_eig_kernel(int N, const cd *A, const cd *V, double *wout, cd *Vout) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)N * N) return;
    int x = (int)(idx / N), i = (int)(idx % N);
    double wi = A[(int64_t)i * N + i].x;
    int rank = 0;
    for (int j = 0; j < N; ++j) {
        double wj = A[(int64_t)j * N + j].x;
        rank += (wj < wi) || (wj == wi && j < i);
    }
    Vout[(int64_t)x * N + rank] = V[(int64_t)x * N + i];
    if (x == 0) wout[rank] = wi;
}

hipError_t launch_jacobi_eig(int N, cd *A, cd *A2, cd *V, cd *V2, double *w, double *red,
                             int max_sweeps, hipStream_t s, int *sweeps_out, cd **Vout) {
    // A (input, destroyed), A2/V/V2 workspaces; on return *Vout = eigenvectors
    // (columns, ascending) in one of V/V2, w = eigenvalues.
    const int N2 = N + (N & 1);
    const int H = N2 / 2;
    int64_t nn = (int64_t)N * N;
    hipLaunchKernelGGL(identity_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, N, V);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    cd *a = A, *a2 = A2, *v = V, *v2 = V2;
    double host[2];
    int sweep = 0;
    const int64_t nthr = (int64_t)H * H + (int64_t)N * H;
    for (; sweep < max_sweeps; ++sweep) {
        hipLaunchKernelGGL(offnorm_kernel, dim3(1), dim3(256), 0, s, N, a, red);
        err = hipMemcpyAsync(host, red, sizeof(host), hipMemcpyDeviceToHost, s);
        if (err != hipSuccess) return err;
        err = hipStreamSynchronize(s);
        if (err != hipSuccess) return err;
        if (!(std::isfinite(host[0]) && std::isfinite(host[1]))) return hipErrorInvalidValue;
        if (host[0] <= 1e-30 * (host[0] + host[1]) || N < 2) break;
        for (int r = 0; r < N2 - 1; ++r) {
            hipLaunchKernelGGL(jacobi_round_kernel, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, N, N2, r,
                               a, a2, v, v2);
            std::swap(a, a2);
            std::swap(v, v2);
        }
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    if (sweeps_out) *sweeps_out = sweep;
    hipLaunchKernelGGL(sort_eig_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, N, a, v, w, v2);
    *Vout = v2;
    return hipGetLastError();
}

}  // namespace chfsi
