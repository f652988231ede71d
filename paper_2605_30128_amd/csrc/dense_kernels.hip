// Small dense FP64 kernels of the Rayleigh-Ritz stage (matrices of the
// subspace size N, row-major complex128): Hermitian equilibration, Cholesky
// factorisation, the triangular inverse that turns a Cholesky factor into
// the orthonormalizing transform, and the conjugate transpose that brings
// the dense eigensolver's column-major eigenvectors into this layout.
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

// Q[x][j] = conj(Z[j][x]): the eigenvectors of a row-major Hermitian A from
// those that a column-major eigensolver returns for the same buffer (it sees
// conj(A), whose eigenvectors are the conjugates of A's).
__global__ void conj_transpose_kernel(int N, const cd *Z, cd *Q) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)N * N) return;
    const int x = (int)(idx / N), j = (int)(idx % N);
    const cd z = Z[(int64_t)j * N + x];
    Q[idx] = cd{z.x, -z.y};
}

hipError_t launch_conj_transpose(int N, const cd *Z, cd *Q, hipStream_t s) {
    const int64_t nn = (int64_t)N * N;
    hipLaunchKernelGGL(conj_transpose_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, N, Z, Q);
    return hipGetLastError();
}

}  // namespace chfsi
