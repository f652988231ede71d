// Streaming kernels of the R-ChFSI filter and of the residual (HBM-bound):
// the three-term update of eq. rChFSIrecurrence without its H term, the
// Chebyshev-filtered Ritz values Lambda_k, the recovery Y = D^{-1} Z_q +
// X Lambda_q, the residual R = HX - MX Lambda with column norms, and small
// helpers.  Column reductions are two-stage with a fixed summation order, so
// every result is deterministic.
#include "internal.h"

namespace chfsi {


template <typename TZ> struct ZT;
template <> struct ZT<cd> { using real = double; };
template <> struct ZT<cf> { using real = float; };

// Znew = beta*Zk + gamma*Zkm + (rscale * lam[c]) * R   (lam == nullptr: 1)
template <typename TZ>
__global__ void filter_init_kernel(int64_t rows, int64_t nvec, int64_t ldz, int64_t ldr, TZ *Znew,
                                   const TZ *Zk, const TZ *Zkm, const cd *R, double beta, double gamma,
                                   const double *lam, double rscale) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nvec) return;
    const double d = rscale * (lam ? lam[c] : 1.0);
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
        int64_t o = r * ldz + c;
        cd rr = R[r * ldr + c];
        double vx = d * rr.x, vy = d * rr.y;
        if (Zk) { vx += beta * (double)Zk[o].x; vy += beta * (double)Zk[o].y; }
        if (Zkm) { vx += gamma * (double)Zkm[o].x; vy += gamma * (double)Zkm[o].y; }
        TZ z;
        z.x = (typename ZT<TZ>::real)vx;
        z.y = (typename ZT<TZ>::real)vy;
        Znew[o] = z;
    }
}

// Two adjacent complex values as doubles (16-byte aligned pairs of cf, or
// two cd), and their store after rounding to TZ.
__device__ __forceinline__ void load2(const cf *p, double v[4]) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 z = *reinterpret_cast<const f4 *>(p);
    v[0] = z[0]; v[1] = z[1]; v[2] = z[2]; v[3] = z[3];
}
__device__ __forceinline__ void load2(const cd *p, double v[4]) {
    const cd a = p[0], b = p[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void store2(cf *p, const double v[4]) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    *reinterpret_cast<f4 *>(p) = f4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
}
__device__ __forceinline__ void store2(cd *p, const double v[4]) {
    p[0] = cd{v[0], v[1]};
    p[1] = cd{v[2], v[3]};
}

// The same update with one wave per row and two columns per lane, so each
// load and store of a wave covers a contiguous piece of the row (nvec, ldz
// and ldr even).  Same arithmetic, in the same order, as filter_init_kernel.
template <typename TZ>
__global__ __launch_bounds__(256) void filter_init_rows_kernel(int64_t rows, int64_t nvec, int64_t ldz,
                                                               int64_t ldr, TZ *Znew, const TZ *Zk,
                                                               const TZ *Zkm, const cd *R, double beta,
                                                               double gamma, const double *lam, double rscale) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t npair = nvec >> 1;
    for (int64_t r = wave; r < rows; r += nwaves) {
#pragma unroll 4
        for (int64_t q = lane; q < npair; q += 64) {
            const int64_t c = 2 * q, o = r * ldz + c;
            double v[4], z[4];
            load2(R + r * ldr + c, v);
            const double d0 = rscale * (lam ? lam[c] : 1.0), d1 = rscale * (lam ? lam[c + 1] : 1.0);
            v[0] *= d0; v[1] *= d0; v[2] *= d1; v[3] *= d1;
            if (Zk) {
                load2(Zk + o, z);
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] += beta * z[i];
            }
            if (Zkm) {
                load2(Zkm + o, z);
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] += gamma * z[i];
            }
            store2(Znew + o, v);
        }
    }
}

static dim3 col_grid(int64_t nvec, int64_t rows, unsigned &threads) {
    threads = nvec >= 256 ? 256 : (nvec >= 128 ? 128 : 64);
    unsigned gx = (unsigned)((nvec + threads - 1) / threads);
    int64_t want = (4096 + gx - 1) / gx;  // enough workgroups to fill the chip
    unsigned gy = (unsigned)(want < rows ? want : rows);
    if (gy < 1) gy = 1;
    if (gy > 65535) gy = 65535;
    return dim3(gx, gy);
}

hipError_t launch_filter_init_ld(int64_t rows, int64_t nvec, int64_t ldz, int64_t ldr, bool zf32,
                                 void *Znew, const void *Zk, const void *Zkm, const cd *R, double beta,
                                 double gamma, const double *delta, double rscale, hipStream_t s) {
    if (nvec % 2 == 0 && ldz % 2 == 0 && ldr % 2 == 0) {
        // 8 workgroups of 4 waves per CU; each wave strides over the rows
        const int64_t want = (rows + 3) / 4;
        const unsigned nb = (unsigned)(want < 2048 ? (want > 0 ? want : 1) : 2048);
        if (zf32)
            hipLaunchKernelGGL(filter_init_rows_kernel<cf>, dim3(nb), dim3(256), 0, s, rows, nvec, ldz, ldr,
                               (cf *)Znew, (const cf *)Zk, (const cf *)Zkm, R, beta, gamma, delta, rscale);
        else
            hipLaunchKernelGGL(filter_init_rows_kernel<cd>, dim3(nb), dim3(256), 0, s, rows, nvec, ldz, ldr,
                               (cd *)Znew, (const cd *)Zk, (const cd *)Zkm, R, beta, gamma, delta, rscale);
        return hipGetLastError();
    }
    unsigned th;
    dim3 g = col_grid(nvec, rows, th);
    if (zf32)
        hipLaunchKernelGGL(filter_init_kernel<cf>, g, dim3(th), 0, s, rows, nvec, ldz, ldr, (cf *)Znew,
                           (const cf *)Zk, (const cf *)Zkm, R, beta, gamma, delta, rscale);
    else
        hipLaunchKernelGGL(filter_init_kernel<cd>, g, dim3(th), 0, s, rows, nvec, ldz, ldr, (cd *)Znew,
                           (const cd *)Zk, (const cd *)Zkm, R, beta, gamma, delta, rscale);
    return hipGetLastError();
}

// lamk[k][c] = C_k-recurrence of the Ritz value ritz[c]: Lambda_0 = 1,
// Lambda_1 = s1 (lambda - c)/e, Lambda_{k+1} = (2 s_{k+1}/e)(lambda - c)
// Lambda_k - s_k s_{k+1} Lambda_{k-1}, s_{k+1} = 1/(2/s1 - s_k).
__global__ void lamk_kernel(const double *ritz, int64_t nvec, int degree, double c, double e,
                            double s1, double *lamk, int64_t ldl) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nvec) return;
    double lam = ritz[j];
    double lm = 1.0, l0 = s1 * (lam - c) / e, sk = s1;
    lamk[j] = 1.0;
    if (degree >= 1) lamk[ldl + j] = l0;
    for (int k = 1; k < degree; ++k) {
        double sn = 1.0 / (2.0 / s1 - sk);
        double ln = 2.0 * sn / e * (lam - c) * l0 - sk * sn * lm;
        lamk[(int64_t)(k + 1) * ldl + j] = ln;
        lm = l0;
        l0 = ln;
        sk = sn;
    }
}

hipError_t launch_lamk_table(const double *ritz, int64_t nvec, int degree, double c, double e,
                             double s1, double *lamk, int64_t ldl, hipStream_t s) {
    hipLaunchKernelGGL(lamk_kernel, dim3((unsigned)((nvec + 255) / 256)), dim3(256), 0, s, ritz, nvec,
                       degree, c, e, s1, lamk, ldl);
    return hipGetLastError();
}

// Y = D^{-1} Z + X diag(lamq)
template <typename TZ>
__global__ void recover_kernel(int64_t rows, int64_t nvec, int64_t ldz, int64_t ld, const TZ *Z,
                               const double *dinv, const cd *X, const double *lamq, cd *Y) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nvec) return;
    const double l = lamq[c];
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
        int64_t o = r * ld + c;
        double di = dinv[r >> 1];
        TZ z = Z[r * ldz + c];
        cd x = X[o];
        cd y;
        y.x = di * (double)z.x + l * x.x;
        y.y = di * (double)z.y + l * x.y;
        Y[o] = y;
    }
}

hipError_t launch_recover_ld(int64_t rows, int64_t nvec, int64_t ldz, int64_t ld, bool zf32, const void *Z,
                             const double *dinv, const cd *X, const double *lamq, cd *Y, hipStream_t s) {
    unsigned th;
    dim3 g = col_grid(nvec, rows, th);
    if (zf32)
        hipLaunchKernelGGL(recover_kernel<cf>, g, dim3(th), 0, s, rows, nvec, ldz, ld, (const cf *)Z, dinv, X,
                           lamq, Y);
    else
        hipLaunchKernelGGL(recover_kernel<cd>, g, dim3(th), 0, s, rows, nvec, ldz, ld, (const cd *)Z, dinv, X,
                           lamq, Y);
    return hipGetLastError();
}

// R = HX - MX diag(ritz); red[rb][c] = sum over the row block of |R|^2
__global__ void residual_kernel(int64_t rows, int64_t nvec, int64_t ld, const cd *HX, const cd *MX,
                                const double *ritz, cd *R, double *red) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nvec) return;
    const double l = ritz[c];
    const int64_t per = (rows + gridDim.y - 1) / gridDim.y;
    const int64_t r0 = blockIdx.y * per, r1 = r0 + per < rows ? r0 + per : rows;
    double s = 0;
    for (int64_t r = r0; r < r1; ++r) {
        int64_t o = r * ld + c;
        cd h = HX[o], m = MX[o];
        cd v;
        v.x = h.x - l * m.x;
        v.y = h.y - l * m.y;
        if (R) R[o] = v;
        s += v.x * v.x + v.y * v.y;
    }
    red[(int64_t)blockIdx.y * nvec + c] = s;
}

__global__ void col_finish_kernel(const double *red, int nb, int64_t nvec, double *out, int do_sqrt) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nvec) return;
    double s = 0;
    for (int b = 0; b < nb; ++b) s += red[(int64_t)b * nvec + c];
    out[c] = do_sqrt ? sqrt(s) : s;
}

hipError_t launch_residual(int64_t rows, int64_t nvec, int64_t ld, const cd *HX, const cd *MX,
                           const double *ritz, cd *R, double *red, double *norms, hipStream_t s) {
    unsigned th = nvec >= 256 ? 256 : 64;
    dim3 g((unsigned)((nvec + th - 1) / th), kRowBlocks);
    hipLaunchKernelGGL(residual_kernel, g, dim3(th), 0, s, rows, nvec, ld, HX, MX, ritz, R, red);
    if (norms)
        hipLaunchKernelGGL(col_finish_kernel, dim3((unsigned)((nvec + 255) / 256)), dim3(256), 0, s, red,
                           kRowBlocks, nvec, norms, 1);
    return hipGetLastError();
}

// sum over rows of w[r/2] |A[r][c]|^2 (w == nullptr: 1)
__global__ void colnorm2_kernel(int64_t rows, int64_t nvec, int64_t ld, const cd *A, const double *w,
                                double *red) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nvec) return;
    const int64_t per = (rows + gridDim.y - 1) / gridDim.y;
    const int64_t r0 = blockIdx.y * per, r1 = r0 + per < rows ? r0 + per : rows;
    double s = 0;
    for (int64_t r = r0; r < r1; ++r) {
        cd v = A[r * ld + c];
        double ww = w ? w[r >> 1] : 1.0;
        s += ww * (v.x * v.x + v.y * v.y);
    }
    red[(int64_t)blockIdx.y * nvec + c] = s;
}

// out[c] = ||A[:, c]||_2 (fixed-order two-stage reduction)
hipError_t launch_colnorm(int64_t rows, int64_t nvec, int64_t ld, const cd *A, double *red, double *out,
                          hipStream_t s) {
    unsigned th = nvec >= 256 ? 256 : 64;
    dim3 g((unsigned)((nvec + th - 1) / th), kRowBlocks);
    hipLaunchKernelGGL(colnorm2_kernel, g, dim3(th), 0, s, rows, nvec, ld, A, (const double *)nullptr, red);
    hipLaunchKernelGGL(col_finish_kernel, dim3((unsigned)((nvec + 255) / 256)), dim3(256), 0, s, red, kRowBlocks,
                       nvec, out, 1);
    return hipGetLastError();
}

hipError_t launch_colnorm2(int64_t rows, int64_t nvec, int64_t ld, const cd *A, const double *w,
                           double *red, double *out, hipStream_t s) {
    unsigned th = nvec >= 256 ? 256 : 64;
    dim3 g((unsigned)((nvec + th - 1) / th), kRowBlocks);
    hipLaunchKernelGGL(colnorm2_kernel, g, dim3(th), 0, s, rows, nvec, ld, A, w, red);
    hipLaunchKernelGGL(col_finish_kernel, dim3((unsigned)((nvec + 255) / 256)), dim3(256), 0, s, red,
                       kRowBlocks, nvec, out, 0);
    return hipGetLastError();
}

template <typename TS, typename TD>
__global__ void cast_kernel(int64_t rows, int64_t nvec, int64_t ld, const TS *src, TD *dst) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nvec) return;
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
        TS v = src[r * ld + c];
        TD o;
        o.x = v.x;
        o.y = v.y;
        dst[r * ld + c] = o;
    }
}

// Mixed-precision subspace rotation helpers: A32[r][c] = (complex64) A[r*ld + c]
// (compact rows of N), and A[r*ld + c] = T[r][c] + C32[r][c] (T compact complex128).
__global__ void sr_to_cf_kernel(int64_t rows, int64_t N, int64_t ld, const cd *A, cf *A32) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
        const cd v = A[r * ld + c];
        A32[r * N + c] = cf{(float)v.x, (float)v.y};
    }
}

__global__ void sr_combine_kernel(int64_t rows, int64_t N, int64_t ld, const cd *T, const cf *C32, cd *A) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
        const cd t = T[r * N + c];
        const cf u = C32[r * N + c];
        A[r * ld + c] = cd{t.x + (double)u.x, t.y + (double)u.y};
    }
}

hipError_t launch_sr_to_cf(int64_t rows, int64_t N, int64_t ld, const cd *A, cf *A32, hipStream_t s) {
    unsigned th;
    dim3 g = col_grid(N, rows, th);
    hipLaunchKernelGGL(sr_to_cf_kernel, g, dim3(th), 0, s, rows, N, ld, A, A32);
    return hipGetLastError();
}

hipError_t launch_sr_combine(int64_t rows, int64_t N, int64_t ld, const cd *T, const cf *C32, cd *A, hipStream_t s) {
    unsigned th;
    dim3 g = col_grid(N, rows, th);
    hipLaunchKernelGGL(sr_combine_kernel, g, dim3(th), 0, s, rows, N, ld, T, C32, A);
    return hipGetLastError();
}

hipError_t launch_cast_block(int64_t rows, int64_t nvec, int64_t ld, const void *src, bool src32,
                             void *dst, bool dst32, hipStream_t s) {
    unsigned th;
    dim3 g = col_grid(nvec, rows, th);
    if (src32 && !dst32)
        hipLaunchKernelGGL((cast_kernel<cf, cd>), g, dim3(th), 0, s, rows, nvec, ld, (const cf *)src, (cd *)dst);
    else if (!src32 && dst32)
        hipLaunchKernelGGL((cast_kernel<cd, cf>), g, dim3(th), 0, s, rows, nvec, ld, (const cd *)src, (cf *)dst);
    else if (src32)
        hipLaunchKernelGGL((cast_kernel<cf, cf>), g, dim3(th), 0, s, rows, nvec, ld, (const cf *)src, (cf *)dst);
    else
        hipLaunchKernelGGL((cast_kernel<cd, cd>), g, dim3(th), 0, s, rows, nvec, ld, (const cd *)src, (cd *)dst);
    return hipGetLastError();
}

// A[r][c] *= w[r/2]
__global__ void scale_rows_kernel(int64_t rows, int64_t nvec, int64_t ld, const double *w, cd *A) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nvec) return;
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
        double ww = w[r >> 1];
        cd v = A[r * ld + c];
        v.x *= ww;
        v.y *= ww;
        A[r * ld + c] = v;
    }
}

hipError_t launch_scale_rows(int64_t rows, int64_t nvec, int64_t ld, const double *w, cd *A,
                             hipStream_t s) {
    unsigned th;
    dim3 g = col_grid(nvec, rows, th);
    hipLaunchKernelGGL(scale_rows_kernel, g, dim3(th), 0, s, rows, nvec, ld, w, A);
    return hipGetLastError();
}

__global__ void finite_kernel(const double *a, int64_t n, int *flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(a[i])) bad = 1;
    if (bad) *flag = 1;  // benign race: every writer stores 1
}

hipError_t launch_check_finite(const double *a, int64_t n, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(finite_kernel, dim3(1024), dim3(256), 0, s, a, n, flag);
    return hipGetLastError();
}

// the first nvec columns of a complex128 [rows][ld] block (the columns past
// nvec may hold anything and are not read)
__global__ void finite_block_kernel(const cd *a, int64_t rows, int64_t nvec, int64_t ld, int *flag) {
    int bad = 0;
    const int64_t n = rows * nvec;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / nvec, c = i - r * nvec;
        const cd v = a[r * ld + c];
        if (!isfinite(v.x) || !isfinite(v.y)) bad = 1;
    }
    if (bad) *flag = 1;
}

hipError_t launch_check_finite_block(const cd *a, int64_t rows, int64_t nvec, int64_t ld, int *flag,
                                     hipStream_t s) {
    hipLaunchKernelGGL(finite_block_kernel, dim3(1024), dim3(256), 0, s, a, rows, nvec, ld, flag);
    return hipGetLastError();
}

// out = Re sum conj(a_i) b_i (two stages, fixed order)
__global__ void dot_partial_kernel(int64_t n, const cd *a, const cd *b, double *red) {
    __shared__ double sm[256];
    double s = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s += a[i].x * b[i].x + a[i].y * b[i].y;
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) red[blockIdx.x] = sm[0];
}

__global__ void dot_finish_kernel(const double *red, int nb, double *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0;
        for (int i = 0; i < nb; ++i) s += red[i];
        *out = s;
    }
}

hipError_t launch_dot_real(int64_t n, const cd *a, const cd *b, double *red, double *out, hipStream_t s) {
    hipLaunchKernelGGL(dot_partial_kernel, dim3(512), dim3(256), 0, s, n, a, b, red);
    hipLaunchKernelGGL(dot_finish_kernel, dim3(1), dim3(64), 0, s, red, 512, out);
    return hipGetLastError();
}

// y = a x + b y
__global__ void axpby_kernel(int64_t n, double a, const cd *x, double b, cd *y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        cd v = y[i];
        cd u = x ? x[i] : cd{0, 0};
        v.x = a * u.x + b * v.x;
        v.y = a * u.y + b * v.y;
        y[i] = v;
    }
}

hipError_t launch_axpby(int64_t n, double a, const cd *x, double b, cd *y, hipStream_t s) {
    hipLaunchKernelGGL(axpby_kernel, dim3(1024), dim3(256), 0, s, n, a, x, b, y);
    return hipGetLastError();
}

}  // namespace chfsi
