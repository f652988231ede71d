// Internal declarations of the MI355X R-ChFSI library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/chfsi.h"

namespace chfsi {

constexpr int kThreads = 256;       // threads per workgroup of the projection and adjoint kernels
constexpr int kMaxN = 512;          // nodes per cell (p <= 7)
constexpr int kMaxBeta = 16;
constexpr int kMaxDegree = 256;     // Chebyshev degree limit (Lambda_k table)
constexpr int kRowBlocks = 256;     // row blocks of the column reductions (partials [kRowBlocks][nvec])
constexpr int kPoiTab = 8 * 8 + 8 * 8 + 8;  // doubles of the Poisson 1D tables (nq1, n1 <= 8)

// complex helpers ------------------------------------------------------------
struct cd { double x, y; };
struct cf { float x, y; };

template <typename T> struct Cplx;
template <> struct Cplx<double> { using type = cd; };
template <> struct Cplx<float> { using type = cf; };

// Byte offsets of the tables in the persistent buffer and of the temporaries
// in the scratch buffer; computed identically by plan and setup.
struct Layout {
    // persistent
    size_t K64, Phi64, PhiT64, M64;          // n-pad square tables (double)
    size_t K32, Phi32, PhiT32;               // float copies
    size_t Kb, Phib, PhiTb;                  // bfloat16 copies
    size_t W64, W32;                         // [ncells][nqpad][4]
    size_t Wq;                               // [nqpad] quadrature weight * |J|
    size_t D64, Dinv64, Dinv32;              // [M]
    size_t colour_cells;                     // int32 [ncells]
    size_t nl_cells;                         // int32 [n_nl_cells]
    size_t cell_pair_ptr, cell_pairs;        // int32 [ncells+1], [npairs]
    size_t pair_atom, atom_pair_ptr;         // int32 [npairs], [natoms+1]
    size_t P64, P32;                         // complex [npairs][npad][2][nbeta]
    size_t PB;                               // bfloat16 [npairs][tile][npad/8][16][32]: projection B operand
    size_t WP64, WP32;                       // real [npairs][4 nbeta][npad]: w|J| phi, k = (j, spin, re|im)
    size_t WPb;                              // bfloat16 [npairs][npad][kpad]: same, k contiguous
    int kpad;                                // 4 nbeta rounded up to 32
    size_t delta64;                          // complex128 [natoms][nbeta][nbeta]
    size_t KdInv64;                          // double [M]: 1 / diag(K) of the Poisson stiffness
    size_t persistent_bytes;
    // scratch
    size_t partial, dcoef;                   // complex128 [npairs|natoms][nbeta][max_nvec]
    size_t Z;                                // two recurrence blocks [2M][filter_block] of the filter's
                                             // complex type; also the rotation and Gram temporaries
    size_t zarea;                            // bytes from Z to the end of the scratch buffer
    size_t lamk;                             // double [kMaxDegree+1][max_nvec]
    size_t small;                            // dense N x N matrices for RR
    size_t red;                              // reduction partials
    size_t flag;                             // int flags
    size_t scratch_bytes;
    size_t small_bytes, red_bytes;
};

struct Mesh {
    int64_t ncell[3];
    double h[3];
    int p, n1, n, nq1, nq, npad, nqpad;
    int64_t ncells, M, Nd[3];
    int64_t natoms, npairs, n_nl_cells;
    int nbeta;
};

}  // namespace chfsi

struct chfsi_ctx {
    chfsi::Mesh m;
    chfsi::Layout L;
    int64_t max_nvec;
    int64_t filter_block;     // columns of one filter pass (<= max_nvec)
    chfsi_prec filter_prec;   // widest filter precision the scratch was sized for
    char *pers;
    char *scr;
    int64_t colour_ptr[9];
    rocblas_handle blas;
    double poi_tab[chfsi::kPoiTab];  // host copy of the Poisson 1D tables (kernel arguments)
    std::string err;
    // typed views
    template <typename T> T *P(size_t off) const { return reinterpret_cast<T *>(pers + off); }
    template <typename T> T *S(size_t off) const { return reinterpret_cast<T *>(scr + off); }
};

namespace chfsi {

// ---------------------------------------------------------------- kernels
// cell operator modes
enum : int {
    MODE_HAM = 0,       // H: kinetic + (V + B.sigma) + nonlocal epilogue
    MODE_MASS = 1,      // M: mass table only
};
enum : int {
    FLAG_ACCUM = 1,     // Y += alpha * (.) at every node (else first touch writes)
    FLAG_DINV = 2,      // gather D^{-1} X
    FLAG_NLOC = 4,      // add the spin-orbit epilogue (needs dcoef)
    FLAG_EPI = 8,       // first touch writes alpha (.) + the recurrence terms of EpiArgs
};

// The recurrence terms of one filter step (eq. rChFSIrecurrence) that the
// cell operator's first touch of a node adds to alpha H D^{-1} Z_k:
// beta Z_k + gamma Z_{k-1} + alpha lam[c] R (formed in double).  Z_k is the
// operator's input block; Zkm (Z_{k-1}, nullable) has its leading dimension
// and may be the output block itself (read before it is overwritten).
struct EpiArgs {
    const void *Zkm;
    const cd *R;
    int64_t ldr;
    const double *lam;
    double beta, gamma;
};

// apply the cell operator for all 8 colours: Y (+)= alpha * Op(X)
hipError_t launch_cell_op(const chfsi_ctx *c, chfsi_prec prec, int mode, int flags, double alpha,
                          const void *X, void *Y, int64_t nvec, int64_t ld, hipStream_t s,
                          const EpiArgs *epi = nullptr);
hipError_t launch_cell_op_bf16(const chfsi_ctx *c, int mode, int flags, double alpha, const void *X,
                               void *Y, int64_t nvec, int64_t ld, hipStream_t s, const EpiArgs *epi = nullptr);
// nonlocal projection + per-atom reduction with Delta: dcoef = Delta * P^H X
hipError_t launch_nonlocal_coeffs(const chfsi_ctx *c, chfsi_prec prec, int flags, const void *X,
                                  int64_t nvec, int64_t ld, hipStream_t s);
// adjoint fields
hipError_t launch_adjoint_fields(const chfsi_ctx *c, chfsi_prec prec, const void *X, const void *G,
                                 int64_t nvec, int64_t ld, double *dV, double *dB, hipStream_t s);
// setup kernels
hipError_t launch_setup_fields(const chfsi_ctx *c, const double *V, const double *B, hipStream_t s);
hipError_t launch_setup_projectors(const chfsi_ctx *c, const cd *phi_dev, hipStream_t s);
hipError_t launch_setup_casts(const chfsi_ctx *c, hipStream_t s);

// elementwise (filter / residual / reductions)
hipError_t launch_filter_init_ld(int64_t rows, int64_t nvec, int64_t ldz, int64_t ldr, bool zf32,
                                 void *Znew, const void *Zk, const void *Zkm, const cd *R, double beta,
                                 double gamma, const double *delta, double rscale, hipStream_t s);
hipError_t launch_lamk_table(const double *ritz, int64_t nvec, int degree, double c, double e,
                             double s1, double *lamk, int64_t ldl, hipStream_t s);
hipError_t launch_recover_ld(int64_t rows, int64_t nvec, int64_t ldz, int64_t ld, bool zf32, const void *Z,
                             const double *dinv, const cd *X, const double *lamq, cd *Y, hipStream_t s);
hipError_t launch_residual(int64_t rows, int64_t nvec, int64_t ld, const cd *HX, const cd *MX,
                           const double *ritz, cd *R, double *red, double *norms, hipStream_t s);
hipError_t launch_colnorm2(int64_t rows, int64_t nvec, int64_t ld, const cd *A, const double *w,
                           double *red, double *out, hipStream_t s);
hipError_t launch_cast_block(int64_t rows, int64_t nvec, int64_t ld, const void *src, bool src32,
                             void *dst, bool dst32, hipStream_t s);
hipError_t launch_scale_rows(int64_t rows, int64_t nvec, int64_t ld, const double *w, cd *A,
                             hipStream_t s);
hipError_t launch_check_finite(const double *a, int64_t n, int *flag, hipStream_t s);
hipError_t launch_check_finite_block(const cd *a, int64_t rows, int64_t nvec, int64_t ld, int *flag,
                                     hipStream_t s);
hipError_t launch_dot_real(int64_t n, const cd *a, const cd *b, double *red, double *out,
                           hipStream_t s);
hipError_t launch_axpby(int64_t n, double a, const cd *x, double b, cd *y, hipStream_t s);

// dense (small N x N, row-major complex128)
hipError_t launch_sum_parts(int64_t n, int nparts, const cd *parts, cd *out, hipStream_t s);
hipError_t launch_herm_equilibrate(int N, cd *S, double *scale, int *flag, hipStream_t s);
hipError_t launch_hermitize(int N, cd *S, hipStream_t s);
hipError_t launch_cholesky_block(int n, int lda, cd *A, int *flag, hipStream_t s);
hipError_t launch_zero_upper(int N, cd *A, hipStream_t s);
hipError_t launch_offdiag_cf(int N, int bs, const cd *Q, cf *Q32, hipStream_t s);
hipError_t launch_sr_to_cf(int64_t rows, int64_t N, int64_t ld, const cd *A, cf *A32, hipStream_t s);
hipError_t launch_sr_combine(int64_t rows, int64_t N, int64_t ld, const cd *T, const cf *C32, cd *A, hipStream_t s);
// block floating-point codec: encode (enc) float[n] -> stream, or decode stream -> float[n]
hipError_t launch_bfp(bool enc, int nbits, const void *src, int64_t n, void *dst, hipStream_t s);
hipError_t launch_fill_lower(int N, cd *A, hipStream_t s);
hipError_t launch_scale_cols(int N, const double *w, const cd *A, cd *B, hipStream_t s);
hipError_t launch_colnorm(int64_t rows, int64_t nvec, int64_t ld, const cd *A, double *red, double *out,
                          hipStream_t s);
hipError_t launch_diag(int N, const double *scale, cd *T, hipStream_t s);
// Poisson (FP64): y = K x, PCG and Chebyshev-Jacobi vector kernels
enum : int { SC_DELTA = 0, SC_ETA = 1, SC_GAMMA = 2, SC_BETA = 3, SC_SUM0 = 4, SC_SUM1 = 5, SC_NSC = 8 };
enum : int { PCG_SUMS = 0, PCG_ETA = 1, PCG_FIRST = 2, PCG_NEXT = 3 };
constexpr int kDotPartials = 2 * 512;  // doubles of partial sums used by launch_dot2
bool kx_supported(int n1, int q1);
hipError_t launch_kx(const chfsi_ctx *c, const double *x, double *y, hipStream_t s);
hipError_t launch_dot2(int64_t n, const double *a, const double *b, const double *c, const double *d, double *part,
                       int op, double *sc, hipStream_t s);
hipError_t launch_pcg_update(int64_t n, const double *sc, const double *p, const double *w, double *x, double *r,
                             hipStream_t s);
hipError_t launch_pcg_dir(int64_t n, const double *sc, bool first, const double *z, double *p, hipStream_t s);
hipError_t launch_pcg_init(int64_t n, const double *sc, const double *Kx, const double *f, double *r,
                           hipStream_t s);
hipError_t launch_sub_mean(int64_t n, const double *sc, double *x, hipStream_t s);
hipError_t launch_cheb_step(int64_t n, bool first, double c1, double c2, const double *dinv, const double *r,
                            const double *Kz, double *d, double *z, hipStream_t s);
hipError_t launch_axpby_real(int64_t n, double alpha, const double *x, double beta, double *y,
                             const double *scale, hipStream_t s);
// last Chebyshev step with the (r.z, r.r) reduction of the PCG (op as in launch_dot2)
hipError_t launch_cheb_last_dot(int64_t n, bool first, double c1, double c2, const double *dinv, const double *r,
                                const double *Kz, const double *d, double *z, double *part, int op, double *sc,
                                hipStream_t s);
hipError_t launch_splitmix(int64_t n, uint64_t seed, double *v, hipStream_t s);
hipError_t launch_sqrt(int64_t n, const double *x, double *y, hipStream_t s);

hipError_t launch_conj_transpose(int N, const cd *Z, cd *Q, hipStream_t s);

}  // namespace chfsi
