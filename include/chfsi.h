/*
 * chfsi.h -- C ABI of the MI355X R-ChFSI library.
 *
 * The library solves the finite-element generalized Hermitian eigenproblem
 * H X = M X Lambda of noncollinear spin-orbit Kohn-Sham DFT (paper Sec.
 * III-A): H is complex Hermitian of size 2M x 2M (M FE nodes, two spinor
 * components), M is the real SPD FE mass matrix.  The solver is the
 * residual-based Chebyshev filtered subspace iteration (R-ChFSI, Sec. III-B2,
 * eq. rChFSIrecurrence and Algorithm RChFSI); its hot path is the
 * matrix-free cell-level Hamiltonian-times-multivector product (Sec. III-C2,
 * eq. cellHam, stages i-iv).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units       Hartree atomic units (Ha, bohr).
 * Mesh        Periodic box of ncell[0] x ncell[1] x ncell[2] hexahedral cells
 *             with edges h[d]; Lagrange elements of degree p on GLL nodes
 *             (Sec. III-A), Gauss-Legendre quadrature with nq1d points per
 *             direction (nq1d = p+1 integrates the kinetic and mass terms
 *             exactly on these cells).  Cell e = ex + ncx*(ey + ncy*ez);
 *             local node I = i + (p+1)*(j + (p+1)*k); quadrature point
 *             q = a + nq1d*(b + nq1d*c) with ascending abscissae.  Global
 *             node g = gx + Nx*(gy + Ny*gz), N_d = ncell[d]*p, gx = (ex*p+i)
 *             mod Nx.  Every ncell[d] must be even (the cell colouring that
 *             makes assembly race-free needs it) and p in 1..7.
 * Vectors     A block of nvec spinor vectors is row-major complex
 *             [M][2][ld] (interleaved re, im): row 2g+alpha holds spin alpha
 *             of node g, the dof numbering of Sec. III-A; the vector index
 *             is fastest, ld >= nvec.  Blocks are complex128 (double pairs)
 *             in CHFSI_FP64 and complex64 (float pairs) in CHFSI_FP32 and
 *             CHFSI_BF16.
 * Fields      V[e][q] and B[e][q][3] (double, device memory): the local
 *             potential and the magnetic field at the quadrature points.
 * Precision   CHFSI_FP64: all products in double on FP64 MFMA.
 *             CHFSI_FP32: cell GEMMs and projector products with float
 *             operands on FP32 MFMA, float accumulation.
 *             CHFSI_BF16: cell-GEMM and projector-product operands rounded
 *             to bfloat16 (nearest even), float accumulation on BF16 MFMA;
 *             the pointwise 2x2 spin term and Delta in float.
 *             The residual, the Chebyshev scalars, orthonormalization and
 *             Rayleigh-Ritz always run in double (Sec. III-C2).
 * Memory      The caller owns every device buffer.  chfsi_plan reports the
 *             sizes of the two buffers the library needs (persistent tables
 *             and scratch); the caller allocates them (e.g. with PyTorch)
 *             and passes them to chfsi_setup.  Host arrays passed to
 *             chfsi_setup are copied; the context keeps device pointers only.
 *             The library itself calls no device allocator except inside
 *             the BLAS handle it creates at setup.
 * Streams     Every call is ordered on the given hipStream_t (NULL = the
 *             null stream) and returns without waiting, unless stated.
 * Errors      Functions return CHFSI_OK (0), a positive warning, or a
 *             negative error code; they never throw.  chfsi_last_error(ctx)
 *             (or (NULL) before a context exists) gives a message.  Argument
 *             errors are detected before any device work is queued.
 * Threads     A context may be used by one host thread at a time.  Calls
 *             on one context that overlap on different streams race on the
 *             scratch buffer.
 */
#ifndef CHFSI_H
#define CHFSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct chfsi_ctx chfsi_ctx;

enum {
    CHFSI_OK = 0,
    CHFSI_NOT_CONVERGED = 1,  /* chfsi_solve: max_iter reached; outputs valid */
    CHFSI_E_ARG = -1,         /* invalid argument (message says which) */
    CHFSI_E_DEVICE = -2,      /* a HIP or BLAS call failed */
    CHFSI_E_NOT_SPD = -3,     /* Cholesky breakdown (rank-deficient block) */
    CHFSI_E_BOUNDS = -4,      /* filter bounds not ordered lmin < lT < lmax */
    CHFSI_E_NONFINITE = -5,   /* NaN or Inf in an input or a residual */
    CHFSI_E_DIVERGED = -6,    /* residual grew by > 1e6 (bad lambda_max) */
    CHFSI_E_WORKSPACE = -7,   /* a buffer is smaller than required */
};

typedef enum { CHFSI_FP64 = 0, CHFSI_FP32 = 1, CHFSI_BF16 = 2 } chfsi_prec;

typedef struct {
    int64_t ncell[3]; /* cells per direction, even, >= 2 */
    double h[3];      /* cell edge lengths (bohr), > 0 */
    int degree;       /* FE degree p, 1..7 */
    int nq1d;         /* quadrature points per direction, 0 means p+1; <= 8 */
} chfsi_mesh;

/* Separable spin-orbit term H_nloc = sum_a P_a Delta_a P_a^H (Sec. II-A eq.
 * hnloc; Sec. III-C2 item iv).  Projector beta_{a,j} (two-component,
 * complex) is given by its samples at the quadrature points of every cell
 * of its support; the library forms the cell projector matrices
 * P_a(e)[I][alpha][j] = sum_q w_q |J| N_I(x_q) beta_{a,j,alpha}(x_q).
 * All arrays are host memory, copied by chfsi_setup. */
typedef struct {
    int64_t natoms;            /* >= 0; 0 disables the term */
    int nbeta;                 /* projectors per atom, 1..16 */
    const int64_t *pair_ptr;   /* [natoms+1], CSR offsets of each atom's cells */
    const int64_t *pair_cell;  /* [npairs], cells (each at most once per atom) */
    const double *phi;         /* complex128 [npairs][nq][2][nbeta] */
    const double *delta;       /* complex128 [natoms][nbeta][nbeta], Hermitian */
} chfsi_projectors;

/* Sizes of the caller-allocated buffers for blocks of up to max_nvec
 * vectors.  persistent: operator tables (all precisions); scratch:
 * temporaries of apply, filter (two recurrence blocks of max_nvec complex128
 * columns) and Rayleigh-Ritz.  Both must be 256-byte aligned device memory.
 * Same as chfsi_plan_ex with {max_nvec, 0, CHFSI_FP64}. */
int chfsi_plan(const chfsi_mesh *mesh, const chfsi_projectors *proj, int64_t max_nvec,
               size_t *persistent_bytes, size_t *scratch_bytes);

/* Scratch sizing for filtering in blocks of wavefunctions (Sec. III-C4: the
 * subspace is processed in column blocks) and for the narrower recurrence
 * blocks of the reduced-precision filters (Sec. III-C2: Z in FP32). */
typedef struct {
    int64_t max_nvec;       /* largest block of any call (the subspace N_s) */
    int64_t filter_block;   /* largest column count of one filter pass
                               (chfsi_filter nvec, chfsi_solve_opts.block);
                               0 means max_nvec; <= max_nvec */
    chfsi_prec filter_prec; /* widest filter precision at filter_block columns:
                               CHFSI_FP64 sizes complex128 recurrence blocks,
                               CHFSI_FP32 / CHFSI_BF16 complex64 (half the
                               bytes; an FP64 filter then fits only half as
                               many columns and reports CHFSI_E_WORKSPACE
                               beyond that) */
} chfsi_plan_opts;

/* Buffer sizes for the options above.  The recurrence area also serves the
 * Rayleigh-Ritz rotations and Gram partials, which run in row chunks when it
 * is smaller than a complex128 block of max_nvec columns. */
int chfsi_plan_ex(const chfsi_mesh *mesh, const chfsi_projectors *proj, const chfsi_plan_opts *opts,
                  size_t *persistent_bytes, size_t *scratch_bytes);

/* Builds the operator tables (Sec. III-A quadrature; Sec. III-C2 cell
 * matrices) into `persistent` and returns a context.  V, B: device fields
 * as above (copied into the tables; the caller may free them afterwards).
 * proj may be NULL (no spin-orbit term).  Synchronizes `stream`.  Returns
 * CHFSI_E_NONFINITE (and no context) if V or B holds NaN or Inf. */
int chfsi_setup(const chfsi_mesh *mesh, const double *V, const double *B,
                const chfsi_projectors *proj, int64_t max_nvec,
                void *persistent, size_t persistent_bytes,
                void *scratch, size_t scratch_bytes, void *stream, chfsi_ctx **out);

/* chfsi_setup with the buffers sized by chfsi_plan_ex for the same opts. */
int chfsi_setup_ex(const chfsi_mesh *mesh, const double *V, const double *B,
                   const chfsi_projectors *proj, const chfsi_plan_opts *opts,
                   void *persistent, size_t persistent_bytes,
                   void *scratch, size_t scratch_bytes, void *stream, chfsi_ctx **out);

/* Replaces the fields V, B (device) of an existing context (same mesh).
 * Synchronizes; CHFSI_E_NONFINITE if V or B holds NaN or Inf, in which case
 * the context keeps its previous fields. */
int chfsi_set_fields(chfsi_ctx *ctx, const double *V, const double *B, void *stream);

/* Y = H X (Sec. III-C2: gather, cell contraction, spin-orbit projectors,
 * colour-ordered assembly).  X, Y: device blocks of the precision's complex
 * type; X and Y must not overlap.  1 <= nvec <= max_nvec, ld >= nvec. */
int chfsi_apply_H(chfsi_ctx *ctx, chfsi_prec prec, const void *X, void *Y,
                  int64_t nvec, int64_t ld, void *stream);

/* Y = M X, the consistent mass matrix (Sec. III-A), complex128 blocks. */
int chfsi_apply_M(chfsi_ctx *ctx, const void *X, void *Y, int64_t nvec, int64_t ld, void *stream);

/* Adjoint of Y = H(V, B) X for the cotangent G (dL = Re sum conj(G) dY):
 *   dX = H G (H is Hermitian),
 *   dV[e][q]    = w_q|J| Re sum_{b,alpha} conj(g_{b,alpha}(x_q)) x_{b,alpha}(x_q),
 *   dB[e][q][d] = w_q|J| Re sum_b g_b(x_q)^H sigma_d x_b(x_q),
 * where x_b(x_q), g_b(x_q) are the fields interpolated to the quadrature
 * points.  With G = X these are w|J| times the densities rho and m of Sec.
 * II-A.  dX may be NULL; dV, dB (double, device) are overwritten. */
int chfsi_apply_H_adjoint(chfsi_ctx *ctx, chfsi_prec prec, const void *X, const void *G,
                          int64_t nvec, int64_t ld, void *dX, double *dV, double *dB, void *stream);

/* Upper bound of the spectrum of D^{-1} H by a k-step Lanczos recurrence on
 * D^{-1/2} H D^{-1/2} (the paper's estimate of the largest eigenvalue, Sec.
 * IV-F): theta_max + |beta_k|.  v0: complex128 device vector [2M] (start
 * vector, any nonzero).  Synchronizes; result in *lambda_max (host). */
int chfsi_estimate_bounds(chfsi_ctx *ctx, int lanczos_steps, const void *v0,
                          double *lambda_max, void *stream);

/* R-ChFSI filter (eq. rChFSIrecurrence) of degree q >= 1 with bounds
 * {lmin, lT, lmax} (host, lmin < lT < lmax):
 *   Z_0 = 0, Z_1 = s1 R / e,
 *   Z_{k+1} = (2 s_{k+1}/e)(H D^{-1} Z_k - c Z_k) - s_k s_{k+1} Z_{k-1}
 *             + (2 s_{k+1}/e) R Lambda_k,
 *   Y = D^{-1} Z_q + X Lambda_q,
 * c = (lmax+lT)/2, e = (lmax-lT)/2, s1 = e/(lmin-c), s_{k+1} = 1/(2/s1-s_k),
 * Lambda_k = C_k(diag(ritz)) by the same three-term rule.  The products
 * H D^{-1} Z_k run in `prec` (Z stored in its complex type); X, R, Y are
 * complex128 and R Lambda_k is formed in double.  ritz: double device [nvec].
 * Y may alias X.  The two recurrence blocks live in the scratch buffer:
 * CHFSI_E_WORKSPACE if nvec columns of the precision's complex type exceed
 * what chfsi_plan_ex sized (filter_block, filter_prec). */
int chfsi_filter(chfsi_ctx *ctx, chfsi_prec prec, int degree, const double bounds[3],
                 const void *X, const double *ritz, const void *R, void *Y,
                 int64_t nvec, int64_t ld, void *stream);

/* Cholesky-QR2 in the M inner product (the orthonormalization step of the
 * Rayleigh-Ritz stage): two passes of S = Y^H MY, s = diag(S)^{-1/2},
 * L L^H = diag(s) S diag(s), (Y, HY, MY) <- (.) diag(s) L^{-H}.  HY, MY:
 * H Y and M Y on entry (MY required, HY may be NULL), updated in place.
 * complex128 blocks.  Returns CHFSI_E_NOT_SPD on breakdown. */
int chfsi_orthonormalize(chfsi_ctx *ctx, void *Y, void *HY, void *MY,
                         int64_t nvec, int64_t ld, void *stream);

/* Rayleigh-Ritz on an M-orthonormal block (Algorithm RChFSI, RR step):
 * Hs = Y^H HY (Hermitian part), Hs Q = Q Lambda with ascending Lambda
 * (dense Hermitian eigensolve by rocSOLVER's divide and conquer; its
 * workspace comes from the rocBLAS handle, and the call synchronizes),
 * Y <- Y Q, HY <- HY Q, MY <- MY Q.  ritz: double device [nvec] output.
 * If R != NULL: R = HY - MY diag(ritz) and resnorm[j] = ||R_j||_2 (double
 * device [nvec]; resnorm may be NULL). */
int chfsi_rayleigh_ritz(chfsi_ctx *ctx, void *Y, void *HY, void *MY, int64_t nvec, int64_t ld,
                        double *ritz, void *R, double *resnorm, void *stream);

/* Rayleigh-Ritz of a block that need not be M-orthonormal (Algorithm
 * RChFSI, RR step: Y^H H Y Q = Y^H M Y Q Lambda): S = Y^H MY, Hs = Y^H HY,
 * s = diag(S)^{-1/2}, L L^H = diag(s) S diag(s), T = diag(s) L^{-H},
 * (T^H Hs T) W = W Lambda, Q = T W, then Y, HY, MY <- (.) Q (so that
 * Y^H M Y = I) and, as in chfsi_rayleigh_ritz, the residual.  Returns
 * CHFSI_E_NOT_SPD if S is numerically singular. */
int chfsi_rayleigh_ritz_general(chfsi_ctx *ctx, void *Y, void *HY, void *MY, int64_t nvec, int64_t ld,
                                double *ritz, void *R, double *resnorm, void *stream);

/* R = HX - MX diag(ritz) and resnorm[j] = ||R_j||_2 (complex128 blocks,
 * double device vectors). */
int chfsi_residual(chfsi_ctx *ctx, const void *HX, const void *MX, const double *ritz,
                   void *R, double *resnorm, int64_t nvec, int64_t ld, void *stream);

/* chfsi_residual for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same R and resnorm, computed by the same kernels in the same order, with
 * the column-norm partials in a static device array of the library (8 MiB
 * per GPU, held until the process ends) instead of the context's scratch.
 * No allocation of any kind.  nvec <= 4096, else CHFSI_E_WORKSPACE.  The
 * array is shared by every call on one GPU: calls that overlap on one GPU
 * (different streams, threads or contexts) race on it. */
int chfsi_residual_noalloc(chfsi_ctx *ctx, const void *HX, const void *MX, const double *ritz,
                           void *R, double *resnorm, int64_t nvec, int64_t ld, void *stream);

typedef struct {
    chfsi_prec prec;    /* precision of the filter's products */
    int degree;         /* Chebyshev degree q per iteration */
    double tol;         /* stop when max_{j < n_wanted} ||R_j||_2 < tol */
    int max_iter;       /* outer iterations (>= 1) */
    int lanczos_steps;  /* steps of the lambda_max estimate (0: use lambda_max) */
    double lambda_max;  /* used when lanczos_steps == 0 */
    int fixed_iters;    /* if != 0, run exactly max_iter iterations (timing) */
    int rr_mode;        /* 0: Cholesky-QR2 then Rayleigh-Ritz on the
                           orthonormal block (chfsi_orthonormalize +
                           chfsi_rayleigh_ritz); 1: Rayleigh-Ritz of the
                           generalized subspace problem through one Cholesky
                           factor of Y^H M Y (chfsi_rayleigh_ritz_general),
                           falling back to mode 0 on a Cholesky breakdown;
                           2: as 1 with the paper's mixed-precision subspace
                           rotation (Sec. III-C4, RR-SR): X <- Y Q with the
                           diagonal 64 x 64 blocks of Q in FP64 and the rest
                           in FP32 (complex64 copies, FP32 MFMA), summed in
                           FP64; the residual products stay FP64.
                           Other values: CHFSI_E_ARG */
    int resume;         /* if != 0, X and the workspace hold the state left by
                           a previous chfsi_solve on the same X and workspace
                           (Ritz vectors, HX, MX, R, Ritz values): the initial
                           orthonormalization, Rayleigh-Ritz and the Lanczos
                           bound are skipped and lambda_max is taken from opts */
    int64_t block;      /* columns per filter pass (blocks of wavefunctions,
                           Sec. III-C4); 0: min(nsub, filter_block).  The
                           filter is column-wise, so blocking changes no
                           result */
    int profile;        /* if != 0, device events on `stream` around the cell-
                           operator launches of every filter step (one pair
                           per step and column block) fill
                           report->t_filter_cell and
                           report->filter_cell_launches; 0: both stay 0 */
} chfsi_solve_opts;

typedef struct {
    int iters;              /* outer iterations done */
    int converged;          /* 1 if the tolerance was met */
    double max_res;         /* final max residual over the wanted columns */
    double lambda_bounds[3];/* last lmin, lT, lmax */
    double t_filter, t_rr, t_total; /* seconds (device events), summed */
    double t_iter_median;   /* median seconds per iteration from the 2nd on */
    double t_filter_cell;   /* with opts.profile: seconds in the filter steps'
                               cell-operator launches (device events), summed */
    int64_t filter_cell_launches; /* with opts.profile: number of those
                               launches (one per non-empty cell colour and step) */
} chfsi_report;

/* Workspace bytes chfsi_solve needs for nsub columns with leading dim ld. */
int chfsi_solve_workspace(chfsi_ctx *ctx, int64_t nsub, int64_t ld, size_t *bytes);

/* Algorithm RChFSI: from the start block X (complex128 [M][2][ld], nsub
 * columns, overwritten with the Ritz vectors, M-orthonormal) and v0 for the
 * Lanczos bound (complex128 [2M], may be NULL when lanczos_steps == 0):
 * orthonormalize and Rayleigh-Ritz, then per iteration: residual (double),
 * stop test, lmin = Lambda_1, lT = Lambda_nsub, filter in opts->prec,
 * H Y and M Y in double, Cholesky-QR2, Rayleigh-Ritz.  eigvals: host
 * [n_wanted] (ascending).  hist_res: optional host [max_iter+1] of the max
 * wanted residual per iteration.  Synchronizes once per iteration.
 * Returns CHFSI_OK, CHFSI_NOT_CONVERGED, or an error: CHFSI_E_NONFINITE if
 * the start block (first nsub columns) or a residual holds NaN or Inf,
 * CHFSI_E_DIVERGED if the largest wanted residual grows past 1e6 times its
 * first value (and past 1), the symptom of a lambda_max below the top of
 * the spectrum, CHFSI_E_BOUNDS if a Ritz value reaches lambda_max,
 * CHFSI_E_NOT_SPD if the filtered block loses rank. */
int chfsi_solve(chfsi_ctx *ctx, int64_t n_wanted, const chfsi_solve_opts *opts,
                void *X, int64_t nsub, int64_t ld, const void *v0,
                double *eigvals, double *hist_res, chfsi_report *report,
                void *workspace, size_t workspace_bytes, void *stream);

/* Instrumentation: performs one chfsi_apply_H(ctx, prec, X, Y, ...) and
 * reports, from device events recorded on `stream` around the launches,
 * ms[0] = milliseconds in the cell-operator launches (gather, cell
 * contraction, projector epilogue, assembly), ms[1] = in the spin-orbit
 * coefficient launches, ms[2] = whole product; *launches = number of
 * cell-operator launches (one per non-empty cell colour).  Synchronizes. */
int chfsi_profile_apply_H(chfsi_ctx *ctx, chfsi_prec prec, const void *X, void *Y, int64_t nvec,
                          int64_t ld, double ms[3], int *launches, void *stream);

/* Mesh sizes of a context: nnodes (M), ncells, n (nodes per cell), nq. */
int chfsi_info(const chfsi_ctx *ctx, int64_t *nnodes, int64_t *ncells, int *n, int *nq);

/* The diagonal D (GLL-integrated mass, Sec. III-B2) as double device [M]. */
int chfsi_mass_diag(chfsi_ctx *ctx, double *D, void *stream);

/* Block floating-point codec (Sec. III-C3, compressed communication, fig.
 * layout).  Four float values form one block of N_bits = 4*nbits bits,
 * nbits in {16, 12, 10}: the low 8 bits hold the shared biased exponent
 * e = e_max + 127 with 2^(e_max-1) <= max|x_i| < 2^e_max (e_max >= -126; 0
 * marks an all-zero block), then four signed coefficients of
 * v = nbits - 2 bits (x_0 first), q_i = round(x_i 2^(v-1-e_max)) with ties
 * to even, clamped to 2^(v-1) - 1 above, stored as their low v bits in two's
 * complement.  Decoding returns q_i 2^(e_max-v+1) exactly.  Blocks are
 * little-endian and back to back, nbits/2 bytes each, so a stream of n
 * values takes n/4 * nbits/2 bytes and block b depends only on x[4b..4b+3].
 * n must be a multiple of 4 and the values finite.  x is 16-byte aligned;
 * the stream is aligned to 8 (nbits 16), 2 (12) or 1 (10) bytes.  Device
 * buffers owned by the caller; stream-ordered; these functions take no
 * context: on failure the message is chfsi_last_error(NULL).
 * Returns CHFSI_E_ARG for a bad nbits, n, NULL or misaligned buffer,
 * CHFSI_E_DEVICE if the launch fails. */
int chfsi_bfp_bytes(int nbits, int64_t n, int64_t *bytes);
int chfsi_bfp_encode(int nbits, const float *x, int64_t n, void *out, void *stream);
int chfsi_bfp_decode(int nbits, const void *in, int64_t n, float *x, void *stream);

/* ------------------------------------------------------------------ Poisson
 * The FE-discretized Poisson problem K V = f of the electrostatics (Sec.
 * III-B1): K_IJ = sum_e int_e grad N_I . grad N_J on the context's periodic
 * mesh, with the same nodes and Gauss quadrature as H.  Vectors are double
 * device arrays [M], node index gx + Nx (gy + Ny gz), owned by the caller.
 * K is assembled matrix-free and sum-factorised (Sec. III-B1; Sec. III-C1, the
 * K x kernel paragraph: extraction, 1D contractions, Jacobian and assembly in one
 * launch); it needs nq1d = degree + 1 or degree + 2 (else CHFSI_E_ARG).  K
 * is symmetric positive semi-definite; its null space is the constants. */

/* y = K x.  x and y must not overlap (y is zeroed first, then assembled with
 * atomic adds, so the last bits of y may differ between calls). */
int chfsi_apply_K(chfsi_ctx *ctx, const double *x, double *y, void *stream);

/* Chebyshev-Jacobi preconditioner (Sec. III-B1; Sec. III-C1): z = P^{-1} r with
 * P^{-1} = chi(D^{-1} K) D^{-1}, D = diag(K), chi the degree-m Chebyshev
 * approximation of 1/lambda on [lmin, lmax] (m steps of the Chebyshev
 * iteration on D^{-1} K z = D^{-1} r from z = 0, m - 1 applications of K;
 * m = 1 is Jacobi scaled by 2/(lmin+lmax)).  0 < lmin < lmax finite,
 * 1 <= degree <= 64; r and z must not overlap. */
int chfsi_poisson_precond(chfsi_ctx *ctx, int degree, double lmin, double lmax, const double *r,
                          double *z, void *stream);

typedef struct {
    double tol;          /* absolute: stop once ||K x - f'||_2 < tol (f' below) */
    int max_iter;        /* >= 0 */
    int cheb_degree;     /* preconditioner degree m, 1..64 */
    int lanczos_steps;   /* steps of the spectral estimate (when lambda_max == 0), 1..1000 */
    double lambda_max;   /* > 0: upper bound of the spectrum of D^{-1} K to use; 0: estimate */
    double range;        /* lmin = lambda_max / range, range > 1 */
} chfsi_pcg_opts;

typedef struct {
    int iters;           /* PCG iterations taken */
    int converged;
    double res_norm;     /* ||r||_2 of the recurrence residual at exit */
    double lambda_min, lambda_max; /* preconditioner interval used */
    double t_lanczos, t_total;     /* seconds (host clock around synchronized work) */
} chfsi_pcg_report;

/* Solves K x = f' with f' = f - mean(f) (the part of f in the range of K) by
 * the PCG of Algorithm pcg_fusion (Sec. III-C1): w = K p; eta = p.w; alpha = delta/eta;
 * x += alpha p and r += alpha w in one pass; z = P^{-1} r, whose last
 * Chebyshev step also reduces (delta_new, gamma) = (r.z, r.r); beta =
 * delta_new/delta; p = -z + beta p; stop when sqrt(gamma) < tol.  r = K x - f' starts from the
 * caller's x (initial guess, e.g. the previous SCF step's potential), and
 * delta, eta, beta live in device memory: the host reads gamma once per
 * iteration.  Without opts->lambda_max the upper bound comes from a
 * Lanczos run on D^{-1/2} K D^{-1/2} (theta_max + |beta_k|) from a fixed
 * splitmix64 start vector.  On return x holds the zero-mean solution (the
 * constant mode is removed).  f and x must not overlap.  Returns CHFSI_OK,
 * CHFSI_NOT_CONVERGED after max_iter iterations (x holds the last iterate),
 * CHFSI_E_NONFINITE on a non-finite or non-positive curvature p.w, or
 * CHFSI_E_ARG.  Synchronizes the stream. */
int chfsi_poisson_solve(chfsi_ctx *ctx, const chfsi_pcg_opts *opts, const double *f, double *x,
                        chfsi_pcg_report *report, void *stream);

const char *chfsi_last_error(const chfsi_ctx *ctx);
void chfsi_destroy(chfsi_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* CHFSI_H */
