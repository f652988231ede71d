// C ABI of the R-ChFSI library: argument checking, operator tables, and the
// host-side drivers of the filter (eq. rChFSIrecurrence), the Rayleigh-Ritz
// stage and the eigensolver loop (Algorithm RChFSI).  Every arithmetic step
// on vectors and subspace matrices runs in this library's kernels; the host
// only carries scalars (Chebyshev coefficients, bounds, a 20x20 Lanczos
// tridiagonal) and the control flow.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <rocsolver/rocsolver.h>

#include "internal.h"

using namespace chfsi;

// ---------------------------------------------------------------------------
// Static scratch of chfsi_residual_noalloc: the column-norm partials
// [kRowBlocks][nvec] of the residual, for callers that cannot allocate.
// Each device holds its own copy of the array until the process ends.  In
// host code `scratch` names a host-side stand-in, not device memory: the
// device address of each GPU's copy is taken once with hipGetSymbolAddress
// (with that device current) and only that address is passed to kernels.
constexpr int64_t kNoAllocMaxCols = 4096;
constexpr int64_t kNoAllocDoubles = (int64_t)chfsi::kRowBlocks * kNoAllocMaxCols;  // 8 MiB
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
double *g_noalloc_ptr[kMaxDevices] = {};

// Device address of the current device's static scratch, taken on first use
// (hipGetSymbolAddress, never the array's name); nullptr and *err on failure.
double *noalloc_scratch(hipError_t *err) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && (dev < 0 || dev >= kMaxDevices)) e = hipErrorInvalidDevice;
    if (e != hipSuccess) {
        *err = e;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        g_noalloc_ptr[dev] = static_cast<double *>(p);
    }
    *err = hipSuccess;
    return g_noalloc_ptr[dev];
}


thread_local std::string g_err;

int fail(chfsi_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    g_err = msg;
    return code;
}

#define HIPCHK(ctx, expr)                                                                          \
    do {                                                                                           \
        hipError_t _e = (expr);                                                                    \
        if (_e != hipSuccess)                                                                      \
            return fail(ctx, CHFSI_E_DEVICE, std::string(#expr " failed: ") + hipGetErrorString(_e)); \
    } while (0)

#define BLASCHK(ctx, expr)                                                                         \
    do {                                                                                           \
        rocblas_status _s = (expr);                                                                \
        if (_s != rocblas_status_success)                                                          \
            return fail(ctx, CHFSI_E_DEVICE, std::string(#expr " failed: ") + rocblas_status_to_string(_s)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ----------------------------------------------------------------- 1D basis
// Legendre polynomial P_n and its derivative (Bonnet recurrence).
void legendre_eval(int n, double x, double &P, double &dP) {
    if (n == 0) { P = 1; dP = 0; return; }
    double pm = 1, pc = x, dm = 0, dc = 1;
    for (int k = 1; k < n; ++k) {
        double pn = ((2 * k + 1) * x * pc - k * pm) / (k + 1);
        double dn = dm + (2 * k + 1) * pc;  // P'_{k+1} = P'_{k-1} + (2k+1) P_k
        pm = pc; pc = pn; dm = dc; dc = dn;
    }
    P = pc;
    dP = dc;
}

// Gauss-Legendre: roots of P_n (Newton from the Chebyshev-like guesses), ascending.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0); w.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        double t = std::cos(M_PI * (4.0 * (n - i) - 1.0) / (4.0 * n + 2.0));
        for (int it = 0; it < 200; ++it) {
            double P, dP;
            legendre_eval(n, t, P, dP);
            double d = P / dP;
            t -= d;
            if (std::fabs(d) < 4e-17) break;
        }
        double P, dP;
        legendre_eval(n, t, P, dP);
        x[i] = t;
        w[i] = 2.0 / ((1 - t * t) * dP * dP);
    }
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return x[a] < x[b]; });
    std::vector<double> xs(n), ws(n);
    for (int i = 0; i < n; ++i) { xs[i] = x[ord[i]]; ws[i] = w[ord[i]]; }
    x = xs; w = ws;
}

// Gauss-Lobatto-Legendre: +-1 and the roots of P_{p-1} - P_{p+1} (which is
// proportional to (1-x^2) P_p'), Newton; w_i = 2/(p(p+1) P_p(x_i)^2).
void gauss_lobatto(int p, std::vector<double> &x, std::vector<double> &w) {
    x.assign(p + 1, 0); w.assign(p + 1, 0);
    x[0] = -1; x[p] = 1;
    for (int i = 1; i < p; ++i) {
        double t = -std::cos(M_PI * i / p);
        for (int it = 0; it < 200; ++it) {
            double Pa, dPa, Pb, dPb;
            legendre_eval(p - 1, t, Pa, dPa);
            legendre_eval(p + 1, t, Pb, dPb);
            double d = (Pa - Pb) / (dPa - dPb);
            t -= d;
            if (std::fabs(d) < 4e-17) break;
        }
        x[i] = t;
    }
    for (int i = 0; i <= p; ++i) {
        double P, dP;
        legendre_eval(p, x[i], P, dP);
        w[i] = 2.0 / (p * (p + 1.0) * P * P);
    }
}

// Lagrange cardinal functions of `nodes` and their derivatives at t
// (barycentric weights; derivative as the sum of the products leaving one
// factor out).
void cardinal(const std::vector<double> &nodes, double t, std::vector<double> &l, std::vector<double> &dl) {
    const int n = (int)nodes.size();
    l.assign(n, 0); dl.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        double bw = 1;
        for (int j = 0; j < n; ++j) if (j != i) bw /= (nodes[i] - nodes[j]);
        double prod = 1;
        for (int j = 0; j < n; ++j) if (j != i) prod *= (t - nodes[j]);
        double d = 0;
        for (int k = 0; k < n; ++k) {
            if (k == i) continue;
            double pk = 1;
            for (int j = 0; j < n; ++j) if (j != i && j != k) pk *= (t - nodes[j]);
            d += pk;
        }
        l[i] = bw * prod;
        dl[i] = bw * d;
    }
}

int pad_size(int need) {
    static const int sizes[] = {32, 64, 128, 224, 352, 512};
    for (int s : sizes) if (need <= s) return s;
    return -1;
}

int build_mesh(const chfsi_mesh *mesh, const chfsi_projectors *proj, Mesh &m, std::string &msg) {
    if (!mesh) { msg = "mesh is NULL"; return CHFSI_E_ARG; }
    for (int d = 0; d < 3; ++d) {
        if (mesh->ncell[d] < 2 || (mesh->ncell[d] & 1)) {
            msg = "ncell[" + std::to_string(d) + "] must be even and >= 2 (cell colouring)";
            return CHFSI_E_ARG;
        }
        if (!(mesh->h[d] > 0) || !std::isfinite(mesh->h[d])) { msg = "h must be positive"; return CHFSI_E_ARG; }
        m.ncell[d] = mesh->ncell[d];
        m.h[d] = mesh->h[d];
    }
    if (mesh->degree < 1 || mesh->degree > 7) { msg = "degree must be in 1..7"; return CHFSI_E_ARG; }
    m.p = mesh->degree;
    m.n1 = m.p + 1;
    m.n = m.n1 * m.n1 * m.n1;
    m.nq1 = mesh->nq1d == 0 ? m.p + 1 : mesh->nq1d;
    if (m.nq1 < 1 || m.nq1 > 8) { msg = "nq1d must be in 1..8"; return CHFSI_E_ARG; }
    m.nq = m.nq1 * m.nq1 * m.nq1;
    m.npad = pad_size(std::max(m.n, m.nq));
    m.nqpad = m.npad;
    m.ncells = m.ncell[0] * m.ncell[1] * m.ncell[2];
    for (int d = 0; d < 3; ++d) m.Nd[d] = m.ncell[d] * m.p;
    m.M = m.Nd[0] * m.Nd[1] * m.Nd[2];
    if (m.ncells > (int64_t)1 << 30) { msg = "too many cells"; return CHFSI_E_ARG; }
    m.natoms = 0; m.npairs = 0; m.nbeta = 0; m.n_nl_cells = 0;
    if (proj && proj->natoms > 0) {
        if (proj->nbeta < 1 || proj->nbeta > kMaxBeta) { msg = "nbeta must be in 1..16"; return CHFSI_E_ARG; }
        if (!proj->pair_ptr || !proj->pair_cell || !proj->phi || !proj->delta) {
            msg = "projector arrays must be non-NULL"; return CHFSI_E_ARG;
        }
        m.natoms = proj->natoms;
        m.nbeta = proj->nbeta;
        if (proj->pair_ptr[0] != 0) { msg = "pair_ptr[0] must be 0"; return CHFSI_E_ARG; }
        for (int64_t a = 0; a < m.natoms; ++a)
            if (proj->pair_ptr[a + 1] < proj->pair_ptr[a]) { msg = "pair_ptr not monotone"; return CHFSI_E_ARG; }
        m.npairs = proj->pair_ptr[m.natoms];
        if (m.npairs > (int64_t)1 << 30) { msg = "too many pairs"; return CHFSI_E_ARG; }
        std::vector<char> has(m.ncells, 0);
        for (int64_t pp = 0; pp < m.npairs; ++pp) {
            int64_t e = proj->pair_cell[pp];
            if (e < 0 || e >= m.ncells) { msg = "pair_cell out of range"; return CHFSI_E_ARG; }
            has[e] = 1;
        }
        for (int64_t e = 0; e < m.ncells; ++e) m.n_nl_cells += has[e];
    }
    return CHFSI_OK;
}

// Bytes of one recurrence block of nvec columns in the filter's complex type.
size_t zblock_bytes(const Mesh &m, int64_t nvec, bool z32) {
    return align256((size_t)(2 * m.M) * nvec * (z32 ? sizeof(cf) : sizeof(cd)));
}

Layout build_layout(const Mesh &m, int64_t max_nvec, int64_t filter_block, chfsi_prec filter_prec) {
    Layout L{};
    size_t o = 0;
    const size_t NP2 = (size_t)m.npad * m.npad;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    L.K64 = take(NP2 * 8); L.Phi64 = take(NP2 * 8); L.PhiT64 = take(NP2 * 8); L.M64 = take(NP2 * 8);
    L.K32 = take(NP2 * 4); L.Phi32 = take(NP2 * 4); L.PhiT32 = take(NP2 * 4);
    L.Kb = take(NP2 * 2); L.Phib = take(NP2 * 2); L.PhiTb = take(NP2 * 2);
    L.W64 = take((size_t)m.ncells * m.npad * 4 * 8);
    L.W32 = take((size_t)m.ncells * m.npad * 4 * 4);
    L.Wq = take((size_t)m.npad * 8);
    L.D64 = take((size_t)m.M * 8);
    L.Dinv64 = take((size_t)m.M * 8);
    L.Dinv32 = take((size_t)m.M * 4);
    L.colour_cells = take((size_t)m.ncells * 4);
    L.nl_cells = take((size_t)std::max<int64_t>(m.n_nl_cells, 1) * 4);
    L.cell_pair_ptr = take((size_t)(m.ncells + 1) * 4);
    L.cell_pairs = take((size_t)std::max<int64_t>(m.npairs, 1) * 4);
    L.pair_atom = take((size_t)std::max<int64_t>(m.npairs, 1) * 4);
    L.atom_pair_ptr = take((size_t)(m.natoms + 1) * 4);
    // projection tables [pair][tile of 8 projectors][node][j % 8][spin]
    L.P64 = take((size_t)m.npairs * ((m.nbeta + 7) / 8) * m.npad * 16 * 16);
    L.P32 = take((size_t)m.npairs * ((m.nbeta + 7) / 8) * m.npad * 16 * 8);
    L.PB = take((size_t)m.npairs * ((m.nbeta + 7) / 8) * m.npad * 64 * 2);
    L.kpad = (4 * m.nbeta + 31) / 32 * 32;
    L.WP64 = take((size_t)m.npairs * 4 * m.nbeta * m.npad * 8);
    L.WP32 = take((size_t)m.npairs * 4 * m.nbeta * m.npad * 4);
    L.WPb = take((size_t)m.npairs * m.npad * L.kpad * 2);
    L.delta64 = take((size_t)m.natoms * m.nbeta * m.nbeta * 16);
    L.KdInv64 = take((size_t)m.M * 8);
    L.persistent_bytes = o;

    o = 0;
    L.partial = take((size_t)m.npairs * m.nbeta * max_nvec * 16);
    L.dcoef = take((size_t)m.natoms * m.nbeta * max_nvec * 16);
    L.lamk = take((size_t)(kMaxDegree + 1) * max_nvec * 8);
    L.small_bytes = (size_t)max_nvec * max_nvec * 16;
    L.small = take(9 * L.small_bytes + 2 * (size_t)max_nvec * 8);
    L.red_bytes = (size_t)256 * std::max<int64_t>(max_nvec, 2) * 8 + 4096 * 8;
    L.red = take(L.red_bytes);
    L.flag = take(256);
    // filter: two recurrence blocks (Z_{k+1} overwrites Z_{k-1} element by
    // element); Lanczos: four vectors and a table of M.  The Rayleigh-Ritz
    // rotations and the split-K Gram partials use the same area in row chunks.
    L.zarea = std::max<size_t>(2 * zblock_bytes(m, filter_block, filter_prec != CHFSI_FP64),
                               5 * (size_t)(2 * m.M) * 16);
    L.Z = take(L.zarea);
    size_t phi_bytes = (size_t)m.npairs * m.nq * 2 * m.nbeta * 16;
    L.scratch_bytes = std::max(o, align256(L.Z + phi_bytes));
    L.zarea = L.scratch_bytes - L.Z;
    return L;
}

// tables of the reference cell (independent host implementation)
struct HostTables {
    std::vector<double> K, Phi, PhiT, Mref, wq, D;
    std::vector<double> poi1d, Kdinv;  // Poisson: 1D tables, 1 / diag(K)
};

void build_tables(const Mesh &m, HostTables &t) {
    std::vector<double> xg, wg, xq, wqd;
    gauss_lobatto(m.p, xg, wg);
    gauss_legendre(m.nq1, xq, wqd);
    const int n1 = m.n1, q1 = m.nq1, NP = m.npad;
    std::vector<double> l1((size_t)q1 * n1), dl1((size_t)q1 * n1), l, dl;
    for (int a = 0; a < q1; ++a) {
        cardinal(xg, xq[a], l, dl);
        for (int i = 0; i < n1; ++i) { l1[a * n1 + i] = l[i]; dl1[a * n1 + i] = dl[i]; }
    }
    std::vector<double> m1((size_t)n1 * n1, 0), k1((size_t)n1 * n1, 0);
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j)
            for (int a = 0; a < q1; ++a) {
                m1[i * n1 + j] += wqd[a] * l1[a * n1 + i] * l1[a * n1 + j];
                k1[i * n1 + j] += wqd[a] * dl1[a * n1 + i] * dl1[a * n1 + j];
            }
    const double detJ = m.h[0] * m.h[1] * m.h[2] / 8.0;
    const double sx = 4.0 / (m.h[0] * m.h[0]), sy = 4.0 / (m.h[1] * m.h[1]), sz = 4.0 / (m.h[2] * m.h[2]);
    t.K.assign((size_t)NP * NP, 0); t.Mref.assign((size_t)NP * NP, 0);
    t.Phi.assign((size_t)NP * NP, 0); t.PhiT.assign((size_t)NP * NP, 0);
    t.wq.assign(NP, 0);
    for (int I = 0; I < m.n; ++I) {
        int i = I % n1, j = (I / n1) % n1, k = I / (n1 * n1);
        for (int J = 0; J < m.n; ++J) {
            int ii = J % n1, jj = (J / n1) % n1, kk = J / (n1 * n1);
            double mx = m1[i * n1 + ii], my = m1[j * n1 + jj], mz = m1[k * n1 + kk];
            double kx = k1[i * n1 + ii], ky = k1[j * n1 + jj], kz = k1[k * n1 + kk];
            t.K[(size_t)I * NP + J] = 0.5 * detJ * (sx * kx * my * mz + sy * mx * ky * mz + sz * mx * my * kz);
            t.Mref[(size_t)I * NP + J] = detJ * mx * my * mz;
        }
    }
    for (int q = 0; q < m.nq; ++q) {
        int a = q % q1, b = (q / q1) % q1, c = q / (q1 * q1);
        t.wq[q] = wqd[a] * wqd[b] * wqd[c] * detJ;
        for (int I = 0; I < m.n; ++I) {
            int i = I % n1, j = (I / n1) % n1, k = I / (n1 * n1);
            double v = l1[a * n1 + i] * l1[b * n1 + j] * l1[c * n1 + k];
            t.Phi[(size_t)q * NP + I] = v;
            t.PhiT[(size_t)I * NP + q] = v;
        }
    }
    // Poisson 1D operators in the even/odd form of the K x kernel: for each
    // of N[q][i] = l_i(x_q), N^T, Dq[a][b] = l'_b(x_a) (collocation
    // derivative: Lagrange basis of the Gauss points) and Dq^T, the first
    // ceil(rows/2) rows of E = (T[a][b] + T[a][ni-1-b]) / 2 (middle column
    // as is) and O = (T[a][b] - T[a][ni-1-b]) / 2; then the Gauss weights.
    {
        std::vector<double> N((size_t)q1 * n1), NT((size_t)n1 * q1), Dq((size_t)q1 * q1), DT((size_t)q1 * q1);
        for (int a = 0; a < q1; ++a) {
            for (int i = 0; i < n1; ++i) N[a * n1 + i] = NT[i * q1 + a] = l1[a * n1 + i];
            cardinal(xq, xq[a], l, dl);
            for (int b = 0; b < q1; ++b) Dq[a * q1 + b] = DT[b * q1 + a] = dl[b];
        }
        t.poi1d.clear();
        auto eo = [&](const std::vector<double> &T, int no, int ni) {
            for (int a = 0; a < (no + 1) / 2; ++a)
                for (int b = 0; b < (ni + 1) / 2; ++b)
                    t.poi1d.push_back(2 * b + 1 == ni ? T[a * ni + b] : 0.5 * (T[a * ni + b] + T[a * ni + ni - 1 - b]));
            for (int a = 0; a < (no + 1) / 2; ++a)
                for (int b = 0; b < ni / 2; ++b) t.poi1d.push_back(0.5 * (T[a * ni + b] - T[a * ni + ni - 1 - b]));
        };
        eo(N, q1, n1);
        eo(NT, n1, q1);
        eo(Dq, q1, q1);
        eo(DT, q1, q1);
        for (int a = 0; a < q1; ++a) t.poi1d.push_back(wqd[a]);
    }
    // diag(K) of the Poisson stiffness K_IJ = sum_e int grad N_I . grad N_J
    // (twice the kinetic table's diagonal), summed over the cells of a node
    std::vector<double> kd((size_t)m.n);
    for (int I = 0; I < m.n; ++I) {
        int i = I % n1, j = (I / n1) % n1, k = I / (n1 * n1);
        kd[I] = detJ * (sx * k1[i * n1 + i] * m1[j * n1 + j] * m1[k * n1 + k] +
                        sy * m1[i * n1 + i] * k1[j * n1 + j] * m1[k * n1 + k] +
                        sz * m1[i * n1 + i] * m1[j * n1 + j] * k1[k * n1 + k]);
    }
    t.Kdinv.assign(m.M, 0);
    t.D.assign(m.M, 0);
    for (int64_t e = 0; e < m.ncells; ++e) {
        int64_t ex = e % m.ncell[0], ey = (e / m.ncell[0]) % m.ncell[1], ez = e / (m.ncell[0] * m.ncell[1]);
        for (int I = 0; I < m.n; ++I) {
            int i = I % n1, j = (I / n1) % n1, k = I / (n1 * n1);
            int64_t gx = (ex * m.p + i) % m.Nd[0], gy = (ey * m.p + j) % m.Nd[1], gz = (ez * m.p + k) % m.Nd[2];
            t.D[gx + m.Nd[0] * (gy + m.Nd[1] * gz)] += detJ * wg[i] * wg[j] * wg[k];
            t.Kdinv[gx + m.Nd[0] * (gy + m.Nd[1] * gz)] += kd[I];
        }
    }
    for (auto &v : t.Kdinv) v = 1.0 / v;
}

// largest eigenvalue of the symmetric tridiagonal (alpha, beta[1..m-1]) by
// Sturm-sequence bisection
double tridiag_max(const std::vector<double> &al, const std::vector<double> &be) {
    const int m = (int)al.size();
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < m; ++i) {
        double r = (i > 0 ? std::fabs(be[i]) : 0) + (i + 1 < m ? std::fabs(be[i + 1]) : 0);
        lo = std::min(lo, al[i] - r);
        hi = std::max(hi, al[i] + r);
    }
    auto count_below = [&](double x) {  // number of eigenvalues < x
        int cnt = 0;
        double d = 1;
        for (int i = 0; i < m; ++i) {
            double b2 = i > 0 ? be[i] * be[i] : 0;
            d = al[i] - x - (i > 0 ? b2 / d : 0);
            if (d == 0) d = -1e-300;
            if (d < 0) ++cnt;
        }
        return cnt;
    };
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (count_below(mid) >= m) hi = mid; else lo = mid;
        if (hi - lo <= 1e-15 * std::max(1.0, std::fabs(hi))) break;
    }
    return hi;
}

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

int check_block(chfsi_ctx *c, const void *p, int64_t nvec, int64_t ld, const char *name) {
    if (!p) return fail(c, CHFSI_E_ARG, std::string(name) + " is NULL");
    if (nvec < 1 || nvec > c->max_nvec)
        return fail(c, CHFSI_E_ARG, "nvec must be in 1..max_nvec (" + std::to_string(c->max_nvec) + ")");
    if (ld < nvec) return fail(c, CHFSI_E_ARG, "ld must be >= nvec");
    return CHFSI_OK;
}

int read_flag(chfsi_ctx *c, hipStream_t s, int *out) {
    int h = 0;
    hipError_t e = hipMemcpyAsync(&h, c->S<int>(c->L.flag), sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(c, CHFSI_E_DEVICE, std::string("flag read failed: ") + hipGetErrorString(e));
    *out = h;
    return CHFSI_OK;
}

// Blocked Cholesky A = L L^H of a row-major N x N Hermitian matrix (lower L,
// strict upper triangle zeroed).  The column-major view of the buffer is
// conj(A) = U^H U with U = L^T upper triangular, so the panels are BLAS-3
// calls on that view: per block column j, the diagonal block is factored by
// one workgroup, then U_12 <- U_11^{-H} A_12 (trsm) and A_22 -= U_12^H U_12
// (herk).  flag = 1 if a pivot is below 64 eps (rank deficiency).
int cholesky_blocked(chfsi_ctx *c, int N, cd *A, int *flag, hipStream_t s) {
    constexpr int NB = 64;
    BLASCHK(c, rocblas_set_stream(c->blas, s));
    const rocblas_double_complex one{1.0, 0.0}, mone{-1.0, 0.0};
    const double dmone = -1.0, done = 1.0;
    auto rb = [](cd *p) { return reinterpret_cast<rocblas_double_complex *>(p); };
    for (int j = 0; j < N; j += NB) {
        const int nb = std::min(NB, N - j), m = N - j - nb;
        cd *Ajj = A + (int64_t)j * N + j;
        HIPCHK(c, launch_cholesky_block(nb, N, Ajj, flag, s));
        if (m == 0) break;
        cd *A12 = A + (int64_t)(j + nb) * N + j;  // column-major (j, j + nb)
        BLASCHK(c, rocblas_ztrsm(c->blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_conjugate_transpose,
                                 rocblas_diagonal_non_unit, nb, m, &one, rb(Ajj), N, rb(A12), N));
        BLASCHK(c, rocblas_zherk(c->blas, rocblas_fill_upper, rocblas_operation_conjugate_transpose, m, nb, &dmone,
                                 rb(A12), N, &done, rb(A + (int64_t)(j + nb) * N + j + nb), N));
    }
    (void)mone;
    HIPCHK(c, launch_zero_upper(N, A, s));
    return CHFSI_OK;
}

// T = diag(scale) L^{-H} for the factor of cholesky_blocked: in the
// column-major view T^T = U^{-H} diag(scale), one triangular solve.
int tri_inv_scaled(chfsi_ctx *c, int N, cd *L, const double *scale, cd *T, hipStream_t s) {
    BLASCHK(c, rocblas_set_stream(c->blas, s));
    const rocblas_double_complex one{1.0, 0.0};
    HIPCHK(c, launch_diag(N, scale, T, s));
    BLASCHK(c, rocblas_ztrsm(c->blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_conjugate_transpose,
                             rocblas_diagonal_non_unit, N, N, &one, reinterpret_cast<rocblas_double_complex *>(L), N,
                             reinterpret_cast<rocblas_double_complex *>(T), N));
    return CHFSI_OK;
}

// S = A^H B (N x N row-major) for [rows][ld] blocks when S is Hermitian
// (B = M A or H A).  Column-major view of a row-major block is its
// transpose, so the upper block rows of S are S^T products Bcm Acm^H in BLAS
// terms: one per block row of width GB, each only for the columns at and
// right of its diagonal block (about 0.67 of the full product at N = 576).
// The reduction dimension (2M rows) is split into up to 128 chunks computed
// as one strided-batched product, so that even the last, narrow block row
// gives the chip several workgroups per CU (measured on the medium mesh,
// N = 576: 96-row blocks in 32 chunks took 50 ms more per pair of Grams than
// 192-row blocks in 128 chunks).  The partial matrices are summed in a fixed
// order and the strict lower triangle is filled with the conjugate of the
// upper one.
int gram(chfsi_ctx *c, const cd *A, const cd *B, int64_t N, int64_t ld, cd *Sm, hipStream_t s) {
    constexpr int64_t GB = 192;
    BLASCHK(c, rocblas_set_stream(c->blas, s));
    const rocblas_double_complex one{1.0, 0.0}, zero{0.0, 0.0};
    const int64_t rows = 2 * c->m.M;
    const size_t zcap = c->L.zarea / sizeof(cd);
    int64_t nb = 128;
    while (nb > 1 && ((size_t)(nb + 1) * N * N > zcap || rows / nb < 4096)) nb /= 2;
    auto rb = [](const cd *p) { return reinterpret_cast<const rocblas_double_complex *>(p); };
    auto wb = [](cd *p) { return reinterpret_cast<rocblas_double_complex *>(p); };
    cd *part = nb == 1 ? Sm : c->S<cd>(c->L.Z);
    const int64_t chunk = rows / nb, tail = rows - nb * chunk;
    for (int64_t i0 = 0; i0 < N; i0 += GB) {
        const rocblas_int m = (rocblas_int)(N - i0), n = (rocblas_int)std::min(GB, N - i0);
        if (nb == 1) {
            BLASCHK(c, rocblas_zgemm(c->blas, rocblas_operation_none, rocblas_operation_conjugate_transpose, m, n,
                                     (rocblas_int)rows, &one, rb(B + i0), (rocblas_int)ld, rb(A + i0),
                                     (rocblas_int)ld, &zero, wb(part + i0 * N + i0), (rocblas_int)N));
            continue;
        }
        BLASCHK(c, rocblas_zgemm_strided_batched(
                       c->blas, rocblas_operation_none, rocblas_operation_conjugate_transpose, m, n,
                       (rocblas_int)chunk, &one, rb(B + i0), (rocblas_int)ld, (rocblas_stride)(chunk * ld),
                       rb(A + i0), (rocblas_int)ld, (rocblas_stride)(chunk * ld), &zero, wb(part + i0 * N + i0),
                       (rocblas_int)N, (rocblas_stride)(N * N), (rocblas_int)nb));
        if (tail > 0)
            BLASCHK(c, rocblas_zgemm(c->blas, rocblas_operation_none, rocblas_operation_conjugate_transpose, m, n,
                                     (rocblas_int)tail, &one, rb(B + nb * chunk * ld + i0), (rocblas_int)ld,
                                     rb(A + nb * chunk * ld + i0), (rocblas_int)ld, &zero,
                                     wb(part + nb * N * N + i0 * N + i0), (rocblas_int)N));
    }
    if (nb > 1) HIPCHK(c, launch_sum_parts(N * N, (int)nb + (tail > 0 ? 1 : 0), part, Sm, s));
    HIPCHK(c, launch_fill_lower(N, Sm, s));
    return CHFSI_OK;
}

// C = A B for row-major N x N matrices (column-major BLAS computes C^T = B^T A^T)
int small_mm(chfsi_ctx *c, const cd *A, const cd *B, cd *Cm, int64_t N, bool conjA, hipStream_t s) {
    BLASCHK(c, rocblas_set_stream(c->blas, s));
    const rocblas_double_complex one{1.0, 0.0}, zero{0.0, 0.0};
    // conjA: C = A^H B, i.e. C^T = B^T conj(A) = (buffer of B) op_C(buffer of A)
    BLASCHK(c, rocblas_zgemm(c->blas, rocblas_operation_none,
                             conjA ? rocblas_operation_conjugate_transpose : rocblas_operation_none, (rocblas_int)N,
                             (rocblas_int)N, (rocblas_int)N, &one, reinterpret_cast<const rocblas_double_complex *>(B),
                             (rocblas_int)N, reinterpret_cast<const rocblas_double_complex *>(A), (rocblas_int)N,
                             &zero, reinterpret_cast<rocblas_double_complex *>(Cm), (rocblas_int)N));
    return CHFSI_OK;
}

// A <- A Q (A: [rows][ld] block with N columns; Q: N x N row-major), through
// the compact temporary Z buffer and a strided copy back.
// Rows of a block whose temporaries (bytes_per_row each) fit the Z area at
// once: the whole block when the scratch was planned for it, else chunks.
int64_t row_chunk(const chfsi_ctx *c, size_t bytes_per_row) {
    const int64_t rows = 2 * c->m.M;
    const int64_t cap = (int64_t)(c->L.zarea / bytes_per_row);
    return std::max<int64_t>(1, std::min(rows, cap));
}

int rotate(chfsi_ctx *c, cd *A, const cd *Q, int64_t N, int64_t ld, hipStream_t s) {
    cd *tmp = c->S<cd>(c->L.Z);
    const int64_t rows = 2 * c->m.M, rc = row_chunk(c, (size_t)N * sizeof(cd));
    BLASCHK(c, rocblas_set_stream(c->blas, s));
    const rocblas_double_complex one{1.0, 0.0}, zero{0.0, 0.0};
    for (int64_t r0 = 0; r0 < rows; r0 += rc) {
        const int64_t nr = std::min(rc, rows - r0);
        BLASCHK(c, rocblas_zgemm(c->blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)N,
                                 (rocblas_int)nr, (rocblas_int)N, &one,
                                 reinterpret_cast<const rocblas_double_complex *>(Q), (rocblas_int)N,
                                 reinterpret_cast<const rocblas_double_complex *>(A + r0 * ld), (rocblas_int)ld,
                                 &zero, reinterpret_cast<rocblas_double_complex *>(tmp), (rocblas_int)N));
        HIPCHK(c, hipMemcpy2DAsync(A + r0 * ld, ld * sizeof(cd), tmp, N * sizeof(cd), N * sizeof(cd), nr,
                                   hipMemcpyDeviceToDevice, s));
    }
    return CHFSI_OK;
}

// A <- A Q with the paper's mixed-precision subspace rotation (RR-SR, Sec.
// III-C4, the Rayleigh-Ritz step): the diagonal SRB x SRB blocks of Q in
// FP64 (one strided-batched zgemm), the off-diagonal part in FP32 (cgemm on
// complex64 copies of A and of Q with its diagonal blocks zeroed), summed in
// FP64.  Q32 is scratch for an N x N complex64 matrix.
constexpr int64_t SRB = 64;
int rotate_mixed(chfsi_ctx *c, cd *A, const cd *Q, int64_t N, int64_t ld, cf *Q32, hipStream_t s) {
    const int64_t rows = 2 * c->m.M, rc = row_chunk(c, (size_t)N * (sizeof(cd) + 2 * sizeof(cf)));
    cd *T = c->S<cd>(c->L.Z);
    cf *A32 = reinterpret_cast<cf *>(T + rc * N), *C32 = A32 + rc * N;
    BLASCHK(c, rocblas_set_stream(c->blas, s));
    const rocblas_double_complex one{1.0, 0.0}, zero{0.0, 0.0};
    const rocblas_float_complex onef{1.0f, 0.0f}, zerof{0.0f, 0.0f};
    auto zc = [](const cd *p) { return reinterpret_cast<const rocblas_double_complex *>(p); };
    const int64_t nfull = N / SRB, rem = N - nfull * SRB;
    HIPCHK(c, launch_offdiag_cf((int)N, (int)SRB, Q, Q32, s));
    for (int64_t r0 = 0; r0 < rows; r0 += rc) {
        const int64_t nr = std::min(rc, rows - r0);
        cd *Ar = A + r0 * ld;
        if (nfull > 0)
            BLASCHK(c, rocblas_zgemm_strided_batched(
                           c->blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)SRB, (rocblas_int)nr,
                           (rocblas_int)SRB, &one, zc(Q), (rocblas_int)N, (rocblas_stride)(SRB * (N + 1)), zc(Ar),
                           (rocblas_int)ld, (rocblas_stride)SRB, &zero, reinterpret_cast<rocblas_double_complex *>(T),
                           (rocblas_int)N, (rocblas_stride)SRB, (rocblas_int)nfull));
        if (rem > 0) {
            const int64_t o = nfull * SRB;
            BLASCHK(c, rocblas_zgemm(c->blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)rem,
                                     (rocblas_int)nr, (rocblas_int)rem, &one, zc(Q + o * N + o), (rocblas_int)N,
                                     zc(Ar + o), (rocblas_int)ld, &zero,
                                     reinterpret_cast<rocblas_double_complex *>(T + o), (rocblas_int)N));
        }
        HIPCHK(c, launch_sr_to_cf(nr, N, ld, Ar, A32, s));
        BLASCHK(c, rocblas_cgemm(c->blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)N,
                                 (rocblas_int)nr, (rocblas_int)N, &onef,
                                 reinterpret_cast<const rocblas_float_complex *>(Q32), (rocblas_int)N,
                                 reinterpret_cast<const rocblas_float_complex *>(A32), (rocblas_int)N, &zerof,
                                 reinterpret_cast<rocblas_float_complex *>(C32), (rocblas_int)N));
        HIPCHK(c, launch_sr_combine(nr, N, ld, T, C32, Ar, s));
    }
    return CHFSI_OK;
}

int apply_H_impl(chfsi_ctx *c, chfsi_prec prec, const void *X, void *Y, int64_t nvec, int64_t ld,
                 hipStream_t s) {
    const int nl = c->m.npairs > 0 ? FLAG_NLOC : 0;
    if (nl) HIPCHK(c, launch_nonlocal_coeffs(c, prec, 0, X, nvec, ld, s));
    HIPCHK(c, launch_cell_op(c, prec, MODE_HAM, nl, 1.0, X, Y, nvec, ld, s));
    return CHFSI_OK;
}

int orthonormalize_impl(chfsi_ctx *c, cd *Y, cd *HY, cd *MY, int64_t nvec, int64_t ld, hipStream_t s) {
    const Layout &L = c->L;
    cd *Sm = c->S<cd>(L.small);
    cd *T = Sm + L.small_bytes / sizeof(cd);
    double *scale = reinterpret_cast<double *>(c->scr + L.small + 9 * L.small_bytes);
    int *flag = c->S<int>(L.flag);
    HIPCHK(c, hipMemsetAsync(flag, 0, sizeof(int), s));
    for (int pass = 0; pass < 2; ++pass) {
        int rc = gram(c, Y, MY, nvec, ld, Sm, s);
        if (rc) return rc;
        HIPCHK(c, launch_herm_equilibrate((int)nvec, Sm, scale, flag, s));
        if ((rc = cholesky_blocked(c, (int)nvec, Sm, flag, s))) return rc;
        int f = 0;
        rc = read_flag(c, s, &f);
        if (rc) return rc;
        if (f) return fail(c, CHFSI_E_NOT_SPD, "Cholesky-QR breakdown: the block is (numerically) rank deficient");
        if ((rc = tri_inv_scaled(c, (int)nvec, Sm, scale, T, s))) return rc;
        if ((rc = rotate(c, Y, T, nvec, ld, s))) return rc;
        if (HY && (rc = rotate(c, HY, T, nvec, ld, s))) return rc;
        if ((rc = rotate(c, MY, T, nvec, ld, s))) return rc;
    }
    return CHFSI_OK;
}

// Eigenpairs of the N x N Hermitian matrix A (row-major, overwritten): w the
// eigenvalues in ascending order, Q (row-major) the eigenvectors as columns
// (Algorithm RChFSI, the subspace eigenproblem of the RR step; the paper
// solves it with ELPA).  rocSOLVER's divide and conquer (zheevd) works on the
// column-major view of the buffer, conj(A); launch_conj_transpose turns its
// eigenvectors into A's.  Synchronizes to read rocSOLVER's status.
int herm_eig(chfsi_ctx *c, int N, cd *A, cd *Q, double *w, hipStream_t s) {
    double *E = c->S<double>(c->L.red);
    int *info = reinterpret_cast<int *>(E + N);
    BLASCHK(c, rocblas_set_stream(c->blas, s));
    BLASCHK(c, rocsolver_zheevd(c->blas, rocblas_evect_original, rocblas_fill_upper, N,
                                reinterpret_cast<rocblas_double_complex *>(A), N, w, E, info));
    HIPCHK(c, launch_conj_transpose(N, A, Q, s));
    int h = 0;
    HIPCHK(c, hipMemcpyAsync(&h, info, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (h != 0)
        return fail(c, CHFSI_E_DEVICE, "subspace eigensolver (rocsolver_zheevd) failed, info = " + std::to_string(h));
    return CHFSI_OK;
}

int rr_impl(chfsi_ctx *c, cd *Y, cd *HY, cd *MY, int64_t nvec, int64_t ld, double *ritz, cd *R,
            double *resnorm, hipStream_t s) {
    const Layout &L = c->L;
    cd *Hs = c->S<cd>(L.small);
    const size_t st = L.small_bytes / sizeof(cd);
    cd *Q = Hs + 2 * st;
    int rc = gram(c, Y, HY, nvec, ld, Hs, s);
    if (rc) return rc;
    HIPCHK(c, launch_hermitize((int)nvec, Hs, s));
    if ((rc = herm_eig(c, (int)nvec, Hs, Q, ritz, s))) return rc;
    if ((rc = rotate(c, Y, Q, nvec, ld, s))) return rc;
    if ((rc = rotate(c, HY, Q, nvec, ld, s))) return rc;
    if ((rc = rotate(c, MY, Q, nvec, ld, s))) return rc;
    if (R || resnorm)
        HIPCHK(c, launch_residual(2 * c->m.M, nvec, ld, HY, MY, ritz, R, c->S<double>(L.red), resnorm, s));
    return CHFSI_OK;
}

// Rayleigh-Ritz on a block that is not M-orthonormal (the generalized
// subspace problem of Algorithm RChFSI, Y^H H Y Q = Y^H M Y Q Lambda):
// S = Y^H MY, Hs = Y^H HY, s = diag(S)^{-1/2}, L L^H = diag(s) S diag(s),
// T = diag(s) L^{-H}, C = T^H Hs T, C W = W Lambda, Q = T W,
// (Y, HY, MY) <- (.) Q.  Two Gram products and three rotations.
// Returns CHFSI_E_NOT_SPD if the Cholesky factorisation breaks down.
int rr_general_impl(chfsi_ctx *c, cd *Y, cd *HY, cd *MY, int64_t nvec, int64_t ld, double *ritz, cd *R,
                    double *resnorm, hipStream_t s, bool rotate_hm = true, bool mixed_sr = false) {
    const Layout &L = c->L;
    const size_t st = L.small_bytes / sizeof(cd);
    cd *Sm = c->S<cd>(L.small), *Hs = Sm + st, *T = Sm + 2 * st, *W = Sm + 3 * st, *Cm = Sm + 4 * st;
    cd *A2 = Sm + 5 * st, *Q = Sm + 6 * st;
    double *scale = reinterpret_cast<double *>(c->scr + L.small + 9 * L.small_bytes);
    int *flag = c->S<int>(L.flag);
    int rc;
    HIPCHK(c, hipMemsetAsync(flag, 0, sizeof(int), s));
    if ((rc = gram(c, Y, MY, nvec, ld, Sm, s))) return rc;
    if ((rc = gram(c, Y, HY, nvec, ld, Hs, s))) return rc;
    HIPCHK(c, launch_herm_equilibrate((int)nvec, Sm, scale, flag, s));
    if ((rc = cholesky_blocked(c, (int)nvec, Sm, flag, s))) return rc;
    int f = 0;
    if ((rc = read_flag(c, s, &f))) return rc;
    if (f) return fail(c, CHFSI_E_NOT_SPD, "Cholesky of Y^H M Y broke down: the block is (numerically) rank deficient");
    if ((rc = tri_inv_scaled(c, (int)nvec, Sm, scale, T, s))) return rc;
    if ((rc = small_mm(c, Hs, T, W, nvec, false, s))) return rc;   // W = Hs T
    if ((rc = small_mm(c, T, W, Cm, nvec, true, s))) return rc;    // C = T^H W
    HIPCHK(c, launch_hermitize((int)nvec, Cm, s));
    if ((rc = herm_eig(c, (int)nvec, Cm, Q, ritz, s))) return rc;
    if ((rc = small_mm(c, T, Q, W, nvec, false, s))) return rc;    // W = T Q
    if (mixed_sr) {
        if ((rc = rotate_mixed(c, Y, W, nvec, ld, reinterpret_cast<cf *>(A2), s))) return rc;
    } else if ((rc = rotate(c, Y, W, nvec, ld, s))) {
        return rc;
    }
    if (!rotate_hm && R) {
        // only the residual is needed from HY and MY: R = HY W - MY (W Lambda),
        // two products straight into R, then its column norms
        cd *WL = Sm + 8 * st;
        HIPCHK(c, launch_scale_cols((int)nvec, ritz, W, WL, s));
        BLASCHK(c, rocblas_set_stream(c->blas, s));
        const rocblas_double_complex one{1.0, 0.0}, mone{-1.0, 0.0}, zero{0.0, 0.0};
        const rocblas_int n = (rocblas_int)nvec, rows = (rocblas_int)(2 * c->m.M), l = (rocblas_int)ld;
        auto rb = [](const cd *p) { return reinterpret_cast<const rocblas_double_complex *>(p); };
        BLASCHK(c, rocblas_zgemm(c->blas, rocblas_operation_none, rocblas_operation_none, n, rows, n, &one, rb(W), n,
                                 rb(HY), l, &zero, reinterpret_cast<rocblas_double_complex *>(R), l));
        BLASCHK(c, rocblas_zgemm(c->blas, rocblas_operation_none, rocblas_operation_none, n, rows, n, &mone, rb(WL),
                                 n, rb(MY), l, &one, reinterpret_cast<rocblas_double_complex *>(R), l));
        if (resnorm) HIPCHK(c, launch_colnorm(2 * c->m.M, nvec, ld, R, c->S<double>(L.red), resnorm, s));
        return CHFSI_OK;
    }
    if ((rc = rotate(c, HY, W, nvec, ld, s))) return rc;
    if ((rc = rotate(c, MY, W, nvec, ld, s))) return rc;
    if (R || resnorm)
        HIPCHK(c, launch_residual(2 * c->m.M, nvec, ld, HY, MY, ritz, R, c->S<double>(L.red), resnorm, s));
    return CHFSI_OK;
}

// Device events around the cell-operator launches of filter steps: pairs
// (start, end) recorded on the filter's stream, read after the caller's
// synchronization.  A step is timed only while the pool has room for its pair.
struct StepEvents {
    std::vector<hipEvent_t> ev;
    size_t used = 0;
    ~StepEvents() {
        for (auto e : ev)
            if (e) hipEventDestroy(e);
    }
};

int filter_impl(chfsi_ctx *c, chfsi_prec prec, int degree, const double *bounds, const cd *X,
                const double *ritz, const cd *R, cd *Y, int64_t nvec, int64_t ld, hipStream_t s,
                StepEvents *pe = nullptr) {
    const Layout &L = c->L;
    const double lmin = bounds[0], lT = bounds[1], lmax = bounds[2];
    const double cc = 0.5 * (lmax + lT), e = 0.5 * (lmax - lT);
    const double s1 = e / (lmin - cc);
    const bool z32 = prec != CHFSI_FP64;
    const int64_t rows = 2 * c->m.M;
    char *zb = c->scr + L.Z;
    const size_t zstride = zblock_bytes(c->m, nvec, z32);
    if (2 * zstride > L.zarea)
        return fail(c, CHFSI_E_WORKSPACE, "the scratch holds two recurrence blocks of " +
                                              std::to_string(L.zarea / 2) + " bytes; this filter needs " +
                                              std::to_string(zstride) + " (plan a larger filter_block or a "
                                              "narrower filter precision)");
    // two blocks: Z_k is read by the products, Z_{k+1} is written over
    // Z_{k-1} element by element (each element of Z_{k-1} is read only by
    // the update that overwrites it)
    void *Zc = zb, *Zn = zb + zstride, *Zp = nullptr;
    double *lamk = c->S<double>(L.lamk);
    HIPCHK(c, launch_lamk_table(ritz, nvec, degree, cc, e, s1, lamk, nvec, s));
    // Z_1 = s1 R / e
    HIPCHK(c, launch_filter_init_ld(rows, nvec, nvec, ld, z32, Zc, nullptr, nullptr, R, 0, 0, nullptr, s1 / e, s));
    double sk = s1;
    const void *dinv = z32 ? (const void *)c->P<float>(L.Dinv32) : (const void *)c->P<double>(L.Dinv64);
    (void)dinv;
    const int nl = c->m.npairs > 0 ? FLAG_NLOC : 0;
    for (int k = 1; k < degree; ++k) {
        const double sn = 1.0 / (2.0 / s1 - sk);
        const double a = 2.0 * sn / e;
        // Z_{k+1} = -a c Z_k - s_k s_{k+1} Z_{k-1} + a R Lambda_k
        if (Zp) Zn = Zp;  // Z_{k+1} over Z_{k-1}
        // Z_{k+1} = a H D^{-1} Z_k - a c Z_k - s_k s_{k+1} Z_{k-1} + a R Lambda_k in one pass of the cell
        // operator: the first colour to reach a node writes all four terms, later colours add a H D^{-1} Z_k
        if (nl) HIPCHK(c, launch_nonlocal_coeffs(c, prec, FLAG_DINV, Zc, nvec, nvec, s));
        const EpiArgs ep{Zp, R, ld, lamk + (int64_t)k * nvec, -a * cc, -sk * sn};
        const bool timed = pe && pe->used + 2 <= pe->ev.size();
        if (timed) HIPCHK(c, hipEventRecord(pe->ev[pe->used], s));
        HIPCHK(c, launch_cell_op(c, prec, MODE_HAM, FLAG_EPI | FLAG_DINV | nl, a, Zc, Zn, nvec, nvec, s, &ep));
        if (timed) {
            HIPCHK(c, hipEventRecord(pe->ev[pe->used + 1], s));
            pe->used += 2;
        }
        Zp = Zc;
        Zc = Zn;
        sk = sn;
    }
    HIPCHK(c, launch_recover_ld(rows, nvec, nvec, ld, z32, Zc, c->P<double>(L.Dinv64), X,
                                lamk + (int64_t)degree * nvec, Y, s));
    return CHFSI_OK;
}

}  // namespace

// =========================================================================
extern "C" {

static int plan_opts_check(const chfsi_plan_opts *po, int64_t &max_nvec, int64_t &fblock, chfsi_prec &fprec) {
    if (!po) return fail(nullptr, CHFSI_E_ARG, "plan options are NULL");
    max_nvec = po->max_nvec;
    fblock = po->filter_block > 0 ? po->filter_block : po->max_nvec;
    fprec = po->filter_prec;
    if (max_nvec < 1) return fail(nullptr, CHFSI_E_ARG, "max_nvec must be >= 1");
    if (fblock > max_nvec) return fail(nullptr, CHFSI_E_ARG, "filter_block must be <= max_nvec");
    if (fprec < CHFSI_FP64 || fprec > CHFSI_BF16) return fail(nullptr, CHFSI_E_ARG, "unknown filter precision");
    return CHFSI_OK;
}

int chfsi_plan_ex(const chfsi_mesh *mesh, const chfsi_projectors *proj, const chfsi_plan_opts *po,
                  size_t *persistent_bytes, size_t *scratch_bytes) {
    Mesh m{};
    std::string msg;
    int rc = build_mesh(mesh, proj, m, msg);
    if (rc) return fail(nullptr, rc, msg);
    int64_t max_nvec, fblock;
    chfsi_prec fprec;
    if ((rc = plan_opts_check(po, max_nvec, fblock, fprec))) return rc;
    if (!persistent_bytes || !scratch_bytes) return fail(nullptr, CHFSI_E_ARG, "size outputs are NULL");
    Layout L = build_layout(m, max_nvec, fblock, fprec);
    *persistent_bytes = L.persistent_bytes;
    *scratch_bytes = L.scratch_bytes;
    return CHFSI_OK;
}

int chfsi_plan(const chfsi_mesh *mesh, const chfsi_projectors *proj, int64_t max_nvec,
               size_t *persistent_bytes, size_t *scratch_bytes) {
    const chfsi_plan_opts po{max_nvec, 0, CHFSI_FP64};
    return chfsi_plan_ex(mesh, proj, &po, persistent_bytes, scratch_bytes);
}

int chfsi_setup(const chfsi_mesh *mesh, const double *V, const double *B, const chfsi_projectors *proj,
                int64_t max_nvec, void *persistent, size_t persistent_bytes, void *scratch,
                size_t scratch_bytes, void *stream, chfsi_ctx **out) {
    const chfsi_plan_opts po{max_nvec, 0, CHFSI_FP64};
    return chfsi_setup_ex(mesh, V, B, proj, &po, persistent, persistent_bytes, scratch, scratch_bytes, stream, out);
}

int chfsi_setup_ex(const chfsi_mesh *mesh, const double *V, const double *B, const chfsi_projectors *proj,
                   const chfsi_plan_opts *po, void *persistent, size_t persistent_bytes, void *scratch,
                   size_t scratch_bytes, void *stream, chfsi_ctx **out) {
    if (!out) return fail(nullptr, CHFSI_E_ARG, "out is NULL");
    *out = nullptr;
    Mesh m{};
    std::string msg;
    int rc = build_mesh(mesh, proj, m, msg);
    if (rc) return fail(nullptr, rc, msg);
    int64_t max_nvec, fblock;
    chfsi_prec fprec;
    if ((rc = plan_opts_check(po, max_nvec, fblock, fprec))) return rc;
    if (!V || !B) return fail(nullptr, CHFSI_E_ARG, "V and B must be device pointers");
    Layout L = build_layout(m, max_nvec, fblock, fprec);
    if (!persistent || persistent_bytes < L.persistent_bytes)
        return fail(nullptr, CHFSI_E_WORKSPACE, "persistent buffer too small: need " + std::to_string(L.persistent_bytes));
    if (!scratch || scratch_bytes < L.scratch_bytes)
        return fail(nullptr, CHFSI_E_WORKSPACE, "scratch buffer too small: need " + std::to_string(L.scratch_bytes));
    if ((reinterpret_cast<uintptr_t>(persistent) & 255) || (reinterpret_cast<uintptr_t>(scratch) & 255))
        return fail(nullptr, CHFSI_E_ARG, "buffers must be 256-byte aligned");

    chfsi_ctx *c = new (std::nothrow) chfsi_ctx();
    if (!c) return fail(nullptr, CHFSI_E_ARG, "out of host memory");
    c->m = m;
    c->L = L;
    c->max_nvec = max_nvec;
    c->filter_block = fblock;
    c->filter_prec = fprec;
    c->pers = static_cast<char *>(persistent);
    c->scr = static_cast<char *>(scratch);
    c->blas = nullptr;
    hipStream_t s = S(stream);
    {
        // the fields must be finite (checked on the device before anything is built)
        int *flag = c->S<int>(L.flag);
        hipError_t fe = hipMemsetAsync(flag, 0, sizeof(int), s);
        if (fe == hipSuccess) fe = launch_check_finite(V, m.ncells * m.nq, flag, s);
        if (fe == hipSuccess) fe = launch_check_finite(B, m.ncells * m.nq * 3, flag, s);
        int f = 0;
        if (fe == hipSuccess) fe = hipMemcpyAsync(&f, flag, sizeof(int), hipMemcpyDeviceToHost, s);
        if (fe == hipSuccess) fe = hipStreamSynchronize(s);
        if (fe != hipSuccess || f) {
            const std::string em = fe != hipSuccess ? std::string("setup failed: ") + hipGetErrorString(fe)
                                                    : std::string("V or B holds NaN or Inf");
            delete c;
            return fail(nullptr, fe != hipSuccess ? CHFSI_E_DEVICE : CHFSI_E_NONFINITE, em);
        }
    }
    HostTables t;
    build_tables(m, t);
    auto up = [&](size_t off, const void *src, size_t bytes) {
        return hipMemcpyAsync(c->pers + off, src, bytes, hipMemcpyHostToDevice, s);
    };
    const size_t NP2 = (size_t)m.npad * m.npad;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up(L.K64, t.K.data(), NP2 * 8);
    if (e == hipSuccess) e = up(L.Phi64, t.Phi.data(), NP2 * 8);
    if (e == hipSuccess) e = up(L.PhiT64, t.PhiT.data(), NP2 * 8);
    if (e == hipSuccess) e = up(L.M64, t.Mref.data(), NP2 * 8);
    if (e == hipSuccess) e = up(L.Wq, t.wq.data(), m.npad * 8);
    if (e == hipSuccess) e = up(L.D64, t.D.data(), m.M * 8);
    for (size_t i = 0; i < t.poi1d.size() && i < (size_t)kPoiTab; ++i) c->poi_tab[i] = t.poi1d[i];
    if (e == hipSuccess) e = up(L.KdInv64, t.Kdinv.data(), m.M * 8);
    // colour classes: cells of equal coordinate parity share no node
    std::vector<int> cells;
    cells.reserve(m.ncells);
    for (int col = 0; col < 8; ++col) {
        c->colour_ptr[col] = (int64_t)cells.size();
        for (int64_t ez = (col >> 2) & 1; ez < m.ncell[2]; ez += 2)
            for (int64_t ey = (col >> 1) & 1; ey < m.ncell[1]; ey += 2)
                for (int64_t ex = col & 1; ex < m.ncell[0]; ex += 2)
                    cells.push_back((int)(ex + m.ncell[0] * (ey + m.ncell[1] * ez)));
    }
    c->colour_ptr[8] = (int64_t)cells.size();
    std::vector<int> cpp(m.ncells + 1, 0), cps(std::max<int64_t>(m.npairs, 1), 0),
        patom(std::max<int64_t>(m.npairs, 1), 0), app(m.natoms + 1, 0), nlc;
    if (m.npairs > 0) {
        for (int64_t a = 0; a < m.natoms; ++a) {
            app[a + 1] = (int)proj->pair_ptr[a + 1];
            for (int64_t pp = proj->pair_ptr[a]; pp < proj->pair_ptr[a + 1]; ++pp) {
                patom[pp] = (int)a;
                cpp[proj->pair_cell[pp] + 1]++;
            }
        }
        for (int64_t e2 = 0; e2 < m.ncells; ++e2) cpp[e2 + 1] += cpp[e2];
        std::vector<int> fill(cpp.begin(), cpp.end() - 1);
        for (int64_t pp = 0; pp < m.npairs; ++pp) cps[fill[proj->pair_cell[pp]]++] = (int)pp;
        for (int64_t e2 = 0; e2 < m.ncells; ++e2)
            if (cpp[e2 + 1] > cpp[e2]) nlc.push_back((int)e2);
    }
    if (nlc.empty()) nlc.push_back(0);
    if (e == hipSuccess) e = up(L.colour_cells, cells.data(), cells.size() * 4);
    if (e == hipSuccess) e = up(L.cell_pair_ptr, cpp.data(), cpp.size() * 4);
    if (e == hipSuccess) e = up(L.cell_pairs, cps.data(), cps.size() * 4);
    if (e == hipSuccess) e = up(L.pair_atom, patom.data(), patom.size() * 4);
    if (e == hipSuccess) e = up(L.atom_pair_ptr, app.data(), app.size() * 4);
    if (e == hipSuccess) e = up(L.nl_cells, nlc.data(), nlc.size() * 4);
    if (e == hipSuccess && m.natoms > 0)
        e = up(L.delta64, proj->delta, (size_t)m.natoms * m.nbeta * m.nbeta * 16);
    if (e == hipSuccess && m.npairs > 0)
        e = hipMemcpyAsync(c->scr + L.Z, proj->phi, (size_t)m.npairs * m.nq * 2 * m.nbeta * 16,
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_setup_casts(c, s);
    if (e == hipSuccess) e = launch_setup_fields(c, V, B, s);
    if (e == hipSuccess) e = launch_setup_projectors(c, reinterpret_cast<const cd *>(c->scr + L.Z), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        std::string em = std::string("setup failed: ") + hipGetErrorString(e);
        delete c;
        return fail(nullptr, CHFSI_E_DEVICE, em);
    }
    {
        // the static scratch of chfsi_residual_noalloc on this device
        hipError_t ge = hipSuccess;
        if (!noalloc_scratch(&ge)) {
            delete c;
            return fail(nullptr, CHFSI_E_DEVICE, std::string("static scratch address: ") + hipGetErrorString(ge));
        }
    }
    if (rocblas_create_handle(&c->blas) != rocblas_status_success) {
        delete c;
        return fail(nullptr, CHFSI_E_DEVICE, "rocblas_create_handle failed");
    }
    *out = c;
    return CHFSI_OK;
}

int chfsi_set_fields(chfsi_ctx *c, const double *V, const double *B, void *stream) {
    if (!c) return fail(nullptr, CHFSI_E_ARG, "ctx is NULL");
    if (!V || !B) return fail(c, CHFSI_E_ARG, "V and B must be device pointers");
    hipStream_t s = S(stream);
    int *flag = c->S<int>(c->L.flag);
    HIPCHK(c, hipMemsetAsync(flag, 0, sizeof(int), s));
    HIPCHK(c, launch_check_finite(V, c->m.ncells * c->m.nq, flag, s));
    HIPCHK(c, launch_check_finite(B, c->m.ncells * c->m.nq * 3, flag, s));
    int f = 0;
    int rc = read_flag(c, s, &f);
    if (rc) return rc;
    if (f) return fail(c, CHFSI_E_NONFINITE, "V or B holds NaN or Inf");
    HIPCHK(c, launch_setup_fields(c, V, B, s));
    return CHFSI_OK;
}

int chfsi_apply_H(chfsi_ctx *c, chfsi_prec prec, const void *X, void *Y, int64_t nvec, int64_t ld, void *stream) {
    if (!c) return fail(nullptr, CHFSI_E_ARG, "ctx is NULL");
    if (prec < CHFSI_FP64 || prec > CHFSI_BF16) return fail(c, CHFSI_E_ARG, "unknown precision");
    int rc;
    if ((rc = check_block(c, X, nvec, ld, "X")) || (rc = check_block(c, Y, nvec, ld, "Y"))) return rc;
    if (X == Y) return fail(c, CHFSI_E_ARG, "X and Y must not overlap");
    return apply_H_impl(c, prec, X, Y, nvec, ld, S(stream));
}

int chfsi_apply_M(chfsi_ctx *c, const void *X, void *Y, int64_t nvec, int64_t ld, void *stream) {
    if (!c) return fail(nullptr, CHFSI_E_ARG, "ctx is NULL");
    int rc;
    if ((rc = check_block(c, X, nvec, ld, "X")) || (rc = check_block(c, Y, nvec, ld, "Y"))) return rc;
    if (X == Y) return fail(c, CHFSI_E_ARG, "X and Y must not overlap");
    HIPCHK(c, launch_cell_op(c, CHFSI_FP64, MODE_MASS, 0, 1.0, X, Y, nvec, ld, S(stream)));
    return CHFSI_OK;
}

int chfsi_apply_H_adjoint(chfsi_ctx *c, chfsi_prec prec, const void *X, const void *G, int64_t nvec, int64_t ld,
                          void *dX, double *dV, double *dB, void *stream) {
    if (!c) return fail(nullptr, CHFSI_E_ARG, "ctx is NULL");
    if (prec < CHFSI_FP64 || prec > CHFSI_BF16) return fail(c, CHFSI_E_ARG, "unknown precision");
    int rc;
    if ((rc = check_block(c, X, nvec, ld, "X")) || (rc = check_block(c, G, nvec, ld, "G"))) return rc;
    if (!dV || !dB) return fail(c, CHFSI_E_ARG, "dV and dB must be device pointers");
    hipStream_t s = S(stream);
    if (dX) {
        if (dX == G || dX == X) return fail(c, CHFSI_E_ARG, "dX must not overlap X or G");
        if ((rc = apply_H_impl(c, prec, G, dX, nvec, ld, s))) return rc;
    }
    HIPCHK(c, launch_adjoint_fields(c, prec, X, G, nvec, ld, dV, dB, s));
    return CHFSI_OK;
}

int chfsi_estimate_bounds(chfsi_ctx *c, int steps, const void *v0, double *lambda_max, void *stream) {
    if (!c) return fail(nullptr, CHFSI_E_ARG, "ctx is NULL");
    if (!v0 || !lambda_max) return fail(c, CHFSI_E_ARG, "v0 and lambda_max must be non-NULL");
    if (steps < 1 || steps > 1000) return fail(c, CHFSI_E_ARG, "lanczos_steps must be in 1..1000");
    hipStream_t s = S(stream);
    const int64_t N = 2 * c->m.M;
    cd *v = c->S<cd>(c->L.Z), *vp = v + N, *w = vp + N, *t = w + N;
    double *red = c->S<double>(c->L.red), *dsc = red + 4000;
    double h = 0;
    auto dot = [&](const cd *a, const cd *b, double &res) -> int {
        HIPCHK(c, launch_dot_real(N, a, b, red, dsc, s));
        HIPCHK(c, hipMemcpyAsync(&res, dsc, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        return CHFSI_OK;
    };
    HIPCHK(c, hipMemcpyAsync(v, v0, N * sizeof(cd), hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemsetAsync(vp, 0, N * sizeof(cd), s));
    int rc = dot(v, v, h);
    if (rc) return rc;
    if (!(h > 0) || !std::isfinite(h)) return fail(c, CHFSI_E_ARG, "v0 must be a nonzero finite vector");
    HIPCHK(c, launch_axpby(N, 0.0, nullptr, 1.0 / std::sqrt(h), v, s));
    std::vector<double> al, be(1, 0.0);
    // D^{-1/2} as a length-M table in the reduction area of the Lanczos vectors
    double *dh = reinterpret_cast<double *>(t + N);
    std::vector<double> Dh(c->m.M);
    HIPCHK(c, hipMemcpyAsync(Dh.data(), c->P<double>(c->L.Dinv64), c->m.M * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    for (auto &x : Dh) x = std::sqrt(x);
    HIPCHK(c, hipMemcpyAsync(dh, Dh.data(), c->m.M * 8, hipMemcpyHostToDevice, s));
    for (int j = 0; j < steps; ++j) {
        HIPCHK(c, hipMemcpyAsync(t, v, N * sizeof(cd), hipMemcpyDeviceToDevice, s));
        HIPCHK(c, launch_scale_rows(N, 1, 1, dh, t, s));
        if ((rc = apply_H_impl(c, CHFSI_FP64, t, w, 1, 1, s))) return rc;
        HIPCHK(c, launch_scale_rows(N, 1, 1, dh, w, s));
        HIPCHK(c, launch_axpby(N, -be[j], vp, 1.0, w, s));
        double a;
        if ((rc = dot(v, w, a))) return rc;
        al.push_back(a);
        HIPCHK(c, launch_axpby(N, -a, v, 1.0, w, s));
        double b2;
        if ((rc = dot(w, w, b2))) return rc;
        double b = std::sqrt(std::max(b2, 0.0));
        be.push_back(b);
        if (b == 0 || !std::isfinite(b)) break;
        HIPCHK(c, hipMemcpyAsync(vp, v, N * sizeof(cd), hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipMemcpyAsync(v, w, N * sizeof(cd), hipMemcpyDeviceToDevice, s));
        HIPCHK(c, launch_axpby(N, 0.0, nullptr, 1.0 / b, v, s));
    }
    if (!std::isfinite(be.back())) return fail(c, CHFSI_E_NONFINITE, "Lanczos produced a non-finite value");
    std::vector<double> bt(be.begin(), be.begin() + al.size());
    *lambda_max = tridiag_max(al, bt) + std::fabs(be[al.size()]);
    return CHFSI_OK;
}

int chfsi_filter(chfsi_ctx *c, chfsi_prec prec, int degree, const double bounds[3], const void *X,
                 const double *ritz, const void *R, void *Y, int64_t nvec, int64_t ld, void *stream) {
    if (!c) return fail(nullptr, CHFSI_E_ARG, "ctx is NULL");
    if (prec < CHFSI_FP64 || prec > CHFSI_BF16) return fail(c, CHFSI_E_ARG, "unknown precision");
    if (degree < 1 || degree > kMaxDegree) return fail(c, CHFSI_E_ARG, "degree must be in 1..256");
    if (!bounds || !ritz) return fail(c, CHFSI_E_ARG, "bounds and ritz must be non-NULL");
    int rc;
    if ((rc = check_block(c, X, nvec, ld, "X")) || (rc = check_block(c, R, nvec, ld, "R")) ||
        (rc = check_block(c, Y, nvec, ld, "Y")))
        return rc;
    if (!(bounds[0] < bounds[1] && bounds[1] < bounds[2]) || !std::isfinite(bounds[0]) || !std::isfinite(bounds[2]))
        return fail(c, CHFSI_E_BOUNDS, "bounds must satisfy lmin < lT < lmax");
    if (R == Y) return fail(c, CHFSI_E_ARG, "Y must not overlap R");
    return filter_impl(c, prec, degree, bounds, (const cd *)X, ritz, (const cd *)R, (cd *)Y, nvec, ld, S(stream));
}

int chfsi_orthonormalize(chfsi_ctx *c, void *Y, void *HY, void *MY, int64_t nvec, int64_t ld, void *stream) {
    if (!c) return fail(nullptr, CHFSI_E_ARG, "ctx is NULL");
    int rc;
    if ((rc = check_block(c, Y, nvec, ld, "Y")) || (rc = check_block(c, MY, nvec, ld, "MY"))) return rc;
    return orthonormalize_impl(c, (cd *)Y, (cd *)HY, (cd *)MY, nvec, ld, S(stream));
}

int chfsi_rayleigh_ritz(chfsi_ctx *c, void *Y, void *HY, void *MY, int64_t nvec, int64_t ld, double *ritz,
                        void *R, double *resnorm, void *stream) {
    if (!c) return fail(nullptr, CHFSI_E_ARG, "ctx is NULL");
    int rc;
    if ((rc = check_block(c, Y, nvec, ld, "Y")) || (rc = check_block(c, HY, nvec, ld, "HY")) ||
        (rc = check_block(c, MY, nvec, ld, "MY")))
        return rc;
    if (!ritz) return fail(c, CHFSI_E_ARG, "ritz is NULL");
    return rr_impl(c, (cd *)Y, (cd *)HY, (cd *)MY, nvec, ld, ritz, (cd *)R, resnorm, S(stream));
}

int chfsi_rayleigh_ritz_general(chfsi_ctx *c, void *Y, void *HY, void *MY, int64_t nvec, int64_t ld, double *ritz,
                                void *R, double *resnorm, void *stream) {
    if (!c) return fail(nullptr, CHFSI_E_ARG, "ctx is NULL");
    int rc;
    if ((rc = check_block(c, Y, nvec, ld, "Y")) || (rc = check_block(c, HY, nvec, ld, "HY")) ||
        (rc = check_block(c, MY, nvec, ld, "MY")))
        return rc;
    if (!ritz) return fail(c, CHFSI_E_ARG, "ritz is NULL");
    return rr_general_impl(c, (cd *)Y, (cd *)HY, (cd *)MY, nvec, ld, ritz, (cd *)R, resnorm, S(stream));
}

int chfsi_residual(chfsi_ctx *c, const void *HX, const void *MX, const double *ritz, void *R, double *resnorm,
                   int64_t nvec, int64_t ld, void *stream) {
    if (!c) return fail(nullptr, CHFSI_E_ARG, "ctx is NULL");
    int rc;
    if ((rc = check_block(c, HX, nvec, ld, "HX")) || (rc = check_block(c, MX, nvec, ld, "MX"))) return rc;
    if (!ritz) return fail(c, CHFSI_E_ARG, "ritz is NULL");
    HIPCHK(c, launch_residual(2 * c->m.M, nvec, ld, (const cd *)HX, (const cd *)MX, ritz, (cd *)R,
                              c->S<double>(c->L.red), resnorm, S(stream)));
    return CHFSI_OK;
}

int chfsi_residual_noalloc(chfsi_ctx *c, const void *HX, const void *MX, const double *ritz, void *R,
                           double *resnorm, int64_t nvec, int64_t ld, void *stream) {
    if (!c) return fail(nullptr, CHFSI_E_ARG, "ctx is NULL");
    int rc;
    if ((rc = check_block(c, HX, nvec, ld, "HX")) || (rc = check_block(c, MX, nvec, ld, "MX"))) return rc;
    if (!ritz) return fail(c, CHFSI_E_ARG, "ritz is NULL");
    if (nvec > kNoAllocMaxCols)
        return fail(c, CHFSI_E_WORKSPACE, "chfsi_residual_noalloc: nvec " + std::to_string(nvec) +
                                              " exceeds the static scratch (at most " +
                                              std::to_string(kNoAllocMaxCols) + " columns)");
    hipError_t ge = hipSuccess;
    double *red = noalloc_scratch(&ge);
    if (!red) return fail(c, CHFSI_E_DEVICE, std::string("static scratch address: ") + hipGetErrorString(ge));
    // every partial [kRowBlocks][nvec] is written by the residual kernel
    // before the norms read it, so nothing needs clearing
    HIPCHK(c, launch_residual(2 * c->m.M, nvec, ld, (const cd *)HX, (const cd *)MX, ritz, (cd *)R, red, resnorm,
                              S(stream)));
    return CHFSI_OK;
}

int chfsi_solve_workspace(chfsi_ctx *c, int64_t nsub, int64_t ld, size_t *bytes) {
    if (!c || !bytes) return fail(c, CHFSI_E_ARG, "ctx and bytes must be non-NULL");
    if (nsub < 1 || nsub > c->max_nvec || ld < nsub) return fail(c, CHFSI_E_ARG, "bad nsub or ld");
    const size_t blk = align256((size_t)(2 * c->m.M) * ld * sizeof(cd));
    *bytes = 3 * blk + align256((size_t)nsub * 8 * 2);
    return CHFSI_OK;
}

int chfsi_solve(chfsi_ctx *c, int64_t n_wanted, const chfsi_solve_opts *o, void *Xv, int64_t nsub, int64_t ld,
                const void *v0, double *eigvals, double *hist_res, chfsi_report *rep, void *workspace,
                size_t workspace_bytes, void *stream) {
    if (!c) return fail(nullptr, CHFSI_E_ARG, "ctx is NULL");
    if (!o) return fail(c, CHFSI_E_ARG, "opts is NULL");
    int rc;
    if ((rc = check_block(c, Xv, nsub, ld, "X"))) return rc;
    if (n_wanted < 1 || n_wanted > nsub) return fail(c, CHFSI_E_ARG, "n_wanted must be in 1..nsub");
    if (nsub < 2) return fail(c, CHFSI_E_ARG, "nsub must be >= 2");
    if (o->degree < 1 || o->degree > kMaxDegree || o->max_iter < 1) return fail(c, CHFSI_E_ARG, "bad degree or max_iter");
    if (o->prec < CHFSI_FP64 || o->prec > CHFSI_BF16) return fail(c, CHFSI_E_ARG, "unknown precision");
    if (o->rr_mode < 0 || o->rr_mode > 2) return fail(c, CHFSI_E_ARG, "rr_mode must be 0, 1 or 2");
    if (o->block < 0) return fail(c, CHFSI_E_ARG, "block must be >= 0");
    const int64_t nb = o->block > 0 ? std::min<int64_t>(o->block, nsub) : std::min<int64_t>(nsub, c->filter_block);
    if (nb > c->filter_block)
        return fail(c, CHFSI_E_ARG, "block exceeds the filter_block the scratch was planned for");
    if (2 * zblock_bytes(c->m, nb, o->prec != CHFSI_FP64) > c->L.zarea)
        return fail(c, CHFSI_E_WORKSPACE, "the scratch cannot hold two recurrence blocks of " + std::to_string(nb) +
                                              " columns in this precision (plan a wider filter precision)");
    if (!eigvals) return fail(c, CHFSI_E_ARG, "eigvals is NULL");
    size_t need = 0;
    if ((rc = chfsi_solve_workspace(c, nsub, ld, &need))) return rc;
    if (!workspace || workspace_bytes < need) return fail(c, CHFSI_E_WORKSPACE, "workspace too small: need " + std::to_string(need));
    hipStream_t s = S(stream);
    const size_t blk = align256((size_t)(2 * c->m.M) * ld * sizeof(cd));
    char *ws = static_cast<char *>(workspace);
    cd *X = (cd *)Xv, *HX = (cd *)ws, *MX = (cd *)(ws + blk), *R = (cd *)(ws + 2 * blk);
    double *ritz = (double *)(ws + 3 * blk), *res = ritz + nsub;
    double lmax = o->lambda_max;
    if (o->lanczos_steps > 0 && !o->resume) {
        if (!v0) return fail(c, CHFSI_E_ARG, "v0 is NULL but lanczos_steps > 0");
        if ((rc = chfsi_estimate_bounds(c, o->lanczos_steps, v0, &lmax, stream))) return rc;
    }
    if (!(std::isfinite(lmax))) return fail(c, CHFSI_E_BOUNDS, "lambda_max is not finite");
    if (!o->resume) {
        // a non-finite start block would surface later as a Cholesky breakdown
        int *flag = c->S<int>(c->L.flag);
        HIPCHK(c, hipMemsetAsync(flag, 0, sizeof(int), s));
        HIPCHK(c, launch_check_finite_block(X, 2 * c->m.M, nsub, ld, flag, s));
        int f = 0;
        if ((rc = read_flag(c, s, &f))) return rc;
        if (f) return fail(c, CHFSI_E_NONFINITE, "the start block X holds NaN or Inf");
    }
    // timing events, destroyed on every return path
    struct Events {
        hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
        ~Events() {
            for (auto &e : ev)
                if (e) hipEventDestroy(e);
        }
    } evs;
    hipEvent_t *ev = evs.ev;
    for (int i = 0; i < 4; ++i) HIPCHK(c, hipEventCreate(&ev[i]));
    // with opts.profile: a (start, end) pair per filter step and column block
    StepEvents steps;
    if (o->profile) {
        steps.ev.resize((size_t)2 * (o->degree - 1) * (size_t)((nsub + nb - 1) / nb), nullptr);
        for (auto &e : steps.ev) HIPCHK(c, hipEventCreate(&e));
    }
    int ncolour = 0;
    for (int col = 0; col < 8; ++col) ncolour += c->colour_ptr[col + 1] > c->colour_ptr[col];
    double t_cell = 0;
    int64_t n_cell = 0;
    HIPCHK(c, hipEventRecord(ev[0], s));
    if (!o->resume) {
        if ((rc = apply_H_impl(c, CHFSI_FP64, X, HX, nsub, ld, s))) return rc;
        HIPCHK(c, launch_cell_op(c, CHFSI_FP64, MODE_MASS, 0, 1.0, X, MX, nsub, ld, s));
        if ((rc = orthonormalize_impl(c, X, HX, MX, nsub, ld, s))) return rc;
        if ((rc = rr_impl(c, X, HX, MX, nsub, ld, ritz, R, res, s))) return rc;
    }
    std::vector<double> hr(nsub), hritz(nsub), titer;
    double t_filter = 0, t_rr = 0, first_res = -1;
    int it = 0, converged = 0;
    double maxres = 0, bounds[3] = {0, 0, lmax};
    int status = CHFSI_OK;
    for (;; ++it) {
        HIPCHK(c, hipMemcpyAsync(hr.data(), res, nsub * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(hritz.data(), ritz, nsub * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        maxres = 0;
        bool finite = true;
        for (int64_t j = 0; j < nsub; ++j) finite = finite && std::isfinite(hr[j]) && std::isfinite(hritz[j]);
        for (int64_t j = 0; j < n_wanted; ++j) maxres = std::max(maxres, hr[j]);
        if (hist_res) hist_res[it] = maxres;
        if (!finite) { status = fail(c, CHFSI_E_NONFINITE, "non-finite residual or Ritz value"); break; }
        if (first_res < 0) first_res = maxres;
        if (maxres > 1e6 * std::max(first_res, 1e-300) && maxres > 1.0) {
            status = fail(c, CHFSI_E_DIVERGED, "residual grew by more than 1e6 (lambda_max too small?)");
            break;
        }
        if (!o->fixed_iters && maxres < o->tol) { converged = 1; break; }
        if (it >= o->max_iter) break;
        bounds[0] = hritz[0];
        bounds[1] = hritz[nsub - 1];
        if (!(bounds[0] < bounds[1] && bounds[1] < bounds[2])) {
            status = fail(c, CHFSI_E_BOUNDS, "Ritz values exceed lambda_max: bounds not ordered");
            break;
        }
        HIPCHK(c, hipEventRecord(ev[1], s));
        // the filter is column-wise (Lambda_k is diagonal): blocks of nb columns
        rc = CHFSI_OK;
        for (int64_t b0 = 0; b0 < nsub && !rc; b0 += nb)
            rc = filter_impl(c, o->prec, o->degree, bounds, X + b0, ritz + b0, R + b0, X + b0,
                             std::min(nb, nsub - b0), ld, s, o->profile ? &steps : nullptr);
        if (rc) { status = rc; break; }
        HIPCHK(c, hipEventRecord(ev[2], s));
        if ((rc = apply_H_impl(c, CHFSI_FP64, X, HX, nsub, ld, s))) { status = rc; break; }
        HIPCHK(c, launch_cell_op(c, CHFSI_FP64, MODE_MASS, 0, 1.0, X, MX, nsub, ld, s));
        rc = CHFSI_E_NOT_SPD;
        // the rotated HX and MX are not needed after the residual: it is formed from HY and MY directly
        if (o->rr_mode >= 1) rc = rr_general_impl(c, X, HX, MX, nsub, ld, ritz, R, res, s, false, o->rr_mode == 2);
        if (rc == CHFSI_E_NOT_SPD) {
            if ((rc = orthonormalize_impl(c, X, HX, MX, nsub, ld, s))) { status = rc; break; }
            rc = rr_impl(c, X, HX, MX, nsub, ld, ritz, R, res, s);
        }
        if (rc) { status = rc; break; }
        HIPCHK(c, hipEventRecord(ev[3], s));
        HIPCHK(c, hipEventSynchronize(ev[3]));
        float ms1 = 0, ms2 = 0;
        hipEventElapsedTime(&ms1, ev[1], ev[2]);
        hipEventElapsedTime(&ms2, ev[2], ev[3]);
        for (size_t i = 0; i + 1 < steps.used; i += 2) {
            float m = 0;
            HIPCHK(c, hipEventElapsedTime(&m, steps.ev[i], steps.ev[i + 1]));
            t_cell += m * 1e-3;
            n_cell += ncolour;
        }
        steps.used = 0;
        t_filter += ms1 * 1e-3;
        t_rr += ms2 * 1e-3;
        titer.push_back((ms1 + ms2) * 1e-3);
    }
    HIPCHK(c, hipEventRecord(ev[3], s));
    HIPCHK(c, hipEventSynchronize(ev[3]));
    float mst = 0;
    hipEventElapsedTime(&mst, ev[0], ev[3]);
    HIPCHK(c, hipMemcpy(eigvals, ritz, n_wanted * 8, hipMemcpyDeviceToHost));
    if (rep) {
        rep->iters = it;
        rep->converged = converged;
        rep->max_res = maxres;
        rep->lambda_bounds[0] = bounds[0];
        rep->lambda_bounds[1] = bounds[1];
        rep->lambda_bounds[2] = lmax;
        rep->t_filter = t_filter;
        rep->t_rr = t_rr;
        rep->t_total = mst * 1e-3;
        rep->t_filter_cell = t_cell;
        rep->filter_cell_launches = n_cell;
        std::vector<double> tt(titer.size() > 1 ? titer.begin() + 1 : titer.begin(), titer.end());
        std::sort(tt.begin(), tt.end());
        rep->t_iter_median = tt.empty() ? 0 : tt[tt.size() / 2];
    }
    if (status != CHFSI_OK) return status;
    return converged || o->fixed_iters ? CHFSI_OK : CHFSI_NOT_CONVERGED;
}

int chfsi_profile_apply_H(chfsi_ctx *c, chfsi_prec prec, const void *X, void *Y, int64_t nvec, int64_t ld,
                          double ms[3], int *launches, void *stream) {
    if (!c) return fail(nullptr, CHFSI_E_ARG, "ctx is NULL");
    if (prec < CHFSI_FP64 || prec > CHFSI_BF16) return fail(c, CHFSI_E_ARG, "unknown precision");
    if (!ms) return fail(c, CHFSI_E_ARG, "ms is NULL");
    int rc;
    if ((rc = check_block(c, X, nvec, ld, "X")) || (rc = check_block(c, Y, nvec, ld, "Y"))) return rc;
    if (X == Y) return fail(c, CHFSI_E_ARG, "X and Y must not overlap");
    hipStream_t s = S(stream);
    hipEvent_t ev[3];
    for (auto &e : ev) HIPCHK(c, hipEventCreate(&e));
    const int nl = c->m.npairs > 0 ? FLAG_NLOC : 0;
    hipError_t err = hipEventRecord(ev[0], s);
    if (err == hipSuccess && nl) err = launch_nonlocal_coeffs(c, prec, 0, X, nvec, ld, s);
    if (err == hipSuccess) err = hipEventRecord(ev[1], s);
    if (err == hipSuccess) err = launch_cell_op(c, prec, MODE_HAM, nl, 1.0, X, Y, nvec, ld, s);
    if (err == hipSuccess) err = hipEventRecord(ev[2], s);
    if (err == hipSuccess) err = hipEventSynchronize(ev[2]);
    float a = 0, b = 0;
    if (err == hipSuccess) err = hipEventElapsedTime(&a, ev[0], ev[1]);
    if (err == hipSuccess) err = hipEventElapsedTime(&b, ev[1], ev[2]);
    for (auto &e : ev) hipEventDestroy(e);
    if (err != hipSuccess) return fail(c, CHFSI_E_DEVICE, std::string("profile failed: ") + hipGetErrorString(err));
    ms[0] = b;
    ms[1] = a;
    ms[2] = a + b;
    if (launches) {
        int n = 0;
        for (int col = 0; col < 8; ++col) n += c->colour_ptr[col + 1] > c->colour_ptr[col];
        *launches = n;
    }
    return CHFSI_OK;
}

int chfsi_info(const chfsi_ctx *c, int64_t *nnodes, int64_t *ncells, int *n, int *nq) {
    if (!c) return fail(nullptr, CHFSI_E_ARG, "ctx is NULL");
    if (nnodes) *nnodes = c->m.M;
    if (ncells) *ncells = c->m.ncells;
    if (n) *n = c->m.n;
    if (nq) *nq = c->m.nq;
    return CHFSI_OK;
}

int chfsi_mass_diag(chfsi_ctx *c, double *D, void *stream) {
    if (!c) return fail(nullptr, CHFSI_E_ARG, "ctx is NULL");
    if (!D) return fail(c, CHFSI_E_ARG, "D is NULL");
    HIPCHK(c, hipMemcpyAsync(D, c->P<double>(c->L.D64), c->m.M * 8, hipMemcpyDeviceToDevice, S(stream)));
    return CHFSI_OK;
}

int chfsi_bfp_bytes(int nbits, int64_t n, int64_t *bytes) {
    if (nbits != 16 && nbits != 12 && nbits != 10) return fail(nullptr, CHFSI_E_ARG, "nbits must be 16, 12 or 10");
    if (n < 0 || n % 4) return fail(nullptr, CHFSI_E_ARG, "n must be a non-negative multiple of 4");
    if (!bytes) return fail(nullptr, CHFSI_E_ARG, "bytes is NULL");
    *bytes = n / 4 * (nbits / 2);
    return CHFSI_OK;
}

static int bfp_call(bool enc, int nbits, const void *src, int64_t n, void *dst, void *stream) {
    int64_t nbytes = 0;
    int rc = chfsi_bfp_bytes(nbits, n, &nbytes);
    if (rc) return rc;
    if (n == 0) return CHFSI_OK;
    if (!src || !dst) return fail(nullptr, CHFSI_E_ARG, "NULL buffer");
    const void *f = enc ? src : (const void *)dst;
    const void *b = enc ? (const void *)dst : src;
    const uintptr_t balign = nbits == 16 ? 8 : (nbits == 12 ? 2 : 1);
    if ((reinterpret_cast<uintptr_t>(f) & 15) || (reinterpret_cast<uintptr_t>(b) & (balign - 1)))
        return fail(nullptr, CHFSI_E_ARG, "float buffer must be 16-byte aligned, stream aligned to its store width");
    hipError_t e = launch_bfp(enc, nbits, src, n, dst, S(stream));
    if (e != hipSuccess) return fail(nullptr, CHFSI_E_DEVICE, std::string("bfp kernel: ") + hipGetErrorString(e));
    return CHFSI_OK;
}

int chfsi_bfp_encode(int nbits, const float *x, int64_t n, void *out, void *stream) {
    return bfp_call(true, nbits, x, n, out, stream);
}

int chfsi_bfp_decode(int nbits, const void *in, int64_t n, float *x, void *stream) {
    return bfp_call(false, nbits, in, n, x, stream);
}

// ------------------------------------------------------------------ Poisson

static int poisson_check(chfsi_ctx *c) {
    if (!c) return fail(nullptr, CHFSI_E_ARG, "ctx is NULL");
    if (!kx_supported(c->m.n1, c->m.nq1))
        return fail(c, CHFSI_E_ARG, "the Poisson operator needs nq1d = degree + 1 or degree + 2");
    return CHFSI_OK;
}

static bool overlap(const double *a, const double *b, int64_t n) { return a < b + n && b < a + n; }

// scratch vectors of length M for the Poisson solver (slot k) and the
// scalar area: partial sums, then the PCG scalars
static double *poi_vec(chfsi_ctx *c, int k) { return c->S<double>(c->L.Z) + (size_t)k * c->m.M; }
static double *poi_part(chfsi_ctx *c) { return c->S<double>(c->L.red); }
static double *poi_sc(chfsi_ctx *c) { return c->S<double>(c->L.red) + kDotPartials; }

static int read_sc(chfsi_ctx *c, hipStream_t s, double *h) {
    HIPCHK(c, hipMemcpyAsync(h, poi_sc(c), SC_NSC * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return CHFSI_OK;
}

// z = chi(D^-1 K) D^-1 r by m steps of the Chebyshev iteration for
// D^-1 K z = D^-1 r from z = 0 on [a, b] (Saad, Iterative Methods for
// Sparse Linear Systems, Chebyshev acceleration): theta = (a+b)/2,
// delta = (b-a)/2, sigma = theta/delta, rho_0 = 1/sigma, d_0 = D^-1 r/theta;
// rho_k = 1/(2 sigma - rho_{k-1}), d_k = rho_k rho_{k-1} d_{k-1}
// + (2 rho_k/delta) D^-1 (r - K z_k), z_{k+1} = z_k + d_k.  d, Kz: scratch.
// With dot_op >= 0 the last step also forms the PCG's (r.z, r.r) and
// updates the device scalars as launch_dot2 with that op would.
static int cheb_precond(chfsi_ctx *c, int m, double a, double b, const double *r, double *z, double *d, double *Kz,
                        hipStream_t s, int dot_op = -1) {
    const int64_t M = c->m.M;
    const double *dinv = c->P<double>(c->L.KdInv64);
    const double theta = 0.5 * (a + b), delta = 0.5 * (b - a), sigma = theta / delta;
    double rho = 1.0 / sigma;
    for (int k = 0; k < m; ++k) {
        double c1 = 0.0, c2 = 1.0 / theta;
        if (k > 0) {
            HIPCHK(c, launch_kx(c, z, Kz, s));
            const double rn = 1.0 / (2.0 * sigma - rho);
            c1 = rn * rho;
            c2 = 2.0 * rn / delta;
            rho = rn;
        }
        if (k == m - 1 && dot_op >= 0)
            HIPCHK(c, launch_cheb_last_dot(M, k == 0, c1, c2, dinv, r, Kz, d, z, poi_part(c), dot_op, poi_sc(c), s));
        else
            HIPCHK(c, launch_cheb_step(M, k == 0, c1, c2, dinv, r, Kz, d, z, s));
    }
    return CHFSI_OK;
}

// Upper bound of the spectrum of D^-1 K: k Lanczos steps on the symmetric
// D^-1/2 K D^-1/2 from the splitmix64 vector, theta_max + |beta_k|.
static int poisson_lanczos(chfsi_ctx *c, int steps, double *out, hipStream_t s) {
    const int64_t M = c->m.M;
    double *v = poi_vec(c, 0), *vp = poi_vec(c, 1), *w = poi_vec(c, 2), *t = poi_vec(c, 3), *dh = poi_vec(c, 4);
    double *part = poi_part(c), *sc = poi_sc(c);
    double h[SC_NSC];
    int rc;
    auto dot = [&](const double *x, const double *y, double &res) -> int {
        HIPCHK(c, launch_dot2(M, x, y, nullptr, nullptr, part, PCG_SUMS, sc, s));
        if ((rc = read_sc(c, s, h))) return rc;
        res = h[SC_SUM0];
        return CHFSI_OK;
    };
    HIPCHK(c, launch_sqrt(M, c->P<double>(c->L.KdInv64), dh, s));
    HIPCHK(c, launch_splitmix(M, 0, v, s));
    HIPCHK(c, hipMemsetAsync(vp, 0, M * sizeof(double), s));
    double nv;
    if ((rc = dot(v, v, nv))) return rc;
    HIPCHK(c, launch_axpby_real(M, 0.0, nullptr, 1.0 / std::sqrt(nv), v, nullptr, s));
    std::vector<double> al, be(1, 0.0);
    for (int j = 0; j < steps; ++j) {
        HIPCHK(c, launch_axpby_real(M, 1.0, v, 0.0, t, dh, s));     // t = D^-1/2 v
        HIPCHK(c, launch_kx(c, t, w, s));                      // w = K t
        HIPCHK(c, launch_axpby_real(M, 0.0, nullptr, 1.0, w, dh, s));  // w = D^-1/2 w
        HIPCHK(c, launch_axpby_real(M, -be[j], vp, 1.0, w, nullptr, s));
        double a;
        if ((rc = dot(v, w, a))) return rc;
        al.push_back(a);
        HIPCHK(c, launch_axpby_real(M, -a, v, 1.0, w, nullptr, s));
        double b2;
        if ((rc = dot(w, w, b2))) return rc;
        const double b = std::sqrt(std::max(b2, 0.0));
        be.push_back(b);
        if (b == 0 || !std::isfinite(b)) break;
        HIPCHK(c, launch_axpby_real(M, 1.0, v, 0.0, vp, nullptr, s));
        HIPCHK(c, launch_axpby_real(M, 1.0 / b, w, 0.0, v, nullptr, s));
    }
    if (!std::isfinite(be.back())) return fail(c, CHFSI_E_NONFINITE, "Lanczos produced a non-finite value");
    std::vector<double> bt(be.begin(), be.begin() + al.size());
    *out = tridiag_max(al, bt) + std::fabs(be[al.size()]);
    return CHFSI_OK;
}

int chfsi_apply_K(chfsi_ctx *c, const double *x, double *y, void *stream) {
    int rc = poisson_check(c);
    if (rc) return rc;
    if (!x || !y) return fail(c, CHFSI_E_ARG, "x and y must be non-NULL");
    if (overlap(x, y, c->m.M)) return fail(c, CHFSI_E_ARG, "x and y must not overlap");
    HIPCHK(c, launch_kx(c, x, y, S(stream)));
    return CHFSI_OK;
}

int chfsi_poisson_precond(chfsi_ctx *c, int degree, double lmin, double lmax, const double *r, double *z,
                          void *stream) {
    int rc = poisson_check(c);
    if (rc) return rc;
    if (!r || !z) return fail(c, CHFSI_E_ARG, "r and z must be non-NULL");
    if (overlap(r, z, c->m.M)) return fail(c, CHFSI_E_ARG, "r and z must not overlap");
    if (degree < 1 || degree > 64) return fail(c, CHFSI_E_ARG, "degree must be in 1..64");
    if (!(lmin > 0 && lmin < lmax && std::isfinite(lmax))) return fail(c, CHFSI_E_ARG, "need 0 < lmin < lmax finite");
    return cheb_precond(c, degree, lmin, lmax, r, z, poi_vec(c, 0), poi_vec(c, 1), S(stream));
}

int chfsi_poisson_solve(chfsi_ctx *c, const chfsi_pcg_opts *o, const double *f, double *x, chfsi_pcg_report *rep,
                        void *stream) {
    int rc = poisson_check(c);
    if (rc) return rc;
    if (!o || !f || !x) return fail(c, CHFSI_E_ARG, "opts, f and x must be non-NULL");
    const int64_t M = c->m.M;
    if (overlap(f, x, M)) return fail(c, CHFSI_E_ARG, "f and x must not overlap");
    if (!(o->tol > 0) || !std::isfinite(o->tol)) return fail(c, CHFSI_E_ARG, "tol must be positive");
    if (o->max_iter < 0) return fail(c, CHFSI_E_ARG, "max_iter must be >= 0");
    if (o->cheb_degree < 1 || o->cheb_degree > 64) return fail(c, CHFSI_E_ARG, "cheb_degree must be in 1..64");
    if (!(o->lambda_max >= 0) || !std::isfinite(o->lambda_max)) return fail(c, CHFSI_E_ARG, "lambda_max must be >= 0");
    if (o->lambda_max == 0 && (o->lanczos_steps < 1 || o->lanczos_steps > 1000))
        return fail(c, CHFSI_E_ARG, "lanczos_steps must be in 1..1000");
    if (!(o->range > 1) || !std::isfinite(o->range)) return fail(c, CHFSI_E_ARG, "range must be > 1");
    hipStream_t s = S(stream);
    using clk = std::chrono::steady_clock;
    HIPCHK(c, hipStreamSynchronize(s));
    const auto t0 = clk::now();
    double lmax = o->lambda_max;
    if (lmax == 0 && (rc = poisson_lanczos(c, o->lanczos_steps, &lmax, s))) return rc;
    const double lmin = lmax / o->range;
    const auto t1 = clk::now();
    double *r = poi_vec(c, 0), *p = poi_vec(c, 1), *w = poi_vec(c, 2), *z = poi_vec(c, 3), *d = poi_vec(c, 4),
           *Kz = poi_vec(c, 5);
    double *part = poi_part(c), *sc = poi_sc(c);
    double h[SC_NSC];
    // r = K x - (f - mean f); z = P^-1 r; delta = r.z, gamma = r.r; p = -z
    HIPCHK(c, launch_dot2(M, f, nullptr, nullptr, nullptr, part, PCG_SUMS, sc, s));
    HIPCHK(c, launch_kx(c, x, w, s));
    HIPCHK(c, launch_pcg_init(M, sc, w, f, r, s));
    if ((rc = cheb_precond(c, o->cheb_degree, lmin, lmax, r, z, d, Kz, s, PCG_FIRST))) return rc;
    HIPCHK(c, launch_pcg_dir(M, sc, true, z, p, s));
    if ((rc = read_sc(c, s, h))) return rc;
    int it = 0;
    bool conv = std::sqrt(h[SC_GAMMA]) < o->tol;
    bool bad = !std::isfinite(h[SC_GAMMA]) || !std::isfinite(h[SC_DELTA]);
    while (!conv && !bad && it < o->max_iter) {
        HIPCHK(c, launch_kx(c, p, w, s));                                 // w = K p
        HIPCHK(c, launch_dot2(M, p, w, nullptr, nullptr, part, PCG_ETA, sc, s));  // eta = p.w
        HIPCHK(c, launch_pcg_update(M, sc, p, w, x, r, s));                    // x += a p, r += a w
        // z = P^-1 r; the last Chebyshev step also forms delta, gamma and beta
        if ((rc = cheb_precond(c, o->cheb_degree, lmin, lmax, r, z, d, Kz, s, PCG_NEXT))) return rc;
        HIPCHK(c, launch_pcg_dir(M, sc, false, z, p, s));                      // p = -z + beta p
        if ((rc = read_sc(c, s, h))) return rc;
        ++it;
        bad = !(h[SC_ETA] > 0) || !std::isfinite(h[SC_ETA]) || !std::isfinite(h[SC_GAMMA]) ||
              !std::isfinite(h[SC_DELTA]);
        conv = !bad && std::sqrt(h[SC_GAMMA]) < o->tol;
    }
    // zero-mean representative
    HIPCHK(c, launch_dot2(M, x, nullptr, nullptr, nullptr, part, PCG_SUMS, sc, s));
    HIPCHK(c, launch_sub_mean(M, sc, x, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const auto t2 = clk::now();
    if (rep) {
        rep->iters = it;
        rep->converged = conv ? 1 : 0;
        rep->res_norm = std::sqrt(std::max(h[SC_GAMMA], 0.0));
        rep->lambda_min = lmin;
        rep->lambda_max = lmax;
        rep->t_lanczos = std::chrono::duration<double>(t1 - t0).count();
        rep->t_total = std::chrono::duration<double>(t2 - t0).count();
    }
    if (bad) return fail(c, CHFSI_E_NONFINITE, "PCG breakdown: non-finite scalar or non-positive p.Kp");
    return conv ? CHFSI_OK : CHFSI_NOT_CONVERGED;
}

const char *chfsi_last_error(const chfsi_ctx *c) {
    if (c) return c->err.c_str();
    return g_err.c_str();
}

void chfsi_destroy(chfsi_ctx *c) {
    if (!c) return;
    if (c->blas) rocblas_destroy_handle(c->blas);
    delete c;
}

}  // extern "C"
