/*
 * CPU oracle for the R-ChFSI eigensolver of the finite-element noncollinear
 * spin-orbit Kohn-Sham problem H X = M X Lambda.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, double-precision
 * statement of what the GPU library computes.  It is used by the tests, the
 * smoke check and the CPU baseline leg of the benchmark; the product path
 * never links or calls it.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * Every routine follows the paper's definitions directly:
 *   - FE basis: 1D Lagrange polynomials on Gauss-Lobatto-Legendre nodes, tensor
 *     products on hexahedra, Gauss-Legendre quadrature (Sec. III-A, eq. FEWfns).
 *   - Operator: H = -1/2 Laplacian + V + B.sigma (eq. hloc, Sec. II-A) plus the
 *     separable spin-orbit term sum_a P_a Delta_a P_a^H (eq. hnloc; Sec.
 *     III-C2 item iv), evaluated cell by cell as the quadrature of the
 *     bilinear form; no precomputed element matrices.
 *   - Mass: M_{2I+a,2J+b} = delta_ab int N_I N_J (Sec. III-A).
 *   - D: the GLL-integrated diagonal, D_I = int N_I (Sec. III-B2).
 *   - R-ChFSI: the residual recurrence (eq. rChFSIrecurrence) inside
 *     Algorithm RChFSI; ChFSI: the plain recurrence (eq. ChFSIrecurrence).
 *   - Densities: rho and m as in Sec. II-A (spinor definitions).
 *
 * Layout: a block X of nvec spinor vectors is complex [2M][ld], row = dof
 * index 2g+alpha (spin alpha of global node g), vectors fastest.
 *
 * Parity pins: every function is checked against closed forms, invariants or
 * brute force by the CPU test-suite (see the tests of the oracle).
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;
/* the imaginary unit; the letter I is kept free for node indices */
#undef I
#define IU _Complex_I

/* ------------------------------------------------------------------------ */
/* 1D polynomials                                                            */
/* ------------------------------------------------------------------------ */

/* Legendre P_n(x) and P_n'(x) by the three-term recurrence. */
static void legendre(int n, double x, double *P, double *dP) {
    double p0 = 1.0, p1 = x;
    if (n == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1; p1 = p2;
    }
    *P = p1;
    /* (1-x^2) P_n' = n (P_{n-1} - x P_n) */
    if (fabs(1.0 - x * x) < 1e-300) *dP = 0.5 * n * (n + 1) * (x > 0 ? 1.0 : (n % 2 ? 1.0 : -1.0));
    else *dP = n * (p0 - x * p1) / (1.0 - x * x);
}

/* Gauss-Lobatto-Legendre nodes (ascending) and weights, p+1 points:
 * end points +-1 and the roots of P_p'; w_i = 2 / (p(p+1) P_p(x_i)^2). */
void orc_gll(int p, double *x, double *w) {
    x[0] = -1.0; x[p] = 1.0;
    for (int i = 1; i < p; ++i) {
        double t = -cos(M_PI * i / p);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(p, t, &P, &dP);
            /* P'' from the Legendre ODE: (1-t^2) P'' = 2 t P' - p(p+1) P */
            double d2P = (2.0 * t * dP - p * (p + 1.0) * P) / (1.0 - t * t);
            double dt = dP / d2P;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        x[i] = t;
    }
    for (int i = 0; i <= p; ++i) {
        double P, dP;
        legendre(p, x[i], &P, &dP);
        w[i] = 2.0 / (p * (p + 1.0) * P * P);
    }
}

/* Gauss-Legendre nodes (ascending) and weights, n points: roots of P_n,
 * w_i = 2 / ((1-x_i^2) P_n'(x_i)^2). */
void orc_gauss(int n, double *x, double *w) {
    for (int i = 0; i < n; ++i) {
        double t = -cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(n, t, &P, &dP);
            double dt = P / dP;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        double P, dP;
        legendre(n, t, &P, &dP);
        x[i] = t;
        w[i] = 2.0 / ((1.0 - t * t) * dP * dP);
    }
}

/* Lagrange basis l_i(x) on the nodes and its derivative l_i'(x). */
void orc_lagrange(int np1, const double *nodes, double x, double *l, double *dl) {
    for (int i = 0; i < np1; ++i) {
        double v = 1.0, d = 0.0;
        for (int j = 0; j < np1; ++j) {
            if (j == i) continue;
            double f = (x - nodes[j]) / (nodes[i] - nodes[j]);
            /* product rule: d(v f) = dv f + v df */
            d = d * f + v / (nodes[i] - nodes[j]);
            v *= f;
        }
        l[i] = v;
        dl[i] = d;
    }
}

/* ------------------------------------------------------------------------ */
/* problem                                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int ncell[3];
    double h[3];
    int p, nq1, n1, n, nq;
    int64_t ncells, M, Nd[3];
    const double *V;   /* [ncells][nq] */
    const double *B;   /* [ncells][nq][3] */
    int natoms, nbeta;
    const int64_t *pair_ptr, *pair_cell;
    const cplx *phi;   /* [npairs][nq][2][nbeta] */
    const cplx *delta; /* [natoms][nbeta][nbeta] */
    double *Nq;        /* basis at quadrature points [nq][n] */
    double *dNq;       /* physical gradient [nq][n][3] */
    double *wJ;        /* quadrature weight times |J| [nq] */
    double *D;         /* diagonal approximation of M [M] */
    cplx *Pall;        /* projector matrices of all pairs, built on first use */
} orc_problem;

static int64_t gnode(const orc_problem *pr, int64_t e, int I) {
    int64_t ex = e % pr->ncell[0], ey = (e / pr->ncell[0]) % pr->ncell[1];
    int64_t ez = e / ((int64_t)pr->ncell[0] * pr->ncell[1]);
    int i = I % pr->n1, j = (I / pr->n1) % pr->n1, k = I / (pr->n1 * pr->n1);
    int64_t gx = (ex * pr->p + i) % pr->Nd[0];
    int64_t gy = (ey * pr->p + j) % pr->Nd[1];
    int64_t gz = (ez * pr->p + k) % pr->Nd[2];
    return gx + pr->Nd[0] * (gy + pr->Nd[1] * gz);
}

void *orc_create(const int *ncell, const double *h, int p, int nq1,
                 const double *V, const double *B, int natoms, int nbeta,
                 const int64_t *pair_ptr, const int64_t *pair_cell,
                 const double *phi, const double *delta) {
    orc_problem *pr = (orc_problem *)calloc(1, sizeof(orc_problem));
    for (int d = 0; d < 3; ++d) { pr->ncell[d] = ncell[d]; pr->h[d] = h[d]; pr->Nd[d] = (int64_t)ncell[d] * p; }
    pr->p = p; pr->nq1 = nq1; pr->n1 = p + 1;
    pr->n = pr->n1 * pr->n1 * pr->n1;
    pr->nq = nq1 * nq1 * nq1;
    pr->ncells = (int64_t)ncell[0] * ncell[1] * ncell[2];
    pr->M = pr->Nd[0] * pr->Nd[1] * pr->Nd[2];
    pr->V = V; pr->B = B;
    pr->natoms = natoms; pr->nbeta = nbeta;
    pr->pair_ptr = pair_ptr; pr->pair_cell = pair_cell;
    pr->phi = (const cplx *)phi; pr->delta = (const cplx *)delta;

    int n1 = pr->n1, n = pr->n, nq = pr->nq;
    double *gx = malloc(sizeof(double) * n1), *gw = malloc(sizeof(double) * n1);
    double *qx = malloc(sizeof(double) * nq1), *qw = malloc(sizeof(double) * nq1);
    orc_gll(p, gx, gw);
    orc_gauss(nq1, qx, qw);
    double *l = malloc(sizeof(double) * nq1 * n1), *dl = malloc(sizeof(double) * nq1 * n1);
    for (int a = 0; a < nq1; ++a) orc_lagrange(n1, gx, qx[a], l + a * n1, dl + a * n1);
    pr->Nq = malloc(sizeof(double) * nq * n);
    pr->dNq = malloc(sizeof(double) * nq * n * 3);
    pr->wJ = malloc(sizeof(double) * nq);
    double detJ = h[0] * h[1] * h[2] / 8.0;
    for (int q = 0; q < nq; ++q) {
        int a = q % nq1, b = (q / nq1) % nq1, c = q / (nq1 * nq1);
        pr->wJ[q] = qw[a] * qw[b] * qw[c] * detJ;
        for (int I = 0; I < n; ++I) {
            int i = I % n1, j = (I / n1) % n1, k = I / (n1 * n1);
            pr->Nq[q * n + I] = l[a * n1 + i] * l[b * n1 + j] * l[c * n1 + k];
            pr->dNq[(q * n + I) * 3 + 0] = (2.0 / h[0]) * dl[a * n1 + i] * l[b * n1 + j] * l[c * n1 + k];
            pr->dNq[(q * n + I) * 3 + 1] = (2.0 / h[1]) * l[a * n1 + i] * dl[b * n1 + j] * l[c * n1 + k];
            pr->dNq[(q * n + I) * 3 + 2] = (2.0 / h[2]) * l[a * n1 + i] * l[b * n1 + j] * dl[c * n1 + k];
        }
    }
    /* D_g = int N_g: GLL weights times |J|, summed over the cells of g */
    pr->D = calloc(pr->M, sizeof(double));
    for (int64_t e = 0; e < pr->ncells; ++e)
        for (int I = 0; I < n; ++I) {
            int i = I % n1, j = (I / n1) % n1, k = I / (n1 * n1);
            pr->D[gnode(pr, e, I)] += gw[i] * gw[j] * gw[k] * detJ;
        }
    free(gx); free(gw); free(qx); free(qw); free(l); free(dl);
    return pr;
}

void orc_destroy(void *vp) {
    orc_problem *pr = (orc_problem *)vp;
    if (!pr) return;
    free(pr->Nq); free(pr->dNq); free(pr->wJ); free(pr->D); free(pr->Pall);
    free(pr);
}

void orc_mass_diag(void *vp, double *D) {
    orc_problem *pr = (orc_problem *)vp;
    memcpy(D, pr->D, sizeof(double) * pr->M);
}

void orc_tables(void *vp, double *Nq, double *dNq, double *wJ) {
    orc_problem *pr = (orc_problem *)vp;
    if (Nq) memcpy(Nq, pr->Nq, sizeof(double) * pr->nq * pr->n);
    if (dNq) memcpy(dNq, pr->dNq, sizeof(double) * pr->nq * pr->n * 3);
    if (wJ) memcpy(wJ, pr->wJ, sizeof(double) * pr->nq);
}

/* ------------------------------------------------------------------------ */
/* operator action, one vector at a time                                    */
/* ------------------------------------------------------------------------ */

enum { ORC_KIN = 1, ORC_POT = 2, ORC_MAG = 4, ORC_NLOC = 8, ORC_ALL = 15 };

/* u_alpha(x_q) and grad u_alpha(x_q) of the field with nodal values xl[I][alpha] */
static void interp(const orc_problem *pr, const cplx *xl, int q, cplx u[2], cplx gu[2][3]) {
    u[0] = u[1] = 0;
    for (int a = 0; a < 2; ++a) for (int d = 0; d < 3; ++d) gu[a][d] = 0;
    for (int I = 0; I < pr->n; ++I) {
        double N = pr->Nq[q * pr->n + I];
        const double *dN = pr->dNq + (q * pr->n + I) * 3;
        for (int a = 0; a < 2; ++a) {
            u[a] += N * xl[2 * I + a];
            for (int d = 0; d < 3; ++d) gu[a][d] += dN[d] * xl[2 * I + a];
        }
    }
}

/* (V + B.sigma) applied to the spinor u */
static void spin_term(double V, const double *B, int flags, const cplx u[2], cplx out[2]) {
    double v = (flags & ORC_POT) ? V : 0.0;
    double bx = 0, by = 0, bz = 0;
    if (flags & ORC_MAG) { bx = B[0]; by = B[1]; bz = B[2]; }
    /* [[v+bz, bx - i by], [bx + i by, v - bz]] */
    out[0] = (v + bz) * u[0] + (bx - IU * by) * u[1];
    out[1] = (bx + IU * by) * u[0] + (v - bz) * u[1];
}

/* projector matrix of one (atom, cell) pair:
 * P[I][alpha][j] = sum_q wJ_q N_I(x_q) phi_{j,alpha}(x_q) */
static void pair_matrix(const orc_problem *pr, int64_t pair, cplx *P) {
    int n = pr->n, nb = pr->nbeta;
    const cplx *ph = pr->phi + (size_t)pair * pr->nq * 2 * nb;
    for (int I = 0; I < n; ++I)
        for (int a = 0; a < 2; ++a)
            for (int j = 0; j < nb; ++j) {
                cplx s = 0;
                for (int q = 0; q < pr->nq; ++q)
                    s += pr->wJ[q] * pr->Nq[q * n + I] * ph[(q * 2 + a) * nb + j];
                P[(I * 2 + a) * nb + j] = s;
            }
}

/* y (length 2M, one vector) = H x; flags select the terms */
static void apply_one(const orc_problem *pr, const cplx *x, cplx *y, int flags, const cplx *Pall) {
    int n = pr->n, nq = pr->nq;
    cplx *xl = malloc(sizeof(cplx) * 2 * n), *yl = malloc(sizeof(cplx) * 2 * n);
    memset(y, 0, sizeof(cplx) * 2 * pr->M);
    for (int64_t e = 0; e < pr->ncells; ++e) {
        for (int I = 0; I < n; ++I) {
            int64_t g = gnode(pr, e, I);
            xl[2 * I] = x[2 * g]; xl[2 * I + 1] = x[2 * g + 1];
        }
        memset(yl, 0, sizeof(cplx) * 2 * n);
        for (int q = 0; q < nq; ++q) {
            cplx u[2], gu[2][3], f[2];
            interp(pr, xl, q, u, gu);
            spin_term(pr->V[e * nq + q], pr->B + (e * nq + q) * 3, flags, u, f);
            double w = pr->wJ[q];
            for (int I = 0; I < n; ++I) {
                double N = pr->Nq[q * n + I];
                const double *dN = pr->dNq + (q * n + I) * 3;
                for (int a = 0; a < 2; ++a) {
                    cplx acc = N * f[a];
                    if (flags & ORC_KIN) acc += 0.5 * (dN[0] * gu[a][0] + dN[1] * gu[a][1] + dN[2] * gu[a][2]);
                    yl[2 * I + a] += w * acc;
                }
            }
        }
        for (int I = 0; I < n; ++I) {
            int64_t g = gnode(pr, e, I);
            y[2 * g] += yl[2 * I]; y[2 * g + 1] += yl[2 * I + 1];
        }
    }
    if ((flags & ORC_NLOC) && pr->natoms > 0) {
        int nb = pr->nbeta;
        cplx *c = malloc(sizeof(cplx) * nb), *d = malloc(sizeof(cplx) * nb);
        for (int at = 0; at < pr->natoms; ++at) {
            for (int j = 0; j < nb; ++j) c[j] = 0;
            for (int64_t pp = pr->pair_ptr[at]; pp < pr->pair_ptr[at + 1]; ++pp) {
                const cplx *P = Pall + (size_t)pp * 2 * n * nb;
                int64_t e = pr->pair_cell[pp];
                for (int I = 0; I < n; ++I) {
                    int64_t g = gnode(pr, e, I);
                    for (int a = 0; a < 2; ++a)
                        for (int j = 0; j < nb; ++j) c[j] += conj(P[(I * 2 + a) * nb + j]) * x[2 * g + a];
                }
            }
            const cplx *Dl = pr->delta + (size_t)at * nb * nb;
            for (int i = 0; i < nb; ++i) {
                d[i] = 0;
                for (int j = 0; j < nb; ++j) d[i] += Dl[i * nb + j] * c[j];
            }
            for (int64_t pp = pr->pair_ptr[at]; pp < pr->pair_ptr[at + 1]; ++pp) {
                const cplx *P = Pall + (size_t)pp * 2 * n * nb;
                int64_t e = pr->pair_cell[pp];
                for (int I = 0; I < n; ++I) {
                    int64_t g = gnode(pr, e, I);
                    for (int a = 0; a < 2; ++a) {
                        cplx s = 0;
                        for (int j = 0; j < nb; ++j) s += P[(I * 2 + a) * nb + j] * d[j];
                        y[2 * g + a] += s;
                    }
                }
            }
        }
        free(c); free(d);
    }
    free(xl); free(yl);
}

static cplx *all_pair_matrices(orc_problem *pr) {
    if (pr->natoms == 0) return NULL;
    if (pr->Pall) return pr->Pall;
    int64_t npairs = pr->pair_ptr[pr->natoms];
    size_t per = (size_t)2 * pr->n * pr->nbeta;
    cplx *P = malloc(sizeof(cplx) * per * (npairs > 0 ? npairs : 1));
#pragma omp parallel for schedule(dynamic)
    for (int64_t pp = 0; pp < npairs; ++pp) pair_matrix(pr, pp, P + per * pp);
    pr->Pall = P;
    return P;
}

/* Y = H X for nvec vectors of the [2M][ld] block; flags pick the terms. */
void orc_apply_H(void *vp, const double *Xd, int64_t ld, int64_t nvec, double *Yd, int64_t ldy, int flags) {
    orc_problem *pr = (orc_problem *)vp;
    const cplx *X = (const cplx *)Xd;
    cplx *Y = (cplx *)Yd;
    cplx *Pall = (flags & ORC_NLOC) ? all_pair_matrices(pr) : NULL;
    int64_t ndof = 2 * pr->M;
#pragma omp parallel
    {
        cplx *x = malloc(sizeof(cplx) * ndof), *y = malloc(sizeof(cplx) * ndof);
#pragma omp for schedule(dynamic)
        for (int64_t b = 0; b < nvec; ++b) {
            for (int64_t r = 0; r < ndof; ++r) x[r] = X[r * ld + b];
            apply_one(pr, x, y, flags, Pall);
            for (int64_t r = 0; r < ndof; ++r) Y[r * ldy + b] = y[r];
        }
        free(x); free(y);
    }
}

/* Y = M X: consistent mass, M_{2I+a,2J+b} = delta_ab int N_I N_J */
void orc_apply_M(void *vp, const double *Xd, int64_t ld, int64_t nvec, double *Yd, int64_t ldy) {
    orc_problem *pr = (orc_problem *)vp;
    const cplx *X = (const cplx *)Xd;
    cplx *Y = (cplx *)Yd;
    int n = pr->n, nq = pr->nq;
    int64_t ndof = 2 * pr->M;
#pragma omp parallel
    {
        cplx *x = malloc(sizeof(cplx) * ndof), *y = malloc(sizeof(cplx) * ndof);
        cplx *xl = malloc(sizeof(cplx) * 2 * n), *yl = malloc(sizeof(cplx) * 2 * n);
#pragma omp for schedule(dynamic)
        for (int64_t b = 0; b < nvec; ++b) {
            for (int64_t r = 0; r < ndof; ++r) x[r] = X[r * ld + b];
            memset(y, 0, sizeof(cplx) * ndof);
            for (int64_t e = 0; e < pr->ncells; ++e) {
                for (int I = 0; I < n; ++I) {
                    int64_t g = gnode(pr, e, I);
                    xl[2 * I] = x[2 * g]; xl[2 * I + 1] = x[2 * g + 1];
                }
                memset(yl, 0, sizeof(cplx) * 2 * n);
                for (int q = 0; q < nq; ++q) {
                    cplx u[2] = {0, 0};
                    for (int I = 0; I < n; ++I) {
                        u[0] += pr->Nq[q * n + I] * xl[2 * I];
                        u[1] += pr->Nq[q * n + I] * xl[2 * I + 1];
                    }
                    for (int I = 0; I < n; ++I) {
                        double wN = pr->wJ[q] * pr->Nq[q * n + I];
                        yl[2 * I] += wN * u[0];
                        yl[2 * I + 1] += wN * u[1];
                    }
                }
                for (int I = 0; I < n; ++I) {
                    int64_t g = gnode(pr, e, I);
                    y[2 * g] += yl[2 * I]; y[2 * g + 1] += yl[2 * I + 1];
                }
            }
            for (int64_t r = 0; r < ndof; ++r) Y[r * ldy + b] = y[r];
        }
        free(x); free(y); free(xl); free(yl);
    }
}

/* (H X) at selected nodes and columns: out[s][alpha][c] for node nodes[s],
 * column cols[c].  Only the cells containing each node and the atoms whose
 * support contains such a cell are visited, so that large meshes can be
 * checked on samples.  Same arithmetic as orc_apply_H. */
void orc_apply_H_sampled(void *vp, const double *Xd, int64_t ld, const int64_t *nodes, int64_t nn,
                         const int64_t *cols, int64_t nc, double *outd) {
    orc_problem *pr = (orc_problem *)vp;
    const cplx *X = (const cplx *)Xd;
    cplx *out = (cplx *)outd;
    int n = pr->n, nq = pr->nq, nb = pr->nbeta;
    /* cells containing each node: scan all cells once */
    int64_t *cellof = malloc(sizeof(int64_t) * nn * 8);
    int *locof = malloc(sizeof(int) * nn * 8);
    int *cnt = calloc(nn, sizeof(int));
    for (int64_t e = 0; e < pr->ncells; ++e)
        for (int I = 0; I < n; ++I) {
            int64_t g = gnode(pr, e, I);
            for (int64_t s = 0; s < nn; ++s)
                if (nodes[s] == g && cnt[s] < 8) {
                    cellof[s * 8 + cnt[s]] = e; locof[s * 8 + cnt[s]] = I; cnt[s]++;
                }
        }
    /* atoms that touch any of these cells */
    int64_t npairs = pr->natoms ? pr->pair_ptr[pr->natoms] : 0;
    char *need = calloc(pr->natoms > 0 ? pr->natoms : 1, 1);
    for (int at = 0; at < pr->natoms; ++at)
        for (int64_t pp = pr->pair_ptr[at]; pp < pr->pair_ptr[at + 1]; ++pp)
            for (int64_t s = 0; s < nn; ++s)
                for (int k = 0; k < cnt[s]; ++k)
                    if (cellof[s * 8 + k] == pr->pair_cell[pp]) need[at] = 1;
    size_t per = (size_t)2 * n * nb;
    cplx *Pall = npairs ? calloc(per * npairs, sizeof(cplx)) : NULL;
#pragma omp parallel for schedule(dynamic)
    for (int64_t pp = 0; pp < npairs; ++pp) {
        int at = 0;
        while (pr->pair_ptr[at + 1] <= pp) ++at;
        if (need[at]) pair_matrix(pr, pp, Pall + per * pp);
    }
#pragma omp parallel for schedule(dynamic)
    for (int64_t ci = 0; ci < nc; ++ci) {
        int64_t b = cols[ci];
        cplx xl[2 * 512];
        cplx *dA = malloc(sizeof(cplx) * (pr->natoms > 0 ? pr->natoms : 1) * (nb > 0 ? nb : 1));
        for (int at = 0; at < pr->natoms; ++at) {
            if (!need[at]) continue;
            cplx c[16] = {0};
            for (int64_t pp = pr->pair_ptr[at]; pp < pr->pair_ptr[at + 1]; ++pp) {
                const cplx *P = Pall + per * pp;
                for (int I = 0; I < n; ++I) {
                    int64_t g = gnode(pr, pr->pair_cell[pp], I);
                    for (int a = 0; a < 2; ++a)
                        for (int j = 0; j < nb; ++j) c[j] += conj(P[(I * 2 + a) * nb + j]) * X[(2 * g + a) * ld + b];
                }
            }
            const cplx *Dl = pr->delta + (size_t)at * nb * nb;
            for (int i = 0; i < nb; ++i) {
                cplx s = 0;
                for (int j = 0; j < nb; ++j) s += Dl[i * nb + j] * c[j];
                dA[at * nb + i] = s;
            }
        }
        for (int64_t s = 0; s < nn; ++s) {
            cplx acc[2] = {0, 0};
            for (int k = 0; k < cnt[s]; ++k) {
                int64_t e = cellof[s * 8 + k];
                int Io = locof[s * 8 + k];
                for (int I = 0; I < n; ++I) {
                    int64_t g = gnode(pr, e, I);
                    xl[2 * I] = X[(2 * g) * ld + b]; xl[2 * I + 1] = X[(2 * g + 1) * ld + b];
                }
                for (int q = 0; q < nq; ++q) {
                    cplx u[2], gu[2][3], f[2];
                    interp(pr, xl, q, u, gu);
                    spin_term(pr->V[e * nq + q], pr->B + (e * nq + q) * 3, ORC_ALL, u, f);
                    double N = pr->Nq[q * n + Io];
                    const double *dN = pr->dNq + (q * n + Io) * 3;
                    for (int a = 0; a < 2; ++a)
                        acc[a] += pr->wJ[q] * (N * f[a] + 0.5 * (dN[0] * gu[a][0] + dN[1] * gu[a][1] + dN[2] * gu[a][2]));
                }
                for (int at = 0; at < pr->natoms; ++at) {
                    if (!need[at]) continue;
                    for (int64_t pp = pr->pair_ptr[at]; pp < pr->pair_ptr[at + 1]; ++pp) {
                        if (pr->pair_cell[pp] != e) continue;
                        const cplx *P = Pall + per * pp;
                        for (int a = 0; a < 2; ++a)
                            for (int j = 0; j < nb; ++j) acc[a] += P[(Io * 2 + a) * nb + j] * dA[at * nb + j];
                    }
                }
            }
            out[(s * 2 + 0) * nc + ci] = acc[0];
            out[(s * 2 + 1) * nc + ci] = acc[1];
        }
        free(dA);
    }
    free(cellof); free(locof); free(cnt); free(need); free(Pall);
}

/* Adjoint of Y = H(V,B) X with respect to the quadrature fields, for the
 * cotangent G (dL = Re sum conj(G) dY):
 *   dV[e][q]    = wJ_q Re sum_{b,alpha} conj(g_{b,alpha}(x_q)) x_{b,alpha}(x_q)
 *   dB[e][q][d] = wJ_q Re sum_b g_b(x_q)^H sigma_d x_b(x_q)
 * (dL/dX = H G is orc_apply_H).  With G = X this is wJ * (rho, m) of Sec. II-A. */
void orc_adjoint_fields(void *vp, const double *Xd, const double *Gd, int64_t ld, int64_t nvec,
                        double *dV, double *dB) {
    orc_problem *pr = (orc_problem *)vp;
    const cplx *X = (const cplx *)Xd, *G = (const cplx *)Gd;
    int n = pr->n, nq = pr->nq;
#pragma omp parallel for schedule(dynamic)
    for (int64_t e = 0; e < pr->ncells; ++e) {
        cplx *xl = malloc(sizeof(cplx) * 2 * n), *gl = malloc(sizeof(cplx) * 2 * n);
        double *sv = calloc(nq, sizeof(double)), *sb = calloc(nq * 3, sizeof(double));
        for (int64_t b = 0; b < nvec; ++b) {
            for (int I = 0; I < n; ++I) {
                int64_t g = gnode(pr, e, I);
                xl[2 * I] = X[(2 * g) * ld + b]; xl[2 * I + 1] = X[(2 * g + 1) * ld + b];
                gl[2 * I] = G[(2 * g) * ld + b]; gl[2 * I + 1] = G[(2 * g + 1) * ld + b];
            }
            for (int q = 0; q < nq; ++q) {
                cplx u[2] = {0, 0}, v[2] = {0, 0};
                for (int I = 0; I < n; ++I) {
                    double N = pr->Nq[q * n + I];
                    u[0] += N * xl[2 * I]; u[1] += N * xl[2 * I + 1];
                    v[0] += N * gl[2 * I]; v[1] += N * gl[2 * I + 1];
                }
                sv[q] += creal(conj(v[0]) * u[0] + conj(v[1]) * u[1]);
                sb[q * 3 + 0] += creal(conj(v[0]) * u[1] + conj(v[1]) * u[0]);
                sb[q * 3 + 1] += creal(conj(v[0]) * (-IU * u[1]) + conj(v[1]) * (IU * u[0]));
                sb[q * 3 + 2] += creal(conj(v[0]) * u[0] - conj(v[1]) * u[1]);
            }
        }
        for (int q = 0; q < nq; ++q) {
            dV[e * nq + q] = pr->wJ[q] * sv[q];
            for (int d = 0; d < 3; ++d) dB[(e * nq + q) * 3 + d] = pr->wJ[q] * sb[q * 3 + d];
        }
        free(xl); free(gl); free(sv); free(sb);
    }
}

/* ------------------------------------------------------------------------ */
/* dense linear algebra (no LAPACK)                                          */
/* ------------------------------------------------------------------------ */

/* Cholesky A = L L^H of a Hermitian positive definite n x n matrix (row-major,
 * lower triangle written to L, upper zeroed).  Returns 0, or -1 if a pivot
 * is not positive. */
int orc_cholesky(int n, const double *Ad, double *Ld) {
    const cplx *A = (const cplx *)Ad;
    cplx *L = (cplx *)Ld;
    memset(L, 0, sizeof(cplx) * n * n);
    for (int j = 0; j < n; ++j) {
        double s = creal(A[j * n + j]);
        for (int k = 0; k < j; ++k) s -= creal(L[j * n + k] * conj(L[j * n + k]));
        if (!(s > 0.0)) return -1;
        double ljj = sqrt(s);
        L[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            cplx t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= L[i * n + k] * conj(L[j * n + k]);
            L[i * n + j] = t / ljj;
        }
    }
    return 0;
}

/* Cyclic Jacobi for a complex Hermitian matrix (Golub & Van Loan, Sec. 8.5,
 * with a phase factor that makes each 2x2 pivot block real).  On return w
 * holds the eigenvalues ascending and V (row-major, columns = eigenvectors)
 * the unitary eigenvector matrix.  Returns the number of sweeps. */
int orc_jacobi(int n, const double *Ad, double *w, double *Vd) {
    cplx *A = malloc(sizeof(cplx) * n * n);
    memcpy(A, Ad, sizeof(cplx) * n * n);
    cplx *V = (cplx *)Vd;
    for (int i = 0; i < n * n; ++i) V[i] = 0;
    for (int i = 0; i < n; ++i) V[i * n + i] = 1;
    double fro = 0;
    for (int i = 0; i < n * n; ++i) fro += creal(A[i] * conj(A[i]));
    fro = sqrt(fro);
    int sweep;
    for (sweep = 0; sweep < 100; ++sweep) {
        double off = 0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                if (i != j) off += creal(A[i * n + j] * conj(A[i * n + j]));
        if (sqrt(off) <= 1e-15 * fro || fro == 0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                cplx apq = A[p * n + q];
                double mag = cabs(apq);
                if (mag == 0.0) continue;
                cplx ph = apq / mag; /* e^{i phi} */
                double app = creal(A[p * n + p]), aqq = creal(A[q * n + q]);
                double tau = (aqq - app) / (2.0 * mag);
                double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                /* G = diag(1, conj(ph)) * [[c, s], [-s, c]] */
                cplx gpp = c, gpq = s, gqp = -s * conj(ph), gqq = c * conj(ph);
                for (int k = 0; k < n; ++k) { /* A <- A G */
                    cplx ap = A[k * n + p], aq = A[k * n + q];
                    A[k * n + p] = ap * gpp + aq * gqp;
                    A[k * n + q] = ap * gpq + aq * gqq;
                }
                for (int k = 0; k < n; ++k) { /* A <- G^H A */
                    cplx ap = A[p * n + k], aq = A[q * n + k];
                    A[p * n + k] = conj(gpp) * ap + conj(gqp) * aq;
                    A[q * n + k] = conj(gpq) * ap + conj(gqq) * aq;
                }
                for (int k = 0; k < n; ++k) { /* V <- V G */
                    cplx vp = V[k * n + p], vq = V[k * n + q];
                    V[k * n + p] = vp * gpp + vq * gqp;
                    V[k * n + q] = vp * gpq + vq * gqq;
                }
                A[p * n + q] = 0; A[q * n + p] = 0;
                A[p * n + p] = creal(A[p * n + p]); A[q * n + q] = creal(A[q * n + q]);
            }
    }
    /* sort ascending (selection sort, columns of V follow) */
    for (int i = 0; i < n; ++i) w[i] = creal(A[i * n + i]);
    for (int i = 0; i < n; ++i) {
        int m = i;
        for (int j = i + 1; j < n; ++j) if (w[j] < w[m]) m = j;
        if (m != i) {
            double t = w[i]; w[i] = w[m]; w[m] = t;
            for (int k = 0; k < n; ++k) { cplx tv = V[k * n + i]; V[k * n + i] = V[k * n + m]; V[k * n + m] = tv; }
        }
    }
    free(A);
    return sweep;
}

/* Generalized Hermitian eigenproblem H v = lambda M v (M Hermitian positive
 * definite), by Cholesky M = L L^H, C = L^{-1} H L^{-H}, Jacobi on C and
 * v = L^{-H} y.  Returns 0 or -1 (M not positive definite). */
int orc_dense_geig(int n, const double *Hd, const double *Md, double *w, double *Vd) {
    const cplx *H = (const cplx *)Hd;
    cplx *L = malloc(sizeof(cplx) * n * n);
    if (orc_cholesky(n, Md, (double *)L)) { free(L); return -1; }
    cplx *T = malloc(sizeof(cplx) * n * n), *C = malloc(sizeof(cplx) * n * n);
    cplx *Y = malloc(sizeof(cplx) * n * n);
    /* T = L^{-1} H (forward substitution on each column) */
    for (int c = 0; c < n; ++c)
        for (int i = 0; i < n; ++i) {
            cplx s = H[i * n + c];
            for (int k = 0; k < i; ++k) s -= L[i * n + k] * T[k * n + c];
            T[i * n + c] = s / L[i * n + i];
        }
    /* C = T L^{-H}, i.e. C^H = L^{-1} T^H: solve for each row of C */
    for (int r = 0; r < n; ++r)
        for (int i = 0; i < n; ++i) {
            cplx s = conj(T[r * n + i]);
            for (int k = 0; k < i; ++k) s -= L[i * n + k] * conj(C[r * n + k]);
            C[r * n + i] = conj(s / L[i * n + i]);
        }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) {
            cplx a = 0.5 * (C[i * n + j] + conj(C[j * n + i]));
            C[i * n + j] = a; C[j * n + i] = conj(a);
        }
    orc_jacobi(n, (double *)C, w, (double *)Y);
    /* v = L^{-H} y: back substitution */
    cplx *V = (cplx *)Vd;
    for (int c = 0; c < n; ++c)
        for (int i = n - 1; i >= 0; --i) {
            cplx s = Y[i * n + c];
            for (int k = i + 1; k < n; ++k) s -= conj(L[k * n + i]) * V[k * n + c];
            V[i * n + c] = s / L[i * n + i];
        }
    free(L); free(T); free(C); free(Y);
    return 0;
}

/* Dense H (complex) and M (complex storage, real values) of a tiny mesh,
 * assembled column by column as the operator applied to unit vectors. */
void orc_dense(void *vp, double *Hd, double *Md, int flags) {
    orc_problem *pr = (orc_problem *)vp;
    int64_t N = 2 * pr->M;
    cplx *E = calloc((size_t)N * N, sizeof(cplx));
    for (int64_t i = 0; i < N; ++i) E[i * N + i] = 1;
    if (Hd) orc_apply_H(vp, (double *)E, N, N, Hd, N, flags);
    if (Md) orc_apply_M(vp, (double *)E, N, N, Md, N);
    free(E);
}

/* ------------------------------------------------------------------------ */
/* subspace routines on [2M][ld] blocks                                      */
/* ------------------------------------------------------------------------ */

/* S = A^H B  (k x k) for [rows][ld] blocks */
static void gram(int64_t rows, int k, const cplx *A, const cplx *B, int64_t ld, cplx *S) {
#pragma omp parallel for collapse(2)
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            cplx s = 0;
            for (int64_t r = 0; r < rows; ++r) s += conj(A[r * ld + i]) * B[r * ld + j];
            S[i * k + j] = s;
        }
}

/* A <- A Q (k x k) in place, row by row */
static void rotate(int64_t rows, int k, cplx *A, int64_t ld, const cplx *Q) {
#pragma omp parallel
    {
        cplx *t = malloc(sizeof(cplx) * k);
#pragma omp for
        for (int64_t r = 0; r < rows; ++r) {
            for (int j = 0; j < k; ++j) {
                cplx s = 0;
                for (int i = 0; i < k; ++i) s += A[r * ld + i] * Q[i * k + j];
                t[j] = s;
            }
            for (int j = 0; j < k; ++j) A[r * ld + j] = t[j];
        }
        free(t);
    }
}

/* One Cholesky-QR pass in the M inner product, with column equilibration:
 * S = Y^H M Y, s_j = S_jj^{-1/2}, L L^H = diag(s) S diag(s),
 * Y, HY, MY <- (.) diag(s) L^{-H}.  Returns 0 or -1. */
static int cholqr_pass(int64_t rows, int k, cplx *Y, cplx *HY, cplx *MY, int64_t ld) {
    cplx *S = malloc(sizeof(cplx) * k * k), *L = malloc(sizeof(cplx) * k * k);
    cplx *T = calloc((size_t)k * k, sizeof(cplx));
    double *sc = malloc(sizeof(double) * k);
    gram(rows, k, Y, MY, ld, S);
    for (int i = 0; i < k; ++i) sc[i] = 1.0 / sqrt(creal(S[i * k + i]));
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) S[i * k + j] *= sc[i] * sc[j];
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < i; ++j) {
            cplx a = 0.5 * (S[i * k + j] + conj(S[j * k + i]));
            S[i * k + j] = a; S[j * k + i] = conj(a);
        }
    int rc = orc_cholesky(k, (double *)S, (double *)L);
    if (rc == 0) {
        /* T = diag(s) L^{-H}: solve L^H T' = I (upper triangular), then scale rows */
        for (int c = 0; c < k; ++c)
            for (int i = k - 1; i >= 0; --i) {
                cplx s = (i == c) ? 1.0 : 0.0;
                for (int m = i + 1; m < k; ++m) s -= conj(L[m * k + i]) * T[m * k + c];
                T[i * k + c] = s / L[i * k + i];
            }
        for (int i = 0; i < k; ++i)
            for (int c = 0; c < k; ++c) T[i * k + c] *= sc[i];
        rotate(rows, k, Y, ld, T);
        if (HY) rotate(rows, k, HY, ld, T);
        if (MY) rotate(rows, k, MY, ld, T);
    }
    free(S); free(L); free(T); free(sc);
    return rc;
}

/* Cholesky-QR2 in the M inner product (two passes). */
int orc_orthonormalize(void *vp, double *Yd, double *HYd, double *MYd, int64_t ld, int k) {
    orc_problem *pr = (orc_problem *)vp;
    int64_t rows = 2 * pr->M;
    for (int pass = 0; pass < 2; ++pass)
        if (cholqr_pass(rows, k, (cplx *)Yd, (cplx *)HYd, (cplx *)MYd, ld)) return -1;
    return 0;
}

/* Rayleigh-Ritz on an M-orthonormal basis Y (with HY, MY): Hs = Y^H HY made
 * Hermitian, Hs Q = Q Lambda (ascending), then X = YQ, HX = HY Q, MX = MY Q
 * in place.  ritz receives Lambda. */
void orc_rayleigh_ritz(void *vp, double *Yd, double *HYd, double *MYd, int64_t ld, int k, double *ritz) {
    orc_problem *pr = (orc_problem *)vp;
    int64_t rows = 2 * pr->M;
    cplx *Hs = malloc(sizeof(cplx) * k * k), *Q = malloc(sizeof(cplx) * k * k);
    gram(rows, k, (cplx *)Yd, (cplx *)HYd, ld, Hs);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j <= i; ++j) {
            cplx a = 0.5 * (Hs[i * k + j] + conj(Hs[j * k + i]));
            Hs[i * k + j] = a; Hs[j * k + i] = conj(a);
        }
    orc_jacobi(k, (double *)Hs, ritz, (double *)Q);
    rotate(rows, k, (cplx *)Yd, ld, Q);
    rotate(rows, k, (cplx *)HYd, ld, Q);
    rotate(rows, k, (cplx *)MYd, ld, Q);
    free(Hs); free(Q);
}

/* R = HX - MX diag(ritz) and the Euclidean column norms. */
void orc_residual(int64_t rows, int k, const double *HXd, const double *MXd, int64_t ld,
                  const double *ritz, double *Rd, double *norms) {
    const cplx *HX = (const cplx *)HXd, *MX = (const cplx *)MXd;
    cplx *R = (cplx *)Rd;
    for (int j = 0; j < k; ++j) norms[j] = 0;
    for (int64_t r = 0; r < rows; ++r)
        for (int j = 0; j < k; ++j) {
            cplx v = HX[r * ld + j] - MX[r * ld + j] * ritz[j];
            if (R) R[r * ld + j] = v;
            norms[j] += creal(v * conj(v));
        }
    for (int j = 0; j < k; ++j) norms[j] = sqrt(norms[j]);
}

/* ------------------------------------------------------------------------ */
/* Chebyshev filters                                                         */
/* ------------------------------------------------------------------------ */

/* apply_Dinv: y = D^{-1} z (row r belongs to node r/2).  With Mdense given
 * (tiny meshes only) the exact M^{-1} is used instead, through the Cholesky
 * factor Lm of M. */
static void apply_inv(const orc_problem *pr, const cplx *Lm, const cplx *z, cplx *y, int64_t ld, int k) {
    int64_t rows = 2 * pr->M;
    if (!Lm) {
        for (int64_t r = 0; r < rows; ++r)
            for (int j = 0; j < k; ++j) y[r * ld + j] = z[r * ld + j] / pr->D[r / 2];
        return;
    }
    int64_t n = rows;
    cplx *t = malloc(sizeof(cplx) * n);
    for (int j = 0; j < k; ++j) {
        for (int64_t i = 0; i < n; ++i) {
            cplx s = z[i * ld + j];
            for (int64_t m = 0; m < i; ++m) s -= Lm[i * n + m] * t[m];
            t[i] = s / Lm[i * n + i];
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            cplx s = t[i];
            for (int64_t m = i + 1; m < n; ++m) s -= conj(Lm[m * n + i]) * y[m * ld + j];
            y[i * ld + j] = s / Lm[i * n + i];
        }
    }
    free(t);
}

/* R-ChFSI filter (eq. rChFSIrecurrence): given X (k columns), Ritz values
 * ritz, residual R = HX - MX Lambda and bounds (lmin, lT, lmax), compute
 *   Z_0 = 0, Z_1 = sigma_1 R / e, Lambda_0 = I, Lambda_1 = sigma_1 (Lambda - c)/e,
 *   Z_{k+1} = (2 s_{k+1}/e)(H D^{-1} Z_k - c Z_k) - s_k s_{k+1} Z_{k-1}
 *             + (2 s_{k+1}/e) R Lambda_k,
 *   Lambda_{k+1} = (2 s_{k+1}/e)(Lambda - c) Lambda_k - s_k s_{k+1} Lambda_{k-1},
 * and the recovery Y = D^{-1} Z_q + X Lambda_q.
 * If exactM != 0 (tiny meshes), D^{-1} is replaced by the exact M^{-1}. */
int orc_filter(void *vp, int degree, const double *bounds, const double *Xd, const double *ritz,
               const double *Rd, int64_t ld, int k, double *Yd, int exactM) {
    orc_problem *pr = (orc_problem *)vp;
    int64_t rows = 2 * pr->M;
    const cplx *X = (const cplx *)Xd, *R = (const cplx *)Rd;
    cplx *Y = (cplx *)Yd;
    double lmin = bounds[0], lT = bounds[1], lmax = bounds[2];
    double c = 0.5 * (lmax + lT), e = 0.5 * (lmax - lT);
    double s1 = e / (lmin - c);
    cplx *Lm = NULL;
    if (exactM) {
        cplx *Md = malloc(sizeof(cplx) * rows * rows);
        orc_dense(vp, NULL, (double *)Md, 0);
        Lm = malloc(sizeof(cplx) * rows * rows);
        int rc = orc_cholesky((int)rows, (double *)Md, (double *)Lm);
        free(Md);
        if (rc) { free(Lm); return -1; }
    }
    size_t sz = (size_t)rows * ld;
    cplx *Zm = calloc(sz, sizeof(cplx)), *Z = calloc(sz, sizeof(cplx)), *Zp = calloc(sz, sizeof(cplx));
    cplx *W = calloc(sz, sizeof(cplx)), *HW = calloc(sz, sizeof(cplx));
    double *Lkm = malloc(sizeof(double) * k), *Lk = malloc(sizeof(double) * k), *Lkp = malloc(sizeof(double) * k);
    for (int j = 0; j < k; ++j) { Lkm[j] = 1.0; Lk[j] = s1 * (ritz[j] - c) / e; }
    for (int64_t r = 0; r < rows; ++r)
        for (int j = 0; j < k; ++j) Z[r * ld + j] = s1 * R[r * ld + j] / e;
    double sk = s1;
    for (int step = 1; step < degree; ++step) {
        double sn = 1.0 / (2.0 / s1 - sk);
        apply_inv(pr, Lm, Z, W, ld, k);
        orc_apply_H(vp, (const double *)W, ld, k, (double *)HW, ld, ORC_ALL);
        double a = 2.0 * sn / e;
        for (int64_t r = 0; r < rows; ++r)
            for (int j = 0; j < k; ++j) {
                size_t o = r * ld + j;
                Zp[o] = a * (HW[o] - c * Z[o]) - sk * sn * Zm[o] + a * R[o] * Lk[j];
            }
        for (int j = 0; j < k; ++j) Lkp[j] = a * (ritz[j] - c) * Lk[j] - sk * sn * Lkm[j];
        cplx *t = Zm; Zm = Z; Z = Zp; Zp = t;
        double *tl = Lkm; Lkm = Lk; Lk = Lkp; Lkp = tl;
        sk = sn;
    }
    apply_inv(pr, Lm, Z, W, ld, k);
    for (int64_t r = 0; r < rows; ++r)
        for (int j = 0; j < k; ++j) Y[r * ld + j] = W[r * ld + j] + X[r * ld + j] * Lk[j];
    free(Zm); free(Z); free(Zp); free(W); free(HW); free(Lkm); free(Lk); free(Lkp); free(Lm);
    return 0;
}

/* Plain ChFSI filter (eq. ChFSIrecurrence) on the exact M^{-1}H (tiny meshes)
 * or on D^{-1}H: Y_0 = X, Y_1 = s1 (Minv H - c) X / e,
 * Y_{k+1} = (2 s_{k+1}/e)(Minv H - c) Y_k - s_k s_{k+1} Y_{k-1}. */
int orc_chebyshev_plain(void *vp, int degree, const double *bounds, const double *Xd,
                        int64_t ld, int k, double *Yd, int exactM) {
    orc_problem *pr = (orc_problem *)vp;
    int64_t rows = 2 * pr->M;
    double lmin = bounds[0], lT = bounds[1], lmax = bounds[2];
    double c = 0.5 * (lmax + lT), e = 0.5 * (lmax - lT);
    double s1 = e / (lmin - c);
    cplx *Lm = NULL;
    if (exactM) {
        cplx *Md = malloc(sizeof(cplx) * rows * rows);
        orc_dense(vp, NULL, (double *)Md, 0);
        Lm = malloc(sizeof(cplx) * rows * rows);
        int rc = orc_cholesky((int)rows, (double *)Md, (double *)Lm);
        free(Md);
        if (rc) { free(Lm); return -1; }
    }
    size_t sz = (size_t)rows * ld;
    cplx *Ym = malloc(sizeof(cplx) * sz), *Yc = malloc(sizeof(cplx) * sz), *Yn = malloc(sizeof(cplx) * sz);
    cplx *HY = malloc(sizeof(cplx) * sz), *W = malloc(sizeof(cplx) * sz);
    memcpy(Ym, Xd, sizeof(cplx) * sz);
    orc_apply_H(vp, (const double *)Ym, ld, k, (double *)HY, ld, ORC_ALL);
    apply_inv(pr, Lm, HY, W, ld, k);
    for (size_t o = 0; o < sz; ++o) Yc[o] = s1 * (W[o] - c * Ym[o]) / e;
    double sk = s1;
    for (int step = 1; step < degree; ++step) {
        double sn = 1.0 / (2.0 / s1 - sk);
        orc_apply_H(vp, (const double *)Yc, ld, k, (double *)HY, ld, ORC_ALL);
        apply_inv(pr, Lm, HY, W, ld, k);
        double a = 2.0 * sn / e;
        for (size_t o = 0; o < sz; ++o) Yn[o] = a * (W[o] - c * Yc[o]) - sk * sn * Ym[o];
        cplx *t = Ym; Ym = Yc; Yc = Yn; Yn = t;
        sk = sn;
    }
    memcpy(Yd, Yc, sizeof(cplx) * sz);
    free(Ym); free(Yc); free(Yn); free(HY); free(W); free(Lm);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* spectrum bound                                                            */
/* ------------------------------------------------------------------------ */

/* k-step Lanczos on the Hermitian D^{-1/2} H D^{-1/2} (similar to D^{-1} H)
 * from the start vector v0 (length 2M, complex).  Returns theta_max + |beta_k|
 * (an upper-bound estimate of the spectrum of D^{-1} H). */
double orc_lanczos(void *vp, int ksteps, const double *v0d) {
    orc_problem *pr = (orc_problem *)vp;
    int64_t N = 2 * pr->M;
    cplx *v = malloc(sizeof(cplx) * N), *vprev = calloc(N, sizeof(cplx));
    cplx *w = malloc(sizeof(cplx) * N), *t = malloc(sizeof(cplx) * N), *Ht = malloc(sizeof(cplx) * N);
    double *alpha = calloc(ksteps, sizeof(double)), *beta = calloc(ksteps + 1, sizeof(double));
    double nrm = 0;
    for (int64_t i = 0; i < N; ++i) { v[i] = ((const cplx *)v0d)[i]; nrm += creal(v[i] * conj(v[i])); }
    nrm = sqrt(nrm);
    for (int64_t i = 0; i < N; ++i) v[i] /= nrm;
    int m = 0;
    for (int j = 0; j < ksteps; ++j) {
        for (int64_t i = 0; i < N; ++i) t[i] = v[i] / sqrt(pr->D[i / 2]);
        orc_apply_H(vp, (const double *)t, 1, 1, (double *)Ht, 1, ORC_ALL);
        for (int64_t i = 0; i < N; ++i) w[i] = Ht[i] / sqrt(pr->D[i / 2]) - beta[j] * vprev[i];
        double a = 0;
        for (int64_t i = 0; i < N; ++i) a += creal(conj(v[i]) * w[i]);
        alpha[j] = a;
        double b = 0;
        for (int64_t i = 0; i < N; ++i) { w[i] -= a * v[i]; b += creal(w[i] * conj(w[i])); }
        b = sqrt(b);
        beta[j + 1] = b;
        m = j + 1;
        if (b == 0) break;
        for (int64_t i = 0; i < N; ++i) { vprev[i] = v[i]; v[i] = w[i] / b; }
    }
    cplx *T = calloc((size_t)m * m, sizeof(cplx)), *Q = malloc(sizeof(cplx) * m * m);
    double *ev = malloc(sizeof(double) * m);
    for (int i = 0; i < m; ++i) {
        T[i * m + i] = alpha[i];
        if (i + 1 < m) { T[i * m + i + 1] = beta[i + 1]; T[(i + 1) * m + i] = beta[i + 1]; }
    }
    orc_jacobi(m, (double *)T, ev, (double *)Q);
    double out = ev[m - 1] + fabs(beta[m]);
    free(v); free(vprev); free(w); free(t); free(Ht); free(alpha); free(beta); free(T); free(Q); free(ev);
    return out;
}

/* ------------------------------------------------------------------------ */
/* the eigensolver loop (Algorithm RChFSI)                                   */
/* ------------------------------------------------------------------------ */

/* Runs R-ChFSI (variant 0) or plain ChFSI with D^{-1} (variant 1) or with the
 * exact M^{-1} (variant 2, tiny meshes) from the start block X (k columns,
 * in/out).  Initial Ritz pairs: X <- orthonormalize(X), Rayleigh-Ritz.
 * Each iteration: residual, convergence test on the first n_wanted columns,
 * bounds lmin = Lambda_1, lT = Lambda_k, filter, H and M of the filtered
 * block, Cholesky-QR2, Rayleigh-Ritz.  Records per iteration the max residual
 * over the wanted columns (hist_res) and the Ritz values (hist_ritz[it][k]).
 * Returns the number of iterations (negative on breakdown). */
int orc_chfsi(void *vp, int variant, int k, int n_wanted, int degree, double lmax, double tol,
              int max_iter, double *Xd, int64_t ld, double *ritz, double *hist_res, double *hist_ritz) {
    orc_problem *pr = (orc_problem *)vp;
    int64_t rows = 2 * pr->M;
    size_t sz = (size_t)rows * ld;
    cplx *X = (cplx *)Xd;
    cplx *HX = calloc(sz, sizeof(cplx)), *MX = calloc(sz, sizeof(cplx)), *R = calloc(sz, sizeof(cplx));
    cplx *Yf = calloc(sz, sizeof(cplx));
    double *norms = malloc(sizeof(double) * k);
    orc_apply_H(vp, Xd, ld, k, (double *)HX, ld, ORC_ALL);
    orc_apply_M(vp, Xd, ld, k, (double *)MX, ld);
    if (orc_orthonormalize(vp, Xd, (double *)HX, (double *)MX, ld, k)) goto fail;
    orc_rayleigh_ritz(vp, Xd, (double *)HX, (double *)MX, ld, k, ritz);
    int it;
    for (it = 0; it < max_iter; ++it) {
        orc_residual(rows, k, (double *)HX, (double *)MX, ld, ritz, (double *)R, norms);
        double mx = 0;
        for (int j = 0; j < n_wanted; ++j) mx = norms[j] > mx ? norms[j] : mx;
        if (hist_res) hist_res[it] = mx;
        if (hist_ritz) memcpy(hist_ritz + (size_t)it * k, ritz, sizeof(double) * k);
        if (mx < tol) break;
        double bounds[3] = {ritz[0], ritz[k - 1], lmax};
        int rc;
        if (variant == 0) rc = orc_filter(vp, degree, bounds, Xd, ritz, (double *)R, ld, k, (double *)Yf, 0);
        else rc = orc_chebyshev_plain(vp, degree, bounds, Xd, ld, k, (double *)Yf, variant == 2);
        if (rc) goto fail;
        memcpy(X, Yf, sizeof(cplx) * sz);
        orc_apply_H(vp, Xd, ld, k, (double *)HX, ld, ORC_ALL);
        orc_apply_M(vp, Xd, ld, k, (double *)MX, ld);
        if (orc_orthonormalize(vp, Xd, (double *)HX, (double *)MX, ld, k)) goto fail;
        orc_rayleigh_ritz(vp, Xd, (double *)HX, (double *)MX, ld, k, ritz);
    }
    free(HX); free(MX); free(R); free(Yf); free(norms);
    return it;
fail:
    free(HX); free(MX); free(R); free(Yf); free(norms);
    return -1;
}
