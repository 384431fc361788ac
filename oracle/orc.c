/*
 * Oracle: plain FP64 element-by-element Gauss-quadrature assembly and
 * matrix-free product for tensor-product B-spline discretisations.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links this file;
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load it.  It shares no code with the GPU path.
 *
 * What it computes is the plain quadrature sum of the bilinear form
 * (Sec. 2, eq. (quadrature:1) with the convection-diffusion pull-back of
 * Example 1), element by element, with no sum factorisation:
 *
 *   mass      M[m][n] = sum_x  w(x) c(G(x)) |det J(x)| phi_n(x) phi_m(x)
 *   stiffness K[m][n] = sum_x  w(x) a(G(x)) |det J(x)|
 *                             (J^-T grad phi_n)(x) . A (J^-T grad phi_m)(x)
 *             (A a constant symmetric matrix, orc_set_diffusion; default I)
 *   convection B[m][n] = sum_x w(x) s(G(x)) |det J(x)|
 *                             (b . J^-T grad phi_n)(x) phi_m(x)
 *
 * (op 1, 2, 4).  The convection term is the b . grad u of the
 * convection-diffusion equation of Example 1, tested with v: the derivative
 * falls on the trial function n, the value on the test function m, so B is
 * not symmetric.  b is a constant vector (orc_set_convection) scaled by the
 * scalar coefficient s.
 *
 * with J_ik = dG_i / dxhat_k, G = sum_n c_n phi_n (Sec. 6.3).  Rows are test
 * functions m, columns trial functions n (Sec. 2, matrix definition), both
 * in lexicographic order with direction 1 fastest (Sec. 3.1).  The sparsity
 * pattern is the structural one: (m,n) is stored iff the supports share an
 * element (Sec. 3.2, set NZ), with explicit zeros kept.
 *
 * The caller supplies, per direction, the 1D tables at the Gauss points of
 * every element (values and first derivatives of the p active B-splines,
 * weights) and the index of the first active function of each element.
 * Those tables are produced on the Python side by the literal Cox-de Boor
 * recursion and numpy's Gauss-Legendre rule.
 *
 * Cost: O(N p^{3d}) for a full assembly, the standard method the paper
 * compares against (Sec. 1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EGEOM (-3)
#define ORC_ENOMEM (-4)

#define MAXD 3
#define MAXLOC 729 /* 9^3 active functions per element */

typedef struct {
    int d;
    int p[MAXD];      /* order per direction */
    int nel[MAXD];    /* elements per direction */
    int nfun[MAXD];   /* functions per direction */
    const int *first[MAXD];      /* [nel] first active function */
    const double *w[MAXD];       /* [nel][p] quadrature weights */
    const double *phi[MAXD];     /* [nel][p][p] phi[e][g][j] */
    const double *dphi[MAXD];    /* [nel][p][p] */
    const double *ctrl;          /* [N][d] */
    int coef_kind;               /* 0: constant coef_val, 1: 1+alpha*prod sin(2 pi x_i) */
    double coef_val;
    /* per direction, per function: first/last support element, first/last column */
    int *elo[MAXD], *ehi[MAXD], *clo[MAXD], *chi[MAXD];
    int64_t nfun_total;
} prob_t;

static void prob_free(prob_t *P)
{
    for (int k = 0; k < MAXD; ++k) {
        free(P->elo[k]); free(P->ehi[k]); free(P->clo[k]); free(P->chi[k]);
        P->elo[k] = P->ehi[k] = P->clo[k] = P->chi[k] = NULL;
    }
}

/* Unpack the flat, direction-concatenated tables into a problem record and
 * derive every function's support (elements whose active range contains it)
 * and its column range (union of the active ranges of those elements). */
static int prob_init(prob_t *P, int d, const int *p, const int *nel, const int *nfun,
                     const int *first, const double *w, const double *phi,
                     const double *dphi, const double *ctrl, int coef_kind,
                     double coef_val)
{
    memset(P, 0, sizeof(*P));
    if (d < 1 || d > MAXD) return ORC_EINVAL;
    P->d = d;
    P->ctrl = ctrl;
    P->coef_kind = coef_kind;
    P->coef_val = coef_val;
    P->nfun_total = 1;
    int64_t off_i = 0, off_w = 0, off_t = 0;
    int nloc = 1;
    for (int k = 0; k < d; ++k) {
        P->p[k] = p[k];
        P->nel[k] = nel[k];
        P->nfun[k] = nfun[k];
        P->first[k] = first + off_i;
        P->w[k] = w + off_w;
        P->phi[k] = phi + off_t;
        P->dphi[k] = dphi + off_t;
        off_i += nel[k];
        off_w += (int64_t)nel[k] * p[k];
        off_t += (int64_t)nel[k] * p[k] * p[k];
        P->nfun_total *= nfun[k];
        nloc *= p[k];
    }
    if (nloc > MAXLOC) return ORC_EINVAL;
    for (int k = 0; k < d; ++k) {
        int nf = P->nfun[k];
        P->elo[k] = malloc(sizeof(int) * nf);
        P->ehi[k] = malloc(sizeof(int) * nf);
        P->clo[k] = malloc(sizeof(int) * nf);
        P->chi[k] = malloc(sizeof(int) * nf);
        if (!P->elo[k] || !P->ehi[k] || !P->clo[k] || !P->chi[k]) { prob_free(P); return ORC_ENOMEM; }
        for (int i = 0; i < nf; ++i) {
            int lo = -1, hi = -1;
            for (int e = 0; e < P->nel[k]; ++e) {
                int f = P->first[k][e];
                if (f <= i && i <= f + P->p[k] - 1) {
                    if (lo < 0) lo = e;
                    hi = e;
                }
            }
            if (lo < 0) { prob_free(P); return ORC_EINVAL; } /* function with empty support */
            P->elo[k][i] = lo;
            P->ehi[k][i] = hi;
            P->clo[k][i] = P->first[k][lo];
            P->chi[k][i] = P->first[k][hi] + P->p[k] - 1;
        }
    }
    return ORC_OK;
}

/* Planted mistakes, for the tests that show the pins catch them (0 = none):
 * 1 pull-back with J^-1 in place of J^-T, 2 weight of the last direction
 * dropped, 3 |det J| dropped, 4 sign slip in one entry of the inverse,
 * 5 coefficient taken at the element centre instead of G(xhat). */
static int orc_defect = 0;

void orc_set_defect(int k) { orc_defect = k; }

/* the constant symmetric diffusion matrix A of the stiffness form (op 2),
 * row-major 3 x 3, its first d rows and columns used; default identity */
static double orc_diff_A[MAXD][MAXD] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
void orc_set_diffusion(const double *A9)
{
    for (int i = 0; i < MAXD; ++i)
        for (int j = 0; j < MAXD; ++j) orc_diff_A[i][j] = A9[3 * i + j];
}

/* g . A h over the first d components */
static inline double diff_dot(const prob_t *P, const double *g, const double *h)
{
    double t = 0.0;
    for (int i = 0; i < P->d; ++i)
        for (int j = 0; j < P->d; ++j) t += g[i] * orc_diff_A[i][j] * h[j];
    return t;
}

/* the constant vector b of the convection form (op 4) */
static double orc_conv_b[MAXD] = {0.0, 0.0, 0.0};
void orc_set_convection(double b1, double b2, double b3)
{
    orc_conv_b[0] = b1;
    orc_conv_b[1] = b2;
    orc_conv_b[2] = b3;
}

/* b . (J^-T grad_hat phi_l): the convection derivative of active function l */
static inline double conv_deriv(const prob_t *P, const double *grad)
{
    double t = 0.0;
    for (int i = 0; i < P->d; ++i) t += orc_conv_b[i] * grad[i];
    return t;
}

static double coefficient(const prob_t *P, const double *x)
{
    if (P->coef_kind == 0) return P->coef_val;
    double s = 1.0;
    for (int i = 0; i < P->d; ++i) s *= sin(2.0 * M_PI * x[i]);
    return 1.0 + P->coef_val * s;
}

/* Everything the quadrature sum needs at one Gauss point of one element. */
typedef struct {
    int nloc;
    int64_t gidx[MAXLOC];       /* global index of each active function */
    int lidx[MAXLOC][MAXD];     /* per-direction global index */
    double val[MAXLOC];         /* phi_n(x) */
    double grad[MAXLOC][MAXD];  /* J^-T grad_hat phi_n(x): physical gradient */
    double wdet;                /* w(x) |det J(x)| */
    double coef;                /* coefficient at G(x) */
    double xphys[MAXD];         /* G(x), the physical point */
} qp_t;

static int eval_qp(const prob_t *P, const int *e, const int *g, qp_t *Q)
{
    const int d = P->d;
    double wq = 1.0;
    for (int k = 0; k < d; ++k)
        if (!(orc_defect == 2 && k == d - 1)) wq *= P->w[k][e[k] * P->p[k] + g[k]];

    /* enumerate active functions lexicographically, direction 1 fastest */
    int nloc = 1;
    for (int k = 0; k < d; ++k) nloc *= P->p[k];
    Q->nloc = nloc;
    double ghat[MAXLOC][MAXD];
    for (int l = 0; l < nloc; ++l) {
        int rem = l;
        int64_t gi = 0, stride = 1;
        double v[MAXD], dv[MAXD];
        for (int k = 0; k < d; ++k) {
            int j = rem % P->p[k];
            rem /= P->p[k];
            int fi = P->first[k][e[k]] + j;
            Q->lidx[l][k] = fi;
            gi += (int64_t)fi * stride;
            stride *= P->nfun[k];
            int64_t t = ((int64_t)e[k] * P->p[k] + g[k]) * P->p[k] + j;
            v[k] = P->phi[k][t];
            dv[k] = P->dphi[k][t];
        }
        Q->gidx[l] = gi;
        double prod = 1.0;
        for (int k = 0; k < d; ++k) prod *= v[k];
        Q->val[l] = prod;
        for (int kk = 0; kk < d; ++kk) {
            double q = 1.0;
            for (int k = 0; k < d; ++k) q *= (k == kk) ? dv[k] : v[k];
            ghat[l][kk] = q;
        }
    }

    /* geometry: G(x) and J_ik = sum_n c_{n,i} d_k phi_n (Sec. 6.3) */
    double G[MAXD] = {0, 0, 0};
    double J[MAXD][MAXD] = {{0}};
    for (int l = 0; l < nloc; ++l) {
        const double *c = P->ctrl + Q->gidx[l] * d;
        for (int i = 0; i < d; ++i) {
            G[i] += c[i] * Q->val[l];
            for (int k = 0; k < d; ++k) J[i][k] += c[i] * ghat[l][k];
        }
    }
    double det, inv[MAXD][MAXD];
    if (d == 1) {
        det = J[0][0];
        if (!(det > 0.0)) return ORC_EGEOM;
        inv[0][0] = 1.0 / det;
    } else if (d == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        if (!(det > 0.0)) return ORC_EGEOM;
        inv[0][0] = J[1][1] / det;
        inv[0][1] = (orc_defect == 4 ? J[0][1] : -J[0][1]) / det;
        inv[1][0] = -J[1][0] / det;
        inv[1][1] = J[0][0] / det;
    } else {
        /* adjugate of J divided by its determinant */
        double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        if (!(det > 0.0)) return ORC_EGEOM;
        inv[0][0] = c00 / det;
        inv[1][0] = c01 / det;
        inv[2][0] = c02 / det;
        inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    }
    for (int i = 0; i < d; ++i) Q->xphys[i] = G[i];
    Q->wdet = orc_defect == 3 ? wq : wq * fabs(det);
    if (orc_defect == 5) {
        /* element centre of a uniform reference mesh, not G(xhat) */
        double xr[MAXD];
        for (int k = 0; k < d; ++k) xr[k] = (e[k] + 0.5) / P->nel[k];
        Q->coef = coefficient(P, xr);
    } else {
        Q->coef = coefficient(P, G);
    }
    /* physical gradient: (J^-T ghat)_i = sum_k inv[k][i] ghat_k */
    for (int l = 0; l < nloc; ++l)
        for (int i = 0; i < d; ++i) {
            double s = 0.0;
            for (int k = 0; k < d; ++k) s += (orc_defect == 1 ? inv[i][k] : inv[k][i]) * ghat[l][k];
            Q->grad[l][i] = s;
        }
    return ORC_OK;
}

static inline void unflatten(const prob_t *P, int64_t m, int *mi)
{
    for (int k = 0; k < P->d; ++k) {
        mi[k] = (int)(m % P->nfun[k]);
        m /= P->nfun[k];
    }
}

static inline int64_t row_len(const prob_t *P, const int *mi)
{
    int64_t len = 1;
    for (int k = 0; k < P->d; ++k) len *= P->chi[k][mi[k]] - P->clo[k][mi[k]] + 1;
    return len;
}

/* position of column n (per-direction indices ni) inside row m's column box */
static inline int64_t box_offset(const prob_t *P, const int *mi, const int *ni)
{
    int64_t off = 0;
    for (int k = P->d - 1; k >= 0; --k) {
        int len = P->chi[k][mi[k]] - P->clo[k][mi[k]] + 1;
        off = off * len + (ni[k] - P->clo[k][mi[k]]);
    }
    return off;
}

/* ---------------- exported entry points ---------------- */

#define PROB_ARGS int d, const int *p, const int *nel, const int *nfun, const int *first, \
                  const double *w, const double *phi, const double *dphi, const double *ctrl, \
                  int coef_kind, double coef_val
#define PROB_PASS d, p, nel, nfun, first, w, phi, dphi, ctrl, coef_kind, coef_val

/* Structural CSR pattern: row_ptr[N+1] (int64), col_ind[nnz] (int64). If
 * col_ind is NULL only row_ptr is filled (row_ptr[N] = nnz). */
int orc_pattern(PROB_ARGS, int64_t *row_ptr, int64_t *col_ind)
{
    prob_t P;
    int st = prob_init(&P, PROB_PASS);
    if (st) return st;
    int64_t N = P.nfun_total;
    row_ptr[0] = 0;
    for (int64_t m = 0; m < N; ++m) {
        int mi[MAXD];
        unflatten(&P, m, mi);
        row_ptr[m + 1] = row_ptr[m] + row_len(&P, mi);
    }
    if (col_ind) {
        for (int64_t m = 0; m < N; ++m) {
            int mi[MAXD], ni[MAXD] = {0, 0, 0};
            unflatten(&P, m, mi);
            int64_t len = row_len(&P, mi);
            for (int64_t t = 0; t < len; ++t) {
                int64_t rem = t, gi = 0, stride = 1;
                for (int k = 0; k < P.d; ++k) {
                    int lk = P.chi[k][mi[k]] - P.clo[k][mi[k]] + 1;
                    ni[k] = P.clo[k][mi[k]] + (int)(rem % lk);
                    rem /= lk;
                    gi += ni[k] * stride;
                    stride *= P.nfun[k];
                }
                col_ind[row_ptr[m] + t] = gi;
            }
        }
    }
    prob_free(&P);
    return ORC_OK;
}

/* Full element-by-element assembly into the oracle's own CSR pattern.
 * op = 1: mass, op = 2: stiffness.  vals has nnz entries; row_ptr from
 * orc_pattern.  Elements are processed in p^d colour classes (element index
 * modulo the order in every direction), so elements of one class share no
 * basis function and can be accumulated in parallel without races. */
int orc_assemble(PROB_ARGS, int op, const int64_t *row_ptr, double *vals, int nthreads)
{
    prob_t P;
    int st = prob_init(&P, PROB_PASS);
    if (st) return st;
    memset(vals, 0, sizeof(double) * row_ptr[P.nfun_total]);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int ncol = 1;
    for (int k = 0; k < P.d; ++k) ncol *= P.p[k];
    int64_t nel_total = 1;
    for (int k = 0; k < P.d; ++k) nel_total *= P.nel[k];
    int err = ORC_OK;
    for (int c = 0; c < ncol; ++c) {
        int col[MAXD] = {0, 0, 0};
        { int r = c; for (int k = 0; k < P.d; ++k) { col[k] = r % P.p[k]; r /= P.p[k]; } }
        #pragma omp parallel for schedule(dynamic, 4)
        for (int64_t el = 0; el < nel_total; ++el) {
            int e[MAXD] = {0, 0, 0};
            int64_t r = el;
            int skip = 0;
            for (int k = 0; k < P.d; ++k) {
                e[k] = (int)(r % P.nel[k]);
                r /= P.nel[k];
                if (e[k] % P.p[k] != col[k]) skip = 1;
            }
            if (skip) continue;
            qp_t *Q = malloc(sizeof(qp_t));
            int nqp = 1;
            for (int k = 0; k < P.d; ++k) nqp *= P.p[k];
            for (int q = 0; q < nqp; ++q) {
                int g[MAXD] = {0, 0, 0};
                int rr = q;
                for (int k = 0; k < P.d; ++k) { g[k] = rr % P.p[k]; rr /= P.p[k]; }
                if (eval_qp(&P, e, g, Q) != ORC_OK) {
                    #pragma omp atomic write
                    err = ORC_EGEOM;
                    break;
                }
                double s = Q->wdet * Q->coef;
                for (int a = 0; a < Q->nloc; ++a) {         /* test function m */
                    int64_t m = Q->gidx[a];
                    double *rowv = vals + row_ptr[m];
                    for (int b = 0; b < Q->nloc; ++b) {     /* trial function n */
                        double t;
                        if (op == 1) {
                            t = Q->val[b] * Q->val[a];
                        } else if (op == 4) {
                            t = orc_defect == 6 ? conv_deriv(&P, Q->grad[a]) * Q->val[b]
                                                : conv_deriv(&P, Q->grad[b]) * Q->val[a];
                        } else {
                            t = 0.0;
                            t = diff_dot(&P, Q->grad[b], Q->grad[a]);
                        }
                        rowv[box_offset(&P, Q->lidx[a], Q->lidx[b])] += s * t;
                    }
                }
            }
            free(Q);
        }
        if (err) break;
    }
    prob_free(&P);
    return err;
}

/* Selected rows only, for sizes where the full matrix is out of reach.
 * For every requested row m: cols[i*maxband + t], vals[i*maxband + t],
 * t < count[i], columns ascending; the sum runs over the elements of the
 * support of phi_m only. */
int orc_rows(PROB_ARGS, int op, int64_t nrows, const int64_t *rows, int maxband,
             int32_t *count, int64_t *cols, double *vals, int nthreads)
{
    prob_t P;
    int st = prob_init(&P, PROB_PASS);
    if (st) return st;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int err = ORC_OK;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nrows; ++i) {
        int mi[MAXD] = {0, 0, 0};
        unflatten(&P, rows[i], mi);
        int64_t len = row_len(&P, mi);
        if (len > maxband) {
            #pragma omp atomic write
            err = ORC_EINVAL;
            continue;
        }
        double *acc = vals + i * maxband;
        int64_t *cc = cols + i * maxband;
        for (int64_t t = 0; t < len; ++t) acc[t] = 0.0;
        /* columns */
        for (int64_t t = 0; t < len; ++t) {
            int64_t rem = t, gi = 0, stride = 1;
            for (int k = 0; k < P.d; ++k) {
                int lk = P.chi[k][mi[k]] - P.clo[k][mi[k]] + 1;
                gi += (P.clo[k][mi[k]] + rem % lk) * stride;
                rem /= lk;
                stride *= P.nfun[k];
            }
            cc[t] = gi;
        }
        count[i] = (int32_t)len;
        qp_t *Q = malloc(sizeof(qp_t));
        int ne[MAXD] = {1, 1, 1}, nqp = 1;
        for (int k = 0; k < P.d; ++k) {
            ne[k] = P.ehi[k][mi[k]] - P.elo[k][mi[k]] + 1;
            nqp *= P.p[k];
        }
        int ntup = ne[0] * ne[1] * ne[2];
        for (int et = 0; et < ntup && !err; ++et) {
            int e[MAXD] = {0, 0, 0};
            int r = et;
            for (int k = 0; k < P.d; ++k) { e[k] = P.elo[k][mi[k]] + r % ne[k]; r /= ne[k]; }
            for (int q = 0; q < nqp; ++q) {
                int g[MAXD] = {0, 0, 0};
                int rr = q;
                for (int k = 0; k < P.d; ++k) { g[k] = rr % P.p[k]; rr /= P.p[k]; }
                if (eval_qp(&P, e, g, Q) != ORC_OK) {
                    #pragma omp atomic write
                    err = ORC_EGEOM;
                    break;
                }
                /* locate the test function m among the active ones */
                int a = -1;
                for (int l = 0; l < Q->nloc; ++l) if (Q->gidx[l] == rows[i]) { a = l; break; }
                if (a < 0) continue;
                double s = Q->wdet * Q->coef;
                for (int b = 0; b < Q->nloc; ++b) {
                    double t;
                    if (op == 1) {
                        t = Q->val[b] * Q->val[a];
                    } else if (op == 4) {
                        t = conv_deriv(&P, Q->grad[b]) * Q->val[a];
                    } else {
                        t = 0.0;
                        t = diff_dot(&P, Q->grad[b], Q->grad[a]);
                    }
                    acc[box_offset(&P, mi, Q->lidx[b])] += s * t;
                }
            }
        }
        free(Q);
    }
    prob_free(&P);
    return err;
}

/* Matrix-free product for selected rows: y[i] = sum_x w c |detJ| (grad phi_m . grad u)
 * (or phi_m u for mass) with u = sum_n x_n phi_n evaluated at each Gauss point
 * directly (Sec. 3.3, matrix-free application). */
int orc_apply_rows(PROB_ARGS, int op, const double *x, int64_t nrows, const int64_t *rows,
                   double *y, int nthreads)
{
    prob_t P;
    int st = prob_init(&P, PROB_PASS);
    if (st) return st;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int err = ORC_OK;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nrows; ++i) {
        int mi[MAXD] = {0, 0, 0};
        unflatten(&P, rows[i], mi);
        qp_t *Q = malloc(sizeof(qp_t));
        int ne[MAXD] = {1, 1, 1}, nqp = 1;
        for (int k = 0; k < P.d; ++k) {
            ne[k] = P.ehi[k][mi[k]] - P.elo[k][mi[k]] + 1;
            nqp *= P.p[k];
        }
        double acc = 0.0;
        int ntup = ne[0] * ne[1] * ne[2];
        for (int et = 0; et < ntup; ++et) {
            int e[MAXD] = {0, 0, 0};
            int r = et;
            for (int k = 0; k < P.d; ++k) { e[k] = P.elo[k][mi[k]] + r % ne[k]; r /= ne[k]; }
            for (int q = 0; q < nqp; ++q) {
                int g[MAXD] = {0, 0, 0};
                int rr = q;
                for (int k = 0; k < P.d; ++k) { g[k] = rr % P.p[k]; rr /= P.p[k]; }
                if (eval_qp(&P, e, g, Q) != ORC_OK) {
                    #pragma omp atomic write
                    err = ORC_EGEOM;
                    break;
                }
                int a = -1;
                for (int l = 0; l < Q->nloc; ++l) if (Q->gidx[l] == rows[i]) { a = l; break; }
                if (a < 0) continue;
                double s = Q->wdet * Q->coef;
                if (op == 1) {
                    double u = 0.0;
                    for (int b = 0; b < Q->nloc; ++b) u += x[Q->gidx[b]] * Q->val[b];
                    acc += s * u * Q->val[a];
                } else if (op == 4) {
                    double bu = 0.0;
                    for (int b = 0; b < Q->nloc; ++b) bu += x[Q->gidx[b]] * conv_deriv(&P, Q->grad[b]);
                    acc += s * bu * Q->val[a];
                } else {
                    double gu[MAXD] = {0, 0, 0};
                    for (int b = 0; b < Q->nloc; ++b)
                        for (int k = 0; k < P.d; ++k) gu[k] += x[Q->gidx[b]] * Q->grad[b][k];
                    double t = 0.0;
                    t = diff_dot(&P, gu, Q->grad[a]);
                    acc += s * t;
                }
            }
        }
        y[i] = acc;
        free(Q);
    }
    prob_free(&P);
    return err;
}

/* Full matrix-free product, element by element (cost N p^{2d}); elements are
 * coloured as in orc_assemble so that the scatter into y is race free. */
int orc_apply(PROB_ARGS, int op, const double *x, double *y, int nthreads)
{
    prob_t P;
    int st = prob_init(&P, PROB_PASS);
    if (st) return st;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    memset(y, 0, sizeof(double) * P.nfun_total);
    int ncol = 1;
    for (int k = 0; k < P.d; ++k) ncol *= P.p[k];
    int64_t nel_total = 1;
    for (int k = 0; k < P.d; ++k) nel_total *= P.nel[k];
    int err = ORC_OK;
    for (int c = 0; c < ncol && !err; ++c) {
        int col[MAXD] = {0, 0, 0};
        { int r = c; for (int k = 0; k < P.d; ++k) { col[k] = r % P.p[k]; r /= P.p[k]; } }
        #pragma omp parallel for schedule(dynamic, 8)
        for (int64_t el = 0; el < nel_total; ++el) {
            int e[MAXD] = {0, 0, 0};
            int64_t r = el;
            int skip = 0;
            for (int k = 0; k < P.d; ++k) {
                e[k] = (int)(r % P.nel[k]);
                r /= P.nel[k];
                if (e[k] % P.p[k] != col[k]) skip = 1;
            }
            if (skip) continue;
            qp_t *Q = malloc(sizeof(qp_t));
            int nqp = 1;
            for (int k = 0; k < P.d; ++k) nqp *= P.p[k];
            for (int q = 0; q < nqp; ++q) {
                int g[MAXD] = {0, 0, 0};
                int rr = q;
                for (int k = 0; k < P.d; ++k) { g[k] = rr % P.p[k]; rr /= P.p[k]; }
                if (eval_qp(&P, e, g, Q) != ORC_OK) {
                    #pragma omp atomic write
                    err = ORC_EGEOM;
                    break;
                }
                double s = Q->wdet * Q->coef;
                if (op == 1) {
                    double u = 0.0;
                    for (int b = 0; b < Q->nloc; ++b) u += x[Q->gidx[b]] * Q->val[b];
                    for (int a = 0; a < Q->nloc; ++a) y[Q->gidx[a]] += s * u * Q->val[a];
                } else if (op == 4) {
                    double bu = 0.0;
                    for (int b = 0; b < Q->nloc; ++b) bu += x[Q->gidx[b]] * conv_deriv(&P, Q->grad[b]);
                    for (int a = 0; a < Q->nloc; ++a) y[Q->gidx[a]] += s * bu * Q->val[a];
                } else {
                    double gu[MAXD] = {0, 0, 0};
                    for (int b = 0; b < Q->nloc; ++b)
                        for (int k = 0; k < P.d; ++k) gu[k] += x[Q->gidx[b]] * Q->grad[b][k];
                    for (int a = 0; a < Q->nloc; ++a) {
                        double t = 0.0;
                        t = diff_dot(&P, gu, Q->grad[a]);
                        y[Q->gidx[a]] += s * t;
                    }
                }
            }
            free(Q);
        }
    }
    prob_free(&P);
    return err;
}

/* sum_x w |det J|: the measure of the physical domain under the rule. */
/* The element-by-element product of orc_apply restricted to a list of
 * elements (flattened, direction 1 fastest): y (length N, overwritten) gets
 * the contributions of those elements only.  A row m of A x is complete in y
 * when the list holds every element of supp phi_m; the Python side passes the
 * union of the supports of the rows it wants, so that rows near each other
 * share their elements' work. */
int orc_apply_elements(PROB_ARGS, int op, const double *x, int64_t nlist, const int64_t *elems,
                       double *y, int nthreads)
{
    prob_t P;
    int st = prob_init(&P, PROB_PASS);
    if (st) return st;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    memset(y, 0, sizeof(double) * P.nfun_total);
    int ncol = 1;
    for (int k = 0; k < P.d; ++k) ncol *= P.p[k];
    int err = ORC_OK;
    /* colour classes (e_k mod p_k): elements of one class share no function */
    for (int c = 0; c < ncol && !err; ++c) {
        int col[MAXD] = {0, 0, 0};
        { int r = c; for (int k = 0; k < P.d; ++k) { col[k] = r % P.p[k]; r /= P.p[k]; } }
        #pragma omp parallel for schedule(dynamic, 1)
        for (int64_t i = 0; i < nlist; ++i) {
            int e[MAXD] = {0, 0, 0};
            int64_t r = elems[i];
            int skip = 0;
            for (int k = 0; k < P.d; ++k) {
                e[k] = (int)(r % P.nel[k]);
                r /= P.nel[k];
                if (e[k] % P.p[k] != col[k]) skip = 1;
            }
            if (skip) continue;
            qp_t *Q = malloc(sizeof(qp_t));
            int nqp = 1;
            for (int k = 0; k < P.d; ++k) nqp *= P.p[k];
            for (int q = 0; q < nqp; ++q) {
                int g[MAXD] = {0, 0, 0};
                int rr = q;
                for (int k = 0; k < P.d; ++k) { g[k] = rr % P.p[k]; rr /= P.p[k]; }
                if (eval_qp(&P, e, g, Q) != ORC_OK) {
                    #pragma omp atomic write
                    err = ORC_EGEOM;
                    break;
                }
                double s = Q->wdet * Q->coef;
                if (op == 1) {
                    double u = 0.0;
                    for (int b = 0; b < Q->nloc; ++b) u += x[Q->gidx[b]] * Q->val[b];
                    for (int a = 0; a < Q->nloc; ++a) y[Q->gidx[a]] += s * u * Q->val[a];
                } else if (op == 4) {
                    double bu = 0.0;
                    for (int b = 0; b < Q->nloc; ++b) bu += x[Q->gidx[b]] * conv_deriv(&P, Q->grad[b]);
                    for (int a = 0; a < Q->nloc; ++a) y[Q->gidx[a]] += s * bu * Q->val[a];
                } else {
                    double gu[MAXD] = {0, 0, 0};
                    for (int b = 0; b < Q->nloc; ++b)
                        for (int k = 0; k < P.d; ++k) gu[k] += x[Q->gidx[b]] * Q->grad[b][k];
                    for (int a = 0; a < Q->nloc; ++a) {
                        double t = 0.0;
                        t = diff_dot(&P, gu, Q->grad[a]);
                        y[Q->gidx[a]] += s * t;
                    }
                }
            }
            free(Q);
        }
    }
    prob_free(&P);
    return err;
}

/* Values and physical gradients of u = sum_n u_n phi_n at every quadrature
 * point (the quantities Algorithm 3 produces, Sec. 6.2), by the plain sums
 * over the p^d active functions of the point's element: u(x) = sum u_n phi_n,
 * grad u = sum u_n J^-T grad_hat phi_n.  Points in lexicographic order,
 * quadrature direction 1 fastest; val [Q], grad [Q][d], xyz [Q][d] (the
 * physical points G(x)); any output may be NULL. */
int orc_eval(PROB_ARGS, const double *u, double *val, double *grad, double *xyz, int nthreads)
{
    prob_t P;
    int st = prob_init(&P, PROB_PASS);
    if (st) return st;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int64_t nel_total = 1;
    int nq[MAXD] = {1, 1, 1};
    for (int k = 0; k < P.d; ++k) {
        nel_total *= P.nel[k];
        nq[k] = P.nel[k] * P.p[k];
    }
    int err = ORC_OK;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t el = 0; el < nel_total; ++el) {
        int e[MAXD] = {0, 0, 0};
        int64_t r = el;
        for (int k = 0; k < P.d; ++k) {
            e[k] = (int)(r % P.nel[k]);
            r /= P.nel[k];
        }
        qp_t *Q = malloc(sizeof(qp_t));
        int nqp = 1;
        for (int k = 0; k < P.d; ++k) nqp *= P.p[k];
        for (int q = 0; q < nqp; ++q) {
            int g[MAXD] = {0, 0, 0};
            int rr = q;
            for (int k = 0; k < P.d; ++k) { g[k] = rr % P.p[k]; rr /= P.p[k]; }
            if (eval_qp(&P, e, g, Q) != ORC_OK) {
                #pragma omp atomic write
                err = ORC_EGEOM;
                break;
            }
            int64_t qlin = 0, stride = 1;
            for (int k = 0; k < P.d; ++k) {
                qlin += (int64_t)(e[k] * P.p[k] + g[k]) * stride;
                stride *= nq[k];
            }
            double v = 0.0, gu[MAXD] = {0, 0, 0};
            for (int b = 0; b < Q->nloc; ++b) {
                v += u[Q->gidx[b]] * Q->val[b];
                for (int k = 0; k < P.d; ++k) gu[k] += u[Q->gidx[b]] * Q->grad[b][k];
            }
            if (val) val[qlin] = v;
            for (int k = 0; k < P.d; ++k) {
                if (grad) grad[qlin * P.d + k] = gu[k];
                if (xyz) xyz[qlin * P.d + k] = Q->xphys[k];
            }
        }
        free(Q);
    }
    prob_free(&P);
    return err;
}

int orc_measure(PROB_ARGS, double *out)
{
    prob_t P;
    int st = prob_init(&P, PROB_PASS);
    if (st) return st;
    int64_t nel_total = 1;
    int nqp = 1;
    for (int k = 0; k < P.d; ++k) { nel_total *= P.nel[k]; nqp *= P.p[k]; }
    double total = 0.0;
    qp_t *Q = malloc(sizeof(qp_t));
    for (int64_t el = 0; el < nel_total && st == ORC_OK; ++el) {
        int e[MAXD] = {0, 0, 0};
        int64_t r = el;
        for (int k = 0; k < P.d; ++k) { e[k] = (int)(r % P.nel[k]); r /= P.nel[k]; }
        for (int q = 0; q < nqp; ++q) {
            int g[MAXD] = {0, 0, 0};
            int rr = q;
            for (int k = 0; k < P.d; ++k) { g[k] = rr % P.p[k]; rr /= P.p[k]; }
            st = eval_qp(&P, e, g, Q);
            if (st) break;
            total += Q->wdet;
        }
    }
    free(Q);
    prob_free(&P);
    *out = total;
    return st;
}
