/*
 * oracle.c -- plain, serial, double-precision reference implementation of the
 * two-level method for B-spline (isogeometric) discretisations of
 *
 *     -div(kappa grad u) = f  in (0,1)^d,   u = 0 on the boundary,
 *
 * from "A two level method for isogeometric discretizations"
 * (A. Pe de la Riva, C. Rodrigo, F. J. Gaspar; arXiv:2009.01499).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference against
 * which the GPU library is checked.  Only the test-suite, the smoke check and
 * the benchmark's CPU-baseline leg load it.  It shares no code, header, table
 * or generator with the GPU library, and the GPU library never calls it.
 *
 * Style: every routine states the definition it follows and computes it in
 * the most direct way (scalar loops, no blocking, no fusion, no reordering
 * beyond what the definition states).  Floating point is IEEE double.
 *
 * Storage conventions
 *   - DOFs are the interior (Dirichlet-reduced) tensor-product B-splines,
 *     numbered lexicographically with the x index fastest.  In one direction
 *     the interior functions are the full-basis functions 1..m+p-2 (0-based),
 *     i.e. the paper's N_2..N_{p+m-1} (Section 2.1, eq. splinespace).
 *   - A sparse operator whose entries couple index i with index i+o for
 *     o in [-q,q]^d is stored "by offset": S[row*W + oidx(o)], W=(2q+1)^d,
 *     oidx(o) = sum_k (o_k+q)(2q+1)^k.  Entries whose column falls outside
 *     the grid are zero.
 *
 * Functions without an independent pin are marked "parity unpinned" below;
 * at present there are none (see the test-suite for the pins).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

#define OR_MAXD 3

/* ------------------------------------------------------------------ */
/* error reporting                                                    */
/* ------------------------------------------------------------------ */
static char or_errbuf[256];
const char *or_last_error(void) { return or_errbuf; }
static int fail(const char *msg) {
    snprintf(or_errbuf, sizeof or_errbuf, "%s", msg);
    return -1;
}

/* ------------------------------------------------------------------ */
/* small multi-index helpers                                          */
/* ------------------------------------------------------------------ */
static long ipow(long b, int e) { long r = 1; while (e-- > 0) r *= b; return r; }

/* linear index -> multi-index, x fastest */
static void unravel(long idx, int d, long n1, int *ix) {
    for (int k = 0; k < d; k++) { ix[k] = (int)(idx % n1); idx /= n1; }
}
static long ravel(const int *ix, int d, long n1) {
    long r = 0;
    for (int k = d - 1; k >= 0; k--) r = r * n1 + ix[k];
    return r;
}
static int inside(const int *ix, int d, int n1) {
    for (int k = 0; k < d; k++) if (ix[k] < 0 || ix[k] >= n1) return 0;
    return 1;
}
/* offset index for o in [-q,q]^d */
static long oidx(const int *o, int d, int q) {
    long r = 0;
    for (int k = d - 1; k >= 0; k--) r = r * (2 * q + 1) + (o[k] + q);
    return r;
}

/* ------------------------------------------------------------------ */
/* knot vector and B-spline basis                                     */
/* ------------------------------------------------------------------ */

/* Open uniform knot vector of Section 2.1: p+1 zeros, the interior knots
 * i/m (i=1..m-1), p+1 ones.  Length 2p+m+1. */
int or_knots(int p, int m, double *t) {
    if (p < 0 || m < 1) return fail("or_knots: bad p or m");
    int k = 0;
    for (int i = 0; i <= p; i++) t[k++] = 0.0;
    for (int i = 1; i < m; i++) t[k++] = (double)i / (double)m;
    for (int i = 0; i <= p; i++) t[k++] = 1.0;
    return 0;
}

/* Cox-de Boor recursion, eqs. (constantspline) and (order_spline) of
 * Section 2.1, with 0-based indices: N_i^0 is the indicator of the half-open
 * span [t_i, t_{i+1}); fractions 0/0 are taken as zero. */
static double cox_de_boor(const double *t, int i, int k, double x) {
    if (k == 0) return (t[i] <= x && x < t[i + 1]) ? 1.0 : 0.0;
    double left = 0.0, right = 0.0;
    double d1 = t[i + k] - t[i];
    double d2 = t[i + k + 1] - t[i + 1];
    if (d1 != 0.0) left = (x - t[i]) / d1 * cox_de_boor(t, i, k - 1, x);
    if (d2 != 0.0) right = (t[i + k + 1] - x) / d2 * cox_de_boor(t, i + 1, k - 1, x);
    return left + right;
}

/* Derivative of N_i^k, the textbook formula obtained by differentiating the
 * recursion (the paper states none):
 *   N_i^k' = k/(t_{i+k}-t_i) N_i^{k-1} - k/(t_{i+k+1}-t_{i+1}) N_{i+1}^{k-1}
 * with 0/0 := 0. */
static double cox_de_boor_deriv(const double *t, int i, int k, double x) {
    if (k == 0) return 0.0;
    double left = 0.0, right = 0.0;
    double d1 = t[i + k] - t[i];
    double d2 = t[i + k + 1] - t[i + 1];
    if (d1 != 0.0) left = k / d1 * cox_de_boor(t, i, k - 1, x);
    if (d2 != 0.0) right = k / d2 * cox_de_boor(t, i + 1, k - 1, x);
    return left - right;
}

double or_bspline(const double *t, int p, int i, double x) { return cox_de_boor(t, i, p, x); }
double or_bspline_deriv(const double *t, int p, int i, double x) { return cox_de_boor_deriv(t, i, p, x); }

/* ------------------------------------------------------------------ */
/* Gauss-Legendre quadrature on [-1,1] (textbook: Newton on P_q)       */
/* ------------------------------------------------------------------ */

/* P_q(z) and P_{q-1}(z) by the three-term recurrence, q >= 1 */
static void legendre_pair(int q, double z, double *pq, double *pqm1) {
    double pk = z, pkm1 = 1.0;
    for (int k = 2; k <= q; k++) {
        double pn = ((2.0 * k - 1.0) * z * pk - (k - 1.0) * pkm1) / k;
        pkm1 = pk;
        pk = pn;
    }
    *pq = pk;
    *pqm1 = pkm1;
}

int or_gauss_legendre(int q, double *x, double *w) {
    if (q < 1 || q > 64) return fail("or_gauss_legendre: q out of range");
    for (int i = 0; i < q; i++) {
        double z = cos(M_PI * (i + 0.75) / (q + 0.5));
        double pq, pqm1, dp;
        for (int it = 0; it < 100; it++) {
            legendre_pair(q, z, &pq, &pqm1);
            dp = q * (z * pq - pqm1) / (z * z - 1.0);
            double dz = pq / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        legendre_pair(q, z, &pq, &pqm1);
        dp = q * (z * pq - pqm1) / (z * z - 1.0);
        x[q - 1 - i] = z;
        w[q - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Galerkin assembly by brute-force d-dimensional quadrature           */
/* ------------------------------------------------------------------ */

/* Evaluate, on element span e (0-based) and at parameter x, the p+1 full-basis
 * functions e..e+p that are non-zero there (open knots: on span e the live
 * functions are N_e..N_{e+p}). */
static void live_basis(const double *t, int p, int e, double x, double *val, double *der) {
    for (int a = 0; a <= p; a++) {
        val[a] = cox_de_boor(t, e + a, p, x);
        if (der) der[a] = cox_de_boor_deriv(t, e + a, p, x);
    }
}

enum { OR_STIFF = 0, OR_MASS = 1 };

/*
 * Assemble the stiffness (a(u,v) = int kappa grad u . grad v, Section 2, the
 * matrix A_p below eq. (approxvariational)) or the mass matrix
 * (int u v, Section 3.1.2) for degree p on the m^d uniform mesh.
 *
 *   dirichlet = 1 : interior functions only (the Dirichlet-reduced space of
 *                   eq. splinespace), n1 = m+p-2 per direction;
 *   dirichlet = 0 : all m+p functions (used only for invariant checks).
 *
 * kappa: per-element coefficient (x fastest), or NULL for kappa = 1.  Each
 * element integral is a tensor Gauss rule with p+1 points per direction,
 * which is exact for these polynomial integrands.  Output by offset, q=p.
 */
int or_assemble(int d, int p, int m, const double *kappa, int kind, int dirichlet, double *out) {
    if (d < 1 || d > OR_MAXD || p < 1 || m < 1) return fail("or_assemble: bad arguments");
    int nt = 2 * p + m + 1;
    double *t = malloc(sizeof(double) * nt);
    or_knots(p, m, t);
    int shift = dirichlet ? 1 : 0;
    int n1 = dirichlet ? m + p - 2 : m + p;
    long n = ipow(n1, d), W = ipow(2 * p + 1, d), ne = ipow(m, d);
    memset(out, 0, sizeof(double) * n * W);
    int q = p + 1;
    double gx[64], gw[64];
    or_gauss_legendre(q, gx, gw);
    double h = 1.0 / m;
    int nl = p + 1;                 /* live functions per direction */
    long nloc = ipow(nl, d), nqp = ipow(q, d);
    double *val = malloc(sizeof(double) * OR_MAXD * nl);
    double *der = malloc(sizeof(double) * OR_MAXD * nl);
    double *phi = malloc(sizeof(double) * nloc);
    double *grad = malloc(sizeof(double) * nloc * OR_MAXD);
    int e[OR_MAXD], qi[OR_MAXD], a[OR_MAXD], b[OR_MAXD], ia[OR_MAXD], ib[OR_MAXD], o[OR_MAXD];
    for (long el = 0; el < ne; el++) {
        unravel(el, d, m, e);
        double coef = kappa ? kappa[el] : 1.0;
        for (long qq = 0; qq < nqp; qq++) {
            unravel(qq, d, q, qi);
            double wq = 1.0;
            for (int k = 0; k < d; k++) {
                double x = (e[k] + 0.5 * (gx[qi[k]] + 1.0)) * h;
                wq *= 0.5 * h * gw[qi[k]];
                live_basis(t, p, e[k], x, val + k * nl, der + k * nl);
            }
            /* tensor-product basis values and gradients, Section 2.1 */
            for (long la = 0; la < nloc; la++) {
                unravel(la, d, nl, a);
                double v = 1.0;
                for (int k = 0; k < d; k++) v *= val[k * nl + a[k]];
                phi[la] = v;
                for (int c = 0; c < d; c++) {
                    double g = 1.0;
                    for (int k = 0; k < d; k++) g *= (k == c) ? der[k * nl + a[k]] : val[k * nl + a[k]];
                    grad[la * OR_MAXD + c] = g;
                }
            }
            for (long la = 0; la < nloc; la++) {
                unravel(la, d, nl, a);
                for (int k = 0; k < d; k++) ia[k] = e[k] + a[k] - shift;
                if (!inside(ia, d, n1)) continue;
                long row = ravel(ia, d, n1);
                for (long lb = 0; lb < nloc; lb++) {
                    unravel(lb, d, nl, b);
                    for (int k = 0; k < d; k++) ib[k] = e[k] + b[k] - shift;
                    if (!inside(ib, d, n1)) continue;
                    double integrand;
                    if (kind == OR_STIFF) {
                        integrand = 0.0;
                        for (int c = 0; c < d; c++) integrand += grad[la * OR_MAXD + c] * grad[lb * OR_MAXD + c];
                        integrand *= coef;
                    } else {
                        integrand = phi[la] * phi[lb];
                    }
                    for (int k = 0; k < d; k++) o[k] = ib[k] - ia[k];
                    out[row * W + oidx(o, d, p)] += wq * integrand;
                }
            }
        }
    }
    free(t); free(val); free(der); free(phi); free(grad);
    return 0;
}

/*
 * Mixed mass matrix M_p^{plow} of Section 3.1.2: entry (i,j) is the integral
 * of phi_i^{plow} phi_j^p over the domain, i a coarse (degree plow) interior
 * function and j a fine (degree p) interior function on the same knots.
 * Stored by offset j - i in [-plow, p]^d: out[i*Wm + sum_k (o_k+plow)(p+plow+1)^k].
 */
int or_assemble_mix(int d, int p, int plow, int m, double *out) {
    if (d < 1 || d > OR_MAXD || p < 1 || plow < 1 || plow > p || m < 1) return fail("or_assemble_mix: bad arguments");
    double *t = malloc(sizeof(double) * (2 * p + m + 1));
    double *tl = malloc(sizeof(double) * (2 * plow + m + 1));
    or_knots(p, m, t);
    or_knots(plow, m, tl);
    int n1 = m + p - 2, n1c = m + plow - 2;
    int wm = p + plow + 1;
    long nc = ipow(n1c, d), Wm = ipow(wm, d), ne = ipow(m, d);
    memset(out, 0, sizeof(double) * nc * Wm);
    int q = p + 1;
    double gx[64], gw[64];
    or_gauss_legendre(q, gx, gw);
    double h = 1.0 / m;
    int nl = p + 1, nlc = plow + 1;
    long nloc = ipow(nl, d), nlocc = ipow(nlc, d), nqp = ipow(q, d);
    double val[OR_MAXD * 16], valc[OR_MAXD * 16];
    int e[OR_MAXD], qi[OR_MAXD], a[OR_MAXD], b[OR_MAXD], ia[OR_MAXD], ib[OR_MAXD];
    for (long el = 0; el < ne; el++) {
        unravel(el, d, m, e);
        for (long qq = 0; qq < nqp; qq++) {
            unravel(qq, d, q, qi);
            double wq = 1.0;
            for (int k = 0; k < d; k++) {
                double x = (e[k] + 0.5 * (gx[qi[k]] + 1.0)) * h;
                wq *= 0.5 * h * gw[qi[k]];
                live_basis(t, p, e[k], x, val + k * nl, NULL);
                live_basis(tl, plow, e[k], x, valc + k * nlc, NULL);
            }
            for (long la = 0; la < nlocc; la++) {
                unravel(la, d, nlc, a);
                for (int k = 0; k < d; k++) ia[k] = e[k] + a[k] - 1;
                if (!inside(ia, d, n1c)) continue;
                double pa = 1.0;
                for (int k = 0; k < d; k++) pa *= valc[k * nlc + a[k]];
                long row = ravel(ia, d, n1c);
                for (long lb = 0; lb < nloc; lb++) {
                    unravel(lb, d, nl, b);
                    for (int k = 0; k < d; k++) ib[k] = e[k] + b[k] - 1;
                    if (!inside(ib, d, n1)) continue;
                    double pb = 1.0;
                    for (int k = 0; k < d; k++) pb *= val[k * nl + b[k]];
                    long off = 0;
                    for (int k = d - 1; k >= 0; k--) off = off * wm + (ib[k] - ia[k] + plow);
                    out[row * Wm + off] += wq * pa * pb;
                }
            }
        }
    }
    free(t); free(tl);
    return 0;
}

/*
 * Load vector b_i = (f, phi_i) for the manufactured right-hand side of the
 * square-domain experiment (Section 5.1) generalised to d dimensions:
 * f = d pi^2 prod_k sin(pi x_k), whose exact solution is prod_k sin(pi x_k).
 * Gauss rule with p+3 points per direction (f is not a polynomial).
 */
int or_load_manufactured(int d, int p, int m, double *bvec) {
    double *t = malloc(sizeof(double) * (2 * p + m + 1));
    or_knots(p, m, t);
    int n1 = m + p - 2;
    long n = ipow(n1, d), ne = ipow(m, d);
    memset(bvec, 0, sizeof(double) * n);
    int q = p + 3;
    double gx[64], gw[64];
    or_gauss_legendre(q, gx, gw);
    double h = 1.0 / m;
    int nl = p + 1;
    long nloc = ipow(nl, d), nqp = ipow(q, d);
    double val[OR_MAXD * 16], xq[OR_MAXD];
    int e[OR_MAXD], qi[OR_MAXD], a[OR_MAXD], ia[OR_MAXD];
    for (long el = 0; el < ne; el++) {
        unravel(el, d, m, e);
        for (long qq = 0; qq < nqp; qq++) {
            unravel(qq, d, q, qi);
            double wq = 1.0, f = d * M_PI * M_PI;
            for (int k = 0; k < d; k++) {
                xq[k] = (e[k] + 0.5 * (gx[qi[k]] + 1.0)) * h;
                wq *= 0.5 * h * gw[qi[k]];
                f *= sin(M_PI * xq[k]);
                live_basis(t, p, e[k], xq[k], val + k * nl, NULL);
            }
            for (long la = 0; la < nloc; la++) {
                unravel(la, d, nl, a);
                for (int k = 0; k < d; k++) ia[k] = e[k] + a[k] - 1;
                if (!inside(ia, d, n1)) continue;
                double ph = 1.0;
                for (int k = 0; k < d; k++) ph *= val[k * nl + a[k]];
                bvec[ravel(ia, d, n1)] += wq * f * ph;
            }
        }
    }
    free(t);
    return 0;
}

/*
 * L2 error of u_h = sum_i u_i phi_i against the exact solution prod sin(pi x_k)
 * of the manufactured problem (Section 5.1), Gauss rule with p+3 points.
 */
double or_l2_error_manufactured(int d, int p, int m, const double *u) {
    double *t = malloc(sizeof(double) * (2 * p + m + 1));
    or_knots(p, m, t);
    int n1 = m + p - 2;
    long ne = ipow(m, d);
    int q = p + 3;
    double gx[64], gw[64];
    or_gauss_legendre(q, gx, gw);
    double h = 1.0 / m;
    int nl = p + 1;
    long nloc = ipow(nl, d), nqp = ipow(q, d);
    double val[OR_MAXD * 16], xq[OR_MAXD];
    int e[OR_MAXD], qi[OR_MAXD], a[OR_MAXD], ia[OR_MAXD];
    double err2 = 0.0;
    for (long el = 0; el < ne; el++) {
        unravel(el, d, m, e);
        for (long qq = 0; qq < nqp; qq++) {
            unravel(qq, d, q, qi);
            double wq = 1.0, ex = 1.0;
            for (int k = 0; k < d; k++) {
                xq[k] = (e[k] + 0.5 * (gx[qi[k]] + 1.0)) * h;
                wq *= 0.5 * h * gw[qi[k]];
                ex *= sin(M_PI * xq[k]);
                live_basis(t, p, e[k], xq[k], val + k * nl, NULL);
            }
            double uh = 0.0;
            for (long la = 0; la < nloc; la++) {
                unravel(la, d, nl, a);
                for (int k = 0; k < d; k++) ia[k] = e[k] + a[k] - 1;
                if (!inside(ia, d, n1)) continue;
                double ph = 1.0;
                for (int k = 0; k < d; k++) ph *= val[k * nl + a[k]];
                uh += u[ravel(ia, d, n1)] * ph;
            }
            err2 += wq * (uh - ex) * (uh - ex);
        }
    }
    free(t);
    return sqrt(err2);
}

/* ------------------------------------------------------------------ */
/* operator application by offset storage                             */
/* ------------------------------------------------------------------ */

/* y = S x for an offset-stored operator of radius q on an n1^d grid. */
static void stencil_apply(int d, int n1, int q, const double *S, const double *x, double *y) {
    long n = ipow(n1, d), W = ipow(2 * q + 1, d);
    int ix[OR_MAXD], o[OR_MAXD], jx[OR_MAXD];
    for (long i = 0; i < n; i++) {
        unravel(i, d, n1, ix);
        double s = 0.0;
        for (long w = 0; w < W; w++) {
            unravel(w, d, 2 * q + 1, o);
            for (int k = 0; k < d; k++) { o[k] -= q; jx[k] = ix[k] + o[k]; }
            if (!inside(jx, d, n1)) continue;
            s += S[i * W + w] * x[ravel(jx, d, n1)];
        }
        y[i] = s;
    }
}

/* entry (i,j) of an offset-stored operator; 0 outside the stencil */
static double stencil_get(int d, int n1, int q, const double *S, long i, long j) {
    int ix[OR_MAXD], jx[OR_MAXD], o[OR_MAXD];
    unravel(i, d, n1, ix);
    unravel(j, d, n1, jx);
    for (int k = 0; k < d; k++) {
        o[k] = jx[k] - ix[k];
        if (o[k] < -q || o[k] > q) return 0.0;
    }
    return S[i * ipow(2 * q + 1, d) + oidx(o, d, q)];
}

/* ------------------------------------------------------------------ */
/* Cholesky factorisations (dense and banded), textbook                */
/* ------------------------------------------------------------------ */

/* in-place dense Cholesky of an n x n row-major SPD matrix (lower factor) */
static int dense_cholesky(int n, double *a) {
    for (int j = 0; j < n; j++) {
        double s = a[j * n + j];
        for (int k = 0; k < j; k++) s -= a[j * n + k] * a[j * n + k];
        if (!(s > 0.0)) return -1;
        double ljj = sqrt(s);
        a[j * n + j] = ljj;
        for (int i = j + 1; i < n; i++) {
            double t = a[i * n + j];
            for (int k = 0; k < j; k++) t -= a[i * n + k] * a[j * n + k];
            a[i * n + j] = t / ljj;
        }
        for (int i = 0; i < j; i++) a[i * n + j] = 0.0;
    }
    return 0;
}
/* solve L L^T x = b with the dense lower factor, in place on b */
static void dense_chol_solve(int n, const double *L, double *b) {
    for (int i = 0; i < n; i++) {
        double s = b[i];
        for (int k = 0; k < i; k++) s -= L[i * n + k] * b[k];
        b[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; i--) {
        double s = b[i];
        for (int k = i + 1; k < n; k++) s -= L[k * n + i] * b[k];
        b[i] = s / L[i * n + i];
    }
}

/* banded Cholesky: L(i,j) stored at L[i*(bw+1) + (i-j)] for 0 <= i-j <= bw */
typedef struct { long n, bw; double *L; } band_chol;

static void band_free(band_chol *c) { if (c) { free(c->L); free(c); } }

static band_chol *band_factor_stencil(int d, int n1, int q, const double *S) {
    long n = ipow(n1, d);
    long bw = 0;
    for (int k = 0; k < d; k++) bw += (long)q * ipow(n1, k);
    if (bw > n - 1) bw = n - 1;
    band_chol *c = malloc(sizeof *c);
    c->n = n; c->bw = bw;
    c->L = calloc((size_t)n * (bw + 1), sizeof(double));
    if (!c->L) { free(c); return NULL; }
    for (long i = 0; i < n; i++) {
        long j0 = i - bw < 0 ? 0 : i - bw;
        for (long j = j0; j <= i; j++) {
            double s = stencil_get(d, n1, q, S, i, j);
            long k0 = j0 > (j - bw) ? j0 : (j - bw);
            for (long k = k0; k < j; k++) s -= c->L[i * (bw + 1) + (i - k)] * c->L[j * (bw + 1) + (j - k)];
            if (j == i) {
                if (!(s > 0.0)) { band_free(c); return NULL; }
                c->L[i * (bw + 1)] = sqrt(s);
            } else {
                c->L[i * (bw + 1) + (i - j)] = s / c->L[j * (bw + 1)];
            }
        }
    }
    return c;
}
static void band_solve(const band_chol *c, double *x) {
    long n = c->n, bw = c->bw;
    for (long i = 0; i < n; i++) {
        double s = x[i];
        long k0 = i - bw < 0 ? 0 : i - bw;
        for (long k = k0; k < i; k++) s -= c->L[i * (bw + 1) + (i - k)] * x[k];
        x[i] = s / c->L[i * (bw + 1)];
    }
    for (long i = n - 1; i >= 0; i--) {
        double s = x[i];
        long k1 = i + bw > n - 1 ? n - 1 : i + bw;
        for (long k = i + 1; k <= k1; k++) s -= c->L[k * (bw + 1) + (k - i)] * x[k];
        x[i] = s / c->L[i * (bw + 1)];
    }
}

/* ------------------------------------------------------------------ */
/* the problem object                                                 */
/* ------------------------------------------------------------------ */
typedef struct {
    int m, n1;            /* n1 interior nodes per side; m = n1 + 1 */
    long n;
    double *S;            /* Q1 operator by offset, radius 1 */
    double *Sfact;        /* dense Cholesky at the coarsest level, else NULL */
} or_level;

typedef struct {
    int d, p, m, plow, bw, lumped;
    int n1, n1c;
    long n, nc, ne, W, Wc, Wm;
    double *kappa;
    double *A;            /* fine stiffness, radius p */
    double *Alow;         /* coarse stiffness, radius plow */
    double *Mlow;         /* coarse mass, radius plow */
    double *Mmix;         /* mixed mass, offsets [-plow,p]^d */
    double *Dlump;        /* row sums of Mlow */
    long *blk_off, *blk_idx, *chol_off;
    double *chol;
    band_chol *coarse_chol;     /* Alow */
    band_chol *mass_chol;       /* Mlow (exact, non-lumped variant) */
    band_chol *agg_chol;        /* degree-1 operator on the 2h grid (aggressive coarsening, exact) */
    int nlev;
    or_level *lev;        /* V-cycle hierarchy for plow = 1 */
} or_problem;

void or_destroy(or_problem *P) {
    if (!P) return;
    free(P->kappa); free(P->A); free(P->Alow); free(P->Mlow); free(P->Mmix); free(P->Dlump);
    free(P->blk_off); free(P->blk_idx); free(P->chol_off); free(P->chol);
    band_free(P->coarse_chol); band_free(P->mass_chol); band_free(P->agg_chol);
    for (int l = 0; l < P->nlev; l++) { free(P->lev[l].S); free(P->lev[l].Sfact); }
    free(P->lev);
    free(P);
}

/* block width chosen per degree as in Sections 3.1.1 / 4.2 / 5.1:
 * 3x3 blocks for p=2..4, 5x5 for p=5,6, 7x7 for p=7,8 (p=1: 3x3). */
int or_default_block_width(int p) {
    if (p <= 4) return 3;
    if (p <= 6) return 5;
    return 7;
}

/*
 * Blocks of the multiplicative Schwarz smoother with maximum overlap
 * (Section 3.1.1): one block per DOF j, made of the DOFs k with
 * |k_c - j_c| <= (bw-1)/2 in every direction, truncated to the interior
 * DOFs, in lexicographic order.  A^{B_j} = V_j A V_j^T is factorised by a
 * dense Cholesky for later local solves.
 */
static int build_blocks(or_problem *P) {
    int d = P->d, n1 = P->n1, hb = (P->bw - 1) / 2;
    long n = P->n;
    long maxnb = ipow(P->bw, d);
    P->blk_off = malloc(sizeof(long) * (n + 1));
    P->chol_off = malloc(sizeof(long) * (n + 1));
    P->blk_off[0] = 0; P->chol_off[0] = 0;
    int jx[OR_MAXD], kx[OR_MAXD], o[OR_MAXD];
    for (long j = 0; j < n; j++) {
        unravel(j, d, n1, jx);
        long cnt = 0;
        for (long w = 0; w < maxnb; w++) {
            unravel(w, d, P->bw, o);
            for (int k = 0; k < d; k++) kx[k] = jx[k] + o[k] - hb;
            if (inside(kx, d, n1)) cnt++;
        }
        P->blk_off[j + 1] = P->blk_off[j] + cnt;
        P->chol_off[j + 1] = P->chol_off[j] + cnt * cnt;
    }
    P->blk_idx = malloc(sizeof(long) * P->blk_off[n]);
    P->chol = malloc(sizeof(double) * P->chol_off[n]);
    if (!P->blk_idx || !P->chol) return fail("build_blocks: out of memory");
    for (long j = 0; j < n; j++) {
        unravel(j, d, n1, jx);
        long c = P->blk_off[j];
        for (long w = 0; w < maxnb; w++) {
            unravel(w, d, P->bw, o);
            for (int k = 0; k < d; k++) kx[k] = jx[k] + o[k] - hb;
            if (inside(kx, d, n1)) P->blk_idx[c++] = ravel(kx, d, n1);
        }
        int nb = (int)(P->blk_off[j + 1] - P->blk_off[j]);
        const long *idx = P->blk_idx + P->blk_off[j];
        double *a = P->chol + P->chol_off[j];
        for (int r = 0; r < nb; r++)
            for (int s = 0; s < nb; s++) a[r * nb + s] = stencil_get(d, n1, P->p, P->A, idx[r], idx[s]);
        if (dense_cholesky(nb, a)) return fail("build_blocks: block matrix not positive definite");
    }
    return 0;
}

/*
 * V-cycle hierarchy for the degree-1 coarse problem (Section 3.2): level 0 is
 * A_{plow} itself.  The paper fixes only "standard" h -> 2h coarsening and
 * analyses three grids; the reading used here, which needs no assumption on
 * m, is: the coarse nodes of a level are its odd-indexed interior nodes
 * (0-based) in every direction, P is linear interpolation between them (the
 * boundary value being zero), the coarse operator is the Galerkin product
 * P^T A P, and coarsening stops at the first level with at most
 * OR_COARSEST_MAX unknowns, which is solved exactly.  For m a power of two
 * this is standard full coarsening of the uniform mesh (and P^T A P equals
 * rediscretisation for kappa = 1); for other m the last coarse cell next to
 * the boundary is narrower.
 */
#ifndef OR_COARSEST_MAX
#define OR_COARSEST_MAX 512
#endif
static double interp_weight(int i_fine, int I_coarse) {
    /* fine interior node i sits at grid node i+1, coarse node I at fine grid
     * node 2(I+1), i.e. fine interior index 2I+1 */
    int dist = i_fine - (2 * I_coarse + 1);
    if (dist == 0) return 1.0;
    if (dist == 1 || dist == -1) return 0.5;
    return 0.0;
}

static int build_levels(or_problem *P) {
    int d = P->d;
    int nl = 1, nn = P->m - 1;
    while (ipow(nn, d) > OR_COARSEST_MAX) { nn /= 2; nl++; }
    P->nlev = nl;
    P->lev = calloc(nl, sizeof(or_level));
    long W3 = ipow(3, d);
    P->lev[0].m = P->m; P->lev[0].n1 = P->m - 1; P->lev[0].n = ipow(P->m - 1, d);
    P->lev[0].S = malloc(sizeof(double) * P->lev[0].n * W3);
    memcpy(P->lev[0].S, P->Alow, sizeof(double) * P->lev[0].n * W3);
    int ix[OR_MAXD], IX[OR_MAXD], a[OR_MAXD], jx[OR_MAXD], o[OR_MAXD], JX[OR_MAXD], bb[OR_MAXD], oc[OR_MAXD];
    for (int l = 1; l < nl; l++) {
        or_level *F = &P->lev[l - 1], *C = &P->lev[l];
        C->n1 = F->n1 / 2; C->m = C->n1 + 1; C->n = ipow(C->n1, d);
        C->S = calloc(C->n * W3, sizeof(double));
        /* A_c(I,J) = sum_{i,j} P(i,I) A_f(i,j) P(j,J) */
        for (long I = 0; I < C->n; I++) {
            unravel(I, d, C->n1, IX);
            for (long ai = 0; ai < W3; ai++) {          /* fine i near 2I+1 */
                unravel(ai, d, 3, a);
                double wI = 1.0;
                for (int k = 0; k < d; k++) { ix[k] = 2 * IX[k] + 1 + a[k] - 1; wI *= interp_weight(ix[k], IX[k]); }
                if (!inside(ix, d, F->n1) || wI == 0.0) continue;
                long i = ravel(ix, d, F->n1);
                for (long w = 0; w < W3; w++) {           /* fine j = i + o */
                    unravel(w, d, 3, o);
                    for (int k = 0; k < d; k++) jx[k] = ix[k] + o[k] - 1;
                    if (!inside(jx, d, F->n1)) continue;
                    double aij = F->S[i * W3 + w];
                    if (aij == 0.0) continue;
                    for (long bj = 0; bj < W3; bj++) {      /* coarse J near I */
                        unravel(bj, d, 3, bb);
                        double wJ = 1.0;
                        for (int k = 0; k < d; k++) { JX[k] = IX[k] + bb[k] - 1; }
                        if (!inside(JX, d, C->n1)) continue;
                        for (int k = 0; k < d; k++) wJ *= interp_weight(jx[k], JX[k]);
                        if (wJ == 0.0) continue;
                        for (int k = 0; k < d; k++) oc[k] = bb[k] - 1;
                        C->S[I * W3 + oidx(oc, d, 1)] += wI * aij * wJ;
                    }
                }
            }
        }
    }
    /* coarsest level: dense Cholesky */
    or_level *Z = &P->lev[nl - 1];
    long nz = Z->n;
    Z->Sfact = malloc(sizeof(double) * nz * nz);
    for (long i = 0; i < nz; i++)
        for (long j = 0; j < nz; j++) Z->Sfact[i * nz + j] = stencil_get(d, Z->n1, 1, Z->S, i, j);
    if (dense_cholesky((int)nz, Z->Sfact)) return fail("build_levels: coarsest matrix not SPD");
    return 0;
}

/*
 * Create the problem: assemble A_p (Section 2), A_{plow}, M_{plow}^{plow},
 * M_p^{plow} (Section 3.1.2), the lumped diagonal (row-sum lumping of
 * M_{plow}^{plow}, Section 3.1.2), the Schwarz blocks (Section 3.1.1), the
 * coarse factorisations and, for plow = 1, the V-cycle hierarchy.
 *   block_width = 0 selects the paper's choice per p.
 *   want_coarse_direct / want_vcycle control which coarse set-ups are built.
 */
or_problem *or_create(int d, int p, int m, const double *kappa, int plow, int block_width,
                      int lumped, int want_coarse_direct, int want_vcycle) {
    if (d < 1 || d > OR_MAXD || p < 1 || p > 8 || m < 2 || plow < 1 || plow > p) { fail("or_create: bad arguments"); return NULL; }
    if (block_width < 0 || (block_width && block_width % 2 == 0)) { fail("or_create: block width must be odd"); return NULL; }
    if (want_vcycle && plow != 1) { fail("or_create: the V-cycle needs plow = 1"); return NULL; }
    or_problem *P = calloc(1, sizeof *P);
    P->d = d; P->p = p; P->m = m; P->plow = plow;
    P->bw = block_width ? block_width : or_default_block_width(p);
    P->lumped = lumped;
    P->n1 = m + p - 2; P->n1c = m + plow - 2;
    P->n = ipow(P->n1, d); P->nc = ipow(P->n1c, d); P->ne = ipow(m, d);
    P->W = ipow(2 * p + 1, d); P->Wc = ipow(2 * plow + 1, d); P->Wm = ipow(p + plow + 1, d);
    if (P->n1 < 1 || P->n1c < 1) { fail("or_create: mesh too small"); free(P); return NULL; }
    P->kappa = malloc(sizeof(double) * P->ne);
    for (long e = 0; e < P->ne; e++) {
        P->kappa[e] = kappa ? kappa[e] : 1.0;
        if (!(P->kappa[e] > 0.0) || !isfinite(P->kappa[e])) { fail("or_create: kappa must be positive and finite"); or_destroy(P); return NULL; }
    }
    P->A = malloc(sizeof(double) * P->n * P->W);
    P->Alow = malloc(sizeof(double) * P->nc * P->Wc);
    P->Mlow = malloc(sizeof(double) * P->nc * P->Wc);
    P->Mmix = malloc(sizeof(double) * P->nc * P->Wm);
    P->Dlump = malloc(sizeof(double) * P->nc);
    if (!P->A || !P->Alow || !P->Mlow || !P->Mmix || !P->Dlump) { fail("or_create: out of memory"); or_destroy(P); return NULL; }
    or_assemble(d, p, m, P->kappa, OR_STIFF, 1, P->A);
    or_assemble(d, plow, m, P->kappa, OR_STIFF, 1, P->Alow);
    or_assemble(d, plow, m, NULL, OR_MASS, 1, P->Mlow);
    or_assemble_mix(d, p, plow, m, P->Mmix);
    for (long i = 0; i < P->nc; i++) {
        double s = 0.0;
        for (long w = 0; w < P->Wc; w++) s += P->Mlow[i * P->Wc + w];
        P->Dlump[i] = s;
    }
    if (build_blocks(P)) { or_destroy(P); return NULL; }
    if (want_coarse_direct) {
        P->coarse_chol = band_factor_stencil(d, P->n1c, plow, P->Alow);
        if (!P->coarse_chol) { fail("or_create: coarse factorisation failed"); or_destroy(P); return NULL; }
    }
    if (!lumped) {
        P->mass_chol = band_factor_stencil(d, P->n1c, plow, P->Mlow);
        if (!P->mass_chol) { fail("or_create: mass factorisation failed"); or_destroy(P); return NULL; }
    }
    if (want_vcycle) {
        if (build_levels(P)) { or_destroy(P); return NULL; }
    }
    return P;
}

long or_n(const or_problem *P) { return P->n; }
long or_nc(const or_problem *P) { return P->nc; }
long or_ne(const or_problem *P) { return P->ne; }
int or_block_width(const or_problem *P) { return P->bw; }
int or_nlevels(const or_problem *P) { return P->nlev; }

/* copies of the assembled operators (offset storage) */
void or_get_A(const or_problem *P, double *out) { memcpy(out, P->A, sizeof(double) * P->n * P->W); }
void or_get_Alow(const or_problem *P, double *out) { memcpy(out, P->Alow, sizeof(double) * P->nc * P->Wc); }
void or_get_Mlow(const or_problem *P, double *out) { memcpy(out, P->Mlow, sizeof(double) * P->nc * P->Wc); }
void or_get_Mmix(const or_problem *P, double *out) { memcpy(out, P->Mmix, sizeof(double) * P->nc * P->Wm); }
void or_get_Dlump(const or_problem *P, double *out) { memcpy(out, P->Dlump, sizeof(double) * P->nc); }
long or_level_n(const or_problem *P, int l) { return P->lev[l].n; }
void or_get_level(const or_problem *P, int l, double *out) {
    memcpy(out, P->lev[l].S, sizeof(double) * P->lev[l].n * ipow(3, P->d));
}

/* ------------------------------------------------------------------ */
/* fine-level operations                                              */
/* ------------------------------------------------------------------ */

void or_apply_A(const or_problem *P, const double *x, double *y) { stencil_apply(P->d, P->n1, P->p, P->A, x, y); }

/* defect d = b - A u (Algorithm 1, second step) */
void or_residual(const or_problem *P, const double *u, const double *b, double *r) {
    stencil_apply(P->d, P->n1, P->p, P->A, u, r);
    for (long i = 0; i < P->n; i++) r[i] = b[i] - r[i];
}

/* residual restricted to one row: b_i - (A u)_i */
static double residual_row(const or_problem *P, const double *u, const double *b, long i) {
    int d = P->d, n1 = P->n1, p = P->p;
    int ix[OR_MAXD], jx[OR_MAXD], o[OR_MAXD];
    unravel(i, d, n1, ix);
    double s = 0.0;
    for (long w = 0; w < P->W; w++) {
        unravel(w, d, 2 * p + 1, o);
        for (int k = 0; k < d; k++) jx[k] = ix[k] + o[k] - p;
        if (!inside(jx, d, n1)) continue;
        s += P->A[i * P->W + w] * u[ravel(jx, d, n1)];
    }
    return b[i] - s;
}

/* colour of block j under COLOUR(s): sum_k (j_k mod s) s^k */
static long block_colour(const or_problem *P, long j, int s) {
    int jx[OR_MAXD];
    unravel(j, P->d, P->n1, jx);
    long c = 0;
    for (int k = P->d - 1; k >= 0; k--) c = c * s + (jx[k] % s);
    return c;
}

/*
 * One sweep of the multiplicative Schwarz smoother (Section 3.1.1): the
 * iteration matrix is the ordered product over blocks of
 * (I - V_j^T (A^{B_j})^{-1} V_j A).
 *
 * The blocks are grouped into an ordered list of classes:
 *   ordering 0 (lexicographic): every block is its own class, in global
 *       index order -- the product formula taken literally;
 *   ordering 1 (coloured, period s >= block width): class c holds the
 *       blocks whose index satisfies sum_k (j_k mod s) s^k = c, c = 0..s^d-1.
 * Within a class all block corrections are computed from the iterate at the
 * start of the class and then added; for s >= block width the blocks of a
 * class are disjoint.  (The paper's three-colour ordering is defined only in
 * its reference [nuestropaper2018]; this parameterised colouring is the
 * reading used throughout.)
 */
int or_sweep(const or_problem *P, double *u, const double *b, int ordering, int s) {
    long n = P->n;
    if (ordering == 0) {
        double rb[400];
        for (long j = 0; j < n; j++) {
            int nb = (int)(P->blk_off[j + 1] - P->blk_off[j]);
            const long *idx = P->blk_idx + P->blk_off[j];
            for (int r = 0; r < nb; r++) rb[r] = residual_row(P, u, b, idx[r]);
            dense_chol_solve(nb, P->chol + P->chol_off[j], rb);
            for (int r = 0; r < nb; r++) u[idx[r]] += rb[r];
        }
        return 0;
    }
    if (ordering != 1) return fail("or_sweep: unknown ordering");
    if (s < P->bw) return fail("or_sweep: colour period must be >= block width");
    long ncol = ipow(s, P->d);
    long *members = malloc(sizeof(long) * n);
    double *corr = malloc(sizeof(double) * P->blk_off[n]);
    for (long c = 0; c < ncol; c++) {
        long cnt = 0;
        for (long j = 0; j < n; j++) if (block_colour(P, j, s) == c) members[cnt++] = j;
        /* all corrections from the class-start iterate ... */
        for (long t = 0; t < cnt; t++) {
            long j = members[t];
            int nb = (int)(P->blk_off[j + 1] - P->blk_off[j]);
            const long *idx = P->blk_idx + P->blk_off[j];
            double *rb = corr + P->blk_off[j];
            for (int r = 0; r < nb; r++) rb[r] = residual_row(P, u, b, idx[r]);
            dense_chol_solve(nb, P->chol + P->chol_off[j], rb);
        }
        /* ... then added */
        for (long t = 0; t < cnt; t++) {
            long j = members[t];
            int nb = (int)(P->blk_off[j + 1] - P->blk_off[j]);
            const long *idx = P->blk_idx + P->blk_off[j];
            const double *rb = corr + P->blk_off[j];
            for (int r = 0; r < nb; r++) u[idx[r]] += rb[r];
        }
    }
    free(members); free(corr);
    return 0;
}

/* ------------------------------------------------------------------ */
/* transfers (Section 3.1.2)                                          */
/* ------------------------------------------------------------------ */

/* y_c = M_p^{plow} x_f */
static void mix_apply(const or_problem *P, const double *xf, double *yc) {
    int d = P->d, wm = P->p + P->plow + 1;
    int IX[OR_MAXD], o[OR_MAXD], jx[OR_MAXD];
    for (long I = 0; I < P->nc; I++) {
        unravel(I, d, P->n1c, IX);
        double s = 0.0;
        for (long w = 0; w < P->Wm; w++) {
            unravel(w, d, wm, o);
            for (int k = 0; k < d; k++) jx[k] = IX[k] + o[k] - P->plow;
            if (!inside(jx, d, P->n1)) continue;
            s += P->Mmix[I * P->Wm + w] * xf[ravel(jx, d, P->n1)];
        }
        yc[I] = s;
    }
}
/* y_f += (M_p^{plow})^T x_c */
static void mix_apply_transpose_add(const or_problem *P, const double *xc, double *yf) {
    int d = P->d, wm = P->p + P->plow + 1;
    int IX[OR_MAXD], o[OR_MAXD], jx[OR_MAXD];
    for (long I = 0; I < P->nc; I++) {
        unravel(I, d, P->n1c, IX);
        for (long w = 0; w < P->Wm; w++) {
            unravel(w, d, wm, o);
            for (int k = 0; k < d; k++) jx[k] = IX[k] + o[k] - P->plow;
            if (!inside(jx, d, P->n1)) continue;
            yf[ravel(jx, d, P->n1)] += P->Mmix[I * P->Wm + w] * xc[I];
        }
    }
}

/* restriction I_p^{plow} = (M_{plow}^{plow})^{-1} M_p^{plow}; the inverse is
 * replaced by the row-sum lumped diagonal when lumped = 1 */
void or_restrict(const or_problem *P, const double *df, double *dc) {
    mix_apply(P, df, dc);
    if (P->lumped) {
        for (long I = 0; I < P->nc; I++) dc[I] /= P->Dlump[I];
    } else {
        band_solve(P->mass_chol, dc);
    }
}

/* prolongation I_{plow}^p = (M_p^{plow})^T (M_{plow}^{plow})^{-T}, the
 * adjoint of the restriction; uf += I_{plow}^p ec */
void or_prolong_add(const or_problem *P, const double *ec, double *uf) {
    double *tmp = malloc(sizeof(double) * P->nc);
    memcpy(tmp, ec, sizeof(double) * P->nc);
    if (P->lumped) {
        for (long I = 0; I < P->nc; I++) tmp[I] /= P->Dlump[I];
    } else {
        band_solve(P->mass_chol, tmp);
    }
    mix_apply_transpose_add(P, tmp, uf);
    free(tmp);
}

/* ------------------------------------------------------------------ */
/* coarse level (Sections 3.1, 3.2)                                   */
/* ------------------------------------------------------------------ */

/* exact solve A_{plow} e = d by banded Cholesky */
int or_coarse_direct(const or_problem *P, const double *dc, double *ec) {
    if (!P->coarse_chol) return fail("or_coarse_direct: not set up");
    memcpy(ec, dc, sizeof(double) * P->nc);
    band_solve(P->coarse_chol, ec);
    return 0;
}

/* red-black Gauss-Seidel on a Q1 level: first all red nodes (sum of indices
 * even), each updated from the iterate at the start of the half step, then
 * all black nodes the same way */
static void rbgs(const or_problem *P, const or_level *L, double *e, const double *rhs) {
    int d = P->d;
    long W3 = ipow(3, d);
    long c0 = (W3 - 1) / 2;
    double *enew = malloc(sizeof(double) * L->n);
    double *r = malloc(sizeof(double) * L->n);
    int ix[OR_MAXD];
    for (int colour = 0; colour < 2; colour++) {
        stencil_apply(d, L->n1, 1, L->S, e, r);
        memcpy(enew, e, sizeof(double) * L->n);
        for (long i = 0; i < L->n; i++) {
            unravel(i, d, L->n1, ix);
            int par = 0;
            for (int k = 0; k < d; k++) par += ix[k];
            if ((par & 1) != colour) continue;
            enew[i] = e[i] + (rhs[i] - r[i]) / L->S[i * W3 + c0];
        }
        memcpy(e, enew, sizeof(double) * L->n);
    }
    free(enew); free(r);
}

/* y_c = P^T x_f and y_f += P x_c for the bilinear interpolation */
static void interp_restrict(const or_problem *P, const or_level *F, const or_level *C, const double *xf, double *yc) {
    int d = P->d;
    long W3 = ipow(3, d);
    int IX[OR_MAXD], a[OR_MAXD], ix[OR_MAXD];
    for (long I = 0; I < C->n; I++) {
        unravel(I, d, C->n1, IX);
        double s = 0.0;
        for (long w = 0; w < W3; w++) {
            unravel(w, d, 3, a);
            double wt = 1.0;
            for (int k = 0; k < d; k++) { ix[k] = 2 * IX[k] + 1 + a[k] - 1; wt *= interp_weight(ix[k], IX[k]); }
            if (!inside(ix, d, F->n1)) continue;
            s += wt * xf[ravel(ix, d, F->n1)];
        }
        yc[I] = s;
    }
}
static void interp_prolong_add(const or_problem *P, const or_level *F, const or_level *C, const double *xc, double *yf) {
    int d = P->d;
    long W3 = ipow(3, d);
    int IX[OR_MAXD], a[OR_MAXD], ix[OR_MAXD];
    for (long I = 0; I < C->n; I++) {
        unravel(I, d, C->n1, IX);
        for (long w = 0; w < W3; w++) {
            unravel(w, d, 3, a);
            double wt = 1.0;
            for (int k = 0; k < d; k++) { ix[k] = 2 * IX[k] + 1 + a[k] - 1; wt *= interp_weight(ix[k], IX[k]); }
            if (!inside(ix, d, F->n1)) continue;
            yf[ravel(ix, d, F->n1)] += wt * xc[I];
        }
    }
}

/* one V(nu1,nu2)-cycle on level l for L_l e = rhs, starting from e = 0 */
static void vcycle_level(const or_problem *P, int l, const double *rhs, double *e, int nu1, int nu2) {
    const or_level *L = &P->lev[l];
    if (l == P->nlev - 1) {
        memcpy(e, rhs, sizeof(double) * L->n);
        dense_chol_solve((int)L->n, L->Sfact, e);
        return;
    }
    const or_level *C = &P->lev[l + 1];
    memset(e, 0, sizeof(double) * L->n);
    for (int k = 0; k < nu1; k++) rbgs(P, L, e, rhs);
    double *r = malloc(sizeof(double) * L->n);
    stencil_apply(P->d, L->n1, 1, L->S, e, r);
    for (long i = 0; i < L->n; i++) r[i] = rhs[i] - r[i];
    double *rc = malloc(sizeof(double) * C->n), *ecl = malloc(sizeof(double) * C->n);
    interp_restrict(P, L, C, r, rc);
    vcycle_level(P, l + 1, rc, ecl, nu1, nu2);
    interp_prolong_add(P, L, C, ecl, e);
    for (int k = 0; k < nu2; k++) rbgs(P, L, e, rhs);
    free(r); free(rc); free(ecl);
}

int or_coarse_vcycle(const or_problem *P, const double *dc, double *ec, int nu1, int nu2) {
    if (!P->lev) return fail("or_coarse_vcycle: not set up");
    vcycle_level(P, 0, dc, ec, nu1, nu2);
    return 0;
}

/*
 * Aggressive coarsening (Section 3.3): the coarse level is the degree-plow
 * discretisation on the grid of size 2h.  Its transfers are the composition
 * of the degree transfer on h (I_p^{plow}, I_{plow}^p of Section 3.1.2) with
 * the h <-> 2h transfers between degree-1 spaces (linear interpolation P_0 of
 * the V-cycle hierarchy and its transpose, Section 3.2); the 2h operator is
 * level 1 of that hierarchy (the Galerkin product P_0^T A_1 P_0, equal to the
 * rediscretised degree-1 operator on 2h for kappa = 1).  Needs plow = 1 and a
 * hierarchy of at least two levels.  The exact 2h solve is a banded
 * Cholesky, factorised on first request.
 */
int or_setup_aggressive_direct(or_problem *P) {
    if (!P->lev || P->nlev < 2) return fail("or_setup_aggressive_direct: needs a V-cycle hierarchy of >= 2 levels");
    if (!P->agg_chol) {
        P->agg_chol = band_factor_stencil(P->d, P->lev[1].n1, 1, P->lev[1].S);
        if (!P->agg_chol) return fail("or_setup_aggressive_direct: factorisation failed");
    }
    return 0;
}

/* e_c = P_0 C P_0^T d_c, C = exact 2h solve (coarse 0) or one V(nu1,nu2)
 * cycle from zero on levels 1, 2, ... (coarse 1) */
static int coarse_aggressive(const or_problem *P, const double *dc, double *ec, int coarse, int nu1, int nu2) {
    if (!P->lev || P->nlev < 2) return fail("aggressive coarsening needs a V-cycle hierarchy of >= 2 levels");
    if (coarse == 0 && !P->agg_chol) return fail("aggressive coarsening: exact 2h solve not set up");
    const or_level *F = &P->lev[0], *C = &P->lev[1];
    double *rc = malloc(sizeof(double) * C->n), *ecl = malloc(sizeof(double) * C->n);
    interp_restrict(P, F, C, dc, rc);
    if (coarse == 0) {
        memcpy(ecl, rc, sizeof(double) * C->n);
        band_solve(P->agg_chol, ecl);
    } else {
        vcycle_level(P, 1, rc, ecl, nu1, nu2);
    }
    memset(ec, 0, sizeof(double) * F->n);
    interp_prolong_add(P, F, C, ecl, ec);
    free(rc); free(ecl);
    return 0;
}

int or_coarse_aggressive(const or_problem *P, const double *dc, double *ec, int coarse, int nu1, int nu2) {
    return coarse_aggressive(P, dc, ec, coarse, nu1, nu2);
}

/* ------------------------------------------------------------------ */
/* the two-level cycle (Algorithm 1, general form of Section 3.1)      */
/* ------------------------------------------------------------------ */

/* options: ordering/s as in or_sweep; coarse 0 = exact, 1 = V(cnu1,cnu2);
 * aggressive = 1: the coarse level is degree 1 on 2h (Section 3.3) */
int or_cycle(const or_problem *P, double *u, const double *b, int ordering, int s,
             int nu1, int nu2, int coarse, int cnu1, int cnu2, int aggressive) {
    long n = P->n, nc = P->nc;
    for (int k = 0; k < nu1; k++) if (or_sweep(P, u, b, ordering, s)) return -1;
    double *d = malloc(sizeof(double) * n), *dc = malloc(sizeof(double) * nc), *ec = malloc(sizeof(double) * nc);
    or_residual(P, u, b, d);
    or_restrict(P, d, dc);
    int rc;
    if (aggressive) rc = coarse_aggressive(P, dc, ec, coarse, cnu1, cnu2);
    else rc = coarse == 0 ? or_coarse_direct(P, dc, ec) : or_coarse_vcycle(P, dc, ec, cnu1, cnu2);
    if (rc == 0) or_prolong_add(P, ec, u);
    free(d); free(dc); free(ec);
    if (rc) return rc;
    for (int k = 0; k < nu2; k++) if (or_sweep(P, u, b, ordering, s)) return -1;
    return 0;
}

static double norm2(const double *x, long n) {
    double s = 0.0;
    for (long i = 0; i < n; i++) s += x[i] * x[i];
    return sqrt(s);
}

/*
 * Iterate two-level cycles until ||b - A u||_2 <= tol ||b - A u^0||_2 or
 * max_cycles cycles (Section 5 stopping rule).  hist (length max_cycles+1,
 * may be NULL) receives the residual norms.  Returns the cycle count, or -1.
 */
int or_solve(const or_problem *P, const double *b, double *u, int ordering, int s, int nu1, int nu2,
             int coarse, int cnu1, int cnu2, int aggressive, double tol, int max_cycles, double *hist) {
    long n = P->n;
    double *r = malloc(sizeof(double) * n);
    or_residual(P, u, b, r);
    double r0 = norm2(r, n), rk = r0;
    if (hist) hist[0] = r0;
    int k = 0;
    while (k < max_cycles && rk > tol * r0) {
        if (or_cycle(P, u, b, ordering, s, nu1, nu2, coarse, cnu1, cnu2, aggressive)) { free(r); return -1; }
        k++;
        or_residual(P, u, b, r);
        rk = norm2(r, n);
        if (hist) hist[k] = rk;
    }
    free(r);
    return k;
}

/* direct solve A_p u = b by banded Cholesky (the fixed point of the cycle) */
int or_direct_solve(const or_problem *P, const double *b, double *u) {
    band_chol *c = band_factor_stencil(P->d, P->n1, P->p, P->A);
    if (!c) return fail("or_direct_solve: factorisation failed");
    memcpy(u, b, sizeof(double) * P->n);
    band_solve(c, u);
    band_free(c);
    return 0;
}

/*
 * Gradient of a loss L(u) with respect to the per-element coefficient, for
 * A(kappa) u = b with A = sum_e kappa_e A_e:  given the adjoint state lambda
 * (A lambda = dL/du, A symmetric), dL/dkappa_e = -lambda^T A_e u
 * = -int_e grad lambda_h . grad u_h.  Element integrals by the tensor Gauss
 * rule with p+1 points per direction (exact).
 */
int or_grad_kappa(const or_problem *P, const double *u, const double *lam, double *g) {
    int d = P->d, p = P->p, m = P->m, n1 = P->n1;
    double *t = malloc(sizeof(double) * (2 * p + m + 1));
    or_knots(p, m, t);
    int q = p + 1;
    double gx[64], gw[64];
    or_gauss_legendre(q, gx, gw);
    double h = 1.0 / m;
    int nl = p + 1;
    long nloc = ipow(nl, d), nqp = ipow(q, d);
    double val[OR_MAXD * 16], der[OR_MAXD * 16];
    int e[OR_MAXD], qi[OR_MAXD], a[OR_MAXD], ia[OR_MAXD];
    for (long el = 0; el < P->ne; el++) {
        unravel(el, d, m, e);
        double acc = 0.0;
        for (long qq = 0; qq < nqp; qq++) {
            unravel(qq, d, q, qi);
            double wq = 1.0;
            for (int k = 0; k < d; k++) {
                double x = (e[k] + 0.5 * (gx[qi[k]] + 1.0)) * h;
                wq *= 0.5 * h * gw[qi[k]];
                live_basis(t, p, e[k], x, val + k * nl, der + k * nl);
            }
            double gu[OR_MAXD] = {0, 0, 0}, gl[OR_MAXD] = {0, 0, 0};
            for (long la = 0; la < nloc; la++) {
                unravel(la, d, nl, a);
                for (int k = 0; k < d; k++) ia[k] = e[k] + a[k] - 1;
                if (!inside(ia, d, n1)) continue;
                long i = ravel(ia, d, n1);
                for (int c = 0; c < d; c++) {
                    double gcomp = 1.0;
                    for (int k = 0; k < d; k++) gcomp *= (k == c) ? der[k * nl + a[k]] : val[k * nl + a[k]];
                    gu[c] += u[i] * gcomp;
                    gl[c] += lam[i] * gcomp;
                }
            }
            double dot = 0.0;
            for (int c = 0; c < d; c++) dot += gu[c] * gl[c];
            acc += wq * dot;
        }
        g[el] = -acc;
    }
    free(t);
    return 0;
}

/*
 * out = A_e u for one element e: (A_e u)_i = integral over e of grad phi_i .
 * grad u_h (unit coefficient), for the interior functions i live on e; zero
 * elsewhere.  A = sum_e kappa_e A_e (Section 2).  Tensor Gauss rule with p+1
 * points per direction (exact).
 */
int or_element_apply(const or_problem *P, long el, const double *u, double *out) {
    int d = P->d, p = P->p, m = P->m, n1 = P->n1;
    if (el < 0 || el >= P->ne) return fail("or_element_apply: element out of range");
    double *t = malloc(sizeof(double) * (2 * p + m + 1));
    or_knots(p, m, t);
    int q = p + 1;
    double gx[64], gw[64];
    or_gauss_legendre(q, gx, gw);
    double h = 1.0 / m;
    int nl = p + 1;
    long nloc = ipow(nl, d), nqp = ipow(q, d);
    double val[OR_MAXD * 16], der[OR_MAXD * 16];
    int e[OR_MAXD], qi[OR_MAXD], a[OR_MAXD], ia[OR_MAXD];
    memset(out, 0, sizeof(double) * P->n);
    unravel(el, d, m, e);
    for (long qq = 0; qq < nqp; qq++) {
        unravel(qq, d, q, qi);
        double wq = 1.0;
        for (int k = 0; k < d; k++) {
            double x = (e[k] + 0.5 * (gx[qi[k]] + 1.0)) * h;
            wq *= 0.5 * h * gw[qi[k]];
            live_basis(t, p, e[k], x, val + k * nl, der + k * nl);
        }
        double gu[OR_MAXD] = {0, 0, 0};
        for (long la = 0; la < nloc; la++) {
            unravel(la, d, nl, a);
            for (int k = 0; k < d; k++) ia[k] = e[k] + a[k] - 1;
            if (!inside(ia, d, n1)) continue;
            long i = ravel(ia, d, n1);
            for (int c = 0; c < d; c++) {
                double g = 1.0;
                for (int k = 0; k < d; k++) g *= (k == c) ? der[k * nl + a[k]] : val[k * nl + a[k]];
                gu[c] += u[i] * g;
            }
        }
        for (long la = 0; la < nloc; la++) {
            unravel(la, d, nl, a);
            for (int k = 0; k < d; k++) ia[k] = e[k] + a[k] - 1;
            if (!inside(ia, d, n1)) continue;
            long i = ravel(ia, d, n1);
            double dot = 0.0;
            for (int c = 0; c < d; c++) {
                double g = 1.0;
                for (int k = 0; k < d; k++) g *= (k == c) ? der[k * nl + a[k]] : val[k * nl + a[k]];
                dot += g * gu[c];
            }
            out[i] += wq * dot;
        }
    }
    free(t);
    return 0;
}

/* ------------------------------------------------------------------ */
/* NURBS discretisation of the quarter annulus (Sections 2.2 and 5.2) */
/* ------------------------------------------------------------------ */
/*
 * Domain: {(x,y) : r^2 <= x^2+y^2 <= R^2, x, y >= 0}.  Geometry: the map
 * F(xi, eta) = rho(eta) (c(xi), s(xi)), rho = r + (R - r) eta, where
 * (c, s) is the quarter of the unit circle written as the rational quadratic
 * with control points (1,0), (1,1), (0,1) and weights 1, sqrt(2)/2, 1 (the
 * standard exact conic; Section 2.2 uses quadratic NURBS for this domain).
 * The radial direction eta is linear, so after raising both directions to
 * degree q and refining to m elements the weight net is w_i(xi) x 1: the
 * weights w_i are the coefficients of the quadratic denominator
 * w(xi) = (1-xi)^2 + sqrt(2) xi (1-xi) + xi^2 in the degree-q basis of the
 * refined knot vector (computed here by the L2 projection onto that basis,
 * which reproduces w exactly because w lies in the spline space).
 *
 * Basis (Section 2.2): R_ij = w_ij N_i(xi) N_j(eta) / W(xi,eta),
 * W = sum_kl w_kl N_k(xi) N_l(eta) over every function of the full basis
 * (the Dirichlet-eliminated ones included).  The discrete space of degree q
 * is the span of the interior R_ij composed with F^{-1}.  Integrals are
 * pulled back to (0,1)^2 with the Jacobian J of F: stiffness
 * int grad_xi R_a^T (J^T J)^{-1} grad_xi R_b |det J|, mass
 * int R_a R_b |det J|.  Quadrature: Gauss with QPTS(pfine) points per
 * direction per element (the integrands are rational; the rule is fixed by
 * the fine degree and shared by every annulus integral of a problem).
 */
#define OR_ANN_QPTS(pf) ((pf) + 3)

static void circle_arc(double xi, double *c, double *s, double *dc, double *ds) {
    const double r2 = sqrt(2.0);
    double nx = (1 - xi) * (1 - xi) + r2 * xi * (1 - xi);
    double ny = r2 * xi * (1 - xi) + xi * xi;
    double w = nx + xi * xi;   /* (1-xi)^2 + sqrt2 xi(1-xi) + xi^2 */
    double dnx = -2 * (1 - xi) + r2 * (1 - 2 * xi);
    double dny = r2 * (1 - 2 * xi) + 2 * xi;
    double dw = dnx + 2 * xi;
    *c = nx / w; *s = ny / w;
    *dc = (dnx * w - nx * dw) / (w * w);
    *ds = (dny * w - ny * dw) / (w * w);
}

static double arc_denominator(double xi) {
    return (1 - xi) * (1 - xi) + sqrt(2.0) * xi * (1 - xi) + xi * xi;
}

/* the weights of the degree-q, m-element basis (all m+q functions): the L2
 * projection of w(xi), Gram system solved by dense Cholesky */
int or_annulus_weights(int q, int m, double *wts) {
    int nb = m + q;
    double *t = malloc(sizeof(double) * (2 * q + m + 1));
    or_knots(q, m, t);
    double *G = calloc((size_t)nb * nb, sizeof(double));
    double *g = calloc(nb, sizeof(double));
    double gx[64], gw[64], val[16];
    int nq = q + 3;
    or_gauss_legendre(nq, gx, gw);
    double h = 1.0 / m;
    for (int e = 0; e < m; e++)
        for (int k = 0; k < nq; k++) {
            double x = (e + 0.5 * (gx[k] + 1.0)) * h, wq = 0.5 * h * gw[k];
            live_basis(t, q, e, x, val, NULL);
            double wx = arc_denominator(x);
            for (int a = 0; a <= q; a++) {
                g[e + a] += wq * val[a] * wx;
                for (int b = 0; b <= q; b++) G[(size_t)(e + a) * nb + e + b] += wq * val[a] * val[b];
            }
        }
    int rc = dense_cholesky(nb, G);
    if (rc == 0) {
        dense_chol_solve(nb, G, g);
        memcpy(wts, g, sizeof(double) * nb);
    }
    free(t); free(G); free(g);
    return rc ? fail("or_annulus_weights: Gram matrix not positive definite") : 0;
}

/* basis values and parametric gradients of the live functions of element
 * (ex, ey) at (xi, eta) for degree q: R[la], dR[la][2], la = a + (q+1) b
 * (a along xi); W includes every live function (boundary ones too) */
static void nurbs_live(const double *t, int q, const double *wts, int ex, int ey, double xi, double eta,
                       double *R, double *dR) {
    double vx[16], dx[16], vy[16], dy[16];
    live_basis(t, q, ex, xi, vx, dx);
    live_basis(t, q, ey, eta, vy, dy);
    double W = 0, Wx = 0, Wy = 0;
    int nl = q + 1;
    for (int b = 0; b < nl; b++)
        for (int a = 0; a < nl; a++) {
            double w = wts[ex + a];   /* w_ij = w_i (xi) x 1 (eta) */
            W += w * vx[a] * vy[b];
            Wx += w * dx[a] * vy[b];
            Wy += w * vx[a] * dy[b];
        }
    for (int b = 0; b < nl; b++)
        for (int a = 0; a < nl; a++) {
            double w = wts[ex + a];
            double Nv = vx[a] * vy[b];
            int la = a + nl * b;
            R[la] = w * Nv / W;
            dR[2 * la + 0] = w * (dx[a] * vy[b] * W - Nv * Wx) / (W * W);
            dR[2 * la + 1] = w * (vx[a] * dy[b] * W - Nv * Wy) / (W * W);
        }
}

/* Jacobian of F at (xi, eta): J[0]=dx/dxi J[1]=dx/deta J[2]=dy/dxi J[3]=dy/deta */
static void annulus_map(double rin, double rout, double xi, double eta, double *x, double *y, double *J) {
    double c, s, dc, ds;
    circle_arc(xi, &c, &s, &dc, &ds);
    double rho = rin + (rout - rin) * eta;
    *x = rho * c; *y = rho * s;
    J[0] = rho * dc; J[1] = (rout - rin) * c;
    J[2] = rho * ds; J[3] = (rout - rin) * s;
}

/*
 * Bilinear form between the interior functions of degree qa (rows) and qb
 * (columns) on the annulus, stored by offset in [-qa, qb]^2 with width
 * qa+qb+1 per direction (for qa == qb this is the symmetric offset storage
 * of radius q).  kind: OR_STIFF or OR_MASS.  pf: the fine degree (fixes the
 * quadrature).
 */
static int annulus_form(int qa, int qb, int pf, int m, double rin, double rout, int kind, double *out) {
    int n1a = m + qa - 2, n1b = m + qb - 2, wd = qa + qb + 1;
    long W = (long)wd * wd;
    memset(out, 0, sizeof(double) * (long)n1a * n1a * W);
    double *ta = malloc(sizeof(double) * (2 * qa + m + 1)), *tb = malloc(sizeof(double) * (2 * qb + m + 1));
    double *wa = malloc(sizeof(double) * (m + qa)), *wb = malloc(sizeof(double) * (m + qb));
    or_knots(qa, m, ta); or_knots(qb, m, tb);
    if (or_annulus_weights(qa, m, wa) || or_annulus_weights(qb, m, wb)) { free(ta); free(tb); free(wa); free(wb); return 1; }
    int nq = OR_ANN_QPTS(pf);
    double gx[64], gw[64];
    or_gauss_legendre(nq, gx, gw);
    double h = 1.0 / m;
    int nla = qa + 1, nlb = qb + 1;
    double Ra[256], dRa[512], Rb[256], dRb[512];
    for (int ey = 0; ey < m; ey++)
        for (int ex = 0; ex < m; ex++)
            for (int ky = 0; ky < nq; ky++)
                for (int kx = 0; kx < nq; kx++) {
                    double xi = (ex + 0.5 * (gx[kx] + 1.0)) * h, eta = (ey + 0.5 * (gx[ky] + 1.0)) * h;
                    double wq = 0.25 * h * h * gw[kx] * gw[ky];
                    double X, Y, J[4];
                    annulus_map(rin, rout, xi, eta, &X, &Y, J);
                    double det = J[0] * J[3] - J[1] * J[2];
                    /* (J^T J)^{-1} */
                    double g00 = J[0] * J[0] + J[2] * J[2], g01 = J[0] * J[1] + J[2] * J[3], g11 = J[1] * J[1] + J[3] * J[3];
                    double gd = g00 * g11 - g01 * g01;
                    double i00 = g11 / gd, i01 = -g01 / gd, i11 = g00 / gd;
                    nurbs_live(ta, qa, wa, ex, ey, xi, eta, Ra, dRa);
                    nurbs_live(tb, qb, wb, ex, ey, xi, eta, Rb, dRb);
                    for (int bA = 0; bA < nla; bA++)
                        for (int aA = 0; aA < nla; aA++) {
                            int I = ex + aA - 1, Jr = ey + bA - 1;
                            if (I < 0 || I >= n1a || Jr < 0 || Jr >= n1a) continue;
                            int la = aA + nla * bA;
                            for (int bB = 0; bB < nlb; bB++)
                                for (int aB = 0; aB < nlb; aB++) {
                                    int K = ex + aB - 1, L = ey + bB - 1;
                                    if (K < 0 || K >= n1b || L < 0 || L >= n1b) continue;
                                    int lb = aB + nlb * bB;
                                    double v;
                                    if (kind == OR_STIFF) {
                                        double ax = dRa[2 * la], ay = dRa[2 * la + 1], bx = dRb[2 * lb], by = dRb[2 * lb + 1];
                                        v = (ax * (i00 * bx + i01 * by) + ay * (i01 * bx + i11 * by)) * fabs(det);
                                    } else {
                                        v = Ra[la] * Rb[lb] * fabs(det);
                                    }
                                    long off = (long)(K - I + qa) + (long)(L - Jr + qa) * wd;
                                    out[((long)Jr * n1a + I) * W + off] += wq * v;
                                }
                        }
                }
    free(ta); free(tb); free(wa); free(wb);
    return 0;
}

/* the exact solution of the annulus experiment and minus its Laplacian
 * (Section 5.2): u = sin(pi x) sin(pi y) (x^2+y^2-r^2)(x^2+y^2-R^2) */
static double annulus_exact(double x, double y, double rin, double rout) {
    double s = x * x + y * y;
    return sin(M_PI * x) * sin(M_PI * y) * (s - rin * rin) * (s - rout * rout);
}
static double annulus_f(double x, double y, double rin, double rout) {
    double s = x * x + y * y, S = sin(M_PI * x) * sin(M_PI * y);
    double Q = (s - rin * rin) * (s - rout * rout);
    double Sx = M_PI * cos(M_PI * x) * sin(M_PI * y), Sy = M_PI * sin(M_PI * x) * cos(M_PI * y);
    double dQ = 2 * s - rin * rin - rout * rout;           /* dQ/ds */
    double Qx = dQ * 2 * x, Qy = dQ * 2 * y;
    double lapS = -2 * M_PI * M_PI * S, lapQ = 16 * s - 4 * (rin * rin + rout * rout);
    return -(Q * lapS + 2 * (Sx * Qx + Sy * Qy) + S * lapQ);
}

/* load vector b_i = int f R_i |det J| (interior functions, degree p) */
int or_load_annulus(int p, int m, double rin, double rout, double *bvec) {
    int n1 = m + p - 2;
    memset(bvec, 0, sizeof(double) * (long)n1 * n1);
    double *t = malloc(sizeof(double) * (2 * p + m + 1)), *wts = malloc(sizeof(double) * (m + p));
    or_knots(p, m, t);
    if (or_annulus_weights(p, m, wts)) { free(t); free(wts); return 1; }
    int nq = OR_ANN_QPTS(p), nl = p + 1;
    double gx[64], gw[64], R[256], dR[512];
    or_gauss_legendre(nq, gx, gw);
    double h = 1.0 / m;
    for (int ey = 0; ey < m; ey++)
        for (int ex = 0; ex < m; ex++)
            for (int ky = 0; ky < nq; ky++)
                for (int kx = 0; kx < nq; kx++) {
                    double xi = (ex + 0.5 * (gx[kx] + 1.0)) * h, eta = (ey + 0.5 * (gx[ky] + 1.0)) * h;
                    double wq = 0.25 * h * h * gw[kx] * gw[ky];
                    double X, Y, J[4];
                    annulus_map(rin, rout, xi, eta, &X, &Y, J);
                    double det = fabs(J[0] * J[3] - J[1] * J[2]);
                    double f = annulus_f(X, Y, rin, rout);
                    nurbs_live(t, p, wts, ex, ey, xi, eta, R, dR);
                    for (int b = 0; b < nl; b++)
                        for (int a = 0; a < nl; a++) {
                            int I = ex + a - 1, Jr = ey + b - 1;
                            if (I < 0 || I >= n1 || Jr < 0 || Jr >= n1) continue;
                            bvec[(long)Jr * n1 + I] += wq * f * R[a + nl * b] * det;
                        }
                }
    free(t); free(wts);
    return 0;
}

/* || u_h - u ||_{L2(Omega)} for the coefficient vector u (interior, degree p) */
double or_l2_error_annulus(int p, int m, double rin, double rout, const double *u) {
    int n1 = m + p - 2;
    double *t = malloc(sizeof(double) * (2 * p + m + 1)), *wts = malloc(sizeof(double) * (m + p));
    or_knots(p, m, t);
    if (or_annulus_weights(p, m, wts)) { free(t); free(wts); return -1.0; }
    int nq = OR_ANN_QPTS(p), nl = p + 1;
    double gx[64], gw[64], R[256], dR[512];
    or_gauss_legendre(nq, gx, gw);
    double h = 1.0 / m, err = 0.0;
    for (int ey = 0; ey < m; ey++)
        for (int ex = 0; ex < m; ex++)
            for (int ky = 0; ky < nq; ky++)
                for (int kx = 0; kx < nq; kx++) {
                    double xi = (ex + 0.5 * (gx[kx] + 1.0)) * h, eta = (ey + 0.5 * (gx[ky] + 1.0)) * h;
                    double wq = 0.25 * h * h * gw[kx] * gw[ky];
                    double X, Y, J[4];
                    annulus_map(rin, rout, xi, eta, &X, &Y, J);
                    double det = fabs(J[0] * J[3] - J[1] * J[2]);
                    nurbs_live(t, p, wts, ex, ey, xi, eta, R, dR);
                    double uh = 0.0;
                    for (int b = 0; b < nl; b++)
                        for (int a = 0; a < nl; a++) {
                            int I = ex + a - 1, Jr = ey + b - 1;
                            if (I < 0 || I >= n1 || Jr < 0 || Jr >= n1) continue;
                            uh += u[(long)Jr * n1 + I] * R[a + nl * b];
                        }
                    double d = uh - annulus_exact(X, Y, rin, rout);
                    err += wq * d * d * det;
                }
    free(t); free(wts);
    return sqrt(err);
}

/* the physical point of parameter (xi, eta) and the NURBS curve of the arc
 * evaluated by the rational formula of Section 2.2 (pins the map) */
void or_annulus_point(double rin, double rout, double xi, double eta, double *xy) {
    double J[4];
    annulus_map(rin, rout, xi, eta, &xy[0], &xy[1], J);
}

/* assembled annulus operators, for tests: kind 0 stiffness, 1 mass, 2 mixed
 * mass (rows degree plow, columns degree p), by offset as in or_create */
int or_assemble_annulus(int p, int plow, int m, double rin, double rout, int kind, double *out) {
    if (kind == 2) return annulus_form(plow, p, p, m, rin, rout, OR_MASS, out);
    return annulus_form(p, p, p, m, rin, rout, kind == 0 ? OR_STIFF : OR_MASS, out);
}

/*
 * The two-level problem on the annulus (Section 5.2): degree p on the fine
 * level, plow (2 in the paper) on the coarse level, both NURBS spaces over
 * the same m x m elements; A, Alow, Mlow and Mmix from the forms above,
 * everything else (Schwarz blocks, lumped restriction, exact coarse solve)
 * as for the square.  The V-cycle hierarchy of the degree-1 coarse problem
 * is for the square only.
 */
or_problem *or_create_annulus(int p, int m, int plow, int block_width, int lumped, int want_coarse_direct,
                              double rin, double rout) {
    const int d = 2;
    if (p < 2 || p > 8 || m < 2 || plow < 1 || plow > p || !(rin > 0.0) || !(rout > rin)) {
        fail("or_create_annulus: bad arguments"); return NULL;
    }
    if (block_width < 0 || (block_width && block_width % 2 == 0)) { fail("or_create_annulus: block width must be odd"); return NULL; }
    or_problem *P = calloc(1, sizeof *P);
    P->d = d; P->p = p; P->m = m; P->plow = plow;
    P->bw = block_width ? block_width : or_default_block_width(p);
    P->lumped = lumped;
    P->n1 = m + p - 2; P->n1c = m + plow - 2;
    P->n = ipow(P->n1, d); P->nc = ipow(P->n1c, d); P->ne = ipow(m, d);
    P->W = ipow(2 * p + 1, d); P->Wc = ipow(2 * plow + 1, d); P->Wm = ipow(p + plow + 1, d);
    if (P->n1 < 1 || P->n1c < 1) { fail("or_create_annulus: mesh too small"); free(P); return NULL; }
    P->kappa = malloc(sizeof(double) * P->ne);
    for (long e = 0; e < P->ne; e++) P->kappa[e] = 1.0;
    P->A = malloc(sizeof(double) * P->n * P->W);
    P->Alow = malloc(sizeof(double) * P->nc * P->Wc);
    P->Mlow = malloc(sizeof(double) * P->nc * P->Wc);
    P->Mmix = malloc(sizeof(double) * P->nc * P->Wm);
    P->Dlump = malloc(sizeof(double) * P->nc);
    if (!P->A || !P->Alow || !P->Mlow || !P->Mmix || !P->Dlump) { fail("or_create_annulus: out of memory"); or_destroy(P); return NULL; }
    if (annulus_form(p, p, p, m, rin, rout, OR_STIFF, P->A) ||
        annulus_form(plow, plow, p, m, rin, rout, OR_STIFF, P->Alow) ||
        annulus_form(plow, plow, p, m, rin, rout, OR_MASS, P->Mlow) ||
        annulus_form(plow, p, p, m, rin, rout, OR_MASS, P->Mmix)) { or_destroy(P); return NULL; }
    for (long i = 0; i < P->nc; i++) {
        double s = 0.0;
        for (long w = 0; w < P->Wc; w++) s += P->Mlow[i * P->Wc + w];
        P->Dlump[i] = s;
    }
    if (build_blocks(P)) { or_destroy(P); return NULL; }
    if (want_coarse_direct) {
        P->coarse_chol = band_factor_stencil(d, P->n1c, plow, P->Alow);
        if (!P->coarse_chol) { fail("or_create_annulus: coarse factorisation failed"); or_destroy(P); return NULL; }
    }
    if (!lumped) {
        P->mass_chol = band_factor_stencil(d, P->n1c, plow, P->Mlow);
        if (!P->mass_chol) { fail("or_create_annulus: mass factorisation failed"); or_destroy(P); return NULL; }
    }
    return P;
}
