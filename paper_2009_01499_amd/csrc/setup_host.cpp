// setup_host.cpp -- host-side set-up of the gfx950 two-level solver: B-spline
// evaluation, 1-D element matrices, assembly of the fine operator in
// symmetric padded-diagonal form, the restriction factor, the degree-1 V-cycle
// hierarchy, the DST tables of the exact coarse solver, Schwarz block classes
// and the lexicographic hyperplane schedule.  Runs once per problem; every
// per-cycle operation runs in the HIP kernels.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "internal.h"

namespace iga2l {

namespace {

int64_t ipow(int64_t b, int e) {
    int64_t r = 1;
    while (e-- > 0) r *= b;
    return r;
}

// Gauss-Legendre rule on [-1,1], nodes by Newton iteration on P_q.
void gauss_rule(int q, double *x, double *w) {
    for (int i = 0; i < q; ++i) {
        double z = std::cos(M_PI * (4.0 * i + 3.0) / (4.0 * q + 2.0));
        double p0 = 1.0, p1 = z, dp = 1.0;
        for (int it = 0; it < 64; ++it) {
            p0 = 1.0;
            p1 = z;
            for (int k = 2; k <= q; ++k) {
                double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (q == 1) { p1 = z; p0 = 1.0; }
            dp = q * (z * p1 - p0) / (z * z - 1.0);
            double step = p1 / dp;
            z -= step;
            if (std::fabs(step) < 1e-17) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Values and first derivatives of the p+1 B-splines of degree p that are live
// on knot span s (t[s] <= x < t[s+1]): out index a <-> function s-p+a.
// The triangle of lower-degree values is built stage by stage with the
// Cox-de Boor step restricted to live functions.
void live_values(const std::vector<double> &t, int p, int s, double x, double *val, double *der) {
    double stage[kMaxP + 1], next[kMaxP + 1], prev_stage[kMaxP + 1];
    stage[0] = 1.0;  // degree 0: only N_s is live
    for (int a = 0; a <= p; ++a) prev_stage[a] = 0.0;
    for (int k = 1; k <= p; ++k) {
        // stage holds N^{k-1}_{s-k+1+b}, b = 0..k-1; next gets N^k_{s-k+a}, a = 0..k
        for (int a = 0; a <= k; ++a) {
            int i = s - k + a;
            double lo = (a >= 1) ? stage[a - 1] : 0.0;      // N^{k-1}_i
            double hi = (a <= k - 1) ? stage[a] : 0.0;      // N^{k-1}_{i+1}
            double d1 = t[i + k] - t[i], d2 = t[i + k + 1] - t[i + 1];
            double v = 0.0;
            if (d1 > 0.0) v += (x - t[i]) / d1 * lo;
            if (d2 > 0.0) v += (t[i + k + 1] - x) / d2 * hi;
            next[a] = v;
        }
        if (k == p) {
            for (int b = 0; b < k; ++b) prev_stage[b] = stage[b];
        }
        for (int a = 0; a <= k; ++a) stage[a] = next[a];
    }
    for (int a = 0; a <= p; ++a) val[a] = stage[a];
    if (der) {
        if (p == 0) {
            der[0] = 0.0;
            return;
        }
        for (int a = 0; a <= p; ++a) {
            int i = s - p + a;
            double lo = (a >= 1) ? prev_stage[a - 1] : 0.0;
            double hi = (a <= p - 1) ? prev_stage[a] : 0.0;
            double d1 = t[i + p] - t[i], d2 = t[i + p + 1] - t[i + 1];
            double v = 0.0;
            if (d1 > 0.0) v += p / d1 * lo;
            if (d2 > 0.0) v -= p / d2 * hi;
            der[a] = v;
        }
    }
}

std::vector<double> open_uniform_knots(int p, int m) {
    std::vector<double> t(2 * p + m + 1);
    for (int i = 0; i < (int)t.size(); ++i) t[i] = std::min(1.0, std::max(0.0, double(i - p) / m));
    return t;
}

// 1-D element stiffness/mass matrices of degree p on all m elements,
// [(p+1) x (p+1)] row-major each; Gauss rule with p+1 points (exact).
void element_matrices(int p, int m, std::vector<std::vector<double>> &Ke, std::vector<std::vector<double>> &Me) {
    auto t = open_uniform_knots(p, m);
    double gx[kMaxP + 4], gw[kMaxP + 4];
    int q = p + 1;
    gauss_rule(q, gx, gw);
    double h = 1.0 / m;
    Ke.assign(m, std::vector<double>((p + 1) * (p + 1), 0.0));
    Me.assign(m, std::vector<double>((p + 1) * (p + 1), 0.0));
    double v[kMaxP + 1], dv[kMaxP + 1];
    for (int e = 0; e < m; ++e) {
        for (int k = 0; k < q; ++k) {
            double x = (e + 0.5 * (gx[k] + 1.0)) * h, wq = 0.5 * h * gw[k];
            live_values(t, p, p + e, x, v, dv);
            for (int a = 0; a <= p; ++a)
                for (int b = a; b <= p; ++b) {
                    Ke[e][a * (p + 1) + b] += wq * dv[a] * dv[b];
                    Me[e][a * (p + 1) + b] += wq * v[a] * v[b];
                }
        }
        // symmetric bit for bit (the assembled 1-D factors then are too)
        for (int a = 0; a <= p; ++a)
            for (int b = 0; b < a; ++b) {
                Ke[e][a * (p + 1) + b] = Ke[e][b * (p + 1) + a];
                Me[e][a * (p + 1) + b] = Me[e][b * (p + 1) + a];
            }
    }
    // Elements p .. m-1-p carry only cardinal (translated) B-splines, so their
    // matrices are equal in exact arithmetic; one copy for all of them makes
    // the assembled interior rows exact translates of each other, bit for bit
    // (the interior stencil then equals every interior row of the operator).
    for (int e = p + 1; e <= m - 1 - p; ++e) {
        Ke[e] = Ke[p];
        Me[e] = Me[p];
    }
}

// ------------------------------------------------------------ annulus --
// The quarter annulus (Section 5.2) is the image of the unit square under
// F(xi, eta) = rho(eta) (c(xi), s(xi)), rho = r_in + (r_out - r_in) eta, with
// (c, s) the quarter of the unit circle written as the rational quadratic
// (control points (1,0), (1,1), (0,1), weights 1, sqrt(2)/2, 1).  The
// NURBS basis of degree q on m elements is R_ij = w_i N_i(xi) N_j(eta) / w(xi):
// the radial direction is linear, so the weight net is w_i x 1 and the
// denominator is the arc's quadratic denominator w(xi), whose coefficients
// in the degree-q basis are the w_i.  The columns of the Jacobian are
// rho (c', s') and (r_out - r_in) (c, s), orthogonal, with |(c', s')| = the
// arc's speed v(xi).  So int grad R_a . grad R_b dx pulls back to
// int phi_i' phi_k' / v  x  int N_j N_l (r_out-r_in)/rho
//   + int phi_i phi_k v  x  int N_j' N_l' rho/(r_out-r_in),
// phi_i = w_i N_i / w, and int R_a R_b dx to int phi_i phi_k v x
// int N_j N_l rho (r_out-r_in): tensor sums/products of weighted 1-D forms.
// Quadrature: kAnnulusExtraPts more Gauss points per element than the fine
// degree, in both directions and for every form of a problem.
constexpr int kAnnulusExtraPts = 3;

struct ArcPoint {
    double w, dw, speed;
};

ArcPoint arc_point(double xi) {
    const double r2 = std::sqrt(2.0), a = 1.0 - xi;
    const double nx = a * a + r2 * xi * a, ny = r2 * xi * a + xi * xi, w = nx + xi * xi;
    const double dnx = -2.0 * a + r2 * (1.0 - 2.0 * xi), dny = r2 * (1.0 - 2.0 * xi) + 2.0 * xi;
    const double dw = dnx + 2.0 * xi;
    const double dc = (dnx * w - nx * dw) / (w * w), ds = (dny * w - ny * dw) / (w * w);
    return {w, dw, std::sqrt(dc * dc + ds * ds)};
}

// coefficients of the arc's denominator in the degree-q basis on m elements
// (all m+q functions): L2 projection, Gram system by dense Cholesky
std::vector<double> arc_weights(int q, int m) {
    const int nb = m + q;
    auto t = open_uniform_knots(q, m);
    std::vector<double> G(size_t(nb) * nb, 0.0), g(nb, 0.0);
    double gx[kMaxP + 4], gw[kMaxP + 4], v[kMaxP + 1];
    const int nq = q + 2;   // exact for the degree-2q Gram entries
    gauss_rule(nq, gx, gw);
    for (int e = 0; e < m; ++e)
        for (int k = 0; k < nq; ++k) {
            const double x = (e + 0.5 * (gx[k] + 1.0)) / m, wq = 0.5 * gw[k] / m;
            live_values(t, q, q + e, x, v, nullptr);
            const double wx = arc_point(x).w;
            for (int a = 0; a <= q; ++a) {
                g[e + a] += wq * v[a] * wx;
                for (int b = 0; b <= q; ++b) G[size_t(e + a) * nb + e + b] += wq * v[a] * v[b];
            }
        }
    for (int j = 0; j < nb; ++j) {   // G = L L^T in place (lower)
        double d = G[size_t(j) * nb + j];
        for (int k = 0; k < j; ++k) d -= G[size_t(j) * nb + k] * G[size_t(j) * nb + k];
        IGA2L_REQUIRE(d > 0.0, IGA2L_ENUMERIC, "annulus weights: Gram matrix not positive definite");
        d = std::sqrt(d);
        G[size_t(j) * nb + j] = d;
        for (int i = j + 1; i < nb; ++i) {
            double t2 = G[size_t(i) * nb + j];
            for (int k = 0; k < j; ++k) t2 -= G[size_t(i) * nb + k] * G[size_t(j) * nb + k];
            G[size_t(i) * nb + j] = t2 / d;
        }
    }
    for (int i = 0; i < nb; ++i) {
        double t2 = g[i];
        for (int k = 0; k < i; ++k) t2 -= G[size_t(i) * nb + k] * g[k];
        g[i] = t2 / G[size_t(i) * nb + i];
    }
    for (int i = nb - 1; i >= 0; --i) {
        double t2 = g[i];
        for (int k = i + 1; k < nb; ++k) t2 -= G[size_t(k) * nb + i] * g[k];
        g[i] = t2 / G[size_t(i) * nb + i];
    }
    return g;
}

enum AnnForm { kAnnStiff = 0, kAnnOpMass = 1, kAnnL2Mass = 2 };

// A weighted 1-D form on the annulus between the interior functions of
// degree qa (rows) and qb (columns), by offset: out[i][j - i + qa], width
// qa + qb + 1.  axis 0: angular (NURBS phi, weights as above), axis 1: radial
// (B-splines).  Weights per form and axis:
//   stiffness       1/v (angular)     rho/(r_out-r_in) (radial)
//   operator mass   v                 (r_out-r_in)/rho
//   L2 mass         v                 rho (r_out-r_in)
std::vector<double> annulus_form_1d(const Problem &P, int qa, int qb, int axis, AnnForm form) {
    const int m = P.m, n1a = m + qa - 2, n1b = m + qb - 2, wd = qa + qb + 1;
    const double rin = P.r_in, dr = P.r_out - P.r_in;
    auto ta = open_uniform_knots(qa, m), tb = open_uniform_knots(qb, m);
    std::vector<double> wa, wb;
    if (axis == 0) {
        wa = arc_weights(qa, m);
        wb = arc_weights(qb, m);
    }
    const int nq = P.p + kAnnulusExtraPts;
    double gx[kMaxP + 4], gw[kMaxP + 4];
    gauss_rule(nq, gx, gw);
    std::vector<double> out(size_t(std::max(n1a, 0)) * wd, 0.0);
    double va[kMaxP + 1], da[kMaxP + 1], vb[kMaxP + 1], db[kMaxP + 1];
    for (int e = 0; e < m; ++e)
        for (int k = 0; k < nq; ++k) {
            const double x = (e + 0.5 * (gx[k] + 1.0)) / m, wq = 0.5 * gw[k] / m;
            live_values(ta, qa, qa + e, x, va, da);
            live_values(tb, qb, qb + e, x, vb, db);
            double wgt;
            if (axis == 0) {
                const ArcPoint ap = arc_point(x);
                // phi = w_i N / w, phi' = w_i (N' w - N w') / w^2
                for (int a = 0; a <= qa; ++a) {
                    const double om = wa[e + a];
                    da[a] = om * (da[a] * ap.w - va[a] * ap.dw) / (ap.w * ap.w);
                    va[a] = om * va[a] / ap.w;
                }
                for (int b = 0; b <= qb; ++b) {
                    const double om = wb[e + b];
                    db[b] = om * (db[b] * ap.w - vb[b] * ap.dw) / (ap.w * ap.w);
                    vb[b] = om * vb[b] / ap.w;
                }
                wgt = (form == kAnnStiff) ? 1.0 / ap.speed : ap.speed;
            } else {
                const double rho = rin + dr * x;
                wgt = (form == kAnnStiff) ? rho / dr : (form == kAnnOpMass ? dr / rho : rho * dr);
            }
            for (int a = 0; a <= qa; ++a) {
                const int i = e + a - 1;
                if (i < 0 || i >= n1a) continue;
                for (int b = 0; b <= qb; ++b) {
                    const int j = e + b - 1;
                    if (j < 0 || j >= n1b) continue;
                    const double f = (form == kAnnStiff) ? da[a] * db[b] : va[a] * vb[b];
                    out[size_t(i) * wd + (j - i + qa)] += wq * wgt * f;
                }
            }
        }
    return out;
}

// linear index <-> multi-index over a box of extent n in each of dim directions
inline void split(int64_t idx, int dim, int64_t n, int *out) {
    for (int k = 0; k < dim; ++k) {
        out[k] = int(idx % n);
        idx /= n;
    }
}

}  // namespace

// ------------------------------------------------------------ transfers --
// 1-D factors of the transfer between the degree-p space and the degree-plow
// space on the same knots (Section 3.1.2): Mmix1 = M_p^{plow} by Gauss
// quadrature, entry (I, j) at [I][j - I + plow], j - I in [-plow, p]; R1 =
// D1^{-1} Mmix1 with D1 the row sums of the Dirichlet-reduced degree-plow
// mass matrix (row-sum lumping).  Sets the coarse grid (m + plow - 2 points
// per direction).
void host_transfer_factors(Problem &P, int plow) {
    const int p = P.p, m = P.m, d = P.dim;
    const int n1 = P.fine.n1, n1c = m + plow - 2, w = p + plow + 1;
    P.plow = plow;
    P.coarse = Grid{d, n1c, ipow(n1c, d)};
    if (P.geometry == kGeomAnnulus) {
        // per axis: the L2 mixed mass and the row sums of the L2 coarse mass
        // (the 2-D mass is their tensor product, so is its row-sum lumping)
        for (int axis = 0; axis < 2; ++axis) {
            const auto mix = annulus_form_1d(P, plow, p, axis, kAnnL2Mass);
            const auto mc = annulus_form_1d(P, plow, plow, axis, kAnnL2Mass);
            std::vector<double> R(mix.size());
            for (int I = 0; I < n1c; ++I) {
                double lump = 0.0;
                for (int a = 0; a < 2 * plow + 1; ++a) lump += mc[size_t(I) * (2 * plow + 1) + a];
                for (int a = 0; a < w; ++a) R[size_t(I) * w + a] = mix[size_t(I) * w + a] / lump;
            }
            if (axis == 0) {
                P.Mx1 = mix;
                P.R1 = R;
            } else {
                P.R1y = R;
            }
        }
        return;
    }
    auto tf = open_uniform_knots(p, m), tc = open_uniform_knots(plow, m);
    double gx[kMaxP + 4], gw[kMaxP + 4];
    const int q = p + 1;   // exact for the degree p + plow <= 2p integrands
    gauss_rule(q, gx, gw);
    const double h = 1.0 / m;
    std::vector<double> mix(size_t(n1c) * w, 0.0), lump(n1c, 0.0);
    double v[kMaxP + 1], vc[kMaxP + 1];
    for (int e = 0; e < m; ++e)
        for (int k = 0; k < q; ++k) {
            double x = (e + 0.5 * (gx[k] + 1.0)) * h, wq = 0.5 * h * gw[k];
            live_values(tf, p, p + e, x, v, nullptr);
            live_values(tc, plow, plow + e, x, vc, nullptr);
            for (int c = 0; c <= plow; ++c) {
                int I = e + c - 1;
                if (I < 0 || I >= n1c) continue;
                for (int c2 = 0; c2 <= plow; ++c2) {
                    int J = e + c2 - 1;
                    if (J < 0 || J >= n1c) continue;
                    lump[I] += wq * vc[c] * vc[c2];
                }
                for (int a = 0; a <= p; ++a) {
                    int j = e + a - 1;
                    if (j < 0 || j >= n1) continue;
                    mix[size_t(I) * w + (j - I + plow)] += wq * vc[c] * v[a];
                }
            }
        }
    P.Mx1 = mix;
    P.R1.assign(mix.size(), 0.0);
    for (int I = 0; I < n1c; ++I)
        for (int a = 0; a < w; ++a) P.R1[size_t(I) * w + a] = mix[size_t(I) * w + a] / lump[I];
}

// ------------------------------------------------------------ assembly --
void host_assemble(Problem &P) {
    const int p = P.p, m = P.m, d = P.dim;
    const int n1 = m + p - 2;
    P.fine = Grid{d, n1, ipow(n1, d)};
    P.ne = ipow(m, d);

    element_matrices(p, m, P.Ke, P.Me);

    // interior 1-D factors K1, M1: entry (i, i+o) at [i][o+p]
    const int w1 = 2 * p + 1;
    const bool annulus = P.geometry == kGeomAnnulus;
    if (annulus) {
        // angular factors in K1, M1, radial in K1y, M1y (operator weights)
        P.K1 = annulus_form_1d(P, p, p, 0, kAnnStiff);
        P.M1 = annulus_form_1d(P, p, p, 0, kAnnOpMass);
        P.K1y = annulus_form_1d(P, p, p, 1, kAnnStiff);
        P.M1y = annulus_form_1d(P, p, p, 1, kAnnOpMass);
    } else {
        P.K1.assign(size_t(n1) * w1, 0.0);
        P.M1.assign(size_t(n1) * w1, 0.0);
        for (int e = 0; e < m; ++e)
            for (int a = 0; a <= p; ++a)
                for (int b = 0; b <= p; ++b) {
                    int i = e + a - 1, j = e + b - 1;
                    if (i < 0 || i >= n1 || j < 0 || j >= n1) continue;
                    P.K1[size_t(i) * w1 + (j - i + p)] += P.Ke[e][a * (p + 1) + b];
                    P.M1[size_t(i) * w1 + (j - i + p)] += P.Me[e][a * (p + 1) + b];
                }
    }

    // the annulus is discretised with a degree-2 coarse space (its geometry is
    // quadratic, Section 5.2); the square starts from degree 1
    host_transfer_factors(P, annulus ? 2 : 1);

    // 1-D element matrices (assembly and gradient kernels): [m][2][(p+1)^2] (K then M)
    const int nl = p + 1;
    std::vector<double> km(size_t(m) * 2 * nl * nl);
    for (int el = 0; el < m; ++el)
        for (int k = 0; k < nl * nl; ++k) {
            km[(size_t(el) * 2 + 0) * nl * nl + k] = P.Ke[el][k];
            km[(size_t(el) * 2 + 1) * nl * nl + k] = P.Me[el][k];
        }
    P.Ke_d.alloc(km.size() * sizeof(double));
    IGA2L_HIP(hipMemcpy(P.Ke_d.ptr, km.data(), km.size() * sizeof(double), hipMemcpyHostToDevice));
    std::vector<double> kap(P.ne, 1.0);
    if (!P.kappa_one) kap = P.kappa;
    P.kappa_d.alloc(kap.size() * sizeof(double));
    IGA2L_HIP(hipMemcpy(P.kappa_d.ptr, kap.data(), kap.size() * sizeof(double), hipMemcpyHostToDevice));

    // fine operator in symmetric padded-diagonal form
    SymDia &A = P.A;
    A.q = p;
    A.W = int(ipow(w1, d));
    A.Wh = (A.W + 1) / 2;
    const int np1 = n1 + 2 * p;
    A.pitch[0] = 1;
    A.pitch[1] = np1;
    A.pitch[2] = np1 * np1;
    A.npad = ipow(np1, d);
    const bool host_dia = P.kappa_one || annulus;
    std::vector<double> val(host_dia ? size_t(A.Wh) * A.npad : 0, 0.0);
    const int c0 = (A.W - 1) / 2;
    // factor of axis k: the stiffness one in the derivative's direction, the
    // mass one elsewhere (the radial axis of the annulus has its own)
    auto factor = [&](int k, bool stiff) -> const std::vector<double> & {
        if (annulus && k == 1) return stiff ? P.K1y : P.M1y;
        return stiff ? P.K1 : P.M1;
    };
    if (host_dia) {
        // kappa = 1: A = sum_c (x)_k (k == c ? K1 : M1), entry by entry from the
        // assembled 1-D factors (O(n Wh) instead of the element loop)
        int ix[kMaxDim] = {0, 0, 0}, o[kMaxDim] = {0, 0, 0};
        for (int64_t i = 0; i < P.fine.n; ++i) {
            split(i, d, n1, ix);
            int64_t padi = 0;
            for (int k = 0; k < d; ++k) padi += int64_t(ix[k] + p) * A.pitch[k];
            for (int w = c0; w < A.W; ++w) {
                split(w, d, w1, o);
                bool in = true;
                for (int k = 0; k < d; ++k) {
                    const int j = ix[k] + o[k] - p;
                    if (j < 0 || j >= n1) in = false;
                }
                if (!in) continue;
                // term c = F_x (F_y F_z) with F = K1 in direction c, M1 otherwise
                // (the grouping the 3-D kernels reproduce when they form rows
                // next to the boundary from the factors)
                double term = 0.0;
                for (int c = 0; c < d; ++c) {
                    double f[kMaxDim];
                    for (int k = 0; k < d; ++k) f[k] = factor(k, k == c)[size_t(ix[k]) * w1 + o[k]];
                    const double prod = (d == 3) ? f[0] * (f[1] * f[2]) : (d == 2) ? f[0] * f[1] : f[0];
                    term += prod;
                }
                val[size_t(w - c0) * A.npad + padi] = term;
            }
        }
        A.v64.alloc(val.size() * sizeof(double));
        IGA2L_HIP(hipMemcpy(A.v64.ptr, val.data(), val.size() * sizeof(double), hipMemcpyHostToDevice));
    } else {
        // variable coefficient: sum over elements on the device
        A.v64.alloc(size_t(A.Wh) * A.npad * sizeof(double));
        launch_assemble_dia(P, nullptr);
        IGA2L_HIP(hipStreamSynchronize(nullptr));
    }

    // kappa = 1: rows whose coordinates lie in [2p-1, n1-2p] couple only
    // translates of the cardinal B-spline and carry one common stencil, read
    // here from the centre row of the assembled operator
    P.ulo = 2 * p - 1;
    P.uhi = n1 - 2 * p;
    P.cs64.free();
    P.cs32.free();
    P.cf64.free();
    P.cf32.free();
    P.fac64.free();
    P.fac32.free();
    if (P.kappa_one && P.uhi >= P.ulo) {
        int64_t padc = 0;
        for (int k = 0; k < d; ++k) padc += int64_t(n1 / 2 + p) * A.pitch[k];
        std::vector<double> cs(A.W);
        std::vector<float> cs32(A.W);
        int o[kMaxDim] = {0, 0, 0};
        for (int w = 0; w < A.W; ++w) {
            split(w, d, w1, o);
            int64_t delta = 0;
            for (int k = 0; k < d; ++k) delta += int64_t(o[k] - p) * A.pitch[k];
            cs[w] = (w >= c0) ? val[size_t(w - c0) * A.npad + padc] : val[size_t(c0 - w) * A.npad + padc + delta];
            cs32[w] = float(cs[w]);
        }
        P.cs64.alloc(cs.size() * sizeof(double));
        P.cs32.alloc(cs32.size() * sizeof(float));
        IGA2L_HIP(hipMemcpy(P.cs64.ptr, cs.data(), cs.size() * sizeof(double), hipMemcpyHostToDevice));
        IGA2L_HIP(hipMemcpy(P.cs32.ptr, cs32.data(), cs32.size() * sizeof(float), hipMemcpyHostToDevice));
        // the same stencil as K1 (x) M1 + M1 (x) K1 of the interior 1-D rows, for
        // kernels that apply it by sum factorisation
        const size_t ic = size_t(n1 / 2) * w1;
        std::vector<double> cf(P.K1.begin() + ic, P.K1.begin() + ic + w1);
        cf.insert(cf.end(), P.M1.begin() + ic, P.M1.begin() + ic + w1);
        std::vector<float> cf32(cf.begin(), cf.end());
        P.cf64.alloc(cf.size() * sizeof(double));
        P.cf32.alloc(cf32.size() * sizeof(float));
        IGA2L_HIP(hipMemcpy(P.cf64.ptr, cf.data(), cf.size() * sizeof(double), hipMemcpyHostToDevice));
        IGA2L_HIP(hipMemcpy(P.cf32.ptr, cf32.data(), cf32.size() * sizeof(float), hipMemcpyHostToDevice));
        if (d == 2) {
            // every row of both factors, for the rows next to the boundary,
            // then again as the y factors: A = K1 (x) M1 + M1 (x) K1 in the
            // layout of the direction-dependent factors of the annulus
            std::vector<double> fac(P.K1);
            fac.insert(fac.end(), P.M1.begin(), P.M1.end());
            fac.insert(fac.end(), P.K1.begin(), P.K1.end());
            fac.insert(fac.end(), P.M1.begin(), P.M1.end());
            std::vector<float> fac32(fac.begin(), fac.end());
            P.fac64.alloc(fac.size() * sizeof(double));
            P.fac32.alloc(fac32.size() * sizeof(float));
            IGA2L_HIP(hipMemcpy(P.fac64.ptr, fac.data(), fac.size() * sizeof(double), hipMemcpyHostToDevice));
            IGA2L_HIP(hipMemcpy(P.fac32.ptr, fac32.data(), fac32.size() * sizeof(float), hipMemcpyHostToDevice));
        }
    } else {
        P.ulo = 1;
        P.uhi = 0;
    }

    // kappa = 1 in 3-D: the 1-D factors, from which the kernels form the rows
    // next to the boundary instead of reading (2p+1)^3 diagonals.  Their
    // entry (i, i+o) and the stored entry (i+o, i) must agree bit for bit (so
    // that an entry formed from row i equals the one the symmetric storage
    // keeps for row i+o); otherwise the kernels read the diagonals.
    P.kron64.free();
    P.kron32.free();
    // IGA2L_DIAGONAL_ROWS=1 keeps the diagonals for every row (the two forms
    // give the same FP64 results bit for bit; the switch lets that be checked)
    const char *diag_rows = std::getenv("IGA2L_DIAGONAL_ROWS");
    if (P.kappa_one && d == 3 && !(diag_rows && diag_rows[0] == '1')) {
        bool sym = true;
        for (int i = 0; i < n1 && sym; ++i)
            for (int o = 0; o < w1; ++o) {
                const int j = i + o - p;
                if (j < 0 || j >= n1) continue;
                const size_t a = size_t(i) * w1 + o, b = size_t(j) * w1 + (2 * p - o);
                if (P.K1[a] != P.K1[b] || P.M1[a] != P.M1[b]) sym = false;
            }
        if (sym) {
            std::vector<double> f(P.K1);
            f.insert(f.end(), P.M1.begin(), P.M1.end());
            P.kron64.alloc(f.size() * sizeof(double));
            IGA2L_HIP(hipMemcpy(P.kron64.ptr, f.data(), f.size() * sizeof(double), hipMemcpyHostToDevice));
            std::vector<float> f32(f.begin(), f.end());
            P.kron32.alloc(f32.size() * sizeof(float));
            IGA2L_HIP(hipMemcpy(P.kron32.ptr, f32.data(), f32.size() * sizeof(float), hipMemcpyHostToDevice));
        }
    }

    P.R1d64.alloc(P.R1.size() * sizeof(double));
    IGA2L_HIP(hipMemcpy(P.R1d64.ptr, P.R1.data(), P.R1.size() * sizeof(double), hipMemcpyHostToDevice));
    if (annulus) {
        P.R1yd64.alloc(P.R1y.size() * sizeof(double));
        IGA2L_HIP(hipMemcpy(P.R1yd64.ptr, P.R1y.data(), P.R1y.size() * sizeof(double), hipMemcpyHostToDevice));
        // the operator's 1-D factor rows, for kernels that form its rows by
        // sum factorisation instead of reading the (2p+1)^2 diagonals
        std::vector<double> f(P.K1);
        f.insert(f.end(), P.M1.begin(), P.M1.end());
        f.insert(f.end(), P.K1y.begin(), P.K1y.end());
        f.insert(f.end(), P.M1y.begin(), P.M1y.end());
        P.fac2d64.alloc(f.size() * sizeof(double));
        IGA2L_HIP(hipMemcpy(P.fac2d64.ptr, f.data(), f.size() * sizeof(double), hipMemcpyHostToDevice));
    }

    // workspaces sized by the fine grid
    const size_t nf = size_t(P.fine.n), nc = size_t(P.coarse.n);
    P.r64.alloc(nf * sizeof(double));
    P.ework[0].alloc(nf * sizeof(double));
    P.ework[1].alloc(nf * sizeof(double));
    P.rhs_w.alloc(nf * sizeof(double));
    P.dfine.alloc(nf * sizeof(double));
    P.lam_tmp.alloc(nf * sizeof(double));
    (void)nc;
    host_coarse_workspaces(P);
    P.npartial = int(residual_workgroups(P));
    P.partial.alloc(size_t(P.npartial) * sizeof(double));
    P.hist_cap = 128;
    P.scal.alloc(status_bytes(P.hist_cap));
    IGA2L_HIP(hipMemset(P.scal.ptr, 0, status_bytes(P.hist_cap)));
    IGA2L_HIP(hipHostMalloc(&P.host_status, status_bytes(P.hist_cap), hipHostMallocDefault));
}

// coarse vectors of the cycle, sized by the coarse grid
void host_coarse_workspaces(Problem &P) {
    const size_t nc = size_t(P.coarse.n);
    P.dc.alloc(nc * sizeof(double));
    P.ec.alloc(nc * sizeof(double));
    P.ctmp.alloc(nc * sizeof(double));
    if (P.fp32_ready) {
        P.dc64.alloc(nc * sizeof(double));
        P.ec64.alloc(nc * sizeof(double));
    }
}

// Changes the degree of the coarse space (1 or 2): new transfer factors and
// coarse vectors; every coarse solver and exact-transfer table is dropped
// (they belong to the previous coarse space) and rebuilt on request.
void host_set_coarse_degree(Problem &P, int plow) {
    if (plow == P.plow) return;
    host_transfer_factors(P, plow);
    P.R1d64.alloc(P.R1.size() * sizeof(double));
    IGA2L_HIP(hipMemcpy(P.R1d64.ptr, P.R1.data(), P.R1.size() * sizeof(double), hipMemcpyHostToDevice));
    if (P.fp32_ready) {
        std::vector<float> f32(P.R1.begin(), P.R1.end());
        P.R1d32.alloc(f32.size() * sizeof(float));
        IGA2L_HIP(hipMemcpy(P.R1d32.ptr, f32.data(), f32.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    if (P.geometry == kGeomAnnulus) {
        P.R1yd64.alloc(P.R1y.size() * sizeof(double));
        IGA2L_HIP(hipMemcpy(P.R1yd64.ptr, P.R1y.data(), P.R1y.size() * sizeof(double), hipMemcpyHostToDevice));
        if (P.fp32_ready) {
            std::vector<float> f32(P.R1y.begin(), P.R1y.end());
            P.R1yd32.alloc(f32.size() * sizeof(float));
            IGA2L_HIP(hipMemcpy(P.R1yd32.ptr, f32.data(), f32.size() * sizeof(float), hipMemcpyHostToDevice));
        }
    }
    host_coarse_workspaces(P);
    P.vcycle_ready = P.direct_ready = P.mass_ready = P.agg_direct_ready = false;
    P.coarse_inv64.free();
    P.levels.clear();
    P.levhost64.clear();
    P.levhost32.clear();
    P.ctmp2.free();
}

// Symmetric eigen-decomposition of the n x n row-major matrix C by cyclic
// Jacobi rotations: on return C holds the eigenvalues on its diagonal and Q
// (row-major) the eigenvectors in its columns.
static void jacobi_eigen(int n, std::vector<double> &C, std::vector<double> &Q) {
    Q.assign(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) Q[size_t(i) * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i) {
            diag += C[size_t(i) * n + i] * C[size_t(i) * n + i];
            for (int j = i + 1; j < n; ++j) off += C[size_t(i) * n + j] * C[size_t(i) * n + j];
        }
        if (off <= 1e-32 * diag) break;
        for (int pp = 0; pp < n - 1; ++pp)
            for (int qq = pp + 1; qq < n; ++qq) {
                const double apq = C[size_t(pp) * n + qq];
                if (std::fabs(apq) < 1e-300) continue;
                const double app = C[size_t(pp) * n + pp], aqq = C[size_t(qq) * n + qq];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {   // columns pp, qq
                    const double ckp = C[size_t(k) * n + pp], ckq = C[size_t(k) * n + qq];
                    C[size_t(k) * n + pp] = c * ckp - sn * ckq;
                    C[size_t(k) * n + qq] = sn * ckp + c * ckq;
                }
                for (int k = 0; k < n; ++k) {   // rows pp, qq
                    const double cpk = C[size_t(pp) * n + k], cqk = C[size_t(qq) * n + k];
                    C[size_t(pp) * n + k] = c * cpk - sn * cqk;
                    C[size_t(qq) * n + k] = sn * cpk + c * cqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double qkp = Q[size_t(k) * n + pp], qkq = Q[size_t(k) * n + qq];
                    Q[size_t(k) * n + pp] = c * qkp - sn * qkq;
                    Q[size_t(k) * n + qq] = sn * qkp + c * qkq;
                }
            }
    }
}

// Degree-2 coarse space, kappa = 1: the Dirichlet-reduced 1-D stiffness K2
// and mass M2 (degree 2 on the same knots) give the generalised eigenvectors V
// with V^T M2 V = I, V^T K2 V = diag(lambda) (M2 = L L^T, C = L^{-1} K2 L^{-T} =
// Q diag(lambda) Q^T, V = L^{-T} Q).  The d-dimensional coarse operator
// sum_c (x)_k (k == c ? K2 : M2) is then (V (x) V ..) diag(sum_k lambda_k)
// (V (x) V ..)^T, inverted by one transform per axis each way ("fast
// diagonalisation"); M2^{-1} = (V V^T) per direction for the exact transfers.
// On the annulus each axis has its own weighted K2, M2 (the coarse operator is
// K2x (x) M2y + M2x (x) K2y), hence its own V and eigenvalues.
void host_build_fdm(Problem &P) {
    IGA2L_REQUIRE(P.plow == 2, IGA2L_EINVAL, "fast diagonalisation is the coarse solver of the degree-2 space");
    const bool annulus = P.geometry == kGeomAnnulus;
    IGA2L_REQUIRE(P.kappa_one || annulus, IGA2L_EUNSUPPORTED, "the exact degree-2 coarse solve needs kappa = 1");
    const int m = P.m, n = P.coarse.n1, d = P.dim;
    IGA2L_REQUIRE(n <= 1024, IGA2L_EUNSUPPORTED, "degree-2 coarse space limited to m <= 1024");
    // generalised eigenvectors of one axis: V^T M V = I, V^T K V = diag(lam)
    auto eigen_axis = [&](const std::vector<double> &K, const std::vector<double> &M, std::vector<double> &V,
                          std::vector<double> &lam) {
        // M = L L^T (dense Cholesky, lower)
        std::vector<double> L(M);
        for (int j = 0; j < n; ++j) {
            double s2 = L[size_t(j) * n + j];
            for (int k = 0; k < j; ++k) s2 -= L[size_t(j) * n + k] * L[size_t(j) * n + k];
            IGA2L_REQUIRE(s2 > 0.0, IGA2L_ENUMERIC, "degree-2 mass matrix not positive definite");
            const double ljj = std::sqrt(s2);
            L[size_t(j) * n + j] = ljj;
            for (int i = j + 1; i < n; ++i) {
                double t = L[size_t(i) * n + j];
                for (int k = 0; k < j; ++k) t -= L[size_t(i) * n + k] * L[size_t(j) * n + k];
                L[size_t(i) * n + j] = t / ljj;
            }
            for (int k = j + 1; k < n; ++k) L[size_t(j) * n + k] = 0.0;
        }
        // C = L^{-1} K L^{-T}: solve L X = K, then C^T: L C^T = X^T (C symmetric)
        auto lower_solve = [&](std::vector<double> &B) {   // B <- L^{-1} B, column by column
            for (int c = 0; c < n; ++c)
                for (int i = 0; i < n; ++i) {
                    double t = B[size_t(i) * n + c];
                    for (int k = 0; k < i; ++k) t -= L[size_t(i) * n + k] * B[size_t(k) * n + c];
                    B[size_t(i) * n + c] = t / L[size_t(i) * n + i];
                }
        };
        std::vector<double> X(K);
        lower_solve(X);
        std::vector<double> C(size_t(n) * n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) C[size_t(i) * n + j] = X[size_t(j) * n + i];
        lower_solve(C);
        for (int i = 0; i < n; ++i)           // symmetrise the rounding
            for (int j = i + 1; j < n; ++j) {
                const double a2 = 0.5 * (C[size_t(i) * n + j] + C[size_t(j) * n + i]);
                C[size_t(i) * n + j] = C[size_t(j) * n + i] = a2;
            }
        std::vector<double> Q;
        jacobi_eigen(n, C, Q);
        lam.resize(n);
        for (int i = 0; i < n; ++i) lam[i] = C[size_t(i) * n + i];
        // V = L^{-T} Q: back substitution with L^T, column by column
        V = Q;
        for (int c = 0; c < n; ++c)
            for (int i = n - 1; i >= 0; --i) {
                double t = V[size_t(i) * n + c];
                for (int k = i + 1; k < n; ++k) t -= L[size_t(k) * n + i] * V[size_t(k) * n + c];
                V[size_t(i) * n + c] = t / L[size_t(i) * n + i];
            }
    };
    // the 1-D degree-2 stiffness and (operator) mass of each axis, dense
    auto dense = [&](const std::vector<double> &off) {   // by offset [i][j-i+2] -> n x n
        std::vector<double> D(size_t(n) * n, 0.0);
        for (int i = 0; i < n; ++i)
            for (int o = -2; o <= 2; ++o)
                if (i + o >= 0 && i + o < n) D[size_t(i) * n + i + o] = off[size_t(i) * 5 + o + 2];
        return D;
    };
    const int naxes = annulus ? d : 1;
    std::vector<std::vector<double>> Vax(naxes), lamax(naxes);
    for (int ax = 0; ax < naxes; ++ax) {
        std::vector<double> K(size_t(n) * n, 0.0), M(size_t(n) * n, 0.0);
        if (annulus) {
            K = dense(annulus_form_1d(P, 2, 2, ax, kAnnStiff));
            M = dense(annulus_form_1d(P, 2, 2, ax, kAnnOpMass));
        } else {
            std::vector<std::vector<double>> Ke, Me;
            element_matrices(2, m, Ke, Me);
            for (int e = 0; e < m; ++e)
                for (int a = 0; a <= 2; ++a)
                    for (int b = 0; b <= 2; ++b) {
                        const int i = e + a - 1, j = e + b - 1;
                        if (i < 0 || i >= n || j < 0 || j >= n) continue;
                        K[size_t(i) * n + j] += Ke[e][a * 3 + b];
                        M[size_t(i) * n + j] += Me[e][a * 3 + b];
                    }
        }
        eigen_axis(K, M, Vax[ax], lamax[ax]);
    }
    // forward transform matrices V^T (row k = column k of V), backward V, one
    // per axis for the annulus (stacked, axis stride n^2), one for all otherwise
    std::vector<double> Vt, V;
    for (int ax = 0; ax < naxes; ++ax) {
        for (int k = 0; k < n; ++k)
            for (int i = 0; i < n; ++i) Vt.push_back(Vax[ax][size_t(i) * n + k]);
        V.insert(V.end(), Vax[ax].begin(), Vax[ax].end());
    }
    P.fdm_axis_stride = annulus ? int64_t(n) * n : 0;
    const int64_t nc = ipow(n, d);
    std::vector<double> mu(nc), ones(nc, 1.0);
    int ix[kMaxDim] = {0, 0, 0};
    for (int64_t i = 0; i < nc; ++i) {
        split(i, d, n, ix);
        double sl = 0.0;
        for (int k = 0; k < d; ++k) sl += lamax[annulus ? k : 0][ix[k]];
        mu[i] = sl;
    }
    P.fdm_Vt.alloc(Vt.size() * sizeof(double));
    P.fdm_V.alloc(V.size() * sizeof(double));
    P.dst_mu.alloc(mu.size() * sizeof(double));
    P.dstM_mu.alloc(ones.size() * sizeof(double));
    IGA2L_HIP(hipMemcpy(P.fdm_Vt.ptr, Vt.data(), Vt.size() * sizeof(double), hipMemcpyHostToDevice));
    IGA2L_HIP(hipMemcpy(P.fdm_V.ptr, V.data(), V.size() * sizeof(double), hipMemcpyHostToDevice));
    IGA2L_HIP(hipMemcpy(P.dst_mu.ptr, mu.data(), mu.size() * sizeof(double), hipMemcpyHostToDevice));
    IGA2L_HIP(hipMemcpy(P.dstM_mu.ptr, ones.data(), ones.size() * sizeof(double), hipMemcpyHostToDevice));
    P.direct_ready = true;
}

// ---------------------------------------------------- V-cycle hierarchy --
// Level 0: the degree-1 stiffness on the same knots and kappa, full 3^d
// stencil.  Coarser levels: coarse nodes are the odd-indexed interior nodes
// (0-based) of the finer level, P = linear interpolation, A_c = P^T A P,
// down to a single node per direction.
// The degree-1 operator on the fine knots with the element coefficients
// kappa, [3^d][(m-1)^d], assembled on the device.
static DevBuf assemble_degree1(Problem &P) {
    const int d = P.dim, m = P.m;
    // degree-1 element matrices: K = (1/h)[1 -1; -1 1], M = (h/6)[2 1; 1 2]
    std::vector<std::vector<double>> Kc, Mc;
    element_matrices(1, m, Kc, Mc);
    std::vector<double> km1(size_t(m) * 8);
    for (int el = 0; el < m; ++el)
        for (int k = 0; k < 4; ++k) {
            km1[(size_t(el) * 2 + 0) * 4 + k] = Kc[el][k];
            km1[(size_t(el) * 2 + 1) * 4 + k] = Mc[el][k];
        }
    DevBuf km1_d;
    km1_d.alloc(km1.size() * sizeof(double));
    IGA2L_HIP(hipMemcpy(km1_d.ptr, km1.data(), km1.size() * sizeof(double), hipMemcpyHostToDevice));
    DevBuf S0;
    S0.alloc(size_t(ipow(3, d)) * ipow(m - 1, d) * sizeof(double));
    launch_assemble_q1(d, km1_d.as<double>(), P.kappa_d.as<double>(), m, S0.as<double>(), nullptr);
    IGA2L_HIP(hipDeviceSynchronize());
    return S0;
}

void host_build_levels(Problem &P) {
    const int d = P.dim, m = P.m;
    const int W3 = int(ipow(3, d));
    // stencils of every level, built on the device: the degree-1 operator on
    // the fine knots, then Galerkin products down to the first level with at
    // most kCoarsestMax unknowns; host copies for the per-level book-keeping
    std::vector<DevBuf> dops;
    std::vector<int> sizes;
    dops.push_back(assemble_degree1(P));
    sizes.push_back(m - 1);
    while (ipow(sizes.back(), d) > kCoarsestMax) {
        const int nf1 = sizes.back(), nc1 = nf1 / 2;
        DevBuf Sc;
        Sc.alloc(size_t(W3) * ipow(nc1, d) * sizeof(double));
        launch_galerkin(d, dops.back().as<double>(), nf1, Sc.as<double>(), nc1, nullptr);
        dops.push_back(std::move(Sc));
        sizes.push_back(nc1);
    }
    std::vector<std::vector<double>> ops(dops.size());
    for (size_t l = 0; l < dops.size(); ++l) {
        ops[l].resize(size_t(W3) * ipow(sizes[l], d));
        IGA2L_HIP(hipMemcpy(ops[l].data(), dops[l].ptr, ops[l].size() * sizeof(double), hipMemcpyDeviceToHost));
    }
    P.levels.clear();
    P.levels.resize(ops.size());
    P.levhost64.assign(ops.size(), LevelDev<double>{});
    P.levhost32.assign(ops.size(), LevelDev<float>{});
    const int cw = (W3 - 1) / 2;
    for (size_t l = 0; l < ops.size(); ++l) {
        Level &L = P.levels[l];
        L.g = Grid{d, sizes[l], ipow(sizes[l], d)};
        const auto &S = ops[l];
        const int64_t n = L.g.n;
        const int n1 = L.g.n1;
        L.S64 = std::move(dops[l]);
        std::vector<float> s32(S.begin(), S.end());
        L.S32.alloc(s32.size() * sizeof(float));
        IGA2L_HIP(hipMemcpy(L.S32.ptr, s32.data(), s32.size() * sizeof(float), hipMemcpyHostToDevice));
        std::vector<double> inv(n);
        std::vector<float> inv32(n);
        for (int64_t i = 0; i < n; ++i) {
            inv[i] = 1.0 / S[size_t(cw) * n + i];
            inv32[i] = 1.0f / float(S[size_t(cw) * n + i]);
        }
        L.invd64.alloc(n * sizeof(double));
        L.invd32.alloc(n * sizeof(float));
        IGA2L_HIP(hipMemcpy(L.invd64.ptr, inv.data(), n * sizeof(double), hipMemcpyHostToDevice));
        IGA2L_HIP(hipMemcpy(L.invd32.ptr, inv32.data(), n * sizeof(float), hipMemcpyHostToDevice));
        // translation invariance: every row carries the centre row's coefficients
        // on all of its in-grid neighbours (rows are truncated at the boundary),
        // to 1e-12 of the largest: the element matrices next to the boundary are
        // computed on their own, and their rounding grows with m (the centre
        // coefficient of the last row of the degree-1 operator is 2.6666666666668792
        // against 2.6666666666666679 at m = 4096); the smoother then reads no
        // stored stencil on such a level
        constexpr double kCstTol = 1e-12;
        L.cst = false;
        double ref[27] = {0};
        if (n1 >= 3) {
            int64_t ic = 0;
            for (int k = d - 1; k >= 0; --k) ic = ic * n1 + n1 / 2;
            double scale = 0.0;
            for (int w = 0; w < W3; ++w) {
                ref[w] = S[size_t(w) * n + ic];
                scale = std::max(scale, std::fabs(ref[w]));
            }
            bool same = true;
            int ix[kMaxDim] = {0, 0, 0}, o[kMaxDim] = {0, 0, 0};
            for (int64_t i = 0; i < n && same; ++i) {
                split(i, d, n1, ix);
                for (int w = 0; w < W3 && same; ++w) {
                    split(w, d, 3, o);
                    bool in = true;
                    for (int k = 0; k < d; ++k) {
                        int j = ix[k] + o[k] - 1;
                        if (j < 0 || j >= n1) in = false;
                    }
                    if (in && std::fabs(S[size_t(w) * n + i] - ref[w]) > kCstTol * scale) {
                        same = false;
                        if (tune_log())
                            std::fprintf(stderr, "[iga2l setup] level %zu row %lld offset %d: %.17g against %.17g\n",
                                         l, (long long)i, w, S[size_t(w) * n + i], ref[w]);
                    }
                }
            }
            L.cst = same;
        }
        if (tune_log())
            std::fprintf(stderr, "[iga2l setup] V-cycle level %zu: n1=%d, %s stencil\n", l, n1,
                         L.cst ? "constant" : "stored");
        const size_t nb = size_t(n) * sizeof(double);
        L.e[0].alloc(nb);
        L.e[1].alloc(nb);
        L.rhs.alloc(nb);
        L.res.alloc(nb);
        LevelDev<double> &h64 = P.levhost64[l];
        LevelDev<float> &h32 = P.levhost32[l];
        h64.n1 = h32.n1 = n1;
        h64.n = h32.n = n;
        h64.cst = h32.cst = L.cst ? 1 : 0;
        h64.S = L.S64.as<double>();
        h32.S = L.S32.as<float>();
        h64.invd = L.invd64.as<double>();
        h32.invd = L.invd32.as<float>();
        for (int w = 0; w < 27; ++w) {
            h64.c[w] = (w < W3) ? ref[w] : 0.0;
            h32.c[w] = float(h64.c[w]);
        }
        h64.cinv = L.cst ? 1.0 / ref[cw] : 0.0;
        h32.cinv = L.cst ? 1.0f / float(ref[cw]) : 0.0f;
        h64.Zinv = nullptr;
        h32.Zinv = nullptr;
        if (l + 1 == ops.size()) {
            // coarsest level: dense matrix, Cholesky factor, explicit inverse
            std::vector<double> Z(size_t(n) * n, 0.0);
            int ix[kMaxDim] = {0, 0, 0}, o[kMaxDim] = {0, 0, 0};
            for (int64_t i = 0; i < n; ++i) {
                split(i, d, n1, ix);
                for (int w = 0; w < W3; ++w) {
                    split(w, d, 3, o);
                    bool in = true;
                    int64_t j = 0;
                    for (int k = d - 1; k >= 0; --k) {
                        const int jk = ix[k] + o[k] - 1;
                        if (jk < 0 || jk >= n1) in = false;
                        j = j * n1 + jk;
                    }
                    if (in) Z[size_t(i) * n + j] = S[size_t(w) * n + i];
                }
            }
            std::vector<double> Lc(Z);  // lower Cholesky factor in place
            for (int64_t j = 0; j < n; ++j) {
                double sdiag = Lc[size_t(j) * n + j];
                for (int64_t k = 0; k < j; ++k) sdiag -= Lc[size_t(j) * n + k] * Lc[size_t(j) * n + k];
                IGA2L_REQUIRE(sdiag > 0.0, IGA2L_ENUMERIC, "coarsest V-cycle level is not positive definite");
                const double ljj = std::sqrt(sdiag);
                Lc[size_t(j) * n + j] = ljj;
                for (int64_t i = j + 1; i < n; ++i) {
                    double t = Lc[size_t(i) * n + j];
                    for (int64_t k = 0; k < j; ++k) t -= Lc[size_t(i) * n + k] * Lc[size_t(j) * n + k];
                    Lc[size_t(i) * n + j] = t / ljj;
                }
            }
            // columns of Z^{-1}: solve L L^T x = e_c
            std::vector<double> Zi(size_t(n) * n), col(n);
            for (int64_t c = 0; c < n; ++c) {
                for (int64_t i = 0; i < n; ++i) col[i] = (i == c) ? 1.0 : 0.0;
                for (int64_t i = 0; i < n; ++i) {
                    double t = col[i];
                    for (int64_t k = 0; k < i; ++k) t -= Lc[size_t(i) * n + k] * col[k];
                    col[i] = t / Lc[size_t(i) * n + i];
                }
                for (int64_t i = n - 1; i >= 0; --i) {
                    double t = col[i];
                    for (int64_t k = i + 1; k < n; ++k) t -= Lc[size_t(k) * n + i] * col[k];
                    col[i] = t / Lc[size_t(i) * n + i];
                }
                for (int64_t i = 0; i < n; ++i) Zi[size_t(i) * n + c] = col[i];
            }
            std::vector<float> Zi32(Zi.begin(), Zi.end());
            L.Zinv64.alloc(Zi.size() * sizeof(double));
            L.Zinv32.alloc(Zi32.size() * sizeof(float));
            IGA2L_HIP(hipMemcpy(L.Zinv64.ptr, Zi.data(), Zi.size() * sizeof(double), hipMemcpyHostToDevice));
            IGA2L_HIP(hipMemcpy(L.Zinv32.ptr, Zi32.data(), Zi32.size() * sizeof(float), hipMemcpyHostToDevice));
            h64.Zinv = L.Zinv64.as<double>();
            h32.Zinv = L.Zinv32.as<float>();
        }
    }
    P.levdev64.alloc(P.levhost64.size() * sizeof(LevelDev<double>));
    P.levdev32.alloc(P.levhost32.size() * sizeof(LevelDev<float>));
    IGA2L_HIP(hipMemcpy(P.levdev64.ptr, P.levhost64.data(), P.levhost64.size() * sizeof(LevelDev<double>),
                        hipMemcpyHostToDevice));
    IGA2L_HIP(hipMemcpy(P.levdev32.ptr, P.levhost32.data(), P.levhost32.size() * sizeof(LevelDev<float>),
                        hipMemcpyHostToDevice));
    // the one-workgroup tail starts at the first level whose whole tail fits in
    // 64 KiB of LDS (and whose half steps need at most the per-thread budget)
    const int64_t lds_budget = 64 * 1024;
    auto pick = [&](size_t elem) {
        for (size_t lb = 0; lb < P.levels.size(); ++lb)
            if (vcycle_bottom_fits(P, lb) && vcycle_bottom_lds(P, lb) * int64_t(elem) <= lds_budget) return lb;
        return P.levels.size() - 1;
    };
    P.vc_bottom64 = pick(sizeof(double));
    P.vc_bottom32 = pick(sizeof(float));
    P.vcycle_ready = true;
}

// ------------------------------------------------------- exact coarse --
// For kappa = 1 the degree-1 operator on the uniform mesh is a sum of
// Kronecker products of (1/h) tridiag(-1,2,-1) and (h/6) tridiag(1,4,1), all
// diagonalised by the orthonormal DST-I matrix S_ik = sqrt(2/m) sin((i+1)(k+1)pi/m).
// The degree-1 stiffness and mass matrices on a uniform grid of m cells with
// homogeneous Dirichlet conditions, (1/h) tridiag(-1, 2, -1) and
// (h/6) tridiag(1, 4, 1) per direction, are diagonalised by the orthonormal
// DST-I matrix S_ik = sqrt(2/m) sin(ik pi/m) with eigenvalues
// (2/h)(1 - cos t_k) and (h/3)(2 + cos t_k), t_k = k pi/m.  stiffness: mu =
// eigenvalues of the d-dimensional stiffness sum_c prod_k (k == c ? K : M);
// otherwise of the mass matrix prod_k M.
static void dst_tables(int m, int d, bool stiffness, DevBuf &Sd, DevBuf &mud) {
    const int n1 = m - 1;
    const double h = 1.0 / m;
    std::vector<double> S(size_t(n1) * n1), lk(n1), lm(n1);
    for (int i = 0; i < n1; ++i)
        for (int k = 0; k < n1; ++k) S[size_t(i) * n1 + k] = std::sqrt(2.0 / m) * std::sin((i + 1.0) * (k + 1.0) * M_PI / m);
    for (int k = 0; k < n1; ++k) {
        double th = (k + 1.0) * M_PI / m;
        lk[k] = (2.0 / h) * (1.0 - std::cos(th));
        lm[k] = (h / 3.0) * (2.0 + std::cos(th));
    }
    const int64_t n = ipow(n1, d);
    std::vector<double> mu(n);
    int ix[kMaxDim] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        split(i, d, n1, ix);
        if (stiffness) {
            double s = 0.0;
            for (int c = 0; c < d; ++c) {
                double prod = 1.0;
                for (int k = 0; k < d; ++k) prod *= (k == c) ? lk[ix[k]] : lm[ix[k]];
                s += prod;
            }
            mu[i] = s;
        } else {
            double prod = 1.0;
            for (int k = 0; k < d; ++k) prod *= lm[ix[k]];
            mu[i] = prod;
        }
    }
    Sd.alloc(S.size() * sizeof(double));
    mud.alloc(mu.size() * sizeof(double));
    IGA2L_HIP(hipMemcpy(Sd.ptr, S.data(), S.size() * sizeof(double), hipMemcpyHostToDevice));
    IGA2L_HIP(hipMemcpy(mud.ptr, mu.data(), mu.size() * sizeof(double), hipMemcpyHostToDevice));
}

// Variable kappa, degree-1 coarse space: A_1 (the degree-1 operator with the
// element coefficients) factored by banded Cholesky, L L^T with L(i, i-k) for
// k <= bw = the largest stencil offset; then A_1^{-1} column by column (one
// banded forward and one backward solve each), uploaded as a dense matrix
// that the exact coarse solve applies on the device.  O(n bw^2) for the
// factor and O(n^2 bw) for the inverse: bounded by kCoarseInvMax unknowns.
static void host_build_coarse_inverse(Problem &P) {
    const int d = P.dim, n1 = P.m - 1;
    const int W3 = int(ipow(3, d));
    const int64_t n = ipow(n1, d);
    IGA2L_REQUIRE(n <= kCoarseInvMax, IGA2L_EUNSUPPORTED,
                  "the exact coarse solve with variable kappa is limited to 4096 coarse unknowns; use the V-cycle");
    DevBuf S0 = assemble_degree1(P);
    std::vector<double> S(size_t(W3) * n);
    IGA2L_HIP(hipMemcpy(S.data(), S0.ptr, S.size() * sizeof(double), hipMemcpyDeviceToHost));
    int64_t bw = 0;  // offset of the (+1, +1, +1) neighbour
    for (int k = 0; k < d; ++k) bw = bw * n1 + 1;
    const int64_t w1 = bw + 1;
    // A(i, i-k) for 0 <= k <= bw, row i: from the stencil entries of row i
    std::vector<double> Lb(size_t(n) * w1, 0.0);
    int ix[kMaxDim] = {0, 0, 0}, o[kMaxDim] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        split(i, d, n1, ix);
        for (int w = 0; w < W3; ++w) {
            split(w, d, 3, o);
            bool in = true;
            int64_t j = 0;
            for (int k = d - 1; k >= 0; --k) {
                const int jk = ix[k] + o[k] - 1;
                if (jk < 0 || jk >= n1) in = false;
                j = j * n1 + jk;
            }
            if (in && j <= i) Lb[size_t(i) * w1 + (i - j)] = S[size_t(w) * n + i];
        }
    }
    auto L = [&](int64_t i, int64_t j) -> double & { return Lb[size_t(i) * w1 + (i - j)]; };
    for (int64_t i = 0; i < n; ++i) {
        const int64_t j0 = std::max<int64_t>(0, i - bw);
        for (int64_t j = j0; j <= i; ++j) {
            double t = L(i, j);
            for (int64_t k = std::max(j0, j - bw); k < j; ++k) t -= L(i, k) * L(j, k);
            if (j == i) {
                IGA2L_REQUIRE(t > 0.0, IGA2L_ENUMERIC, "coarse operator is not positive definite");
                L(i, i) = std::sqrt(t);
            } else {
                L(i, j) = t / L(j, j);
            }
        }
    }
    std::vector<double> Zi(size_t(n) * n), col(n);
    for (int64_t c = 0; c < n; ++c) {
        std::fill(col.begin(), col.end(), 0.0);
        col[c] = 1.0;
        for (int64_t i = c; i < n; ++i) {
            double t = col[i];
            for (int64_t k = std::max(c, i - bw); k < i; ++k) t -= L(i, k) * col[k];
            col[i] = t / L(i, i);
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            double t = col[i];
            for (int64_t k = i + 1; k <= std::min(n - 1, i + bw); ++k) t -= L(k, i) * col[k];
            col[i] = t / L(i, i);
        }
        for (int64_t i = 0; i < n; ++i) Zi[size_t(i) * n + c] = col[i];
    }
    P.coarse_inv64.alloc(Zi.size() * sizeof(double));
    IGA2L_HIP(hipMemcpy(P.coarse_inv64.ptr, Zi.data(), Zi.size() * sizeof(double), hipMemcpyHostToDevice));
    P.direct_ready = true;
}

void host_build_dst(Problem &P) {
    if (P.plow == 2) {
        host_build_fdm(P);
        return;
    }
    if (!P.kappa_one && P.geometry == kGeomSquare) {
        host_build_coarse_inverse(P);
        return;
    }
    dst_tables(P.m, P.dim, true, P.dst_S, P.dst_mu);
    P.direct_ready = true;
}

// exact transfers (Section 3.1.2 without lumping): the unlumped factor and
// the DST-I of the degree-1 mass matrix
void host_build_mass(Problem &P) {
    if (P.plow == 2) {
        // M2^{-1} = (V V^T) per direction: the fast-diagonalisation tables with unit eigenvalues
        if (!P.direct_ready) host_build_fdm(P);
    } else {
        dst_tables(P.m, P.dim, false, P.dstM_S, P.dstM_mu);
    }
    P.Mx64.alloc(P.Mx1.size() * sizeof(double));
    IGA2L_HIP(hipMemcpy(P.Mx64.ptr, P.Mx1.data(), P.Mx1.size() * sizeof(double), hipMemcpyHostToDevice));
    std::vector<float> f32(P.Mx1.begin(), P.Mx1.end());
    P.Mx32.alloc(f32.size() * sizeof(float));
    IGA2L_HIP(hipMemcpy(P.Mx32.ptr, f32.data(), f32.size() * sizeof(float), hipMemcpyHostToDevice));
    P.ctmp2.alloc(size_t(P.coarse.n) * sizeof(double));
    P.mass_ready = true;
}

// aggressive coarsening, exact 2h solve: level 1 of the hierarchy is the
// degree-1 operator on m/2 cells (Galerkin = rediscretisation for kappa = 1
// with full coarsening of an even m), solved by its DST-I
void host_build_agg_direct(Problem &P) {
    IGA2L_REQUIRE(P.kappa_one, IGA2L_EUNSUPPORTED, "the exact 2h solve of aggressive coarsening needs kappa = 1");
    IGA2L_REQUIRE(P.m % 2 == 0, IGA2L_EUNSUPPORTED, "the exact 2h solve of aggressive coarsening needs an even m");
    IGA2L_REQUIRE(P.levels.size() >= 2 && P.levels[1].g.n1 == P.m / 2 - 1, IGA2L_EUNSUPPORTED,
                  "aggressive coarsening needs a V-cycle hierarchy with a 2h level");
    dst_tables(P.m / 2, P.dim, true, P.dst2_S, P.dst2_mu);
    const size_t n2 = size_t(P.levels[1].g.n);
    P.agg64.alloc(4 * n2 * sizeof(double));   // rhs, solution, transform buffer, FP64 staging
    P.agg_direct_ready = true;
}

// ------------------------------------------------------- block classes --
// A block matrix depends only on the 1-D position class of its centre in each
// direction when kappa = 1 (the operator is a sum of Kronecker products of
// 1-D factors).  Centres within L = p-1+hb of either end form individual
// classes; all others share the uniform interior class.  With a variable
// coefficient every DOF is its own class.  reps gets one representative
// centre (linear DOF index) per inverse slot; slot = sum_k cls[j_k] ncls^k.
void host_block_classes(Problem &P, std::vector<int> &cls1, std::vector<int64_t> &reps) {
    const int n1 = P.fine.n1, d = P.dim, hb = (P.bw - 1) / 2;
    const int L = P.p - 1 + hb;
    std::vector<int> rep1;
    cls1.assign(n1, 0);
    if (P.kappa_one && n1 >= 2 * L + 2) {
        P.shared_inverses = true;
        P.ncls1 = 2 * L + 1;
        for (int j = 0; j < n1; ++j) {
            if (j < L) cls1[j] = j;
            else if (j > n1 - 1 - L) cls1[j] = L + 1 + (j - (n1 - L));
            else cls1[j] = L;
        }
        rep1.resize(P.ncls1);
        for (int j = n1 - 1; j >= 0; --j) rep1[cls1[j]] = j;
    } else {
        P.shared_inverses = false;
        P.ncls1 = n1;
        rep1.resize(n1);
        for (int j = 0; j < n1; ++j) cls1[j] = rep1[j] = j;
    }
    P.nslots = ipow(P.ncls1, d);
    reps.resize(P.nslots);
    int c[kMaxDim] = {0, 0, 0};
    for (int64_t s = 0; s < P.nslots; ++s) {
        split(s, d, P.ncls1, c);
        int64_t j = 0;
        for (int k = d - 1; k >= 0; --k) j = j * n1 + rep1[c[k]];
        reps[s] = j;
    }
}

// ------------------------------------------------- lexicographic schedule --
// Block j runs at step t(j) = j_x + S j_y + S^2 j_z with S = bw + p: two blocks
// that interact (centres closer than bw + p in every direction) are then
// ordered as in the lexicographic sequence, and blocks of one step never
// interact, so each step may run all its blocks at once.
void host_lex_schedule(Problem &P) {
    const int n1 = P.fine.n1, d = P.dim;
    const int64_t S = P.bw + P.p;
    const int64_t n = P.fine.n;
    std::vector<int64_t> tj(n);
    int64_t tmax = 0;
    int ix[kMaxDim] = {0, 0, 0};
    for (int64_t j = 0; j < n; ++j) {
        split(j, d, n1, ix);
        int64_t t = 0;
        for (int k = d - 1; k >= 0; --k) t = t * S + ix[k];
        tj[j] = t;
        tmax = std::max(tmax, t);
    }
    std::vector<int> count(tmax + 2, 0);
    for (int64_t j = 0; j < n; ++j) count[tj[j] + 1]++;
    // compress empty steps away
    std::vector<int> off;
    off.push_back(0);
    std::vector<int64_t> order(n);
    std::vector<int> start(tmax + 2, 0);
    for (int64_t t = 0; t <= tmax; ++t) start[t + 1] = start[t] + count[t + 1];
    std::vector<int> fill(start.begin(), start.end());
    for (int64_t j = 0; j < n; ++j) order[fill[tj[j]]++] = j;
    for (int64_t t = 0; t <= tmax; ++t)
        if (count[t + 1] > 0) off.push_back(start[t + 1]);
    P.lex_off = off;
    std::vector<int> blocks(order.begin(), order.end());
    P.lex_blocks.alloc(blocks.size() * sizeof(int));
    IGA2L_HIP(hipMemcpy(P.lex_blocks.ptr, blocks.data(), blocks.size() * sizeof(int), hipMemcpyHostToDevice));
    P.lex_off_d.alloc(off.size() * sizeof(int));
    IGA2L_HIP(hipMemcpy(P.lex_off_d.ptr, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice));
    P.lex_maxcnt = 0;
    for (size_t k = 0; k + 1 < off.size(); ++k) P.lex_maxcnt = std::max(P.lex_maxcnt, off[k + 1] - off[k]);
}

}  // namespace iga2l
