// Host-side 1D spline layer (see spline.h).
#include "spline.h"

#include <cmath>

namespace sfiga {

// Gauss-Legendre rule with p points on [-1, 1]: Newton's method on the
// Legendre polynomial P_p, evaluated by its three-term (Bonnet) recurrence,
// started from the classical cosine approximation of the roots; weights
// 2 / ((1 - z^2) P_p'(z)^2).  A textbook method (e.g. Abramowitz & Stegun,
// 25.4.29, and the Gauss-Legendre routines of Numerical Recipes), restated.
void gauss_legendre(int p, std::vector<double> &nodes, std::vector<double> &weights)
{
    nodes.assign(p, 0.0);
    weights.assign(p, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < (p + 1) / 2; ++i) {
        // Chebyshev-like initial guess for the i-th largest root of P_p
        double z = std::cos(pi * (i + 0.75) / (p + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            // P_p(z) and P_p'(z) from (k+1) P_{k+1} = (2k+1) z P_k - k P_{k-1}
            double pk = z, pkm1 = 1.0;
            for (int k = 1; k < p; ++k) {
                double pkp1 = ((2.0 * k + 1.0) * z * pk - k * pkm1) / (k + 1.0);
                pkm1 = pk;
                pk = pkp1;
            }
            dp = p * (z * pk - pkm1) / (z * z - 1.0);
            double dz = pk / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                // one more recurrence pass for the derivative at the converged root
                pk = z; pkm1 = 1.0;
                for (int k = 1; k < p; ++k) {
                    double pkp1 = ((2.0 * k + 1.0) * z * pk - k * pkm1) / (k + 1.0);
                    pkm1 = pk;
                    pk = pkp1;
                }
                dp = p * (z * pk - pkm1) / (z * z - 1.0);
                break;
            }
        }
        nodes[i] = -z;
        nodes[p - 1 - i] = z;
        double wi = 2.0 / ((1.0 - z * z) * dp * dp);
        weights[i] = wi;
        weights[p - 1 - i] = wi;
    }
    if (p % 2 == 1) nodes[p / 2] = 0.0;
}

// Values and first derivatives of the p B-splines of order p that are
// nonzero on knot span [t[k], t[k+1]) at x, by de Boor's triangular scheme
// (left/right differences), then the derivative from the order p-1 values.
// This is the textbook basis-function table (de Boor, "A Practical Guide to
// Splines"; Piegl & Tiller, "The NURBS Book", algorithms A2.2 and A2.3, whose
// layout keeps the knot differences in the lower triangle), restated.
static void basis_funs(const double *t, int k, int p, double x, double *val, double *der)
{
    const int deg = p - 1;
    std::vector<double> left(p + 1), right(p + 1);
    // ndu[r][c]: column c = basis of degree r (upper triangle), knot differences below
    std::vector<double> ndu((p) * (p), 0.0);
    auto N = [&](int r, int c) -> double & { return ndu[r * p + c]; };
    N(0, 0) = 1.0;
    for (int j = 1; j <= deg; ++j) {
        left[j] = x - t[k + 1 - j];
        right[j] = t[k + j] - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            N(j, r) = right[r + 1] + left[j - r];    // lower triangle: knot differences
            double tmp = N(r, j - 1) / N(j, r);
            N(r, j) = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        N(j, j) = saved;
    }
    for (int j = 0; j <= deg; ++j) val[j] = N(j, deg);
    if (deg == 0) {
        der[0] = 0.0;
        return;
    }
    // first derivative: deg * (N_{j,deg-1}/(t_{j+deg}-t_j) - N_{j+1,deg-1}/(t_{j+deg+1}-t_{j+1}))
    for (int j = 0; j <= deg; ++j) {
        double d = 0.0;
        if (j >= 1) d += N(j - 1, deg - 1) / N(deg, j - 1);
        if (j <= deg - 1) d -= N(j, deg - 1) / N(deg, j);
        der[j] = deg * d;
    }
}

std::string build_tables_1d(const double *t, int64_t nk, int p, Tables1D &out, bool &unsupported)
{
    unsupported = false;
    if (p < 1) return "order must be >= 1";
    if (nk < 2 * p) return "knot vector shorter than 2*order";
    for (int64_t i = 0; i + 1 < nk; ++i)
        if (!(t[i] <= t[i + 1])) return "knot vector not nondecreasing";
    for (int i = 1; i < p; ++i)
        if (t[i] != t[0] || t[nk - 1 - i] != t[nk - 1]) return "knot vector is not open";
    if (!(t[0] < t[nk - 1])) return "knot vector spans an empty interval";
    if (t[p] == t[0] || t[nk - 1 - p] == t[nk - 1]) return "knot multiplicity at an end exceeds the order";
    // interior knots: the kernels assume maximal smoothness (simple knots)
    for (int64_t i = p; i + 1 < nk - p; ++i)
        if (t[i] == t[i + 1]) { unsupported = true; return "interior knot multiplicity > 1 is not supported"; }

    const int K = (int)(nk - 2 * p + 1);
    out.p = p;
    out.nel = K;
    out.nfun = K + p - 1;
    out.B.assign((size_t)K * p * p, 0.0);
    out.D.assign((size_t)K * p * p, 0.0);
    out.w.assign((size_t)K * p, 0.0);
    out.x.assign((size_t)K * p, 0.0);
    std::vector<double> gn, gw;
    gauss_legendre(p, gn, gw);
    std::vector<double> val(p), der(p);
    for (int e = 0; e < K; ++e) {
        const int k = e + p - 1;              // span index: [t_k, t_{k+1})
        const double a = t[k], b = t[k + 1];
        for (int g = 0; g < p; ++g) {
            double x = a + 0.5 * (b - a) * (gn[g] + 1.0);
            out.x[(size_t)e * p + g] = x;
            out.w[(size_t)e * p + g] = 0.5 * (b - a) * gw[g];
            basis_funs(t, k, p, x, val.data(), der.data());
            for (int j = 0; j < p; ++j) {
                out.B[((size_t)e * p + g) * p + j] = val[j];
                out.D[((size_t)e * p + g) * p + j] = der[j];
            }
        }
    }
    return std::string();
}

}  // namespace sfiga
