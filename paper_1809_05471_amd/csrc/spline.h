// Host-side 1D spline layer: knot validation, Gauss-Legendre rule and the
// per-element value/derivative tables at the Gauss points (Sec. 6.1: the
// univariate tables are precomputed once, at cost sum_k p^2 #X_k).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace sfiga {

struct Tables1D {
    int p = 0;          // order
    int nel = 0;        // elements K
    int nfun = 0;       // basis functions N = K + p - 1
    // [e][g][j], j = local index of the active function first(e) + j = e + j
    std::vector<double> B, D;
    std::vector<double> w, x;   // [e][g] weights and points
};

// Returns an empty string on success, else the reason.  `unsupported` is set
// when the knot vector is valid but outside what the kernels handle
// (interior knot multiplicity above one).
std::string build_tables_1d(const double *knots, int64_t nk, int p, Tables1D &out, bool &unsupported);

// p-point Gauss-Legendre rule on [-1, 1] (Newton on the three-term recurrence).
void gauss_legendre(int p, std::vector<double> &nodes, std::vector<double> &weights);

}  // namespace sfiga
