// Device-side common definitions shared by the sfiga kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace sfiga {

constexpr int kMaxOrder = 9;

// 1D Gauss tables of one direction, device memory (Sec. 6.1).  Element e
// activates functions e .. e+P-1 (open knots, simple interior knots).
struct Dir {
    const double *B;   // [K][P][P]: B[(e*P+g)*P+j] = phi_{e+j}(x_{e,g})
    const double *D;   // [K][P][P]: first derivative
    const double *W;   // [K][P]: Gauss weights mapped to the element
    const double *X;   // [K][P]: Gauss points
    const float *Bf;   // B and D rounded to FP32, for the FP32-computing kernels
    const float *Df;
    int K, N, Q;       // elements, functions (K+P-1), quadrature points (K*P)
};

// CSR row offsets in closed form: per direction, S[i] = sum_{i'<i} len(i'),
// len(i) = min(N-1, i+P-1) - max(0, i-P+1) + 1 (Corollary on #NZ), T = S[N].
struct RowIndex {
    const int64_t *S[3];
    int64_t T[3];
    int N[3];
    int P;
    int d;
};

__device__ __forceinline__ int band_lo(int i, int P) { return i - P + 1 > 0 ? i - P + 1 : 0; }
__device__ __forceinline__ int band_hi(int i, int P, int N) { return i + P - 1 < N - 1 ? i + P - 1 : N - 1; }
__device__ __forceinline__ int band_len(int i, int P, int N) { return band_hi(i, P, N) - band_lo(i, P) + 1; }

// First nonzero of row m = (m0, m1, m2) in the lexicographic CSR layout.
__device__ __forceinline__ int64_t row_start(const RowIndex &ri, int m0, int m1, int m2)
{
    const int P = ri.P;
    if (ri.d == 1) return ri.S[0][m0];
    const int64_t l0 = band_len(m0, P, ri.N[0]);
    (void)l0;
    if (ri.d == 2) return ri.S[1][m1] * ri.T[0] + (int64_t)band_len(m1, P, ri.N[1]) * ri.S[0][m0];
    const int64_t l2 = band_len(m2, P, ri.N[2]);
    const int64_t l1 = band_len(m1, P, ri.N[1]);
    return ri.S[2][m2] * ri.T[1] * ri.T[0] + l2 * (ri.S[1][m1] * ri.T[0] + l1 * ri.S[0][m0]);
}

// Position of column n inside row m (columns ascending, direction 1 fastest).
__device__ __forceinline__ int64_t col_offset(const RowIndex &ri, int m0, int m1, int m2, int n0, int n1, int n2)
{
    const int P = ri.P;
    int64_t off = n0 - band_lo(m0, P);
    if (ri.d >= 2) off += (int64_t)(n1 - band_lo(m1, P)) * band_len(m0, P, ri.N[0]);
    if (ri.d >= 3)
        off += (int64_t)(n2 - band_lo(m2, P)) * band_len(m1, P, ri.N[1]) * band_len(m0, P, ri.N[0]);
    return off;
}

// Component order of the symmetric stiffness coefficient tensor.
// d = 3: 00 11 22 01 02 12;  d = 2: 00 11 01;  d = 1: 00.
template <int DIM>
__host__ __device__ constexpr int sym_comp(int i, int j)
{
    if (DIM == 1) return 0;
    if (i == j) return i;
    int a = i < j ? i : j, b = i < j ? j : i;
    if (DIM == 2) return 2;
    return (a == 0) ? (b == 1 ? 3 : 4) : 5;
}

template <typename T>
__device__ __forceinline__ T from_double(double v) { return (T)v; }

// Coefficient descriptors (SF_COEF_*).
struct Coef {
    int kind;           // 0 const, 1 sinprod, 2 qp values
    double value;       // constant value or alpha
    const double *qp;   // [Q] lexicographic quadrature values (kind 2)
};

__device__ __forceinline__ double eval_coef(const Coef &c, const double *x, int d, int64_t qlin)
{
    if (c.kind == 0) return c.value;
    if (c.kind == 2) return c.qp[qlin];
    double s = 1.0;
    // sin(2 pi x) as sinpi(2 x): the argument reduction is exact in FP64 and
    // cheaper than reducing a multiple of pi
    for (int i = 0; i < d; ++i) s *= sinpi(2.0 * x[i]);
    return 1.0 + c.value * s;
}

}  // namespace sfiga
