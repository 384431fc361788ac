// Matrix-free product of the convection form, d = 3, FP64: the b . grad u
// term of the convection-diffusion equation of Sec. 2, Example 1, tested
// with v.  With u = sum_n x_n phi_n,
//   y_m = sum_x c(x) . grad_hat u(x) phi_m(x),   c = w s(G) |det J| J^-1 b,
// c folded per quadrature point by the geometry step (conv_coef_index
// layout).  The trial side needs the three reference derivatives of u
// (Algorithm 3 with the derivative table in one direction at a time), the
// test side only values (Algorithm 2 with value tables), so the form is not
// symmetric and is computed by a pair of kernels over the same grid (element
// tile of E x E elements in directions 1 and 2, E = apply_tile_elems(P), one
// element layer in direction 3 per workgroup):
//   conv_forward_kernel   the tile's x block (E+p-1)^2 x p, contracted
//                         3 -> 2 -> 1 through LDS into the three derivatives
//                         at the tile's points, dotted with c, stored to the
//                         point buffer h (one contiguous block per tile and
//                         layer);
//   conv_backward_kernel  h of the tile and layer, contracted with the value
//                         tables 1 -> 2 -> 3 (the sums over the elements that
//                         share a function formed inside the tile), added into
//                         y with FP64 atomics (tiles and layers overlap in p-1
//                         functions per direction).
// HBM per quadrature point: c (24 B) and h written and read (16 B), plus
// the x block and the y atomics (about 43 and 43 values per element at
// order 6, E = 3).
#include "kernels.h"

namespace sfiga {

template <int P>
struct ConvTile {
    static constexpr int E = apply_tile_elems(P);
    static constexpr int T = E * P;         // quadrature points per tile side
    static constexpr int NF = E + P - 1;    // functions per tile side
    static constexpr int NT = 256;
};

template <int P>
__global__ __launch_bounds__(256) void conv_forward_kernel(PatchView pv, const double *__restrict__ cv,
                                                           const double *__restrict__ x, double *__restrict__ h)
{
    using CT = ConvTile<P>;
    constexpr int E = CT::E, T = CT::T, NF = CT::NF, NT = CT::NT, NFF = NF * NF, TT = T * T;
    constexpr int SB = P * T * NF;           // one field of the direction-2 results
    __shared__ double xs[P * NFF];           // x rows e3 .. e3+p-1 of the tile: [s][ly][lx]
    __shared__ double sa[2 * P * NFF];       // B3 x, D3 x: [2][g3][ly][lx]
    __shared__ double sb[3 * SB];            // B2 B3 x, D2 B3 x, B2 D3 x: [3][g3][yy][lx]
    const Dir &d0 = pv.dir[0], &d1 = pv.dir[1], &d2 = pv.dir[2];
    const int bx = blockIdx.x, by = blockIdx.y, e3 = blockIdx.z;
    const int e1b = bx * E, e2b = by * E;
    const int64_t N0 = d0.N, N01 = (int64_t)d0.N * d1.N;
    const int tid = threadIdx.x;

    for (int i = tid; i < P * NFF; i += NT) {
        const int s = i / NFF, j = i % NFF;
        const int n0 = e1b + j % NF, n1 = e2b + j / NF;
        xs[i] = (n0 < d0.N && n1 < d1.N) ? x[n0 + N0 * n1 + N01 * (e3 + s)] : 0.0;
    }
    __syncthreads();
    // direction 3: a = B3 x, b = D3 x per plane g3 and function column
    const double *B3 = d2.B + (int64_t)e3 * P * P, *D3 = d2.D + (int64_t)e3 * P * P;
    for (int i = tid; i < P * NFF; i += NT) {
        const int g3 = i / NFF, j = i % NFF;
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int s = 0; s < P; ++s) {
            const double v = xs[s * NFF + j];
            a += B3[g3 * P + s] * v;
            b += D3[g3 * P + s] * v;
        }
        sa[i] = a;
        sa[P * NFF + i] = b;
    }
    __syncthreads();
    // direction 2, per point row yy = (element l2, point h2): B2 a (for d1),
    // D2 a (d2), B2 b (d3)
    for (int i = tid; i < SB; i += NT) {
        const int lx = i % NF, yy = (i / NF) % T, g3 = i / (NF * T);
        const int l2 = yy / P, h2 = yy % P;
        const int e2 = min(e2b + l2, d1.K - 1);     // rows outside the patch: any table, results unused
        const double *B2 = d1.B + ((int64_t)e2 * P + h2) * P, *D2 = d1.D + ((int64_t)e2 * P + h2) * P;
        const double *ca = sa + g3 * NFF + l2 * NF + lx, *cb = ca + P * NFF;
        double f0 = 0.0, f1 = 0.0, f2 = 0.0;
#pragma unroll
        for (int s = 0; s < P; ++s) {
            f0 += B2[s] * ca[s * NF];
            f1 += D2[s] * ca[s * NF];
            f2 += B2[s] * cb[s * NF];
        }
        sb[i] = f0;
        sb[SB + i] = f1;
        sb[2 * SB + i] = f2;
    }
    __syncthreads();
    // direction 1 and the pointwise product, per point (g3, yy, xx)
    const int64_t tile = (int64_t)by * gridDim.x + bx;
    const int64_t hb = (tile * d2.Q + (int64_t)e3 * P) * TT;           // first point of the layer
    const int64_t cb0 = (tile * d2.Q + (int64_t)e3 * P) * 3 * TT;
    for (int i = tid; i < P * TT; i += NT) {
        const int xx = i % T, yy = (i / T) % T, g3 = i / TT;
        const int l1 = xx / P, h1 = xx % P;
        const int e1 = min(e1b + l1, d0.K - 1);
        const double *B1 = d0.B + ((int64_t)e1 * P + h1) * P, *D1 = d0.D + ((int64_t)e1 * P + h1) * P;
        const double *r = sb + (g3 * T + yy) * NF + l1;
        double u1 = 0.0, u2 = 0.0, u3 = 0.0;
#pragma unroll
        for (int s = 0; s < P; ++s) {
            u1 += D1[s] * r[s];
            u2 += B1[s] * r[SB + s];
            u3 += B1[s] * r[2 * SB + s];
        }
        // points outside the patch have c = 0
        const double *c = cv + cb0 + (int64_t)g3 * 3 * TT + yy * T + xx;
        h[hb + i] = c[0] * u1 + c[TT] * u2 + c[2 * TT] * u3;
    }
}

template <int P>
__global__ __launch_bounds__(256) void conv_backward_kernel(PatchView pv, const double *__restrict__ h,
                                                            double *__restrict__ y)
{
    using CT = ConvTile<P>;
    constexpr int E = CT::E, T = CT::T, NF = CT::NF, NT = CT::NT, NFF = NF * NF, TT = T * T;
    __shared__ double hs[P * TT];            // the tile's point values: [g3][yy][xx]
    __shared__ double r1[P * T * NF];        // direction-1 sums: [g3][yy][lx]
    __shared__ double r2[P * NFF];           // direction-2 sums: [g3][ly][lx]
    const Dir &d0 = pv.dir[0], &d1 = pv.dir[1], &d2 = pv.dir[2];
    const int bx = blockIdx.x, by = blockIdx.y, e3 = blockIdx.z;
    const int e1b = bx * E, e2b = by * E;
    const int64_t N0 = d0.N, N01 = (int64_t)d0.N * d1.N;
    const int tid = threadIdx.x;
    const int64_t tile = (int64_t)by * gridDim.x + bx;
    const double *hb = h + (tile * d2.Q + (int64_t)e3 * P) * TT;
    for (int i = tid; i < P * TT; i += NT) hs[i] = hb[i];
    __syncthreads();
    // direction 1: function column lx gets sum over the elements l1 that
    // activate it (local function j = lx - l1) and their points h1
    for (int i = tid; i < P * T * NF; i += NT) {
        const int lx = i % NF, row = i / NF;                 // row = g3 * T + yy
        const double *hr = hs + row * T;
        double acc = 0.0;
#pragma unroll
        for (int l1 = 0; l1 < E; ++l1) {
            const int j = lx - l1;
            if (j < 0 || j >= P) continue;
            const double *B1 = d0.B + (int64_t)min(e1b + l1, d0.K - 1) * P * P + j;   // [h1][j], stride P
#pragma unroll
            for (int h1 = 0; h1 < P; ++h1) acc += B1[h1 * P] * hr[l1 * P + h1];
        }
        r1[i] = acc;
    }
    __syncthreads();
    // direction 2: function row ly, the same over l2 and h2
    for (int i = tid; i < P * NFF; i += NT) {
        const int lx = i % NF, ly = (i / NF) % NF, g3 = i / NFF;
        double acc = 0.0;
#pragma unroll
        for (int l2 = 0; l2 < E; ++l2) {
            const int j = ly - l2;
            if (j < 0 || j >= P) continue;
            const double *B2 = d1.B + (int64_t)min(e2b + l2, d1.K - 1) * P * P + j;
#pragma unroll
            for (int h2 = 0; h2 < P; ++h2) acc += B2[h2 * P] * r1[(g3 * T + l2 * P + h2) * NF + lx];
        }
        r2[i] = acc;
    }
    __syncthreads();
    // direction 3: function layer e3 + s, into y
    const double *B3 = d2.B + (int64_t)e3 * P * P;
    for (int i = tid; i < P * NFF; i += NT) {
        const int s = i / NFF, j = i % NFF;
        const int n0 = e1b + j % NF, n1 = e2b + j / NF;
        double acc = 0.0;
#pragma unroll
        for (int g3 = 0; g3 < P; ++g3) acc += B3[g3 * P + s] * r2[g3 * NFF + j];
        if (n0 < d0.N && n1 < d1.N) atomicAdd(&y[n0 + N0 * n1 + N01 * (e3 + s)], acc);
    }
}

template <int P>
static hipError_t launch_conv_p(const PatchView &pv, const double *cv, double *h, const double *x, double *y,
                                hipStream_t s)
{
    constexpr int E = ConvTile<P>::E;
    const dim3 grid((pv.dir[0].K + E - 1) / E, (pv.dir[1].K + E - 1) / E, pv.dir[2].K);
    hipError_t e = launch_fill(y, pv.N, 0.0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(conv_forward_kernel<P>, grid, dim3(ConvTile<P>::NT), 0, s, pv, cv, x, h);
    hipLaunchKernelGGL(conv_backward_kernel<P>, grid, dim3(ConvTile<P>::NT), 0, s, pv, (const double *)h, y);
    return hipGetLastError();
}

hipError_t launch_conv_apply(const PatchView &pv, const double *cv, double *h, const double *x, double *y,
                             hipStream_t s)
{
    if (pv.d != 3) return hipErrorInvalidValue;
    switch (pv.P) {
    case 2: return launch_conv_p<2>(pv, cv, h, x, y, s);
    case 3: return launch_conv_p<3>(pv, cv, h, x, y, s);
    case 4: return launch_conv_p<4>(pv, cv, h, x, y, s);
    case 5: return launch_conv_p<5>(pv, cv, h, x, y, s);
    case 6: return launch_conv_p<6>(pv, cv, h, x, y, s);
    case 7: return launch_conv_p<7>(pv, cv, h, x, y, s);
    case 8: return launch_conv_p<8>(pv, cv, h, x, y, s);
    case 9: return launch_conv_p<9>(pv, cv, h, x, y, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sfiga
