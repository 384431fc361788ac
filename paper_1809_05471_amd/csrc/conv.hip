// Matrix-free product of the convection form, d = 3, FP64: the b . grad u
// term of the convection-diffusion equation of Sec. 2, Example 1, tested
// with v.  With u = sum_n x_n phi_n,
//   y_m = sum_x c(x) . grad_hat u(x) phi_m(x),   c = w s(G) |det J| J^-1 b,
// c folded per quadrature point by the geometry step (conv_coef_index
// layout).  The trial side needs the three reference derivatives of u
// (Algorithm 3 with the derivative table in one direction at a time), the
// test side only values (Algorithm 2 with value tables): the form is not
// symmetric and has a kernel of its own.
//
// One workgroup per (tile of E x E elements in directions 1 and 2, element
// layer e3), E = conv_tile_elems(P); everything between the loads of x and c
// and the atomic adds into y stays in LDS:
//   forward   the tile's x block ((E+p-1)^2 functions x p layers) contracted
//             3 -> 2 -> 1 (B3/D3, then B2/D2, then D1/B1) into the three
//             reference derivatives at the tile's points, dotted with c;
//   backward  those point values contracted with the value tables 1 -> 2 -> 3
//             (the sums over the elements that share a function formed inside
//             the tile), added into y with FP64 atomics (tiles and layers
//             overlap in p - 1 functions per direction).
// The element tables of the tile are staged in LDS (a lane's table row
// depends on its point, so global loads would go one per operand through
// the vector memory path).  HBM per quadrature point: c, 24 bytes; the x
// block and the y atomics add about ((E+p-1)/(E p))^2 of a value each per
// point and layer.
#include "kernels.h"

namespace sfiga {

// A table read by a whole wavefront at one address: through the constant
// address space the compiler turns the reads into scalar loads.
template <typename T>
using conv_uniform_ptr = const __attribute__((address_space(4))) T *;

template <int P>
struct ConvTile {
    static constexpr int E = conv_tile_elems(P);
    static constexpr int T = E * P;          // quadrature points per tile side
    static constexpr int NF = E + P - 1;     // functions per tile side
    static constexpr int NT = 256;
    static constexpr int PP = P * P, NFF = NF * NF, TT = T * T;
    static constexpr int SB = P * T * NF;    // one field of the direction-2 results
    static constexpr int NPT = (P * TT + NT - 1) / NT;   // points per thread
    // ROWF1: directions 2 and 1 (with the pointwise product) per element row
    // (element, plane, function column or point row), the element uniform
    // across a wavefront and its tables in scalar registers, rows padded to
    // whole wavefronts per element: fewer LDS reads per multiply-add, but
    // idle lanes and strided coefficient loads.  Measured per order at
    // N = 126^3 against one item per point: 0.84 / 0.87 ms at order 4, 5.96 /
    // 6.10 at 7, 21.9 / 24.8 at 9, and at 8 (two elements per tile side, with
    // ROWB) 9.79 against 10.6 with one element and one item per point; slower
    // at 2, 5 and 6 (order 6: 4.11 / 3.06 ms), equal at 3.
    static constexpr bool ROWF1 = P == 4 || P >= 7;
    // ROWB: backward directions 1 and 2 per element row as well, each item
    // adding its p sums into the shared rows with LDS atomics.  Measured at
    // N = 126^3 against the gather per function: 0.110 / 0.126 ms at order 2,
    // 0.41 / 0.43 at 3, 0.80 / 0.85 at 4, 3.07 / 3.10 at 6, 5.68 / 5.96 at 7,
    // equal at 5; at 9 it spills (26.4 / 22.0 ms).
    static constexpr bool ROWB = P <= 8;
    static constexpr int R = P * T, R64 = (R + 63) / 64 * 64;
    static constexpr int NIT = (E * R64 + NT - 1) / NT;  // element rows per thread
    // the same for direction 2 (element l2, plane g3, function column lx)
    static constexpr int C2 = P * NF, C64 = (C2 + 63) / 64 * 64;
    static constexpr int NIT2 = (E * C64 + NT - 1) / NT;
    // LDS in doubles: tables, x rows, direction-3 results, direction-2 results, point values
    static constexpr int LDS = 4 * E * PP + 2 * PP + P * NFF + 2 * P * NFF + 3 * SB + P * TT;
};

template <int P>
__global__ __launch_bounds__(256) void conv_kernel(PatchView pv, const double *__restrict__ cv,
                                                   const double *__restrict__ x, double *__restrict__ y)
{
    using CT = ConvTile<P>;
    constexpr int E = CT::E, T = CT::T, NF = CT::NF, NT = CT::NT, PP = CT::PP, NFF = CT::NFF, TT = CT::TT;
    constexpr int SB = CT::SB, NPT = CT::NPT;
    constexpr bool ROWF1 = CT::ROWF1, ROWB = CT::ROWB;
    constexpr int R = CT::R, R64 = CT::R64, NIT = CT::NIT;
    constexpr int C2 = CT::C2, C64 = CT::C64, NIT2 = CT::NIT2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *t1B = reinterpret_cast<double *>(smem_raw);   // [element l][point h][function j]
    double *t1D = t1B + E * PP, *t2B = t1D + E * PP, *t2D = t2B + E * PP;
    double *t3B = t2D + E * PP, *t3D = t3B + PP;           // [point g][function j] of layer e3
    double *xs = t3D + PP;                                 // x rows e3 .. e3+p-1: [s][ly][lx]
    double *sa = xs + P * NFF;     // B3 x, D3 x: [2][g3][ly][lx]; then the direction-2 sums r2 [g3][ly][lx]
    double *sb = sa + 2 * P * NFF; // B2 B3 x, D2 B3 x, B2 D3 x: [3][g3][yy][lx]; then the direction-1 sums r1
    double *hs = sb + 3 * SB;      // point values c . grad_hat u: [g3][yy][xx]
    const Dir &d0 = pv.dir[0], &d1 = pv.dir[1], &d2 = pv.dir[2];
    const int bx = blockIdx.x, by = blockIdx.y, e3 = blockIdx.z;
    const int e1b = bx * E, e2b = by * E;
    const int64_t N0 = d0.N, N01 = (int64_t)d0.N * d1.N;
    const int tid = threadIdx.x;

    // The layer's coefficients of the thread's points are loaded first, into
    // registers, and arrive while the forward stages run (the last thread's
    // surplus points re-read the layer's last point and are not used).
    const int64_t tile = (int64_t)by * gridDim.x + bx;
    const double *cl = cv + (tile * d2.Q + (int64_t)e3 * P) * 3 * TT;     // c of the layer's first plane
    double cr[ROWF1 ? 1 : NPT][3];
    double crr[ROWF1 ? NIT : 1][3][ROWF1 ? P : 1];
    if constexpr (ROWF1) {
#pragma unroll
        for (int k = 0; k < NIT; ++k) {
            const int idx = min(tid + k * NT, E * R64 - 1);
            const int l1 = idx / R64, r = min(idx % R64, R - 1);
            const double *c = cl + (int64_t)(r / T) * 3 * TT + (r % T) * T + l1 * P;
#pragma unroll
            for (int h1 = 0; h1 < P; ++h1) {
                crr[k][0][h1] = c[h1];
                crr[k][1][h1] = c[TT + h1];
                crr[k][2][h1] = c[2 * TT + h1];
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int i = min(tid + k * NT, P * TT - 1);
            const int xx = i % T, yy = (i / T) % T, g3 = i / TT;
            const double *c = cl + (int64_t)g3 * 3 * TT + yy * T + xx;
            cr[k][0] = c[0];
            cr[k][1] = c[TT];
            cr[k][2] = c[2 * TT];
        }
    }
    // element tables (elements past the patch edge take the last element's:
    // their points have c = 0 and their functions are not stored)
    for (int i = tid; i < E * PP; i += NT) {
        const int l = i / PP, r = i % PP;
        const int64_t a1 = (int64_t)min(e1b + l, d0.K - 1) * PP + r;
        const int64_t a2 = (int64_t)min(e2b + l, d1.K - 1) * PP + r;
        t1B[i] = d0.B[a1];
        t1D[i] = d0.D[a1];
        t2B[i] = d1.B[a2];
        t2D[i] = d1.D[a2];
    }
    for (int i = tid; i < PP; i += NT) {
        t3B[i] = d2.B[(int64_t)e3 * PP + i];
        t3D[i] = d2.D[(int64_t)e3 * PP + i];
    }
    for (int i = tid; i < P * NFF; i += NT) {
        const int s = i / NFF, j = i % NFF;
        const int n0 = e1b + j % NF, n1 = e2b + j / NF;
        xs[i] = (n0 < d0.N && n1 < d1.N) ? x[n0 + N0 * n1 + N01 * (e3 + s)] : 0.0;
    }
    __syncthreads();
    // ---- forward, direction 3: a = B3 x, b = D3 x per plane g3 and function column
    for (int i = tid; i < P * NFF; i += NT) {
        const int g3 = i / NFF, j = i % NFF;
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int s = 0; s < P; ++s) {
            const double v = xs[s * NFF + j];
            a += t3B[g3 * P + s] * v;
            b += t3D[g3 * P + s] * v;
        }
        sa[i] = a;
        sa[P * NFF + i] = b;
    }
    __syncthreads();
    // ---- direction 2: B2 a (for d1), D2 a (d2), B2 b (d3) at the point rows
    // yy = (element l2, point h2)
    if constexpr (ROWF1) {
        // per (element l2, plane, function column): the p values of a and b
        // read once, the element's tables from scalar registers
#pragma unroll
        for (int k = 0; k < NIT2; ++k) {
            const int idx = tid + k * NT;
            if (idx >= E * C64) break;                        // whole wavefronts
            const int l2 = __builtin_amdgcn_readfirstlane(idx / C64), c = idx % C64;
            if (c < C2) {
                const int g3 = c / NF, lx = c % NF;
                const int e2 = min(e2b + l2, d1.K - 1);
                const conv_uniform_ptr<double> B2 = (conv_uniform_ptr<double>)(d1.B + (int64_t)e2 * PP);
                const conv_uniform_ptr<double> D2 = (conv_uniform_ptr<double>)(d1.D + (int64_t)e2 * PP);
                const double *ca = sa + g3 * NFF + l2 * NF + lx, *cb = ca + P * NFF;
                double va[P], vb[P];
#pragma unroll
                for (int s = 0; s < P; ++s) {
                    va[s] = ca[s * NF];
                    vb[s] = cb[s * NF];
                }
                double *o = sb + (g3 * T + l2 * P) * NF + lx;
#pragma unroll
                for (int h2 = 0; h2 < P; ++h2) {
                    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
#pragma unroll
                    for (int s = 0; s < P; ++s) {
                        f0 += B2[h2 * P + s] * va[s];
                        f1 += D2[h2 * P + s] * va[s];
                        f2 += B2[h2 * P + s] * vb[s];
                    }
                    o[h2 * NF] = f0;
                    o[SB + h2 * NF] = f1;
                    o[2 * SB + h2 * NF] = f2;
                }
            }
        }
    } else {
    for (int i = tid; i < SB; i += NT) {
        const int lx = i % NF, yy = (i / NF) % T, g3 = i / (NF * T);
        const int l2 = yy / P;
        const double *B2 = t2B + yy * P, *D2 = t2D + yy * P;     // (l2 P + h2) P = yy P
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
    }
    __syncthreads();
    // ---- direction 1 and the pointwise product
    if constexpr (ROWB) {
        // the backward direction-1 sums are added into the x / direction-3
        // region (free from here on): cleared now
        static_assert(SB <= 3 * P * NFF, "direction-1 sums fit in the x and direction-3 buffers");
        for (int i = tid; i < SB; i += NT) xs[i] = 0.0;
    }
    if constexpr (ROWF1) {
        // per element row: the p direction-2 values of each field read once,
        // the element's tables from scalar registers
#pragma unroll
        for (int k = 0; k < NIT; ++k) {
            const int idx = tid + k * NT;
            if (idx >= E * R64) break;                        // whole wavefronts
            const int l1 = __builtin_amdgcn_readfirstlane(idx / R64), r = idx % R64;
            if (r < R) {
                const int e1 = min(e1b + l1, d0.K - 1);
                const conv_uniform_ptr<double> B1 = (conv_uniform_ptr<double>)(d0.B + (int64_t)e1 * PP);
                const conv_uniform_ptr<double> D1 = (conv_uniform_ptr<double>)(d0.D + (int64_t)e1 * PP);
                const double *rw = sb + r * NF + l1;          // r = g3 T + yy
                double v0[P], v1[P], v2[P];
#pragma unroll
                for (int s = 0; s < P; ++s) {
                    v0[s] = rw[s];
                    v1[s] = rw[SB + s];
                    v2[s] = rw[2 * SB + s];
                }
                double *ho = hs + r * T + l1 * P;
#pragma unroll
                for (int h1 = 0; h1 < P; ++h1) {
                    double u1 = 0.0, u2 = 0.0, u3 = 0.0;
#pragma unroll
                    for (int s = 0; s < P; ++s) {
                        u1 += D1[h1 * P + s] * v0[s];
                        u2 += B1[h1 * P + s] * v1[s];
                        u3 += B1[h1 * P + s] * v2[s];
                    }
                    ho[h1] = crr[k][0][h1] * u1 + crr[k][1][h1] * u2 + crr[k][2][h1] * u3;
                }
            }
        }
    } else {
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int i = tid + k * NT;
        if (i >= P * TT) break;
        const int xx = i % T, yy = (i / T) % T, g3 = i / TT;
        const int l1 = xx / P;
        const double *B1 = t1B + xx * P, *D1 = t1D + xx * P;     // (l1 P + h1) P = xx P
        const double *r = sb + (g3 * T + yy) * NF + l1;
        double u1 = 0.0, u2 = 0.0, u3 = 0.0;
#pragma unroll
        for (int s = 0; s < P; ++s) {
            u1 += D1[s] * r[s];
            u2 += B1[s] * r[SB + s];
            u3 += B1[s] * r[2 * SB + s];
        }
        hs[i] = cr[k][0] * u1 + cr[k][1] * u2 + cr[k][2] * u3;
    }
    }
    __syncthreads();
    // ---- backward, direction 1: function column lx gets the sum over the
    // elements l1 that activate it (local function j = lx - l1) and their
    // points h1
    double *r1 = ROWB ? xs : sb;
    double *r2 = ROWB ? sb : sa;
    if constexpr (ROWB) {
        // per element row (element l1, row g3 T + yy): its p point values read
        // once, its p sums added into the row with LDS atomics (the elements
        // that share a column meet there); the direction-2 sums' buffer (the
        // direction-2 forward region, free now) cleared meanwhile
        for (int i = tid; i < P * NFF; i += NT) r2[i] = 0.0;
#pragma unroll
        for (int k = 0; k < NIT; ++k) {
            const int idx = tid + k * NT;
            if (idx >= E * R64) break;                        // whole wavefronts
            const int l1 = __builtin_amdgcn_readfirstlane(idx / R64), r = idx % R64;
            if (r < R) {
                const int e1 = min(e1b + l1, d0.K - 1);
                const conv_uniform_ptr<double> B1 = (conv_uniform_ptr<double>)(d0.B + (int64_t)e1 * PP);
                double v[P];
#pragma unroll
                for (int h1 = 0; h1 < P; ++h1) v[h1] = hs[r * T + l1 * P + h1];
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    double acc = 0.0;
#pragma unroll
                    for (int h1 = 0; h1 < P; ++h1) acc += B1[h1 * P + j] * v[h1];
                    atomicAdd(&r1[r * NF + l1 + j], acc);
                }
            }
        }
    } else {
    for (int i = tid; i < SB; i += NT) {
        const int lx = i % NF, row = i / NF;                  // row = g3 T + yy
        const double *hr = hs + row * T;
        double acc = 0.0;
#pragma unroll
        for (int l1 = 0; l1 < E; ++l1) {
            const int j = lx - l1;
            if (j < 0 || j >= P) continue;
            const double *B1 = t1B + l1 * PP + j;             // [h1][j], stride P
#pragma unroll
            for (int h1 = 0; h1 < P; ++h1) acc += B1[h1 * P] * hr[l1 * P + h1];
        }
        r1[i] = acc;
    }
    }
    __syncthreads();
    // ---- direction 2: function row ly, the same over l2 and h2
    if constexpr (ROWB) {
        // per (element l2, plane, function column), atomics as above
#pragma unroll
        for (int k = 0; k < NIT2; ++k) {
            const int idx = tid + k * NT;
            if (idx >= E * C64) break;                        // whole wavefronts
            const int l2 = __builtin_amdgcn_readfirstlane(idx / C64), c = idx % C64;
            if (c < C2) {
                const int g3 = c / NF, lx = c % NF;
                const int e2 = min(e2b + l2, d1.K - 1);
                const conv_uniform_ptr<double> B2 = (conv_uniform_ptr<double>)(d1.B + (int64_t)e2 * PP);
                double v[P];
#pragma unroll
                for (int h2 = 0; h2 < P; ++h2) v[h2] = r1[(g3 * T + l2 * P + h2) * NF + lx];
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    double acc = 0.0;
#pragma unroll
                    for (int h2 = 0; h2 < P; ++h2) acc += B2[h2 * P + j] * v[h2];
                    atomicAdd(&r2[g3 * NFF + (l2 + j) * NF + lx], acc);
                }
            }
        }
    } else {
    for (int i = tid; i < P * NFF; i += NT) {
        const int lx = i % NF, ly = (i / NF) % NF, g3 = i / NFF;
        double acc = 0.0;
#pragma unroll
        for (int l2 = 0; l2 < E; ++l2) {
            const int j = ly - l2;
            if (j < 0 || j >= P) continue;
            const double *B2 = t2B + l2 * PP + j;
#pragma unroll
            for (int h2 = 0; h2 < P; ++h2) acc += B2[h2 * P] * r1[(g3 * T + l2 * P + h2) * NF + lx];
        }
        r2[i] = acc;
    }
    }
    __syncthreads();
    // ---- direction 3: function layer e3 + s, into y
    for (int i = tid; i < P * NFF; i += NT) {
        const int s = i / NFF, j = i % NFF;
        const int n0 = e1b + j % NF, n1 = e2b + j / NF;
        double acc = 0.0;
#pragma unroll
        for (int g3 = 0; g3 < P; ++g3) acc += t3B[g3 * P + s] * r2[g3 * NFF + j];
        if (n0 < d0.N && n1 < d1.N) atomicAdd(&y[n0 + N0 * n1 + N01 * (e3 + s)], acc);
    }
}

template <int P>
static hipError_t launch_conv_p(const PatchView &pv, const double *cv, const double *x, double *y, hipStream_t s)
{
    using CT = ConvTile<P>;
    const size_t lds = sizeof(double) * CT::LDS;
    hipError_t e = allow_dynamic_lds((const void *)conv_kernel<P>, lds);
    if (e == hipSuccess) e = launch_fill(y, pv.N, 0.0, s);
    if (e != hipSuccess) return e;
    const dim3 grid((pv.dir[0].K + CT::E - 1) / CT::E, (pv.dir[1].K + CT::E - 1) / CT::E, pv.dir[2].K);
    hipLaunchKernelGGL(conv_kernel<P>, grid, dim3(CT::NT), lds, s, pv, cv, x, y);
    return hipGetLastError();
}

hipError_t launch_conv_apply(const PatchView &pv, const double *cv, const double *x, double *y, hipStream_t s)
{
    if (pv.d != 3) return hipErrorInvalidValue;
    switch (pv.P) {
    case 2: return launch_conv_p<2>(pv, cv, x, y, s);
    case 3: return launch_conv_p<3>(pv, cv, x, y, s);
    case 4: return launch_conv_p<4>(pv, cv, x, y, s);
    case 5: return launch_conv_p<5>(pv, cv, x, y, s);
    case 6: return launch_conv_p<6>(pv, cv, x, y, s);
    case 7: return launch_conv_p<7>(pv, cv, x, y, s);
    case 8: return launch_conv_p<8>(pv, cv, x, y, s);
    case 9: return launch_conv_p<9>(pv, cv, x, y, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sfiga
