// Matrix-free product y = A x (Sec. 3.3).  Forward: u or grad u at the
// quadrature points by sum factorization (Algorithm 3 with value and
// derivative tables); pointwise product with the folded coefficient tensor;
// backward: the transposed contractions (Algorithm 2, weights already folded
// into the coefficient), accumulated into y.
//
// d = 3 kernel: one workgroup per (E1 x E2 element tile, element layer e3) -
// a localized box in the sense of Sec. 4 - with one thread per quadrature
// column (q1, q2).  The x values of the box's functions are staged in LDS,
// contractions run direction 3 -> 2 -> 1 and back 1 -> 2 -> 3 one
// quadrature plane g3 at a time, and the box's partial y is added to global
// memory with FP64 atomics (the accumulation step of eq. (loc-basis-change)).
// The coefficient tensor is the only stream that scales with Q; every
// thread issues its 6 p (stiffness) or p (mass) coefficient loads before the
// first contraction so they overlap with the forward sweep.
#include "kernels.h"

namespace sfiga {

template <int P, bool STIFF, typename CT>
__global__ __launch_bounds__(Tile<P>::NT) void apply3d_kernel(PatchView pv, const CT *__restrict__ C,
                                                             const double *__restrict__ x, double *__restrict__ y)
{
    using TL = Tile<P>;
    constexpr int NX = TL::NX, NY = TL::NY, TX = TL::TX, TY = TL::TY, NT = TL::NT;
    constexpr int NF = STIFF ? 3 : 1;      // gradient components or value
    constexpr int NC = STIFF ? 6 : 1;      // coefficient components
    extern __shared__ __align__(16) unsigned char smem_raw[];
    CT *xw = reinterpret_cast<CT *>(smem_raw);   // [P][NY][NX] x on the box's functions
    CT *yw = xw + P * NY * NX;                   // [P][NY][NX] partial y
    CT *sa = yw + P * NY * NX;                   // [max(2 NY NX, NF TY NX)] dir-3 results / backward dir-1 results
    constexpr int SA = (2 * NY * NX > NF * TY * NX) ? 2 * NY * NX : NF * TY * NX;
    CT *sb = sa + SA;                            // [NF][TY][NX] forward dir-2 results
    CT *sh = sb + NF * TY * NX;                  // [NF][TY][TX] pointwise results

    const Dir &d0 = pv.dir[0], &d1 = pv.dir[1], &d2 = pv.dir[2];
    const int e1b = blockIdx.x * TL::E1, e2b = blockIdx.y * TL::E2, e3 = blockIdx.z;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int le1 = tx / P, g1 = tx % P, le2 = ty / P, g2 = ty % P;
    const int e1 = e1b + le1, e2 = e2b + le2;
    const bool active = e1 < d0.K && e2 < d1.K;
    const int Q0 = d0.Q, Q1 = d1.Q;

    // coefficient loads for the whole column, issued first
    CT creg[P][NC];
    if (active) {
        const int q0 = e1 * P + g1, q1 = e2 * P + g2;
#pragma unroll
        for (int g3 = 0; g3 < P; ++g3)
#pragma unroll
            for (int c = 0; c < NC; ++c) creg[g3][c] = C[coef_index(3, NC, c, q0, q1, e3 * P + g3, Q0, Q1)];
    } else {
#pragma unroll
        for (int g3 = 0; g3 < P; ++g3)
#pragma unroll
            for (int c = 0; c < NC; ++c) creg[g3][c] = CT(0);
    }

    for (int idx = tid; idx < P * NY * NX; idx += NT) {
        int lx = idx % NX, r = idx / NX;
        int ly = r % NY, s3 = r / NY;
        int n0 = e1b + lx, n1 = e2b + ly, n2 = e3 + s3;
        CT v = CT(0);
        if (n0 < d0.N && n1 < d1.N) v = (CT)x[(int64_t)n0 + (int64_t)d0.N * (n1 + (int64_t)d1.N * n2)];
        xw[idx] = v;
        yw[idx] = CT(0);
    }
    __syncthreads();

    for (int g3 = 0; g3 < P; ++g3) {
        const double *b3 = d2.B + ((int64_t)e3 * P + g3) * P;
        const double *db3 = d2.D + ((int64_t)e3 * P + g3) * P;
        // forward, direction 3: a = B3 x (and b = D3 x)
        for (int idx = tid; idx < NY * NX; idx += NT) {
            CT a = CT(0), b = CT(0);
#pragma unroll
            for (int s = 0; s < P; ++s) {
                CT v = xw[s * NY * NX + idx];
                a += (CT)b3[s] * v;
                if (STIFF) b += (CT)db3[s] * v;
            }
            sa[idx] = a;
            if (STIFF) sa[NY * NX + idx] = b;
        }
        __syncthreads();
        // forward, direction 2: B2 a (-> d1 and value), D2 a (-> d2), B2 b (-> d3)
        for (int idx = tid; idx < TY * NX; idx += NT) {
            int lx = idx % NX, yy = idx / NX;
            int l2 = yy / P, h2 = yy % P, ee2 = e2b + l2;
            CT vb = CT(0), vd = CT(0), wb = CT(0);
            if (ee2 < d1.K) {
                const double *b2 = d1.B + ((int64_t)ee2 * P + h2) * P;
                const double *db2 = d1.D + ((int64_t)ee2 * P + h2) * P;
#pragma unroll
                for (int s = 0; s < P; ++s) {
                    CT a = sa[(l2 + s) * NX + lx];
                    vb += (CT)b2[s] * a;
                    if (STIFF) {
                        CT b = sa[(NY + l2 + s) * NX + lx];
                        vd += (CT)db2[s] * a;
                        wb += (CT)b2[s] * b;
                    }
                }
            }
            sb[yy * NX + lx] = vb;
            if (STIFF) {
                sb[(TY + yy) * NX + lx] = vd;
                sb[(2 * TY + yy) * NX + lx] = wb;
            }
        }
        __syncthreads();
        // forward, direction 1, and the pointwise coefficient
        {
            CT h[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) h[f] = CT(0);
            if (active) {
                const double *b1 = d0.B + ((int64_t)e1 * P + g1) * P;
                const double *db1 = d0.D + ((int64_t)e1 * P + g1) * P;
                if (STIFF) {
                    CT gr0 = CT(0), gr1 = CT(0), gr2 = CT(0);
#pragma unroll
                    for (int s = 0; s < P; ++s) {
                        gr0 += (CT)db1[s] * sb[ty * NX + le1 + s];
                        gr1 += (CT)b1[s] * sb[(TY + ty) * NX + le1 + s];
                        gr2 += (CT)b1[s] * sb[(2 * TY + ty) * NX + le1 + s];
                    }
                    const CT *c = creg[g3];
                    // components 00 11 22 01 02 12
                    h[0] = c[0] * gr0 + c[3] * gr1 + c[4] * gr2;
                    h[1] = c[3] * gr0 + c[1] * gr1 + c[5] * gr2;
                    h[2] = c[4] * gr0 + c[5] * gr1 + c[2] * gr2;
                } else {
                    CT u = CT(0);
#pragma unroll
                    for (int s = 0; s < P; ++s) u += (CT)b1[s] * sb[ty * NX + le1 + s];
                    h[0] = creg[g3][0] * u;
                }
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) sh[(f * TY + ty) * TX + tx] = h[f];
        }
        __syncthreads();
        // backward, direction 1: r1 = D1^T h1, r2 = B1^T h2, r3 = B1^T h3 (mass: B1^T h)
        for (int idx = tid; idx < TY * NX; idx += NT) {
            int lx = idx % NX, yy = idx / NX;
            CT r[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) r[f] = CT(0);
#pragma unroll
            for (int j = 0; j < P; ++j) {
                const int l1 = lx - j, ee1 = e1b + l1;   // element whose local function j is lx
                if (l1 < 0 || l1 >= TL::E1 || ee1 >= d0.K) continue;
                for (int h1 = 0; h1 < P; ++h1) {
                    const double bv = d0.B[((int64_t)ee1 * P + h1) * P + j];
                    const int col = l1 * P + h1;
                    if (STIFF) {
                        const double dv = d0.D[((int64_t)ee1 * P + h1) * P + j];
                        r[0] += (CT)dv * sh[(0 * TY + yy) * TX + col];
                        r[1] += (CT)bv * sh[(1 * TY + yy) * TX + col];
                        r[2] += (CT)bv * sh[(2 * TY + yy) * TX + col];
                    } else {
                        r[0] += (CT)bv * sh[yy * TX + col];
                    }
                }
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) sa[(f * TY + yy) * NX + lx] = r[f];
        }
        __syncthreads();
        // backward, direction 2 then direction 3 into the partial y
        for (int idx = tid; idx < NY * NX; idx += NT) {
            int lx = idx % NX, ly = idx / NX;
            CT sB = CT(0), sD = CT(0);
#pragma unroll
            for (int j = 0; j < P; ++j) {
                const int l2 = ly - j, ee2 = e2b + l2;
                if (l2 < 0 || l2 >= TL::E2 || ee2 >= d1.K) continue;
                for (int h2 = 0; h2 < P; ++h2) {
                    const double bv = d1.B[((int64_t)ee2 * P + h2) * P + j];
                    const int row = l2 * P + h2;
                    if (STIFF) {
                        const double dv = d1.D[((int64_t)ee2 * P + h2) * P + j];
                        sB += (CT)bv * sa[(0 * TY + row) * NX + lx] + (CT)dv * sa[(1 * TY + row) * NX + lx];
                        sD += (CT)bv * sa[(2 * TY + row) * NX + lx];
                    } else {
                        sB += (CT)bv * sa[row * NX + lx];
                    }
                }
            }
#pragma unroll
            for (int s = 0; s < P; ++s) {
                CT v = (CT)b3[s] * sB;
                if (STIFF) v += (CT)db3[s] * sD;
                yw[s * NY * NX + idx] += v;
            }
        }
        __syncthreads();
    }

    for (int idx = tid; idx < P * NY * NX; idx += NT) {
        int lx = idx % NX, r = idx / NX;
        int ly = r % NY, s3 = r / NY;
        int n0 = e1b + lx, n1 = e2b + ly, n2 = e3 + s3;
        if (n0 < d0.N && n1 < d1.N)
            atomicAdd(&y[(int64_t)n0 + (int64_t)d0.N * (n1 + (int64_t)d1.N * n2)], (double)yw[idx]);
    }
}

// d = 1, 2: one thread per element, element-local sum factorization,
// atomics into y.
template <int DIM, int P, bool STIFF, typename CT>
__global__ void apply_small_kernel(PatchView pv, const CT *__restrict__ C, const double *__restrict__ x,
                                   double *__restrict__ y)
{
    const int64_t el = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const Dir &d0 = pv.dir[0], &d1 = pv.dir[1];
    const int64_t nel = (int64_t)d0.K * (DIM == 2 ? d1.K : 1);
    if (el >= nel) return;
    const int e0 = (int)(el % d0.K), e1 = DIM == 2 ? (int)(el / d0.K) : 0;
    constexpr int NC = STIFF ? DIM * (DIM + 1) / 2 : 1;
    constexpr int P2 = DIM == 2 ? P : 1;
    double xl[P2][P], yl[P2][P];
    for (int s1 = 0; s1 < P2; ++s1)
        for (int s0 = 0; s0 < P; ++s0) {
            xl[s1][s0] = x[(e0 + s0) + (int64_t)d0.N * (e1 + s1)];
            yl[s1][s0] = 0.0;
        }
    for (int g1 = 0; g1 < P2; ++g1) {
        double b1[P2], db1[P2];
        for (int s1 = 0; s1 < P2; ++s1) {
            b1[s1] = DIM == 2 ? d1.B[((int64_t)e1 * P + g1) * P + s1] : 1.0;
            db1[s1] = DIM == 2 ? d1.D[((int64_t)e1 * P + g1) * P + s1] : 0.0;
        }
        // direction 2 first: tv = B1 x, td = D1 x at this g1
        double tv[P], td[P], px[P], py[P];
        for (int s0 = 0; s0 < P; ++s0) {
            double a = 0.0, b = 0.0;
            for (int s1 = 0; s1 < P2; ++s1) {
                a += b1[s1] * xl[s1][s0];
                b += db1[s1] * xl[s1][s0];
            }
            tv[s0] = a;
            td[s0] = b;
            px[s0] = py[s0] = 0.0;
        }
        for (int g0 = 0; g0 < P; ++g0) {
            const double *b0 = d0.B + ((int64_t)e0 * P + g0) * P;
            const double *db0 = d0.D + ((int64_t)e0 * P + g0) * P;
            const int q0 = e0 * P + g0, q1 = e1 * P + g1;
            double u = 0.0, gx = 0.0, gy = 0.0;
            for (int s0 = 0; s0 < P; ++s0) {
                u += b0[s0] * tv[s0];
                gx += db0[s0] * tv[s0];
                gy += b0[s0] * td[s0];
            }
            if (STIFF) {
                double c[3] = {0.0, 0.0, 0.0};
                for (int k = 0; k < NC; ++k) c[k] = (double)C[coef_index(DIM, NC, k, q0, q1, 0, d0.Q, d1.Q)];
                double hx = DIM == 2 ? c[0] * gx + c[2] * gy : c[0] * gx;
                double hy = DIM == 2 ? c[2] * gx + c[1] * gy : 0.0;
                for (int s0 = 0; s0 < P; ++s0) {
                    px[s0] += db0[s0] * hx;
                    py[s0] += b0[s0] * hy;
                }
            } else {
                double hv = (double)C[coef_index(DIM, 1, 0, q0, q1, 0, d0.Q, d1.Q)] * u;
                for (int s0 = 0; s0 < P; ++s0) px[s0] += b0[s0] * hv;
            }
        }
        // back through direction 2: the d1-part and value pair with B, the d2-part with D
        for (int s1 = 0; s1 < P2; ++s1)
            for (int s0 = 0; s0 < P; ++s0) yl[s1][s0] += b1[s1] * px[s0] + db1[s1] * py[s0];
    }
    for (int s1 = 0; s1 < P2; ++s1)
        for (int s0 = 0; s0 < P; ++s0) atomicAdd(&y[(e0 + s0) + (int64_t)d0.N * (e1 + s1)], yl[s1][s0]);
}

template <int P, bool STIFF, typename CT>
static hipError_t launch_apply_t(const PatchView &pv, const CT *C, const double *x, double *y, hipStream_t s)
{
    if (pv.d == 3) {
        using TL = Tile<P>;
        constexpr int NF = STIFF ? 3 : 1;
        constexpr int SA = (2 * TL::NY * TL::NX > NF * TL::TY * TL::NX) ? 2 * TL::NY * TL::NX : NF * TL::TY * TL::NX;
        size_t lds = sizeof(CT) * (2 * P * TL::NY * TL::NX + SA + NF * TL::TY * TL::NX + NF * TL::TY * TL::TX);
        dim3 grid((pv.dir[0].K + TL::E1 - 1) / TL::E1, (pv.dir[1].K + TL::E2 - 1) / TL::E2, pv.dir[2].K);
        hipLaunchKernelGGL((apply3d_kernel<P, STIFF, CT>), grid, dim3(TL::NT), lds, s, pv, C, x, y);
    } else {
        int64_t nel = (int64_t)pv.dir[0].K * pv.dir[1].K;
        int64_t nb = (nel + 127) / 128;
        if (pv.d == 2)
            hipLaunchKernelGGL((apply_small_kernel<2, P, STIFF, CT>), dim3((unsigned)nb), dim3(128), 0, s, pv, C, x, y);
        else
            hipLaunchKernelGGL((apply_small_kernel<1, P, STIFF, CT>), dim3((unsigned)nb), dim3(128), 0, s, pv, C, x, y);
    }
    return hipGetLastError();
}

template <int P>
static hipError_t launch_apply_p(const PatchView &pv, int op, Prec prec, const void *C, const double *x, double *y,
                                 hipStream_t s)
{
    if (prec == Prec::F64) {
        if (op == 2) return launch_apply_t<P, true, double>(pv, (const double *)C, x, y, s);
        return launch_apply_t<P, false, double>(pv, (const double *)C, x, y, s);
    }
    if (op == 2) return launch_apply_t<P, true, float>(pv, (const float *)C, x, y, s);
    return launch_apply_t<P, false, float>(pv, (const float *)C, x, y, s);
}

hipError_t launch_apply(const PatchView &pv, int op, Prec prec, const void *C, const double *x, double *y,
                        hipStream_t s)
{
    hipError_t e = launch_fill(y, pv.N, 0.0, s);
    if (e != hipSuccess) return e;
    switch (pv.P) {
    case 2: return launch_apply_p<2>(pv, op, prec, C, x, y, s);
    case 3: return launch_apply_p<3>(pv, op, prec, C, x, y, s);
    case 4: return launch_apply_p<4>(pv, op, prec, C, x, y, s);
    case 5: return launch_apply_p<5>(pv, op, prec, C, x, y, s);
    case 6: return launch_apply_p<6>(pv, op, prec, C, x, y, s);
    case 7: return launch_apply_p<7>(pv, op, prec, C, x, y, s);
    case 8: return launch_apply_p<8>(pv, op, prec, C, x, y, s);
    case 9: return launch_apply_p<9>(pv, op, prec, C, x, y, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sfiga
