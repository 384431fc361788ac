// Geometry step (Sec. 6.3): G and its Jacobian at every quadrature point by
// sum factorization (Algorithm 3 applied to the control points, with value
// and derivative tables), then per point: det J (flag if <= 0), J^-1, the
// coefficient at the physical point G(x), and the folded quadrature
// coefficients (Example 1 with A = a I):
//   mass:      w c |det J|
//   stiffness: w a |det J| (J^-1 A J^-T)_ij, i <= j   (J_ik = dG_i/dxhat_k,
//              A the constant symmetric diffusion matrix, the identity by default)
//   convection: w s |det J| (J^-1 b)_k, k = 1..3 (b . grad u = (J^-1 b) . grad_hat u)
#include <hip/hip_fp16.h>

#include "kernels.h"

namespace sfiga {

template <typename T>
__device__ __forceinline__ void store_coef(void *base, int64_t idx, double v)
{
    static_cast<T *>(base)[idx] = (T)v;
}

__device__ __forceinline__ void pointwise_3d(const double G[3], const double J[3][3], double w, int64_t qlin,
                                             int q0, int q1, int q2, const PatchView &pv, const GeomOut &o,
                                             bool f32, const double *uh)
{
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    if (!(det > 0.0) && o.bad_det) *o.bad_det = 1;
    const double id = 1.0 / det;
    double inv[3][3];
    inv[0][0] = c00 * id;
    inv[1][0] = c01 * id;
    inv[2][0] = c02 * id;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    const double wd = w * fabs(det);
    const int Q0 = pv.dir[0].Q, Q1 = pv.dir[1].Q;
    if (uh) {
        // u and its physical gradient J^-T grad_hat u: (J^-T g)_i = sum_k (J^-1)_ki g_k
        if (o.uval) o.uval[qlin] = uh[0];
        if (o.ugrad)
            for (int i = 0; i < 3; ++i) o.ugrad[qlin * 3 + i] = inv[0][i] * uh[1] + inv[1][i] * uh[2] + inv[2][i] * uh[3];
    }
    if (o.xyz) {
        o.xyz[qlin * 3 + 0] = G[0];
        o.xyz[qlin * 3 + 1] = G[1];
        o.xyz[qlin * 3 + 2] = G[2];
    }
    const int P = pv.P, K0 = pv.dir[0].K, Q2 = pv.dir[2].Q;
    if (o.c_mass) {
        double v = wd * eval_coef(o.coef_mass, G, 3, qlin);
        int64_t idx = coef_index(3, 1, 0, q0, q1, q2, Q0, Q1);
        if (f32) store_coef<float>(o.c_mass, idx, v); else store_coef<double>(o.c_mass, idx, v);
        if (o.ca_mass) {
            idx = apply_coef_index(1, 0, q0, q1, q2, P, K0, Q2);
            if (f32) store_coef<float>(o.ca_mass, idx, v); else store_coef<double>(o.ca_mass, idx, v);
        }
    }
    if (o.c_conv) {
        const double s = wd * eval_coef(o.coef_conv, G, 3, qlin);
        for (int k = 0; k < 3; ++k)
            o.c_conv[conv_coef_index(k, q0, q1, q2, P, K0, Q2)] =
                s * (inv[k][0] * o.bconv[0] + inv[k][1] * o.bconv[1] + inv[k][2] * o.bconv[2]);
    }
    if (o.c_stiff) {
        double s = wd * eval_coef(o.coef_stiff, G, 3, qlin);
        // rows of J^-1 A: ai[j][k] = sum_l A_kl (J^-1)_jl (equal to J^-1 for A = I)
        double ai[3][3];
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                ai[j][k] = o.adiff[3 * k] * inv[j][0] + o.adiff[3 * k + 1] * inv[j][1] + o.adiff[3 * k + 2] * inv[j][2];
        for (int i = 0; i < 3; ++i)
            for (int j = i; j < 3; ++j) {
                double v = s * (inv[i][0] * ai[j][0] + inv[i][1] * ai[j][1] + inv[i][2] * ai[j][2]);
                const int c = sym_comp<3>(i, j);
                int64_t idx = coef_index(3, 6, c, q0, q1, q2, Q0, Q1);
                if (f32) store_coef<float>(o.c_stiff, idx, v); else store_coef<double>(o.c_stiff, idx, v);
                if (o.ca_stiff) {
                    idx = apply_coef_index(6, c, q0, q1, q2, P, K0, Q2);
                    if (f32) store_coef<float>(o.ca_stiff, idx, v); else store_coef<double>(o.ca_stiff, idx, v);
                }
            }
    }
}

// One workgroup per (E1 x E2 element tile, element layer e3).  Threads own a
// quadrature column (q1, q2); the three contractions run 3 -> 2 -> 1 through
// LDS for NPS quadrature planes g3 at a time (all p planes of the layer for
// p <= 4, so that each stage has several items per thread and the layer
// needs three barriers; one plane at a time above, to bound LDS).
template <int P> struct GeomPlanes { static constexpr int NPS = P <= 4 ? P : 1; };

// EVAL: a fourth field, the coefficients u_n of a discrete function, goes
// through the same contractions (Algorithm 3 evaluates u = sum u_n phi_n and
// its reference derivatives on the grid of quadrature points).
template <int P, bool EVAL>
constexpr size_t geom3d_lds()
{
    using TL = Tile<P>;
    constexpr int NPS = GeomPlanes<P>::NPS;
    constexpr int NFL = EVAL ? 4 : 3;
    return sizeof(double) * (NFL * P * TL::NY * TL::NX + 2 * NFL * NPS * TL::NY * TL::NX +
                             3 * NFL * NPS * TL::TY * TL::NX + 2 * (TL::E1 + TL::E2) * P * P);
}

template <int P, bool EVAL>
__global__ __launch_bounds__(Tile<P>::NT) void geom3d_kernel(PatchView pv, GeomOut o)
{
    using TL = Tile<P>;
    constexpr int NX = TL::NX, NY = TL::NY, TX = TL::TX, TY = TL::TY;
    constexpr int NPS = GeomPlanes<P>::NPS;
    constexpr int NYX = NY * NX, TYX = TY * NX;
    constexpr int NFL = EVAL ? 4 : 3;          // fields: the 3 coordinates of the control points (and u)
    extern __shared__ double smem[];
    double *cw = smem;                         // [NFL][P][NY][NX] control points (and u)
    double *sa = cw + NFL * P * NYX;           // [NPS][2 NFL][NY][NX]   B3 c, D3 c at g3
    double *sb = sa + 2 * NFL * NPS * NYX;     // [NPS][3 NFL][TY][NX]   B2 B3 c, D2 B3 c, B2 D3 c
    double *t1B = sb + 3 * NFL * NPS * TYX, *t1D = t1B + TL::E1 * P * P;   // tile tables [elem][g][j]
    double *t2B = t1D + TL::E1 * P * P, *t2D = t2B + TL::E2 * P * P;

    const Dir &d0 = pv.dir[0], &d1 = pv.dir[1], &d2 = pv.dir[2];
    const int e1b = blockIdx.x * TL::E1, e2b = blockIdx.y * TL::E2, e3 = blockIdx.z;
    const int tid = threadIdx.x;
    const bool f32 = o.prec == Prec::F32;

    for (int idx = tid; idx < NFL * P * NYX; idx += TL::NT) {
        int lx = idx % NX, r = idx / NX;
        int ly = r % NY; r /= NY;
        int s3 = r % P, c = r / P;
        int n0 = e1b + lx, n1 = e2b + ly, n2 = e3 + s3;
        double v = 0.0;
        if (n0 < d0.N && n1 < d1.N) {
            const int64_t n = (int64_t)n0 + (int64_t)d0.N * (n1 + (int64_t)d1.N * n2);
            v = c < 3 ? pv.ctrl[n * 3 + c] : o.u[n];
        }
        cw[idx] = v;
    }
    {
        constexpr int PP = P * P;
        for (int i = tid; i < TL::E1 * PP; i += TL::NT) {
            const int e = e1b + i / PP;
            const int64_t src = (int64_t)(e < d0.K ? e : 0) * PP + i % PP;   // in-bounds address
            t1B[i] = e < d0.K ? d0.B[src] : 0.0;
            t1D[i] = e < d0.K ? d0.D[src] : 0.0;
        }
        for (int i = tid; i < TL::E2 * PP; i += TL::NT) {
            const int e = e2b + i / PP;
            const int64_t src = (int64_t)(e < d1.K ? e : 0) * PP + i % PP;
            t2B[i] = e < d1.K ? d1.B[src] : 0.0;
            t2D[i] = e < d1.K ? d1.D[src] : 0.0;
        }
    }
    __syncthreads();

    const int tx = tid % TX, ty = tid / TX;
    const int le1 = tx / P, g1 = tx % P, le2 = ty / P, g2 = ty % P;
    const int e1 = e1b + le1, e2 = e2b + le2;
    const bool active = tid < TX * TY && e1 < d0.K && e2 < d1.K;

    for (int g3b = 0; g3b < P; g3b += NPS) {
        // direction 3: value and derivative of the control-point columns
        for (int it = tid; it < NPS * NYX; it += TL::NT) {
            const int gg = it / NYX, idx = it % NYX;
            const int g3 = g3b + gg;
            const double *b3 = d2.B + ((int64_t)e3 * P + g3) * P;
            const double *db3 = d2.D + ((int64_t)e3 * P + g3) * P;
            for (int c = 0; c < NFL; ++c) {
                double a = 0.0, b = 0.0;
#pragma unroll
                for (int s = 0; s < P; ++s) {
                    double v = cw[(c * P + s) * NYX + idx];
                    a += b3[s] * v;
                    b += db3[s] * v;
                }
                sa[(gg * 2 * NFL + c) * NYX + idx] = a;
                sa[(gg * 2 * NFL + NFL + c) * NYX + idx] = b;
            }
        }
        __syncthreads();
        // direction 2
        for (int it = tid; it < NPS * TYX; it += TL::NT) {
            const int gg = it / TYX, idx = it % TYX;
            const int lx = idx % NX, yy = idx / NX;
            const int l2 = yy / P, h2 = yy % P, ee2 = e2b + l2;
            if (ee2 >= d1.K) continue;
            const double *b2 = t2B + (l2 * P + h2) * P;
            const double *db2 = t2D + (l2 * P + h2) * P;
            const double *sg = sa + gg * 2 * NFL * NYX;
            double *so = sb + gg * 3 * NFL * TYX;
            for (int c = 0; c < NFL; ++c) {
                double vb = 0.0, vd = 0.0, wb = 0.0;
#pragma unroll
                for (int s = 0; s < P; ++s) {
                    double a = sg[(c * NY + l2 + s) * NX + lx];
                    double b = sg[((NFL + c) * NY + l2 + s) * NX + lx];
                    vb += b2[s] * a;
                    vd += db2[s] * a;
                    wb += b2[s] * b;
                }
                so[(3 * c + 0) * TYX + idx] = vb;
                so[(3 * c + 1) * TYX + idx] = vd;
                so[(3 * c + 2) * TYX + idx] = wb;
            }
        }
        __syncthreads();
        // direction 1 and the pointwise quantities
        if (active) {
            const double *b1 = t1B + (le1 * P + g1) * P;
            const double *db1 = t1D + (le1 * P + g1) * P;
            const int q0 = e1 * P + g1, q1 = e2 * P + g2;
            const double w01 = d0.W[q0] * d1.W[q1];
            for (int gg = 0; gg < NPS; ++gg) {
                const double *sg = sb + gg * 3 * NFL * TYX;
                double G[NFL], J[NFL][3];
                for (int c = 0; c < NFL; ++c) {
                    double gv = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
#pragma unroll
                    for (int s = 0; s < P; ++s) {
                        double vb = sg[((3 * c + 0) * TY + ty) * NX + le1 + s];
                        double vd = sg[((3 * c + 1) * TY + ty) * NX + le1 + s];
                        double wb = sg[((3 * c + 2) * TY + ty) * NX + le1 + s];
                        gv += b1[s] * vb;
                        j0 += db1[s] * vb;
                        j1 += b1[s] * vd;
                        j2 += b1[s] * wb;
                    }
                    G[c] = gv;
                    J[c][0] = j0;
                    J[c][1] = j1;
                    J[c][2] = j2;
                }
                const int q2 = e3 * P + g3b + gg;
                const double w = w01 * d2.W[q2];
                const int64_t qlin = (int64_t)q0 + (int64_t)d0.Q * (q1 + (int64_t)d1.Q * q2);
                const double uh[4] = {G[NFL - 1], J[NFL - 1][0], J[NFL - 1][1], J[NFL - 1][2]};   // u, grad_hat u
                pointwise_3d(G, J, w, qlin, q0, q1, q2, pv, o, f32, EVAL ? uh : nullptr);
            }
        }
        __syncthreads();
    }
}

// d = 1, 2: one thread per quadrature point, direct sums over the p^d active
// control points (these sizes are small; d = 3 uses the tile kernel above).
template <int DIM, int P>
__global__ void geom_small_kernel(PatchView pv, GeomOut o)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= pv.Q) return;
    const Dir &d0 = pv.dir[0], &d1 = pv.dir[1];
    int q0 = (int)(q % d0.Q), q1 = (DIM == 2) ? (int)(q / d0.Q) : 0;
    int e0 = q0 / P, g0 = q0 % P, e1 = q1 / P, g1 = q1 % P;
    double G[2] = {0, 0}, J[2][2] = {{0, 0}, {0, 0}};
    double U = 0.0, UG[2] = {0, 0};                // u and grad_hat u (evaluation)
    const double *b0 = d0.B + ((int64_t)e0 * P + g0) * P, *db0 = d0.D + ((int64_t)e0 * P + g0) * P;
    if (DIM == 1) {
        for (int s = 0; s < P; ++s) {
            double c = pv.ctrl[e0 + s];
            G[0] += b0[s] * c;
            J[0][0] += db0[s] * c;
            if (o.u) {
                U += b0[s] * o.u[e0 + s];
                UG[0] += db0[s] * o.u[e0 + s];
            }
        }
    } else {
        const double *b1 = d1.B + ((int64_t)e1 * P + g1) * P, *db1 = d1.D + ((int64_t)e1 * P + g1) * P;
        for (int s1 = 0; s1 < P; ++s1) {
            double t0[3] = {0, 0, 0}, t1[3] = {0, 0, 0};     // coordinates, then u
            for (int s0 = 0; s0 < P; ++s0) {
                const int64_t n = (int64_t)(e0 + s0) + (int64_t)d0.N * (e1 + s1);
                const double *c = pv.ctrl + n * 2;
                for (int i = 0; i < 2; ++i) {
                    t0[i] += b0[s0] * c[i];
                    t1[i] += db0[s0] * c[i];
                }
                if (o.u) {
                    t0[2] += b0[s0] * o.u[n];
                    t1[2] += db0[s0] * o.u[n];
                }
            }
            for (int i = 0; i < 2; ++i) {
                G[i] += b1[s1] * t0[i];
                J[i][0] += b1[s1] * t1[i];
                J[i][1] += db1[s1] * t0[i];
            }
            U += b1[s1] * t0[2];
            UG[0] += b1[s1] * t1[2];
            UG[1] += db1[s1] * t0[2];
        }
    }
    double det, inv[2][2];
    if (DIM == 1) {
        det = J[0][0];
        inv[0][0] = 1.0 / det;
    } else {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        inv[0][0] = J[1][1] / det;
        inv[0][1] = -J[0][1] / det;
        inv[1][0] = -J[1][0] / det;
        inv[1][1] = J[0][0] / det;
    }
    if (!(det > 0.0) && o.bad_det) *o.bad_det = 1;
    double w = d0.W[q0] * (DIM == 2 ? d1.W[q1] : 1.0);
    double wd = w * fabs(det);
    const bool f32 = o.prec == Prec::F32;
    if (o.xyz)
        for (int i = 0; i < DIM; ++i) o.xyz[q * DIM + i] = G[i];
    if (o.u && o.uval) o.uval[q] = U;
    if (o.u && o.ugrad)
        for (int i = 0; i < DIM; ++i) {
            double g = 0.0;
            for (int k = 0; k < DIM; ++k) g += inv[k][i] * UG[k];     // J^-T grad_hat u
            o.ugrad[q * DIM + i] = g;
        }
    if (o.c_mass) {
        double v = wd * eval_coef(o.coef_mass, G, DIM, q);
        int64_t idx = coef_index(DIM, 1, 0, q0, q1, 0, d0.Q, d1.Q);
        if (f32) store_coef<float>(o.c_mass, idx, v); else store_coef<double>(o.c_mass, idx, v);
    }
    if (o.c_stiff) {
        double s = wd * eval_coef(o.coef_stiff, G, DIM, q);
        constexpr int NC = DIM * (DIM + 1) / 2;
        for (int i = 0; i < DIM; ++i)
            for (int j = i; j < DIM; ++j) {
                // (J^-1 A J^-T)_ij, A the symmetric diffusion matrix
                double v = 0.0;
                for (int k = 0; k < DIM; ++k) {
                    double a = 0.0;
                    for (int l = 0; l < DIM; ++l) a += o.adiff[3 * k + l] * inv[j][l];
                    v += inv[i][k] * a;
                }
                int64_t idx = coef_index(DIM, NC, sym_comp<DIM>(i, j), q0, q1, 0, d0.Q, d1.Q);
                if (f32) store_coef<float>(o.c_stiff, idx, s * v); else store_coef<double>(o.c_stiff, idx, s * v);
            }
    }
}

template <int P, bool EVAL>
static hipError_t launch_geom3d(const PatchView &pv, const GeomOut &o, hipStream_t s)
{
    using TL = Tile<P>;
    dim3 grid((pv.dir[0].K + TL::E1 - 1) / TL::E1, (pv.dir[1].K + TL::E2 - 1) / TL::E2, pv.dir[2].K);
    constexpr size_t lds = geom3d_lds<P, EVAL>();
    hipError_t e = allow_dynamic_lds((const void *)geom3d_kernel<P, EVAL>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((geom3d_kernel<P, EVAL>), grid, dim3(TL::NT), lds, s, pv, o);
    return hipGetLastError();
}

template <int P>
static hipError_t launch_geom_p(const PatchView &pv, const GeomOut &o, hipStream_t s)
{
    if (pv.d == 3) {
        hipError_t e = o.u ? launch_geom3d<P, true>(pv, o, s) : launch_geom3d<P, false>(pv, o, s);
        if (e != hipSuccess) return e;
    } else {
        int64_t nb = (pv.Q + 255) / 256;
        if (pv.d == 2)
            hipLaunchKernelGGL((geom_small_kernel<2, P>), dim3((unsigned)nb), dim3(256), 0, s, pv, o);
        else
            hipLaunchKernelGGL((geom_small_kernel<1, P>), dim3((unsigned)nb), dim3(256), 0, s, pv, o);
    }
    return hipGetLastError();
}

// FP16-split storage of a coefficient tensor (see launch_split_coef), in two
// passes.  First the range of C / w per (element, component): one thread per
// pair, the threads of a wavefront on consecutive elements in direction 1 so
// that each (g3, g2) row of their points is one contiguous run.
__global__ void split_range_kernel(PatchView pv, int nc, const float *__restrict__ c32, float *__restrict__ rs)
{
    const Dir &d0 = pv.dir[0], &d1 = pv.dir[1], &d2 = pv.dir[2];
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)d0.K * d1.K * d2.K * nc;
    if (t >= total) return;
    const int P = pv.P;
    const int e1 = (int)(t % d0.K);
    int64_t r = t / d0.K;
    const int c = (int)(r % nc);
    r /= nc;
    const int e2 = (int)(r % d1.K), e3 = (int)(r / d1.K);
    double lo = 0.0, hi = 0.0;
    for (int g3 = 0; g3 < P; ++g3)
        for (int g2 = 0; g2 < P; ++g2) {
            const int q1 = e2 * P + g2, q2 = e3 * P + g3;
            const double w23 = d1.W[q1] * d2.W[q2];
            for (int g1 = 0; g1 < P; ++g1) {
                const int q0 = e1 * P + g1;
                const double v = (double)c32[coef_index(3, nc, c, q0, q1, q2, d0.Q, d1.Q)] / (d0.W[q0] * w23);
                if (g1 == 0 && g2 == 0 && g3 == 0) lo = hi = v;
                lo = fmin(lo, v);
                hi = fmax(hi, v);
            }
        }
    double scl = 0.5 * (hi - lo);
    if (!(scl > 0.0)) scl = 1.0;                   // constant over the element: residual 0
    const int64_t e = ((int64_t)e3 * d1.K + e2) * d0.K + e1;
    rs[(e * nc + c) * 2 + 0] = (float)(0.5 * (hi + lo));
    rs[(e * nc + c) * 2 + 1] = (float)scl;
}

// Then the residuals, the stored values in the tile-major order with the
// threads of the grid striding over them (coalesced stores; the loads of a
// tile row are one run of the FP32 tensor).  The grid is bounded: a 1D
// dispatch addresses fewer than 2^32 work-items, and 118^3 elements at order 9
// store 7.2e9 values.
__global__ void split_store_kernel(PatchView pv, int nc, const float *__restrict__ c32, const float *__restrict__ rs,
                                   __half *__restrict__ h16, int64_t total)
{
    const Dir &d0 = pv.dir[0], &d1 = pv.dir[1], &d2 = pv.dir[2];
    const int P = pv.P;
    const int T = apply_tile_elems(P) * P;
    const int gx = (d0.Q + T - 1) / T, gy = (d1.Q + T - 1) / T;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int tx = (int)(t % T);
        int64_t r = t / T;
        const int ty = (int)(r % T);
        r /= T;
        const int bx = (int)(r % gx);
        r /= gx;
        const int by = (int)(r % gy);
        r /= gy;
        const int c = (int)(r % nc), q2 = (int)(r / nc);
        const int q0 = bx * T + tx, q1 = by * T + ty;
        float h = 0.0f;                            // padding of the edge tiles
        if (q0 < d0.Q && q1 < d1.Q) {
            const int64_t e = ((int64_t)(q2 / P) * d1.K + q1 / P) * d0.K + q0 / P;
            const double w = d0.W[q0] * d1.W[q1] * d2.W[q2];
            const double v = (double)c32[coef_index(3, nc, c, q0, q1, q2, d0.Q, d1.Q)] / w;
            h = (float)((v - (double)rs[(e * nc + c) * 2]) / (double)rs[(e * nc + c) * 2 + 1]);
        }
        h16[t] = __float2half_rn(h);
    }
}

hipError_t launch_split_coef(const PatchView &pv, int op, const float *c32, void *h16, float *rs, hipStream_t s)
{
    if (pv.d != 3) return hipErrorInvalidValue;
    const int nc = op == 2 ? 6 : 1;
    const int64_t npair = (int64_t)pv.dir[0].K * pv.dir[1].K * pv.dir[2].K * nc;
    hipLaunchKernelGGL(split_range_kernel, dim3((unsigned)((npair + 255) / 256)), dim3(256), 0, s, pv, nc, c32, rs);
    const int64_t total = split_size(nc, pv.P, pv.dir[0].K, pv.dir[1].K, pv.dir[2].K);
    const int64_t nb = (total + 255) / 256;
    hipLaunchKernelGGL(split_store_kernel, dim3((unsigned)(nb < 65536 ? nb : 65536)), dim3(256), 0, s, pv, nc, c32,
                       rs, static_cast<__half *>(h16), total);
    return hipGetLastError();
}

hipError_t launch_geometry(const PatchView &pv, const GeomOut &o, hipStream_t s)
{
    switch (pv.P) {
    case 2: return launch_geom_p<2>(pv, o, s);
    case 3: return launch_geom_p<3>(pv, o, s);
    case 4: return launch_geom_p<4>(pv, o, s);
    case 5: return launch_geom_p<5>(pv, o, s);
    case 6: return launch_geom_p<6>(pv, o, s);
    case 7: return launch_geom_p<7>(pv, o, s);
    case 8: return launch_geom_p<8>(pv, o, s);
    case 9: return launch_geom_p<9>(pv, o, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sfiga
