// Matrix-free product y = A x (Sec. 3.3).  Forward: u or grad u at the
// quadrature points by sum factorization (Algorithm 3 with value and
// derivative tables); pointwise product with the folded coefficient tensor;
// backward: the transposed contractions (Algorithm 2, weights already folded
// into the coefficient), accumulated into y.
//
// d = 3 kernel: one workgroup per (E x E element tile in directions 1 and 2,
// segment of LZ element layers in direction 3) - a localized box in the
// sense of Sec. 4 - with one thread per quadrature column (q1, q2).  The
// workgroup walks its layers in order with sliding windows of the p rows of x
// and of partial y that the current layer touches; every stage handles all
// p quadrature planes of the layer at once (6 to 8 barriers per layer).  The
// coefficient tensor is the only stream that scales with Q; it is read plane
// by plane in the pointwise stage (prefetched a layer ahead only where that
// costs no occupancy).  LZ is tuned per patch by the caller.  Partial y rows
// leave the window through FP64 atomics (the accumulation of eq.
// (loc-basis-change)), because boxes share functions.
#include "kernels.h"

namespace sfiga {

template <int P>
struct STile {
    static constexpr int E = (16 + P - 1) / P;                 // elements per direction
    static constexpr int TX = E * P, TY = E * P;               // quadrature columns
    static constexpr int NX = E + P - 1, NY = E + P - 1;       // functions
    static constexpr int NT = (TX * TY + 63) / 64 * 64;
};

template <int P, bool STIFF, typename CT>
__device__ __forceinline__ void apply3d_block(const PatchView &pv, const CT *__restrict__ C,
                                              const double *__restrict__ x, double *__restrict__ y, int LZ, int bx,
                                              int by, int bz)
{
    using TL = STile<P>;
    constexpr int E = TL::E, NX = TL::NX, NY = TL::NY, TX = TL::TX, TY = TL::TY, NT = TL::NT;
    constexpr int NF = STIFF ? 3 : 1;      // gradient components or value
    constexpr int NC = STIFF ? 6 : 1;      // coefficient components
    constexpr int PP = P * P, NXY = NX * NY;
    // stage buffers: sa holds the forward direction-3 results, then the
    // pointwise results; sb the forward direction-2 results, then the
    // backward direction-1 results
    constexpr int SA = (2 * P * NXY > NF * P * TY * TX) ? 2 * P * NXY : NF * P * TY * TX;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    CT *xw = reinterpret_cast<CT *>(smem_raw);   // [P slots][NY][NX], slot = n3 mod p
    CT *yw = xw + P * NXY;                       // [P slots][NY][NX]
    CT *sa = yw + P * NXY;                       // [2][P][NY][NX] forward dir 3
    CT *sh = sa;                                 // [NF][P][TY][TX] pointwise (sa is dead by then)
    CT *sb = sa + SA;                            // [NF][P][TY][NX] forward dir 2
    CT *sr = sb;                                 // [NF][P][TY][NX] backward dir 1 (sb is dead by then)
    CT *t1B = sb + NF * P * TY * NX, *t1D = t1B + E * PP;   // tables [elem][g][j]
    CT *t2B = t1D + E * PP, *t2D = t2B + E * PP;
    CT *t3B = t2D + E * PP, *t3D = t3B + PP;

    const Dir &d0 = pv.dir[0], &d1 = pv.dir[1], &d2 = pv.dir[2];
    const int e1b = bx * E, e2b = by * E;
    const int e3a = bz * LZ;
    const int e3z = (e3a + LZ < d2.K ? e3a + LZ : d2.K) - 1;      // last layer
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int le1 = tx / P, g1 = tx % P, le2 = ty / P, g2 = ty % P;
    const bool active = tid < TX * TY && e1b + le1 < d0.K && e2b + le2 < d1.K;
    const int Q0 = d0.Q, Q1 = d1.Q;
    const int64_t N0 = d0.N, N01 = (int64_t)d0.N * d1.N;

    // coefficients of one layer for this column: when they are few (order 2
    // stiffness, mass) all planes are held in registers and the next layer's
    // are fetched during this one; otherwise they are read plane by plane in
    // the pointwise stage, which keeps the registers low enough for more
    // resident waves (measured faster from order 3 on)
    constexpr bool PRE = P * NC <= 12;
    // FP64 at order 4 and FP32 at order 3: the current layer's coefficients
    // are held in registers at little or no cost in occupancy (at FP64 order
    // 4 the LDS already limits the kernel to 3 waves per SIMD); they are
    // loaded at the start of the layer and have the two forward stages to
    // arrive.  Measured slower for the other orders.
    constexpr bool LAYER = !PRE && (sizeof(CT) == sizeof(double) ? P == 4 : P == 3);
    // Backward directions 1 and 2 in two steps (per-element sums, then sums
    // over the elements sharing a function) where it pays: FP64 from order 3,
    // FP32 from order 5 (measured).
    constexpr bool TWOSTEP = sizeof(CT) == sizeof(double) ? P >= 3 : P >= 5;
    constexpr int NCR = (PRE || LAYER) ? P : 1;
    CT cur[NCR][NC], nxt[PRE ? NCR : 1][NC];
    const int cq0 = active ? (e1b + le1) * P + g1 : 0, cq1 = active ? (e2b + le2) * P + g2 : 0;
    auto load_plane = [&](int e3, int g3, CT *dst) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            dst[c] = active ? C[coef_index(3, NC, c, cq0, cq1, e3 * P + g3, Q0, Q1)] : CT(0);
    };
    auto load_layer = [&](int e3, CT (*dst)[NC]) {
#pragma unroll
        for (int g3 = 0; g3 < NCR; ++g3) load_plane(e3, g3, dst[g3]);
    };
    auto load_xrow = [&](int n3) {
        for (int idx = tid; idx < NXY; idx += NT) {
            const int lx = idx % NX, ly = idx / NX;
            const int n0 = e1b + lx, n1 = e2b + ly;
            CT v = CT(0);
            if (n0 < d0.N && n1 < d1.N) v = (CT)x[n0 + N0 * n1 + N01 * n3];
            xw[(n3 % P) * NXY + idx] = v;
        }
    };
    auto flush_yrow = [&](int n3) {          // add the finished row to y and clear its slot
        for (int idx = tid; idx < NXY; idx += NT) {
            const int lx = idx % NX, ly = idx / NX;
            const int n0 = e1b + lx, n1 = e2b + ly;
            CT *slot = yw + (n3 % P) * NXY + idx;
            if (n0 < d0.N && n1 < d1.N) atomicAdd(&y[n0 + N0 * n1 + N01 * n3], (double)*slot);
            *slot = CT(0);
        }
    };

    if (PRE) load_layer(e3a, cur);
    for (int i = tid; i < E * PP; i += NT) {
        const int ea = e1b + i / PP, eb = e2b + i / PP;
        const int64_t sa1 = (int64_t)(ea < d0.K ? ea : 0) * PP + i % PP;   // in-bounds addresses
        const int64_t sb2 = (int64_t)(eb < d1.K ? eb : 0) * PP + i % PP;
        t1B[i] = ea < d0.K ? (CT)d0.B[sa1] : CT(0);
        t1D[i] = ea < d0.K ? (CT)d0.D[sa1] : CT(0);
        t2B[i] = eb < d1.K ? (CT)d1.B[sb2] : CT(0);
        t2D[i] = eb < d1.K ? (CT)d1.D[sb2] : CT(0);
    }
    for (int i = tid; i < P * NXY; i += NT) yw[i] = CT(0);
    for (int r = 0; r < P - 1; ++r) load_xrow(e3a + r);

    for (int e3 = e3a; e3 <= e3z; ++e3) {
        // ---- new x row entering the window, tables of this layer, next coefficients
        load_xrow(e3 + P - 1);
        for (int i = tid; i < PP; i += NT) {
            t3B[i] = (CT)d2.B[(int64_t)e3 * PP + i];
            t3D[i] = (CT)d2.D[(int64_t)e3 * PP + i];
        }
        if (PRE && e3 < e3z) load_layer(e3 + 1, nxt);
        if (LAYER) load_layer(e3, cur);
        __syncthreads();
        // ---- forward, direction 3: a = B3 x, b = D3 x, every plane
        for (int idx = tid; idx < P * NXY; idx += NT) {
            const int g3 = idx / NXY, j = idx % NXY;
            CT a = CT(0), b = CT(0);
#pragma unroll
            for (int s = 0; s < P; ++s) {
                const CT v = xw[((e3 + s) % P) * NXY + j];
                a += t3B[g3 * P + s] * v;
                if (STIFF) b += t3D[g3 * P + s] * v;
            }
            sa[g3 * NXY + j] = a;
            if (STIFF) sa[(P + g3) * NXY + j] = b;
        }
        __syncthreads();
        // ---- forward, direction 2: B2 a (d1 and value), D2 a (d2), B2 b (d3)
        for (int idx = tid; idx < P * TY * NX; idx += NT) {
            const int lx = idx % NX, yy = (idx / NX) % TY, g3 = idx / (NX * TY);
            const int l2 = yy / P, h2 = yy % P;
            CT vb = CT(0), vd = CT(0), wb = CT(0);
#pragma unroll
            for (int s = 0; s < P; ++s) {
                const CT a = sa[g3 * NXY + (l2 + s) * NX + lx];
                const CT bv = t2B[(l2 * P + h2) * P + s];
                vb += bv * a;
                if (STIFF) {
                    vd += t2D[(l2 * P + h2) * P + s] * a;
                    wb += bv * sa[(P + g3) * NXY + (l2 + s) * NX + lx];
                }
            }
            sb[(0 * P + g3) * TY * NX + yy * NX + lx] = vb;
            if (STIFF) {
                sb[(1 * P + g3) * TY * NX + yy * NX + lx] = vd;
                sb[(2 * P + g3) * TY * NX + yy * NX + lx] = wb;
            }
        }
        __syncthreads();
        // ---- forward, direction 1, and the pointwise coefficient, every plane
        if (tid < TX * TY) {
            const CT *b1 = t1B + (le1 * P + g1) * P, *db1 = t1D + (le1 * P + g1) * P;
            constexpr int UNR = (PRE || LAYER) ? P : 1;   // planes unrolled (registers hold cur)
#pragma unroll UNR
            for (int g3 = 0; g3 < P; ++g3) {
                CT cpl[NC];
                if (!PRE && !LAYER) load_plane(e3, g3, cpl);
                const CT *cg = (PRE || LAYER) ? cur[g3 < NCR ? g3 : 0] : cpl;
                CT h[NF];
                if (STIFF) {
                    CT gr0 = CT(0), gr1 = CT(0), gr2 = CT(0);
#pragma unroll
                    for (int s = 0; s < P; ++s) {
                        gr0 += db1[s] * sb[(0 * P + g3) * TY * NX + ty * NX + le1 + s];
                        gr1 += b1[s] * sb[(1 * P + g3) * TY * NX + ty * NX + le1 + s];
                        gr2 += b1[s] * sb[(2 * P + g3) * TY * NX + ty * NX + le1 + s];
                    }
                    const CT *c = cg;             // components 00 11 22 01 02 12
                    h[0] = c[0] * gr0 + c[3] * gr1 + c[4] * gr2;
                    h[NF > 1 ? 1 : 0] = c[3] * gr0 + c[1] * gr1 + c[5] * gr2;
                    h[NF > 2 ? 2 : 0] = c[4] * gr0 + c[5] * gr1 + c[2] * gr2;
                } else {
                    CT u = CT(0);
#pragma unroll
                    for (int s = 0; s < P; ++s) u += b1[s] * sb[g3 * TY * NX + ty * NX + le1 + s];
                    h[0] = cg[0] * u;
                }
#pragma unroll
                for (int f = 0; f < NF; ++f) sh[(f * P + g3) * TY * TX + ty * TX + tx] = active ? h[f] : CT(0);
            }
        }
        __syncthreads();
        // ---- backward, direction 1: D1^T h1, B1^T h2, B1^T h3 (mass: B1^T h)
        if constexpr (TWOSTEP) {
            // In two steps in place over sh.  First, per (plane, row, element l1), the
            // p sums over the element's points, part[f][j] = sum_h T_f(l1, h, j)
            // v[f][h], written over the element's own p values; then, per function
            // column lx, the sum over the <= p elements that share it.
            for (int idx = tid; idx < P * TY * E; idx += NT) {
                const int l1 = idx % E, rest = idx / E;
                const int yy = rest % TY, g3 = rest / TY;
                const int col0 = (g3 * TY + yy) * TX + l1 * P;
                CT v[NF][P];
#pragma unroll
                for (int f = 0; f < NF; ++f)
#pragma unroll
                    for (int h = 0; h < P; ++h) v[f][h] = sh[f * P * TY * TX + col0 + h];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const CT *T = (STIFF && f == 0) ? t1D : t1B;
#pragma unroll
                    for (int j = 0; j < P; ++j) {
                        CT part = CT(0);
#pragma unroll
                        for (int h = 0; h < P; ++h) part += T[(l1 * P + h) * P + j] * v[f][h];
                        sh[f * P * TY * TX + col0 + j] = part;
                    }
                }
            }
            __syncthreads();
            for (int idx = tid; idx < P * TY * NX; idx += NT) {
                const int lx = idx % NX, yy = (idx / NX) % TY, g3 = idx / (NX * TY);
                CT r[NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) r[f] = CT(0);
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    const int l1 = lx - j;                    // element whose local function j is lx
                    if (l1 < 0 || l1 >= E) continue;
                    const int col = (g3 * TY + yy) * TX + l1 * P + j;
#pragma unroll
                    for (int f = 0; f < NF; ++f) r[f] += sh[f * P * TY * TX + col];
                }
#pragma unroll
                for (int f = 0; f < NF; ++f) sr[(f * P + g3) * TY * NX + yy * NX + lx] = r[f];
            }
            __syncthreads();
        } else {
            // one item per (plane, row, function column), p^2 terms each
            for (int idx = tid; idx < P * TY * NX; idx += NT) {
                const int lx = idx % NX, yy = (idx / NX) % TY, g3 = idx / (NX * TY);
                CT r[NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) r[f] = CT(0);
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    const int l1 = lx - j;                    // element whose local function j is lx
                    if (l1 < 0 || l1 >= E) continue;
#pragma unroll
                    for (int h1 = 0; h1 < P; ++h1) {
                        const CT bv = t1B[(l1 * P + h1) * P + j];
                        const int col = (g3 * TY + yy) * TX + l1 * P + h1;
                        if (STIFF) {
                            r[0] += t1D[(l1 * P + h1) * P + j] * sh[0 * P * TY * TX + col];
                            r[NF > 1 ? 1 : 0] += bv * sh[1 * P * TY * TX + col];
                            r[NF > 2 ? 2 : 0] += bv * sh[2 * P * TY * TX + col];
                        } else {
                            r[0] += bv * sh[col];
                        }
                    }
                }
#pragma unroll
                for (int f = 0; f < NF; ++f) sr[(f * P + g3) * TY * NX + yy * NX + lx] = r[f];
            }
            __syncthreads();
        }
        // ---- backward, direction 2 into sq (the pointwise results in sa are
        // dead once direction 1 has run)
        CT *sq = sa;                                 // [2][P][NY][NX]
        if constexpr (TWOSTEP) {
            // In two steps, in place over sr: per (plane, element l2, column lx)
            // the p sums over the element's points (sB into field 0, sD into
            // field 1 of the element's own rows), then per function row the sum
            // over the <= p elements that share it.
            for (int idx = tid; idx < P * E * NX; idx += NT) {
                const int lx = idx % NX, rest = idx / NX;
                const int l2 = rest % E, g3 = rest / E;
                const int row0 = (g3 * TY + l2 * P) * NX + lx;          // point h: row0 + h NX
                CT v[NF][P];
#pragma unroll
                for (int f = 0; f < NF; ++f)
#pragma unroll
                    for (int h = 0; h < P; ++h) v[f][h] = sr[f * P * TY * NX + row0 + h * NX];
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    CT pB = CT(0), pD = CT(0);
#pragma unroll
                    for (int h = 0; h < P; ++h) {
                        const CT bv = t2B[(l2 * P + h) * P + j];
                        if (STIFF) {
                            pB += bv * v[0][h] + t2D[(l2 * P + h) * P + j] * v[NF > 1 ? 1 : 0][h];
                            pD += bv * v[NF > 2 ? 2 : 0][h];
                        } else {
                            pB += bv * v[0][h];
                        }
                    }
                    sr[row0 + j * NX] = pB;
                    if (STIFF) sr[1 * P * TY * NX + row0 + j * NX] = pD;
                }
            }
            __syncthreads();
            for (int idx = tid; idx < P * NXY; idx += NT) {
                const int j2 = idx % NXY, g3 = idx / NXY;
                const int lx = j2 % NX, ly = j2 / NX;
                CT sB = CT(0), sD = CT(0);
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    const int l2 = ly - j;
                    if (l2 < 0 || l2 >= E) continue;
                    const int row = (g3 * TY + l2 * P + j) * NX + lx;
                    sB += sr[row];
                    if (STIFF) sD += sr[1 * P * TY * NX + row];
                }
                sq[g3 * NXY + j2] = sB;
                if (STIFF) sq[(P + g3) * NXY + j2] = sD;
            }
            __syncthreads();
        } else {
            // one item per (plane, function column), p^2 terms each
            for (int idx = tid; idx < P * NXY; idx += NT) {
                const int j2 = idx % NXY, g3 = idx / NXY;
                const int lx = j2 % NX, ly = j2 / NX;
                CT sB = CT(0), sD = CT(0);
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    const int l2 = ly - j;
                    if (l2 < 0 || l2 >= E) continue;
#pragma unroll
                    for (int h2 = 0; h2 < P; ++h2) {
                        const CT bv = t2B[(l2 * P + h2) * P + j];
                        const int row = (g3 * TY + l2 * P + h2) * NX + lx;
                        if (STIFF) {
                            sB += bv * sr[0 * P * TY * NX + row] + t2D[(l2 * P + h2) * P + j] * sr[1 * P * TY * NX + row];
                            sD += bv * sr[2 * P * TY * NX + row];
                        } else {
                            sB += bv * sr[row];
                        }
                    }
                }
                sq[g3 * NXY + j2] = sB;
                if (STIFF) sq[(P + g3) * NXY + j2] = sD;
            }
            __syncthreads();
        }
        // ---- backward, direction 3 into the y window
        for (int idx = tid; idx < NXY; idx += NT) {
            CT acc[P];
#pragma unroll
            for (int s = 0; s < P; ++s) acc[s] = CT(0);
#pragma unroll
            for (int g3 = 0; g3 < P; ++g3) {
                const CT sB = sq[g3 * NXY + idx], sD = STIFF ? sq[(P + g3) * NXY + idx] : CT(0);
#pragma unroll
                for (int s = 0; s < P; ++s) {
                    acc[s] += t3B[g3 * P + s] * sB;
                    if (STIFF) acc[s] += t3D[g3 * P + s] * sD;
                }
            }
#pragma unroll
            for (int s = 0; s < P; ++s) yw[((e3 + s) % P) * NXY + idx] += acc[s];
        }
        __syncthreads();
        // ---- row e3 is complete for this box
        flush_yrow(e3);
        if (PRE && e3 < e3z) {
#pragma unroll
            for (int g3 = 0; g3 < P; ++g3)
#pragma unroll
                for (int c = 0; c < NC; ++c) cur[g3 < NCR ? g3 : 0][c] = nxt[PRE && g3 < NCR ? g3 : 0][c];
        }
    }
    __syncthreads();
    for (int r = 1; r < P; ++r) flush_yrow(e3z + r);
}

// d = 1, 2: one thread per element, element-local sum factorization,
// atomics into y.

template <int P, bool STIFF, typename CT>
__global__ __launch_bounds__(STile<P>::NT) void apply3d_kernel(PatchView pv, const CT *__restrict__ C,
                                                              const double *__restrict__ x, double *__restrict__ y,
                                                              int LZ)
{
    apply3d_block<P, STIFF, CT>(pv, C, x, y, LZ, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Persistent form over the concatenated per-patch grids of a batch.
template <int P, bool STIFF, typename CT>
__global__ __launch_bounds__(STile<P>::NT) void apply3d_persistent(TaskList tl)
{
    for (int64_t it = blockIdx.x; it < tl.nitems; it += gridDim.x) {
        const int t = task_of(tl.off, tl.ntask, it);
        const BatchTask &T = tl.tasks[t];
        const int64_t l = it - tl.off[t];
        const int bx = (int)(l % T.gx);
        const int64_t r = l / T.gx;
        apply3d_block<P, STIFF, CT>(T.pv, (const CT *)T.C, T.x, T.out, T.arg, bx, (int)(r % T.gy), (int)(r / T.gy));
        __syncthreads();   // LDS of the next block
    }
}

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
static size_t apply3d_lds()
{
    using TL = STile<P>;
    constexpr int NF = STIFF ? 3 : 1;
    constexpr int NXY = TL::NX * TL::NY;
    constexpr int SA = (2 * P * NXY > NF * P * TL::TY * TL::TX) ? 2 * P * NXY : NF * P * TL::TY * TL::TX;
    return sizeof(CT) * (size_t)(2 * P * NXY + SA + NF * P * TL::TY * TL::NX + 4 * TL::E * P * P + 2 * P * P);
}

template <int P> static int apply_tile_elems() { return STile<P>::E; }

void apply_blocks(const PatchView &pv, int lz, int &gx, int &gy, int &gz, int &LZ)
{
    int E = 0;
    switch (pv.P) {
    case 2: E = apply_tile_elems<2>(); break;
    case 3: E = apply_tile_elems<3>(); break;
    case 4: E = apply_tile_elems<4>(); break;
    case 5: E = apply_tile_elems<5>(); break;
    case 6: E = apply_tile_elems<6>(); break;
    case 7: E = apply_tile_elems<7>(); break;
    case 8: E = apply_tile_elems<8>(); break;
    default: E = apply_tile_elems<9>(); break;
    }
    gx = (pv.dir[0].K + E - 1) / E;
    gy = (pv.dir[1].K + E - 1) / E;
    if (lz <= 0) {
        // layers per workgroup: long enough to amortise the window start-up,
        // short enough to give every CU a few workgroups
        lz = (int)((int64_t)gx * gy * pv.dir[2].K / 2048);
        lz = lz < 2 ? 2 : (lz > 16 ? 16 : lz);
    }
    LZ = lz;
    gz = (pv.dir[2].K + LZ - 1) / LZ;
}

template <int P, bool STIFF, typename CT>
static hipError_t launch_apply_t(const PatchView &pv, const CT *C, const double *x, double *y, hipStream_t s, int lz)
{
    if (pv.d == 3) {
        const size_t lds = apply3d_lds<P, STIFF, CT>();
        hipError_t e = allow_dynamic_lds((const void *)apply3d_kernel<P, STIFF, CT>, lds);
        if (e != hipSuccess) return e;
        int gx, gy, gz, LZ;
        apply_blocks(pv, lz, gx, gy, gz, LZ);
        hipLaunchKernelGGL((apply3d_kernel<P, STIFF, CT>), dim3(gx, gy, gz), dim3(STile<P>::NT), lds, s, pv, C, x, y,
                           LZ);
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

template <int P, bool STIFF, typename CT>
static hipError_t launch_apply_batch_t(const TaskList &tl, int nblocks, hipStream_t s)
{
    const size_t lds = apply3d_lds<P, STIFF, CT>();
    hipError_t e = allow_dynamic_lds((const void *)apply3d_persistent<P, STIFF, CT>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((apply3d_persistent<P, STIFF, CT>), dim3(nblocks), dim3(STile<P>::NT), lds, s, tl);
    return hipGetLastError();
}

template <int P>
static hipError_t launch_apply_batch_p(const TaskList &tl, int op, Prec prec, int nblocks, hipStream_t s)
{
    if (prec == Prec::F64)
        return op == 2 ? launch_apply_batch_t<P, true, double>(tl, nblocks, s)
                       : launch_apply_batch_t<P, false, double>(tl, nblocks, s);
    return op == 2 ? launch_apply_batch_t<P, true, float>(tl, nblocks, s)
                   : launch_apply_batch_t<P, false, float>(tl, nblocks, s);
}

hipError_t launch_apply_batch(const TaskList &tl, int P, int op, Prec prec, int nblocks, hipStream_t s)
{
    if (tl.nitems == 0) return hipSuccess;
    switch (P) {
    case 2: return launch_apply_batch_p<2>(tl, op, prec, nblocks, s);
    case 3: return launch_apply_batch_p<3>(tl, op, prec, nblocks, s);
    case 4: return launch_apply_batch_p<4>(tl, op, prec, nblocks, s);
    case 5: return launch_apply_batch_p<5>(tl, op, prec, nblocks, s);
    case 6: return launch_apply_batch_p<6>(tl, op, prec, nblocks, s);
    case 7: return launch_apply_batch_p<7>(tl, op, prec, nblocks, s);
    case 8: return launch_apply_batch_p<8>(tl, op, prec, nblocks, s);
    case 9: return launch_apply_batch_p<9>(tl, op, prec, nblocks, s);
    default: return hipErrorInvalidValue;
    }
}

template <int P>
static hipError_t launch_apply_p(const PatchView &pv, int op, Prec prec, const void *C, const double *x, double *y,
                                 hipStream_t s, int lz)
{
    if (prec == Prec::F64) {
        if (op == 2) return launch_apply_t<P, true, double>(pv, (const double *)C, x, y, s, lz);
        return launch_apply_t<P, false, double>(pv, (const double *)C, x, y, s, lz);
    }
    if (op == 2) return launch_apply_t<P, true, float>(pv, (const float *)C, x, y, s, lz);
    return launch_apply_t<P, false, float>(pv, (const float *)C, x, y, s, lz);
}

hipError_t launch_apply(const PatchView &pv, int op, Prec prec, const void *C, const double *x, double *y,
                        hipStream_t s, int lz)
{
    hipError_t e = launch_fill(y, pv.N, 0.0, s);
    if (e != hipSuccess) return e;
    switch (pv.P) {
    case 2: return launch_apply_p<2>(pv, op, prec, C, x, y, s, lz);
    case 3: return launch_apply_p<3>(pv, op, prec, C, x, y, s, lz);
    case 4: return launch_apply_p<4>(pv, op, prec, C, x, y, s, lz);
    case 5: return launch_apply_p<5>(pv, op, prec, C, x, y, s, lz);
    case 6: return launch_apply_p<6>(pv, op, prec, C, x, y, s, lz);
    case 7: return launch_apply_p<7>(pv, op, prec, C, x, y, s, lz);
    case 8: return launch_apply_p<8>(pv, op, prec, C, x, y, s, lz);
    case 9: return launch_apply_p<9>(pv, op, prec, C, x, y, s, lz);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sfiga
