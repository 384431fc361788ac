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
#include <hip/hip_fp16.h>

#include <type_traits>

#include "kernels.h"

namespace sfiga {

template <int P>
struct STile {
    static constexpr int E = apply_tile_elems(P);              // elements per direction
    static constexpr int TX = E * P, TY = E * P;               // quadrature columns
    static constexpr int NX = E + P - 1, NY = E + P - 1;       // functions
    static constexpr int NT = (TX * TY + 63) / 64 * 64;
};

// Per (order, operator, storage type) shape of the d = 3 kernel, chosen by
// measurement (stiffness, N = 126^3, and 128^3 at order 6):
//   ROWS   the element-row form (apply3d_rows_block): the stiffness apply at
//          every order in FP64, and from order 3 in FP32 and FP16 split
//          (N = 126^3, ms FP64 / FP32 before -> after: order 4 1.55 -> 1.23 /
//          0.94 -> 0.70, order 6 6.58 -> 4.98 / 4.18 -> 2.90, order 8 38.9
//          -> 23.2 / 10.8 -> 7.3, order 9 42.7 -> 28.1 / 20.3 -> 16.9); the
//          mass apply and order 2 in FP32 keep apply3d_block;
//   ALAY   with ROWS, the coefficients in the tiled copy (apply_coef_index);
//   G      the layer's p quadrature planes go through the plane stages
//          in G groups of ceil(p / G) planes: less LDS per workgroup (a
//          second workgroup per CU at orders 8 and 9), but more barriers
//          (FP64 order 8, N = 126^3: 19.1 ms with 2 groups, 16.6 with 3);
//   CMODE  how the coefficients reach the pointwise stage: 0 loaded in that
//          stage; 1 the layer's (apply3d_block: the group's) planes loaded at
//          the start of the layer; 2 the next layer's (apply3d_block: the next
//          group's) planes loaded from the pointwise stage on, so that they
//          have the backward stages to arrive;
//   TWOSTEP (apply3d_block) backward directions 1 and 2 in two steps
//          (per-element sums in place, then sums over the elements sharing a
//          function);
//   UNRJ   (apply3d_block) the output loop of those per-element sums
//          unrolled: more independent work per item, but the compiler then
//          holds all p^2 table values of an element in registers;
//   XCD    tiles dealt to the XCDs in contiguous ranges (xcd_tile): a tile
//          row of row-layout coefficients is TX values, not a whole number of
//          128-byte lines, so neighbouring tiles share the lines at their
//          ends; on one XCD those are fetched once;
//   JU, FU (apply3d_block, UNRJ = 0) the unroll counts of that loop and of the
//          field loop of backward direction 1;
//   W      minimum resident waves per SIMD asked of the compiler (register
//          cap).  A workgroup of six waves spreads 2, 2, 1, 1 over the four
//          SIMDs, so two of them per CU need four waves per SIMD: 128 VGPRs.
// Measured at 128^3 order 6 FP64 (ms per apply): 12.43 in the first
// apply3d_block, 7.57 in its last form, 6.68 in the element-row form on the
// row layout and 5.54 on the tiled copy.
struct ApplyShape {
    int G, CMODE, TWOSTEP, UNRJ, W, XCD;
    int JU = 1;            // with UNRJ = 0: unroll count of the per-element output loops
    int FU = 1;            // with UNRJ = 0: unroll count of the field loop of backward direction 1
    int ROWS = 0;          // the element-row form (apply3d_rows_block); TWOSTEP, UNRJ, JU, FU unused
    int ALAY = 0;          // with ROWS: the coefficients in the tiled layout of apply_coef_index
};

// storage: 0 FP64, 1 FP32, 2 FP16 split
constexpr ApplyShape apply_shape(int P, int storage, bool stiff)
{
    const bool f64 = storage == 0;
    // BEGIN SHAPES
    // element-row form with the tiled coefficient copy (FP64, FP32) or the
    // FP16-split storage; coefficients a layer ahead (CMODE 2), or plane
    // groups with their own loads where one workgroup per CU would be left
    if (stiff && (f64 || P > 2)) {
        const int alay = storage == 2 ? 0 : 1;
        if (P == 8 && f64) return ApplyShape{3, 0, 1, 0, 4, 1, 1, 1, 1, alay};
        if (P == 8 && storage == 1) return ApplyShape{2, 0, 1, 0, 4, 1, 1, 1, 1, alay};
        if (P == 9 && storage == 1) return ApplyShape{3, 0, 1, 0, 4, 1, 1, 1, 1, alay};
        return ApplyShape{1, 2, 1, 0, P <= 6 ? 4 : 2, 1, 1, 1, 1, alay};
    }
    if (!stiff || P == 2) return ApplyShape{1, 2, f64 ? P >= 3 : P >= 5, 1, 1, P == 2 || (!f64 && P <= 4)};
    return ApplyShape{1, 1, P >= 5, 1, 1, P <= 4};
    // END SHAPES
}

template <int P, bool STIFF, typename CS>
struct ApplyCfg {
    static constexpr ApplyShape S =
        apply_shape(P, sizeof(CS) == sizeof(double) ? 0 : (sizeof(CS) == sizeof(float) ? 1 : 2), STIFF);
    static constexpr int G = S.G;
    static constexpr int CMODE = S.CMODE;
    static constexpr bool TWOSTEP = S.TWOSTEP != 0;
    static constexpr bool UNRJ = S.UNRJ != 0;
    static constexpr int JU = S.JU, FU = S.FU;
    static constexpr int W = S.W;
    static constexpr bool XCD = S.XCD != 0;
    static constexpr bool ROWS = S.ROWS != 0;
    static constexpr bool ALAY = S.ROWS != 0 && S.ALAY != 0;
};

// Storage of the coefficient tensor: double or float (computed in that type),
// or __half in the FP16-split form (computed in float): per element and
// component a reference r and a scale s (FP32, `rs`), per point an FP16
// residual h, with C = w (r + s h) where w is the product of the point's
// Gauss weights.
template <typename CS> struct ComputeOf { using T = CS; };
template <> struct ComputeOf<__half> { using T = float; };

template <int P, bool STIFF, typename CS>
__device__ __forceinline__ void apply3d_block(const PatchView &pv, const CS *__restrict__ C,
                                              const float *__restrict__ rs, const double *__restrict__ x,
                                              double *__restrict__ y, int LZ, int bx, int by, int bz)
{
    using CT = typename ComputeOf<CS>::T;
    constexpr bool SPLIT = !std::is_same<CS, CT>::value;
    using TL = STile<P>;
    using CF = ApplyCfg<P, STIFF, CS>;
    constexpr int E = TL::E, NX = TL::NX, NY = TL::NY, TX = TL::TX, TY = TL::TY, NT = TL::NT;
    constexpr int NF = STIFF ? 3 : 1;      // gradient components or value
    constexpr int NC = STIFF ? 6 : 1;      // coefficient components
    constexpr int PP = P * P, NXY = NX * NY;
    constexpr int G = CF::G, PG = (P + G - 1) / G;     // plane groups, planes per group
    constexpr int CMODE = CF::CMODE;
    constexpr bool TWOSTEP = CF::TWOSTEP;
    // stage buffers: sa the forward direction-3 results of all planes; sh the
    // pointwise results and sb the forward direction-2 / backward direction-1
    // results of one group; sq the backward direction-2 results of all planes.
    // With one group sa, sh and sq share one buffer (each is dead when the
    // next one is written).
    constexpr int SA = 2 * P * NXY, SH = NF * PG * TY * TX, SB = NF * PG * TY * NX;
    constexpr int SAHQ = G == 1 ? (SA > SH ? SA : SH) : 2 * SA + SH;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    CT *xw = reinterpret_cast<CT *>(smem_raw);   // [P slots][NY][NX], slot = n3 mod p
    CT *yw = xw + P * NXY;                       // [P slots][NY][NX]
    CT *sa = yw + P * NXY;                       // [2][P][NY][NX]
    CT *sh = G == 1 ? sa : sa + SA;              // [NF][PG][TY][TX]
    CT *sq = G == 1 ? sa : sh + SH;              // [2][P][NY][NX]
    CT *sb = sa + SAHQ;                          // [NF][PG][TY][NX]
    CT *sr = sb;
    CT *t1B = sb + SB, *t1D = t1B + E * PP;      // tables [elem][g][j]
    CT *t2B = t1D + E * PP, *t2D = t2B + E * PP;
    CT *t3Bb = t2D + E * PP, *t3Db = t3Bb + 2 * PP;   // direction-3 tables, [layer parity][g][j]
    CT *t3Wb = t3Db + 2 * PP;                         // direction-3 weights, [layer parity][g] (FP16 split)
    static_assert(NXY <= NT && PP <= NT, "one prefetched x value and table entry per thread");

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

    const int cq0 = active ? (e1b + le1) * P + g1 : 0, cq1 = active ? (e2b + le2) * P + g2 : 0;
    // stored values are kept raw in registers and converted where they are
    // used, so that a prefetch never waits for its loads
    // FP16 split: the tile's plane of one component is one contiguous block
    // (split_index), read by the workgroup's threads in order
    const int64_t tile0 = SPLIT ? split_index(NC, 0, e1b * P, e2b * P, 0, P, d0.K, d1.K) : 0;
    const int64_t plane_stride = SPLIT ? split_index(NC, 1, 0, 0, 0, P, d0.K, d1.K) : 0;
    auto load_plane = [&](int e3, int g3, CS *dst) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if constexpr (SPLIT)
                dst[c] = active ? C[tile0 + ((int64_t)(e3 * P + g3) * NC + c) * plane_stride + tid] : CS(0);
            else
                dst[c] = active ? C[coef_index(3, NC, c, cq0, cq1, e3 * P + g3, Q0, Q1)] : CS(0);
        }
    };
    // FP16 split: the element's reference and scale of the current layer, and
    // the weights of the thread's column in directions 1 and 2
    CT rsr[SPLIT ? 2 * NC : 1];
    const CT w12 = SPLIT && active ? (CT)(d0.W[cq0] * d1.W[cq1]) : CT(0);
    const int64_t rs_col = SPLIT && active ? ((int64_t)(e2b + le2) * d0.K + e1b + le1) * 2 * NC : 0;
    auto load_rs = [&](int e3) {
        if constexpr (SPLIT) {
#pragma unroll
            for (int k = 0; k < 2 * NC; ++k)
                rsr[k] = active ? rs[(int64_t)e3 * d1.K * d0.K * 2 * NC + rs_col + k] : CT(0);
        }
    };
    auto coef = [&](CS raw, int c, CT w3v) -> CT {
        if constexpr (SPLIT) return w12 * w3v * (rsr[2 * c] + rsr[2 * c + 1] * __half2float(raw));
        else return (CT)raw;
    };
    // coefficients of the planes of group grp of layer e3 (CMODE 1, 2)
    constexpr int NCR = CMODE ? PG : 1;
    CS cur[NCR][NC], nxt[CMODE == 2 ? NCR : 1][NC];
    auto load_group = [&](int e3, int grp, CS (*dst)[NC]) {
#pragma unroll
        for (int gl = 0; gl < NCR; ++gl) {
            const int g3 = grp * PG + gl;
            if (g3 < P) load_plane(e3, g3, dst[gl]);
        }
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

    if (CMODE == 2) load_group(e3a, 0, cur);
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
    for (int r = 0; r < P; ++r) load_xrow(e3a + r);
    if (tid < PP) {
        t3Bb[(e3a & 1) * PP + tid] = (CT)d2.B[(int64_t)e3a * PP + tid];
        t3Db[(e3a & 1) * PP + tid] = (CT)d2.D[(int64_t)e3a * PP + tid];
    }
    if (SPLIT && tid < P) t3Wb[(e3a & 1) * P + tid] = (CT)d2.W[(int64_t)e3a * P + tid];
    // the x row and the direction-3 tables of the next layer are loaded into
    // registers at the start of a layer and stored to LDS once the forward
    // direction-3 stage no longer reads the slot, so that no layer waits for
    // a global load before its first stage
    const int xlx = tid % NX, xly = tid / NX;
    const bool xin = tid < NXY && e1b + xlx < d0.N && e2b + xly < d1.N;
    const int64_t xoff = xin ? (e1b + xlx) + N0 * (e2b + xly) : 0;
    __syncthreads();

    for (int e3 = e3a; e3 <= e3z; ++e3) {
        const CT *t3B = t3Bb + (e3 & 1) * PP, *t3D = t3Db + (e3 & 1) * PP, *t3W = t3Wb + (e3 & 1) * P;
        const bool more = e3 < e3z;
        double xn = 0.0, tnB = 0.0, tnD = 0.0, tnW = 0.0;
        if (more) {
            if (xin) xn = x[xoff + N01 * (e3 + P)];
            if (tid < PP) {
                tnB = d2.B[(int64_t)(e3 + 1) * PP + tid];
                tnD = d2.D[(int64_t)(e3 + 1) * PP + tid];
            }
            if (SPLIT && tid < P) tnW = d2.W[(int64_t)(e3 + 1) * P + tid];
        }
        load_rs(e3);
        // the first group's coefficients (CMODE 1) have the forward stages to
        // arrive; with one group, CMODE 2 fetches the next layer's here, a
        // whole layer ahead
        if (CMODE == 1) load_group(e3, 0, cur);
        if (CMODE == 2 && G == 1) {
            if (e3 > e3a) {
#pragma unroll
                for (int gl = 0; gl < NCR; ++gl)
#pragma unroll
                    for (int c = 0; c < NC; ++c) cur[gl][c] = nxt[CMODE == 2 ? gl : 0][c];
            }
            if (more) load_group(e3 + 1, 0, nxt);
        }
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
        // ---- the slot of x row e3 and the other table buffer are free now
        if (more) {
            if (tid < NXY) xw[((e3 + P) % P) * NXY + tid] = (CT)xn;
            if (tid < PP) {
                t3Bb[((e3 + 1) & 1) * PP + tid] = (CT)tnB;
                t3Db[((e3 + 1) & 1) * PP + tid] = (CT)tnD;
            }
            if (SPLIT && tid < P) t3Wb[((e3 + 1) & 1) * P + tid] = (CT)tnW;
        }
#pragma unroll 1
        for (int grp = 0; grp < G; ++grp) {
            const int g0 = grp * PG;
            const int npl = (P - g0 < PG) ? P - g0 : PG;         // planes in this group
            if (CMODE == 1 && grp > 0) load_group(e3, grp, cur);
            if (CMODE == 2 && G > 1 && (grp > 0 || e3 > e3a)) {
#pragma unroll
                for (int gl = 0; gl < NCR; ++gl)
#pragma unroll
                    for (int c = 0; c < NC; ++c) cur[gl][c] = nxt[CMODE == 2 ? gl : 0][c];
            }
            // ---- forward, direction 2: B2 a (d1 and value), D2 a (d2), B2 b (d3)
            for (int idx = tid; idx < npl * TY * NX; idx += NT) {
                const int lx = idx % NX, yy = (idx / NX) % TY, gl = idx / (NX * TY);
                const int g3 = g0 + gl;
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
                sb[(0 * PG + gl) * TY * NX + yy * NX + lx] = vb;
                if (STIFF) {
                    sb[(1 * PG + gl) * TY * NX + yy * NX + lx] = vd;
                    sb[(2 * PG + gl) * TY * NX + yy * NX + lx] = wb;
                }
            }
            __syncthreads();
            // ---- forward, direction 1, and the pointwise coefficient, every plane of the group
            if (tid < TX * TY) {
                const CT *b1 = t1B + (le1 * P + g1) * P, *db1 = t1D + (le1 * P + g1) * P;
#pragma unroll
                for (int gl = 0; gl < PG; ++gl) {
                    if (gl >= npl) break;
                    CS cpl[NC];
                    if (CMODE == 0) load_plane(e3, g0 + gl, cpl);
                    const CS *cr = CMODE ? cur[CMODE ? gl : 0] : cpl;
                    const CT w3v = SPLIT ? t3W[g0 + gl] : CT(0);
                    CT cg[NC];
#pragma unroll
                    for (int c = 0; c < NC; ++c) cg[c] = coef(cr[c], c, w3v);
                    CT h[NF];
                    if (STIFF) {
                        CT gr0 = CT(0), gr1 = CT(0), gr2 = CT(0);
#pragma unroll
                        for (int s = 0; s < P; ++s) {
                            gr0 += db1[s] * sb[(0 * PG + gl) * TY * NX + ty * NX + le1 + s];
                            gr1 += b1[s] * sb[(1 * PG + gl) * TY * NX + ty * NX + le1 + s];
                            gr2 += b1[s] * sb[(2 * PG + gl) * TY * NX + ty * NX + le1 + s];
                        }
                        const CT *c = cg;             // components 00 11 22 01 02 12
                        h[0] = c[0] * gr0 + c[3] * gr1 + c[4] * gr2;
                        h[NF > 1 ? 1 : 0] = c[3] * gr0 + c[1] * gr1 + c[5] * gr2;
                        h[NF > 2 ? 2 : 0] = c[4] * gr0 + c[5] * gr1 + c[2] * gr2;
                    } else {
                        CT u = CT(0);
#pragma unroll
                        for (int s = 0; s < P; ++s) u += b1[s] * sb[gl * TY * NX + ty * NX + le1 + s];
                        h[0] = cg[0] * u;
                    }
#pragma unroll
                    for (int f = 0; f < NF; ++f) sh[(f * PG + gl) * TY * TX + ty * TX + tx] = active ? h[f] : CT(0);
                }
            }
            // the coefficients of the next group (or of the next layer's first
            // group) are on their way during the backward stages
            if (CMODE == 2 && G > 1) {
                if (grp + 1 < G) load_group(e3, grp + 1, nxt);
                else if (more) load_group(e3 + 1, 0, nxt);
            }
            __syncthreads();
            // ---- backward, direction 1: D1^T h1, B1^T h2, B1^T h3 (mass: B1^T h)
            if constexpr (TWOSTEP) {
                // In two steps in place over sh.  First, per (plane, row, element l1),
                // the p sums over the element's points, part[f][j] = sum_h
                // T_f(l1, h, j) v[f][h], written over the element's own p values;
                // then, per function column lx, the sum over the <= p elements
                // that share it.
                for (int idx = tid; idx < npl * TY * E; idx += NT) {
                    const int l1 = idx % E, rest = idx / E;
                    const int yy = rest % TY, gl = rest / TY;
                    const int col0 = (gl * TY + yy) * TX + l1 * P;
                    if constexpr (CF::UNRJ) {
                        // every field's p values first, then all outputs
                        CT v[NF][P];
#pragma unroll
                        for (int f = 0; f < NF; ++f)
#pragma unroll
                            for (int hh = 0; hh < P; ++hh) v[f][hh] = sh[f * PG * TY * TX + col0 + hh];
#pragma unroll
                        for (int f = 0; f < NF; ++f) {
                            const CT *T = (STIFF && f == 0) ? t1D : t1B;
#pragma unroll
                            for (int j = 0; j < P; ++j) {
                                CT part = CT(0);
#pragma unroll
                                for (int hh = 0; hh < P; ++hh) part += T[(l1 * P + hh) * P + j] * v[f][hh];
                                sh[f * PG * TY * TX + col0 + j] = part;
                            }
                        }
                    } else {
                        // one field at a time, one output at a time: its p values are
                        // read before any is overwritten, and only p table values are
                        // live at once
#pragma unroll (CF::FU)
                        for (int f = 0; f < NF; ++f) {
                            const CT *T = (STIFF && f == 0) ? t1D : t1B;
                            CT *col = sh + f * PG * TY * TX + col0;
                            CT v[P];
#pragma unroll
                            for (int hh = 0; hh < P; ++hh) v[hh] = col[hh];
#pragma unroll (CF::JU)
                            for (int j = 0; j < P; ++j) {
                                CT part = CT(0);
#pragma unroll
                                for (int hh = 0; hh < P; ++hh) part += T[(l1 * P + hh) * P + j] * v[hh];
                                col[j] = part;
                            }
                        }
                    }
                }
                __syncthreads();
                for (int idx = tid; idx < npl * TY * NX; idx += NT) {
                    const int lx = idx % NX, yy = (idx / NX) % TY, gl = idx / (NX * TY);
                    CT r[NF];
#pragma unroll
                    for (int f = 0; f < NF; ++f) r[f] = CT(0);
#pragma unroll
                    for (int j = 0; j < P; ++j) {
                        const int l1 = lx - j;                    // element whose local function j is lx
                        if (l1 < 0 || l1 >= E) continue;
                        const int col = (gl * TY + yy) * TX + l1 * P + j;
#pragma unroll
                        for (int f = 0; f < NF; ++f) r[f] += sh[f * PG * TY * TX + col];
                    }
#pragma unroll
                    for (int f = 0; f < NF; ++f) sr[(f * PG + gl) * TY * NX + yy * NX + lx] = r[f];
                }
                __syncthreads();
            } else {
                // one item per (plane, row, function column), p^2 terms each
                for (int idx = tid; idx < npl * TY * NX; idx += NT) {
                    const int lx = idx % NX, yy = (idx / NX) % TY, gl = idx / (NX * TY);
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
                            const int col = (gl * TY + yy) * TX + l1 * P + h1;
                            if (STIFF) {
                                r[0] += t1D[(l1 * P + h1) * P + j] * sh[0 * PG * TY * TX + col];
                                r[NF > 1 ? 1 : 0] += bv * sh[1 * PG * TY * TX + col];
                                r[NF > 2 ? 2 : 0] += bv * sh[2 * PG * TY * TX + col];
                            } else {
                                r[0] += bv * sh[col];
                            }
                        }
                    }
#pragma unroll
                    for (int f = 0; f < NF; ++f) sr[(f * PG + gl) * TY * NX + yy * NX + lx] = r[f];
                }
                __syncthreads();
            }
            // ---- backward, direction 2 into sq at the group's planes
            if constexpr (TWOSTEP) {
                // In two steps, in place over sr: per (plane, element l2, column lx)
                // the p sums over the element's points (sB into field 0, sD into
                // field 1 of the element's own rows), then per function row the sum
                // over the <= p elements that share it.
                for (int idx = tid; idx < npl * E * NX; idx += NT) {
                    const int lx = idx % NX, rest = idx / NX;
                    const int l2 = rest % E, gl = rest / E;
                    const int row0 = (gl * TY + l2 * P) * NX + lx;          // point h: row0 + h NX
                    if constexpr (CF::UNRJ) {
                        CT v[NF][P];
#pragma unroll
                        for (int f = 0; f < NF; ++f)
#pragma unroll
                            for (int hh = 0; hh < P; ++hh) v[f][hh] = sr[f * PG * TY * NX + row0 + hh * NX];
#pragma unroll
                        for (int j = 0; j < P; ++j) {
                            CT pB = CT(0), pD = CT(0);
#pragma unroll
                            for (int hh = 0; hh < P; ++hh) {
                                const CT bv = t2B[(l2 * P + hh) * P + j];
                                if (STIFF) {
                                    pB += bv * v[0][hh] + t2D[(l2 * P + hh) * P + j] * v[NF > 1 ? 1 : 0][hh];
                                    pD += bv * v[NF > 2 ? 2 : 0][hh];
                                } else {
                                    pB += bv * v[0][hh];
                                }
                            }
                            sr[row0 + j * NX] = pB;
                            if (STIFF) sr[1 * PG * TY * NX + row0 + j * NX] = pD;
                        }
                        continue;
                    }
                    // sB from fields 0 and 1 into field 0, then sD from field 2 into
                    // field 1: each step reads its inputs before it overwrites them
                    {
                        CT v0[P], v1[P];
#pragma unroll
                        for (int hh = 0; hh < P; ++hh) {
                            v0[hh] = sr[row0 + hh * NX];
                            v1[hh] = STIFF ? sr[1 * PG * TY * NX + row0 + hh * NX] : CT(0);
                        }
#pragma unroll (CF::JU)
                        for (int j = 0; j < P; ++j) {
                            CT pB = CT(0);
#pragma unroll
                            for (int hh = 0; hh < P; ++hh) {
                                pB += t2B[(l2 * P + hh) * P + j] * v0[hh];
                                if (STIFF) pB += t2D[(l2 * P + hh) * P + j] * v1[hh];
                            }
                            sr[row0 + j * NX] = pB;
                        }
                    }
                    if (STIFF) {
                        CT v2[P];
#pragma unroll
                        for (int hh = 0; hh < P; ++hh) v2[hh] = sr[(NF - 1) * PG * TY * NX + row0 + hh * NX];
#pragma unroll (CF::JU)
                        for (int j = 0; j < P; ++j) {
                            CT pD = CT(0);
#pragma unroll
                            for (int hh = 0; hh < P; ++hh) pD += t2B[(l2 * P + hh) * P + j] * v2[hh];
                            sr[1 * PG * TY * NX + row0 + j * NX] = pD;
                        }
                    }
                }
                __syncthreads();
                for (int idx = tid; idx < npl * NXY; idx += NT) {
                    const int j2 = idx % NXY, gl = idx / NXY;
                    const int g3 = g0 + gl;
                    const int lx = j2 % NX, ly = j2 / NX;
                    CT sB = CT(0), sD = CT(0);
#pragma unroll
                    for (int j = 0; j < P; ++j) {
                        const int l2 = ly - j;
                        if (l2 < 0 || l2 >= E) continue;
                        const int row = (gl * TY + l2 * P + j) * NX + lx;
                        sB += sr[row];
                        if (STIFF) sD += sr[1 * PG * TY * NX + row];
                    }
                    sq[g3 * NXY + j2] = sB;
                    if (STIFF) sq[(P + g3) * NXY + j2] = sD;
                }
            } else {
                // one item per (plane, function column), p^2 terms each
                for (int idx = tid; idx < npl * NXY; idx += NT) {
                    const int j2 = idx % NXY, gl = idx / NXY;
                    const int g3 = g0 + gl;
                    const int lx = j2 % NX, ly = j2 / NX;
                    CT sB = CT(0), sD = CT(0);
#pragma unroll
                    for (int j = 0; j < P; ++j) {
                        const int l2 = ly - j;
                        if (l2 < 0 || l2 >= E) continue;
#pragma unroll
                        for (int h2 = 0; h2 < P; ++h2) {
                            const CT bv = t2B[(l2 * P + h2) * P + j];
                            const int row = (gl * TY + l2 * P + h2) * NX + lx;
                            if (STIFF) {
                                sB += bv * sr[0 * PG * TY * NX + row] +
                                      t2D[(l2 * P + h2) * P + j] * sr[1 * PG * TY * NX + row];
                                sD += bv * sr[2 * PG * TY * NX + row];
                            } else {
                                sB += bv * sr[row];
                            }
                        }
                    }
                    sq[g3 * NXY + j2] = sB;
                    if (STIFF) sq[(P + g3) * NXY + j2] = sD;
                }
            }
            __syncthreads();
        }
        // ---- backward, direction 3 into the y window, one item per (row s, column)
        for (int idx = tid; idx < P * NXY; idx += NT) {
            const int s3 = idx / NXY, j = idx % NXY;
            CT acc = CT(0);
#pragma unroll
            for (int g3 = 0; g3 < P; ++g3) {
                acc += t3B[g3 * P + s3] * sq[g3 * NXY + j];
                if (STIFF) acc += t3D[g3 * P + s3] * sq[(P + g3) * NXY + j];
            }
            yw[((e3 + s3) % P) * NXY + j] += acc;
        }
        __syncthreads();
        // ---- row e3 is complete for this box
        flush_yrow(e3);
    }
    __syncthreads();
    for (int r = 1; r < P; ++r) flush_yrow(e3z + r);
}

// Tables read by a whole wavefront at one address: through the constant
// address space the compiler turns these reads into scalar loads, so an
// element's tables cost neither LDS traffic nor vector registers.
template <typename T>
using uniform_ptr = const __attribute__((address_space(4))) T *;

template <typename CT> __device__ __forceinline__ const CT *table_B(const Dir &d);
template <typename CT> __device__ __forceinline__ const CT *table_D(const Dir &d);
template <> __device__ __forceinline__ const double *table_B<double>(const Dir &d) { return d.B; }
template <> __device__ __forceinline__ const double *table_D<double>(const Dir &d) { return d.D; }
template <> __device__ __forceinline__ const float *table_B<float>(const Dir &d) { return d.Bf; }
template <> __device__ __forceinline__ const float *table_D<float>(const Dir &d) { return d.Df; }

// The element's p x p table of direction d as a scalar-load pointer; e is
// wave-uniform (clamped into range: an element beyond the patch only meets
// zero values, any finite table gives zero there).
template <typename CT>
__device__ __forceinline__ uniform_ptr<CT> elem_table(const CT *base, int e, int K, int PP)
{
    e = __builtin_amdgcn_readfirstlane(e < K ? e : K - 1);
    return (uniform_ptr<CT>)(base + (int64_t)e * PP);
}

// Thread mappings of the element-row form of the d = 3 apply, for PG planes
// at a time.  A stage whose items belong to one element (its p x p table)
// gives every element a whole number of wavefronts: lanes per element are the
// item count rounded up to 64, so the element index, and with it the table
// address, is the same across a wavefront.
template <int P, int PG>
struct RowsMap {
    using TL = STile<P>;
    static constexpr int pad64(int n) { return (n + 63) / 64 * 64; }
    static constexpr int NXY = TL::NX * TL::NY;
    static constexpr int R2 = pad64(PG * TL::NX);  // direction-2 stages: (plane, function column) per element row l2
    static constexpr int R1 = pad64(PG * TL::TY);  // direction-1 stages: (plane, point row) per element l1
    static constexpr int RXY = pad64(NXY);         // direction-3 stages: function columns per plane group
    static constexpr int GS = TL::NT / RXY >= P ? P : (TL::NT / RXY >= 1 ? TL::NT / RXY : 1);
    static constexpr int PG3 = (P + GS - 1) / GS;  // planes (forward) or rows (backward) per group
};

// LDS of the element-row form, in compute-type elements: x and y windows,
// the direction-3 results (aliasing the point values when all planes go at
// once), the direction-2 values and the point values of a plane group, and
// the direction-3 weights.
template <int P, bool STIFF, int G>
constexpr int rows_lds_elems()
{
    using TL = STile<P>;
    constexpr int PG = (P + G - 1) / G, NF = STIFF ? 3 : 1, NA = STIFF ? 2 : 1, NXY = TL::NX * TL::NY;
    constexpr int SA = NA * P * (NXY | 1), SH = NF * PG * TL::TY * (TL::TX | 1), SB = NF * PG * TL::TY * (TL::NX | 1);
    return 2 * P * NXY + (G == 1 ? (SA > SH ? SA : SH) : SA + SH) + SB + 2 * P + 4 * P * P;
}

// Element-row form of the d = 3 apply (same box, window and layer walk as
// apply3d_block).  Each stage that contracts one direction gives a work item
// one element's whole 1D slice: it reads the slice's p values once, keeps them
// in registers and forms all p outputs with the element's table in scalar
// registers, instead of reading a value and a table entry from LDS for every
// multiply-add.  Stages per layer (F2 to B2 for each group of PG planes):
//   F3  a = B3 x, b = D3 x (function column, group of planes)
//   F2  B2 a, D2 a, B2 b (element row l2 and output field: plane, function
//       column)
//   F1  gradients (element l1: plane, point row)
//   PW  pointwise product with C (one thread per quadrature column)
//   B1  per-element transposed sums over an element's points (element l1)
//   B2  the same in direction 2 (element row l2), each input formed from the
//       per-element parts of the elements that share its function column;
//       in FP64 the results go into the direction-2 sums with LDS atomics,
//       otherwise the sums over the elements that share a function row get a
//       stage of their own (orders 2 and 3 also sum the direction-1 parts in
//       a stage of their own)
//   B3  the transposed direction-3 sums into the y window (function column,
//       group of rows)
template <int P, bool STIFF, typename CS, bool ALAY, int CM>
__device__ __forceinline__ void apply3d_rows_block(const PatchView &pv, const CS *__restrict__ C,
                                                   const float *__restrict__ rs, const double *__restrict__ x,
                                                   double *__restrict__ y, int LZ, int bx, int by, int bz)
{
    using CT = typename ComputeOf<CS>::T;
    constexpr bool SPLIT = !std::is_same<CS, CT>::value;
    using TL = STile<P>;
    using CF = ApplyCfg<P, STIFF, CS>;
    constexpr int G = CF::G, PG = (P + G - 1) / G;
    using RM = RowsMap<P, PG>;
    constexpr int E = TL::E, NX = TL::NX, NY = TL::NY, TX = TL::TX, TY = TL::TY, NT = TL::NT;
    constexpr int NF = STIFF ? 3 : 1;      // gradient components or value
    constexpr int NA = STIFF ? 2 : 1;      // forward direction-3 results (B3 x, D3 x)
    constexpr int NC = STIFF ? 6 : 1;      // coefficient components
    constexpr int PP = P * P, NXY = NX * NY;
    // Row strides of the stage buffers, rounded up to an odd number of
    // elements so that items on consecutive rows fall into different LDS banks.
    constexpr int AS = NXY | 1, HS = TX | 1, BS = NX | 1;
    constexpr int SHF = PG * TY * HS;      // one field of the point values of a group
    constexpr int SBF = PG * TY * BS;      // one field of the direction-2 values of a group
    constexpr int SA = NA * P * AS, SH = NF * SHF;
    static_assert(G == 1 || CM == 0, "plane groups load their coefficients in the pointwise stage");
    // LDS: x and y windows [P slots][NY][NX]; ra the forward direction-3
    // results sa and then the backward direction-2 sums sq, [NA][P][AS]; rh
    // the point values sh [NF][PG][TY][HS]; rb the forward direction-2
    // results sb and then (without ATOM2) the backward direction-1 sums and
    // the per-element backward direction-2 rows, [NF][PG][TY][BS].  With one
    // group ra lies inside rh (sa is dead before sh is written, sh before
    // sq), and with ATOM2 sq lies in rb (see below).
    extern __shared__ __align__(16) unsigned char smem_raw[];
    CT *xw = reinterpret_cast<CT *>(smem_raw);
    CT *yw = xw + P * NXY;
    CT *rh = yw + P * NXY;
    CT *ra = G == 1 ? rh : rh + SH;
    CT *rb = rh + (G == 1 ? (SA > SH ? SA : SH) : SA + SH);
    // FOLD1 (elements per tile <= p): backward direction 2 forms the sums
    // over the elements that share a function column as it reads its inputs.
    // ATOM2 (FOLD1 in FP64): it also adds its results straight into the
    // direction-2 sums sq with LDS atomics (the <= p elements that share a
    // function row meet there); sq then lies in rb with one plane group (rb is
    // free from the pointwise stage on) and in ra with several.  The FP32 LDS
    // atomics measured slower than the separate sum (order 6: 4.03 against
    // 2.63 ms at N = 126^3).
    constexpr bool FOLD1 = E <= P;
    constexpr bool ATOM2 = FOLD1 && sizeof(CT) == sizeof(double);
    constexpr int NQ2 = STIFF ? 3 : 1;     // output fields of forward direction 2 (one item each)
    constexpr bool MERGE3 = ATOM2 && G == 1 && CM == 2;
    static_assert(!(ATOM2 && G == 1) || NA * P * AS <= NF * SBF, "sq fits in rb");
    CT *sq = (ATOM2 && G == 1) ? rb : ra;
    CT *t3Wb = rb + NF * SBF;              // direction-3 weights, [layer parity][g] (FP16 split)
    CT *t3s = t3Wb + 2 * P;                // direction-3 tables with CMODE 2, [layer parity][B, D][g][j]
    static_assert(NXY <= NT, "one prefetched x value per thread");

    const Dir &d0 = pv.dir[0], &d1 = pv.dir[1], &d2 = pv.dir[2];
    const CT *B1g = table_B<CT>(d0), *D1g = table_D<CT>(d0);
    const CT *B2g = table_B<CT>(d1), *D2g = table_D<CT>(d1);
    const CT *B3g = table_B<CT>(d2), *D3g = table_D<CT>(d2);
    const int e1b = bx * E, e2b = by * E;
    const int e3a = bz * LZ;
    const int e3z = (e3a + LZ < d2.K ? e3a + LZ : d2.K) - 1;      // last layer
    const int Q0 = d0.Q, Q1 = d1.Q;
    const int64_t N0 = d0.N, N01 = (int64_t)d0.N * d1.N;
    const int64_t tile0 = SPLIT ? split_index(NC, 0, e1b * P, e2b * P, 0, P, d0.K, d1.K) : 0;
    const int64_t plane_stride = SPLIT ? split_index(NC, 1, 0, 0, 0, P, d0.K, d1.K) : 0;

    // Per-thread offsets are recomputed inside each stage from an opaque copy
    // of the thread index: hoisted out of the layer loop, the offsets of all
    // stages would hold registers for the whole kernel.
    auto thread_index = [&]() {
        int t = threadIdx.x;
        asm volatile("" : "+v"(t));
        return t;
    };
    // The thread's quadrature column (pointwise stage).  Loads are issued
    // without a condition (an inactive thread reads an in-range address, its
    // results are zeroed where they are stored): under a branch the compiler
    // waits for every load in flight at the next use of any of them.
    struct Col {
        int tid, tx, ty, le1;
        bool active;
        int64_t cq0, cq1;
    };
    auto column = [&]() {
        Col c;
        c.tid = thread_index();
        c.tx = c.tid % TX;
        c.ty = c.tid / TX;
        c.le1 = c.tx / P;
        c.active = c.tid < TX * TY && e1b + c.le1 < d0.K && e2b + c.ty / P < d1.K;
        c.cq0 = c.active ? (int64_t)e1b * P + c.tx : 0;
        c.cq1 = c.active ? (int64_t)e2b * P + c.ty : 0;
        return c;
    };
    // tiled layout (ALAY): the tile's block of plane q3, a pair of components
    // per load
    constexpr int W = STIFF ? 2 : 1;
    const int64_t tile_base = (int64_t)(by * ((d0.K + E - 1) / E) + bx) * d2.Q;
    auto load_plane = [&](const Col &c, int e3, int g3, CS *dst) {
        if constexpr (ALAY && !SPLIT) {
            const int64_t t = c.tid < TX * TY ? c.tid : TX * TY - 1;
            const int64_t b0 = (tile_base + e3 * P + g3) * (NC / W) * (TX * TY);
#pragma unroll
            for (int kp = 0; kp < NC / W; ++kp) {
                const CS *src = C + (b0 + kp * (TX * TY) + t) * W;
                if constexpr (W == 2) {
                    using V2 = typename std::conditional<sizeof(CS) == 8, double2, float2>::type;
                    const V2 v = *reinterpret_cast<const V2 *>(src);
                    dst[2 * kp] = v.x;
                    dst[2 * kp + 1] = v.y;
                } else {
                    dst[kp] = src[0];
                }
            }
            return;
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            if constexpr (SPLIT)
                dst[k] = C[tile0 + ((int64_t)(e3 * P + g3) * NC + k) * plane_stride +
                           (c.tid < TX * TY ? c.tid : TX * TY - 1)];
            else
                dst[k] = C[coef_index(3, NC, k, (int)c.cq0, (int)c.cq1, e3 * P + g3, Q0, Q1)];
        }
    };
    auto flush_yrow = [&](int n3) {          // add the finished row to y and clear its slot
        for (int idx = thread_index(); idx < NXY; idx += NT) {
            const int lx = idx % NX, ly = idx / NX;
            const int n0 = e1b + lx, n1 = e2b + ly;
            CT *slot = yw + (n3 % P) * NXY + idx;
            if (n0 < d0.N && n1 < d1.N) atomicAdd(&y[n0 + N0 * n1 + N01 * n3], (double)*slot);
            *slot = CT(0);
        }
    };

    {
        const int tid = threadIdx.x;
        for (int i = tid; i < P * NXY; i += NT) yw[i] = CT(0);
        for (int r = 0; r < P; ++r) {
            const int n3 = e3a + r;
            for (int idx = tid; idx < NXY; idx += NT) {
                const int n0 = e1b + idx % NX, n1 = e2b + idx / NX;
                xw[(n3 % P) * NXY + idx] = (n0 < d0.N && n1 < d1.N) ? (CT)x[n0 + N0 * n1 + N01 * n3] : CT(0);
            }
        }
        if (SPLIT && tid < P) t3Wb[(e3a & 1) * P + tid] = (CT)d2.W[(int64_t)e3a * P + tid];
    }
    // Global loads are issued in the order they are needed (the memory
    // counter retires in order) and without a condition: the x row that
    // enters the window after layer e3's forward direction-3 stage (row e3 +
    // P) and the direction-3 weights of layer e3 + 1, then the coefficients
    // of layer e3 (CMODE 1 and 2; CMODE 0 loads each group's in its
    // pointwise stage).  With CMODE 2 they are issued at the end of the
    // pointwise stage of layer e3 - 1, so that they have a whole layer to
    // arrive.  Rows and layers past the end are clamped into range; their
    // values are not used.
    // With CMODE 2 the direction-3 tables of the next layer come the same way
    // (into registers, then into LDS during the last stage of the layer), and
    // the coefficient loads are spread over three stages (planes [0, p/3) at
    // the end of the pointwise stage, then the rest after backward stages 1
    // and 2) so that their issue does not stall one stage.
    constexpr bool T3L = CM == 2;
    double xn, tnW, tnB = 0.0, tnD = 0.0;
    CS cur[CM ? P : PG][NC];
    auto load_layer_head = [&](int e3) {
        const int tid = thread_index();
        const int xlx = tid % NX, xly = tid / NX;
        const bool xin = tid < NXY && e1b + xlx < d0.N && e2b + xly < d1.N;
        const int64_t xoff = xin ? (e1b + xlx) + N0 * (e2b + xly) : 0;
        const int e3c = e3 <= e3z ? e3 : e3z;
        xn = x[xoff + N01 * (e3c + P < d2.N ? e3c + P : d2.N - 1)];
        xn = xin ? xn : 0.0;
        tnW = SPLIT ? d2.W[(int64_t)(e3c < e3z ? e3c + 1 : e3c) * P + (tid % P)] : 0.0;
        if constexpr (T3L) {
            const int64_t o = (int64_t)e3c * PP + (tid < PP ? tid : 0);
            tnB = B3g[o];
            tnD = D3g[o];
        }
    };
    auto load_planes = [&](int e3, int lo, int hi) {
        if constexpr (CM != 0) {
            const int e3c = e3 <= e3z ? e3 : e3z;
            const Col c = column();
#pragma unroll
            for (int gl = 0; gl < P; ++gl)
                if (gl >= lo && gl < hi) load_plane(c, e3c, gl, cur[gl]);
        }
    };
    auto store_t3 = [&](int e3) {          // the direction-3 tables of layer e3, loaded by load_layer_head
        if constexpr (T3L) {
            const int tid = thread_index();
            if (tid < PP) {
                t3s[(e3 & 1) * 2 * PP + tid] = (CT)tnB;
                t3s[(e3 & 1) * 2 * PP + PP + tid] = (CT)tnD;
            }
        }
    };
    if constexpr (CM == 2) {
        load_layer_head(e3a);
        store_t3(e3a);
        load_planes(e3a, 0, P);
    }
    // ---- F3 of layer e: a = B3 x, b = D3 x into sa, per function column and
    // group of planes.  With MERGE3 it runs in the last stage of the previous
    // layer, beside backward direction 3 (they touch different buffers: sq
    // lies in rb, sa in rh, and the x window of layer e is complete once the
    // previous layer's first stage stored its last row), which saves one
    // barrier per layer.
    auto forward3 = [&](int e, const CT *t3Le, uniform_ptr<CT> T3Be, uniform_ptr<CT> T3De) {
        auto tb3 = [&](int i) -> CT { if constexpr (T3L) return t3Le[i]; else return T3Be[i]; };
        auto td3 = [&](int i) -> CT { if constexpr (T3L) return t3Le[PP + i]; else return T3De[i]; };
        for (int idx = thread_index(); idx < RM::GS * RM::RXY; idx += NT) {
            const int grp = __builtin_amdgcn_readfirstlane(idx / RM::RXY), j = idx % RM::RXY;
            if (j < NXY) {
                CT v[P];
#pragma unroll
                for (int s = 0; s < P; ++s) v[s] = xw[((e + s) % P) * NXY + j];
#pragma unroll
                for (int k = 0; k < RM::PG3; ++k) {
                    const int g3 = grp * RM::PG3 + k;
                    if (g3 < P) {
                        CT a = CT(0), b = CT(0);
#pragma unroll
                        for (int s = 0; s < P; ++s) {
                            a += tb3(g3 * P + s) * v[s];
                            if (STIFF) b += td3(g3 * P + s) * v[s];
                        }
                        ra[g3 * AS + j] = a;
                        if (STIFF) ra[(P + g3) * AS + j] = b;
                    }
                }
            }
        }
    };
    __syncthreads();
    if constexpr (MERGE3) {
        forward3(e3a, t3s + (e3a & 1) * 2 * PP, elem_table(B3g, e3a, d2.K, PP), elem_table(D3g, e3a, d2.K, PP));
        __syncthreads();
    }

    for (int e3 = e3a; e3 <= e3z; ++e3) {
        const bool more = e3 < e3z;
        const CT *t3W = t3Wb + (e3 & 1) * P;
        if constexpr (CM != 2) {
            load_layer_head(e3);
            load_planes(e3, 0, P);
        }
        // direction-3 tables of this layer: from LDS (CMODE 2) or scalar loads
        const CT *t3L = t3s + (e3 & 1) * 2 * PP;
        const uniform_ptr<CT> T3Bs = elem_table(B3g, e3, d2.K, PP), T3Ds = elem_table(D3g, e3, d2.K, PP);
        auto t3b = [&](int i) -> CT { if constexpr (T3L) return t3L[i]; else return T3Bs[i]; };
        auto t3d = [&](int i) -> CT { if constexpr (T3L) return t3L[PP + i]; else return T3Ds[i]; };

        // ---- F3 (without MERGE3; with it, the previous layer's last stage ran it)
        if constexpr (!MERGE3) {
            forward3(e3, t3L, T3Bs, T3Ds);
            __syncthreads();
        }
        // the slot of x row e3 is free now
        if (more) {
            const int tid = thread_index();
            if (tid < NXY) xw[((e3 + P) % P) * NXY + tid] = (CT)xn;
            if (SPLIT && tid < P) t3Wb[((e3 + 1) & 1) * P + tid] = (CT)tnW;
        }
#pragma unroll 1
        for (int grp = 0; grp < G; ++grp) {
            const int g0 = grp * PG;
            const int npl = P - g0 < PG ? P - g0 : PG;          // planes in this group

            // ---- F2: per element row l2, output field q and (plane, function
            // column): B2 a (q = 0), D2 a (q = 1) or B2 b (q = 2) at the
            // element's p points.  (l2, q) is the same across a wavefront, so
            // the table of the item is uniform, and the three fields of the
            // stiffness run on three times the lanes.
            for (int idx = thread_index(); idx < E * NQ2 * RM::R2; idx += NT) {
                const int w = __builtin_amdgcn_readfirstlane(idx / RM::R2), r = idx % RM::R2;
                const int l2 = w / NQ2, q = w % NQ2;
                const uniform_ptr<CT> T2 = elem_table(q == 1 ? D2g : B2g, e2b + l2, d1.K, PP);
                if (r < npl * NX) {
                    const int gl = r / NX, lx = r % NX;
                    const CT *in = ra + ((q == 2 ? P : 0) + g0 + gl) * AS + l2 * NX + lx;
                    CT a[P];
#pragma unroll
                    for (int s2 = 0; s2 < P; ++s2) a[s2] = in[s2 * NX];
                    CT *o = rb + q * SBF + (gl * TY + l2 * P) * BS + lx;
#pragma unroll
                    for (int h2 = 0; h2 < P; ++h2) {
                        CT v = CT(0);
#pragma unroll
                        for (int s2 = 0; s2 < P; ++s2) v += T2[h2 * P + s2] * a[s2];
                        o[h2 * BS] = v;
                    }
                }
            }
            __syncthreads();
            // ---- F1, per element l1 and (plane, point row): the gradient (mass:
            // the value) at the element's p points from the p function values of
            // each field, into sh
            if constexpr (ATOM2 && G > 1) {
                // this group's planes of sq (in ra; their sa values are dead
                // now) start from zero: backward direction 2 adds into them
                for (int i = thread_index(); i < NA * npl * AS; i += NT) {
                    const int k = i / (npl * AS), rem = i % (npl * AS);
                    sq[(k * P + g0) * AS + rem] = CT(0);
                }
            }
            for (int idx = thread_index(); idx < E * RM::R1; idx += NT) {
                const int l1 = idx / RM::R1, r = idx % RM::R1;
                const uniform_ptr<CT> T1B = elem_table(B1g, e1b + l1, d0.K, PP);
                const uniform_ptr<CT> T1D = elem_table(D1g, e1b + l1, d0.K, PP);
                if (r < npl * TY) {
                    const CT *in = rb + r * BS + l1;         // r = gl * TY + yy; function l1 + s at in[s]
                    CT *out = rh + r * HS + l1 * P;          // point g1 at out[g1]
#pragma unroll
                    for (int f = 0; f < NF; ++f) {
                        CT v[P];
#pragma unroll
                        for (int s2 = 0; s2 < P; ++s2) v[s2] = in[f * SBF + s2];
#pragma unroll
                        for (int g = 0; g < P; ++g) {
                            CT acc = CT(0);
#pragma unroll
                            for (int s2 = 0; s2 < P; ++s2)
                                acc += ((STIFF && f == 0) ? T1D[g * P + s2] : T1B[g * P + s2]) * v[s2];
                            out[f * SHF + g] = acc;
                        }
                    }
                }
            }
            __syncthreads();
            // ---- PW: the pointwise coefficient, one thread per quadrature column, in place
            if constexpr (ATOM2 && G == 1) {
                // sq (in rb, whose forward direction-2 values are dead) starts from zero
                for (int i = thread_index(); i < NA * P * AS; i += NT) sq[i] = CT(0);
            }
            {
                const Col c = column();
                if constexpr (CM == 0) {
#pragma unroll
                    for (int gl = 0; gl < PG; ++gl) load_plane(c, e3, g0 + gl < P ? g0 + gl : P - 1, cur[gl]);
                }
                if (c.tid < TX * TY) {
                    // FP16 split: the element's reference and scale of this layer
                    // and the weight of the column in directions 1 and 2
                    CT rsr[SPLIT ? 2 * NC : 1];
                    CT w12 = CT(0);
                    if constexpr (SPLIT) {
                        const int64_t rs_col =
                            c.active ? ((int64_t)(e2b + c.ty / P) * d0.K + e1b + c.le1) * 2 * NC : 0;
#pragma unroll
                        for (int k = 0; k < 2 * NC; ++k)
                            rsr[k] = rs[(int64_t)e3 * d1.K * d0.K * 2 * NC + rs_col + k];
                        w12 = (CT)(d0.W[c.cq0] * d1.W[c.cq1]);
                    }
#pragma unroll
                    for (int gl = 0; gl < PG; ++gl) {
                        if (gl >= npl) break;
                        const CS *cr = cur[CM ? (G == 1 ? gl : 0) : gl];
                        CT cg[NC];
#pragma unroll
                        for (int k = 0; k < NC; ++k) {
                            if constexpr (SPLIT)
                                cg[k] = w12 * t3W[g0 + gl] * (rsr[2 * k] + rsr[2 * k + 1] * __half2float(cr[k]));
                            else
                                cg[k] = (CT)cr[k];
                        }
                        CT *pt = rh + (gl * TY + c.ty) * HS + c.tx;
                        CT h[NF];
                        if (STIFF) {
                            const CT gr0 = pt[0], gr1 = pt[SHF], gr2 = pt[2 * SHF];
                            const CT *q = cg;             // components 00 11 22 01 02 12
                            h[0] = q[0] * gr0 + q[3] * gr1 + q[4] * gr2;
                            h[NF > 1 ? 1 : 0] = q[3] * gr0 + q[1] * gr1 + q[5] * gr2;
                            h[NF > 2 ? 2 : 0] = q[4] * gr0 + q[5] * gr1 + q[2] * gr2;
                        } else {
                            h[0] = cg[0] * pt[0];
                        }
#pragma unroll
                        for (int f = 0; f < NF; ++f) pt[f * SHF] = c.active ? h[f] : CT(0);
                    }
                }
            }
            if constexpr (CM == 2) {
                load_layer_head(e3 + 1);
                load_planes(e3 + 1, 0, P / 3);
            }
            __syncthreads();
            // ---- B1, per element l1 and (plane, point row): the p transposed sums
            // over the element's points, written over the element's own p values
            for (int idx = thread_index(); idx < E * RM::R1; idx += NT) {
                const int l1 = idx / RM::R1, r = idx % RM::R1;
                const uniform_ptr<CT> T1B = elem_table(B1g, e1b + l1, d0.K, PP);
                const uniform_ptr<CT> T1D = elem_table(D1g, e1b + l1, d0.K, PP);
                if (r < npl * TY) {
                    CT *col = rh + r * HS + l1 * P;          // r = gl * TY + yy
                    // one field at a time (field 0 with D for stiffness, the others
                    // with B), one row of the table (point hh, all functions j) at a time
#pragma unroll
                    for (int f = 0; f < NF; ++f) {
                        CT v[P], part[P];
#pragma unroll
                        for (int hh = 0; hh < P; ++hh) {
                            v[hh] = col[f * SHF + hh];
                            part[hh] = CT(0);
                        }
#pragma unroll
                        for (int hh = 0; hh < P; ++hh)
#pragma unroll
                            for (int j = 0; j < P; ++j)
                                part[j] += ((STIFF && f == 0) ? T1D[hh * P + j] : T1B[hh * P + j]) * v[hh];
#pragma unroll
                        for (int j = 0; j < P; ++j) col[f * SHF + j] = part[j];
                    }
                }
            }
            if constexpr (CM == 2) load_planes(e3 + 1, P / 3, 2 * P / 3);
            __syncthreads();
            // With more elements per tile than points per element (orders 2
            // and 3), the sums over the elements that share a function column
            // get a stage of their own (into rb); otherwise backward direction
            // 2 forms them as it reads its inputs.
            if constexpr (!FOLD1) {
                for (int idx = thread_index(); idx < npl * TY * NX; idx += NT) {
                    const int lx = idx % NX, rr = idx / NX;          // rr = gl * TY + yy
                    CT rv[NF];
#pragma unroll
                    for (int f = 0; f < NF; ++f) rv[f] = CT(0);
#pragma unroll
                    for (int j = 0; j < P; ++j) {
                        const int l1 = lx - j;                       // element whose local function j is lx
                        if (l1 < 0 || l1 >= E) continue;
#pragma unroll
                        for (int f = 0; f < NF; ++f) rv[f] += rh[f * SHF + rr * HS + l1 * P + j];
                    }
#pragma unroll
                    for (int f = 0; f < NF; ++f) rb[f * SBF + rr * BS + lx] = rv[f];
                }
                __syncthreads();
            }
            // ---- B2 with ATOM2: per element row l2, input field q and (plane,
            // function column), the p transposed sums over the element's points
            // of field q's direction-1 sums (formed from the per-element parts
            // of the <= p elements that share the column), added into the
            // direction-2 sums sq: B-part from fields 0 (B table) and 1 (D
            // table), D-part from field 2 (B table).  (l2, q) is the same
            // across a wavefront.
            if constexpr (ATOM2) {
            for (int idx = thread_index(); idx < E * NQ2 * RM::R2; idx += NT) {
                const int w = __builtin_amdgcn_readfirstlane(idx / RM::R2), r = idx % RM::R2;
                const int l2 = w / NQ2, q = w % NQ2;
                const uniform_ptr<CT> T2 = elem_table(q == 1 ? D2g : B2g, e2b + l2, d1.K, PP);
                if (r < npl * NX) {
                    const int gl = r / NX, lx = r % NX;
                    const CT *hrow = rh + q * SHF + (gl * TY + l2 * P) * HS;   // point row hh: hrow[hh HS]
                    CT v[P], pt[P];
#pragma unroll
                    for (int hh = 0; hh < P; ++hh) {
                        CT acc = CT(0);
#pragma unroll
                        for (int l1 = 0; l1 < E; ++l1) {
                            const int j = lx - l1;
                            const bool ok = j >= 0 && j < P;
                            const CT t = hrow[hh * HS + l1 * P + (ok ? j : 0)];
                            acc += ok ? t : CT(0);
                        }
                        v[hh] = acc;
                        pt[hh] = CT(0);
                    }
#pragma unroll
                    for (int hh = 0; hh < P; ++hh)
#pragma unroll
                        for (int j = 0; j < P; ++j) pt[j] += T2[hh * P + j] * v[hh];
                    CT *qo = sq + ((q == 2 ? P : 0) + g0 + gl) * AS + l2 * NX + lx;   // function row l2 + j
#pragma unroll
                    for (int j = 0; j < P; ++j) atomicAdd(qo + j * NX, pt[j]);
                }
            }
            } else {
            // ---- B2, per element row l2 and (plane, function column): the p
            // transposed sums over the element's points of the backward
            // direction-1 results, into the element's own rows of rb (the
            // B-part from fields 0 and 1 into field 0, the D-part from field 2
            // into field 1; each field is read before it is overwritten).
            // With FOLD1 each input, the direction-1 sum at function column lx,
            // is formed here from the per-element parts of the <= p elements
            // that share lx.
            for (int idx = thread_index(); idx < E * RM::R2; idx += NT) {
                const int l2 = idx / RM::R2, r = idx % RM::R2;
                const uniform_ptr<CT> T2B = elem_table(B2g, e2b + l2, d1.K, PP);
                const uniform_ptr<CT> T2D = elem_table(D2g, e2b + l2, d1.K, PP);
                if (r < npl * NX) {
                    const int gl = r / NX, lx = r % NX;
                    const CT *hrow = rh + (gl * TY + l2 * P) * HS;   // point row hh: hrow[hh HS]
                    auto sum1 = [&](int f, int hh) -> CT {
                        if constexpr (!FOLD1) return rb[f * SBF + (gl * TY + l2 * P + hh) * BS + lx];
                        CT v = CT(0);
                        if constexpr (E <= P) {
#pragma unroll
                            for (int l1 = 0; l1 < E; ++l1) {
                                const int j = lx - l1;
                                const bool ok = j >= 0 && j < P;
                                const CT t = hrow[f * SHF + hh * HS + l1 * P + (ok ? j : 0)];
                                v += ok ? t : CT(0);
                            }
                        } else {
#pragma unroll
                            for (int j = 0; j < P; ++j) {
                                const int l1 = lx - j;
                                const bool ok = l1 >= 0 && l1 < E;
                                const CT t = hrow[f * SHF + hh * HS + (ok ? l1 : 0) * P + j];
                                v += ok ? t : CT(0);
                            }
                        }
                        return v;
                    };
                    CT *o = rb + (gl * TY + l2 * P) * BS + lx;   // output function row j: o[j BS]
                    // ATOM2: function row l2 + j of sq
                    CT *qo = sq + (g0 + gl) * AS + l2 * NX + lx;
                    {
                        CT v0[P], v1[P], pB[P];
#pragma unroll
                        for (int hh = 0; hh < P; ++hh) {
                            v0[hh] = sum1(0, hh);
                            if (STIFF) v1[hh] = sum1(1, hh);
                            pB[hh] = CT(0);
                        }
#pragma unroll
                        for (int hh = 0; hh < P; ++hh)
#pragma unroll
                            for (int j = 0; j < P; ++j) {
                                pB[j] += T2B[hh * P + j] * v0[hh];
                                if (STIFF) pB[j] += T2D[hh * P + j] * v1[hh];
                            }
#pragma unroll
                        for (int j = 0; j < P; ++j) {
                            if constexpr (ATOM2) atomicAdd(qo + j * NX, pB[j]);
                            else o[j * BS] = pB[j];
                        }
                    }
                    if constexpr (STIFF) {
                        CT v[P], pD[P];
#pragma unroll
                        for (int hh = 0; hh < P; ++hh) {
                            v[hh] = sum1(2, hh);
                            pD[hh] = CT(0);
                        }
#pragma unroll
                        for (int hh = 0; hh < P; ++hh)
#pragma unroll
                            for (int j = 0; j < P; ++j) pD[j] += T2B[hh * P + j] * v[hh];
#pragma unroll
                        for (int j = 0; j < P; ++j) {
                            if constexpr (ATOM2) atomicAdd(qo + P * AS + j * NX, pD[j]);
                            else o[SBF + j * BS] = pD[j];
                        }
                    }
                }
            }
            }
            if constexpr (CM == 2) load_planes(e3 + 1, 2 * P / 3, P);
            if constexpr (MERGE3) {
                if (more) store_t3(e3 + 1);   // read by the next layer's F3 in the last stage
            }
            __syncthreads();
            // then (without ATOM2) per function row the sum over the <= p
            // elements that share it, into sq
            if constexpr (!ATOM2) {
            for (int idx = thread_index(); idx < npl * NXY; idx += NT) {
                const int j2 = idx % NXY, gl = idx / NXY;
                const int lx = j2 % NX, ly = j2 / NX;
                CT sB = CT(0), sD = CT(0);
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    const int l2 = ly - j;
                    if (l2 < 0 || l2 >= E) continue;
                    const int row = (gl * TY + l2 * P + j) * BS + lx;
                    sB += rb[row];
                    if (STIFF) sD += rb[SBF + row];
                }
                sq[(g0 + gl) * AS + j2] = sB;
                if (STIFF) sq[(P + g0 + gl) * AS + j2] = sD;
            }
            __syncthreads();
            }
        }
        // ---- B3: per function column and group of rows s3, into the y window
        for (int idx = thread_index(); idx < RM::GS * RM::RXY; idx += NT) {
            const int grp = __builtin_amdgcn_readfirstlane(idx / RM::RXY), j = idx % RM::RXY;
            if (j < NXY) {
                CT q[NA][P];
#pragma unroll
                for (int g3 = 0; g3 < P; ++g3) {
                    q[0][g3] = sq[g3 * AS + j];
                    if (STIFF) q[NA - 1][g3] = sq[(P + g3) * AS + j];
                }
                CT acc[RM::PG3];
#pragma unroll
                for (int k = 0; k < RM::PG3; ++k) acc[k] = CT(0);
#pragma unroll
                for (int g3 = 0; g3 < P; ++g3) {
#pragma unroll
                    for (int k = 0; k < RM::PG3; ++k) {
                        const int s3 = grp * RM::PG3 + k < P ? grp * RM::PG3 + k : P - 1;
                        acc[k] += t3b(g3 * P + s3) * q[0][g3];
                        if (STIFF) acc[k] += t3d(g3 * P + s3) * q[NA - 1][g3];
                    }
                }
#pragma unroll
                for (int k = 0; k < RM::PG3; ++k) {
                    const int s3 = grp * RM::PG3 + k;
                    if (s3 < P) yw[((e3 + s3) % P) * NXY + j] += acc[k];
                }
            }
        }
        if constexpr (MERGE3) {
            if (more) forward3(e3 + 1, t3s + ((e3 + 1) & 1) * 2 * PP, T3Bs, T3Ds);
        } else {
            if (more) store_t3(e3 + 1);
        }
        __syncthreads();
        // ---- row e3 is complete for this box
        flush_yrow(e3);
    }
    __syncthreads();
    for (int r = 1; r < P; ++r) flush_yrow(e3z + r);
}

// d = 1, 2: one thread per element, element-local sum factorization,
// atomics into y.

template <int P, bool STIFF, typename CS>
using ApplyCfgS = ApplyCfg<P, STIFF, CS>;

template <int P, bool STIFF, typename CS, bool ALAY>
__global__ __launch_bounds__(STile<P>::NT, (ApplyCfgS<P, STIFF, CS>::W)) void apply3d_kernel(
    PatchView pv, const CS *__restrict__ C, const float *__restrict__ rs, const double *__restrict__ x,
    double *__restrict__ y, int LZ)
{
    // neighbouring tiles in direction 1 share the cache lines at the ends of
    // their coefficient rows (a tile row is TX values, not a whole number of
    // 128-byte lines): on one XCD those lines are fetched once
    int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
    if (ApplyCfgS<P, STIFF, CS>::XCD) xcd_tile(bx, by, bz);
    if constexpr (ApplyCfgS<P, STIFF, CS>::ROWS)
        apply3d_rows_block<P, STIFF, CS, ALAY, ApplyCfgS<P, STIFF, CS>::CMODE>(pv, C, rs, x, y, LZ, bx, by, bz);
    else
        apply3d_block<P, STIFF, CS>(pv, C, rs, x, y, LZ, bx, by, bz);
}

// Persistent form over the concatenated per-patch grids of a batch.
template <int P, bool STIFF, typename CS>
__global__ __launch_bounds__(STile<P>::NT, (ApplyCfgS<P, STIFF, CS>::W)) void apply3d_persistent(TaskList tl)
{
    for (int64_t it = blockIdx.x; it < tl.nitems; it += gridDim.x) {
        const int t = task_of(tl.off, tl.ntask, it);
        const BatchTask &T = tl.tasks[t];
        const int64_t l = it - tl.off[t];
        const int bx = (int)(l % T.gx);
        const int64_t r = l / T.gx;
        if constexpr (ApplyCfgS<P, STIFF, CS>::ROWS)
            // the coefficients in the pointwise stage: the persistent loop
            // leaves no registers for a layer of them in flight
            apply3d_rows_block<P, STIFF, CS, false, 0>(T.pv, (const CS *)T.C, T.rs, T.x, T.out, T.arg, bx,
                                                       (int)(r % T.gy), (int)(r / T.gy));
        else
            apply3d_block<P, STIFF, CS>(T.pv, (const CS *)T.C, T.rs, T.x, T.out, T.arg, bx, (int)(r % T.gy),
                                        (int)(r / T.gy));
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

template <int P, bool STIFF, typename CS>
static size_t apply3d_lds()
{
    using CT = typename ComputeOf<CS>::T;
    using TL = STile<P>;
    using CF = ApplyCfg<P, STIFF, CS>;
    constexpr int NF = STIFF ? 3 : 1;
    constexpr int NXY = TL::NX * TL::NY;
    constexpr int PG = (P + CF::G - 1) / CF::G;
    constexpr int SA = 2 * P * NXY, SH = NF * PG * TL::TY * TL::TX, SB = NF * PG * TL::TY * TL::NX;
    constexpr int SAHQ = CF::G == 1 ? (SA > SH ? SA : SH) : 2 * SA + SH;
    if constexpr (CF::ROWS) return sizeof(CT) * (size_t)rows_lds_elems<P, STIFF, CF::G>();
    return sizeof(CT) * (size_t)(2 * P * NXY + SAHQ + SB + 4 * TL::E * P * P + 4 * P * P + 2 * P);
}

void apply_blocks(const PatchView &pv, int lz, int &gx, int &gy, int &gz, int &LZ)
{
    const int E = apply_tile_elems(pv.P);
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

template <int P, bool STIFF, typename CS, bool ALAY>
static hipError_t launch_apply3d(const PatchView &pv, const CS *C, const float *rs, const double *x, double *y,
                                 hipStream_t s, int lz)
{
    const size_t lds = apply3d_lds<P, STIFF, CS>();
    hipError_t e = allow_dynamic_lds((const void *)apply3d_kernel<P, STIFF, CS, ALAY>, lds);
    if (e != hipSuccess) return e;
    int gx, gy, gz, LZ;
    apply_blocks(pv, lz, gx, gy, gz, LZ);
    hipLaunchKernelGGL((apply3d_kernel<P, STIFF, CS, ALAY>), dim3(gx, gy, gz), dim3(STile<P>::NT), lds, s, pv, C, rs,
                       x, y, LZ);
    return hipGetLastError();
}

template <int P, bool STIFF, typename CS>
static hipError_t launch_apply_t(const PatchView &pv, const CS *C, const float *rs, const double *x, double *y,
                                 hipStream_t s, int lz, bool tiled)
{
    if (pv.d == 3) {
        if constexpr (ApplyCfg<P, STIFF, CS>::ALAY) {
            if (tiled) return launch_apply3d<P, STIFF, CS, true>(pv, C, rs, x, y, s, lz);
        }
        if (tiled) return hipErrorInvalidValue;       // this shape reads the coef_index layout
        return launch_apply3d<P, STIFF, CS, false>(pv, C, rs, x, y, s, lz);
    } else {
        if constexpr (std::is_same<CS, __half>::value) {
            return hipErrorInvalidValue;           // FP16 split is built for d = 3
        } else {
            int64_t nel = (int64_t)pv.dir[0].K * pv.dir[1].K;
            int64_t nb = (nel + 127) / 128;
            if (pv.d == 2)
                hipLaunchKernelGGL((apply_small_kernel<2, P, STIFF, CS>), dim3((unsigned)nb), dim3(128), 0, s, pv, C, x,
                                   y);
            else
                hipLaunchKernelGGL((apply_small_kernel<1, P, STIFF, CS>), dim3((unsigned)nb), dim3(128), 0, s, pv, C, x,
                                   y);
        }
    }
    return hipGetLastError();
}

template <int P, bool STIFF, typename CS>
static hipError_t launch_apply_batch_t(const TaskList &tl, int nblocks, hipStream_t s)
{
    const size_t lds = apply3d_lds<P, STIFF, CS>();
    hipError_t e = allow_dynamic_lds((const void *)apply3d_persistent<P, STIFF, CS>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((apply3d_persistent<P, STIFF, CS>), dim3(nblocks), dim3(STile<P>::NT), lds, s, tl);
    return hipGetLastError();
}

template <int P, bool STIFF>
static hipError_t launch_apply_batch_o(const TaskList &tl, Prec prec, int nblocks, hipStream_t s)
{
    if (prec == Prec::F64) return launch_apply_batch_t<P, STIFF, double>(tl, nblocks, s);
    if (prec == Prec::F16S) return launch_apply_batch_t<P, STIFF, __half>(tl, nblocks, s);
    return launch_apply_batch_t<P, STIFF, float>(tl, nblocks, s);
}

template <int P>
static hipError_t launch_apply_batch_p(const TaskList &tl, int op, Prec prec, int nblocks, hipStream_t s)
{
    return op == 2 ? launch_apply_batch_o<P, true>(tl, prec, nblocks, s)
                   : launch_apply_batch_o<P, false>(tl, prec, nblocks, s);
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

template <int P, bool STIFF>
static hipError_t launch_apply_o(const PatchView &pv, Prec prec, const void *C, const float *rs, const double *x,
                                 double *y, hipStream_t s, int lz, bool tiled)
{
    if (prec == Prec::F64) return launch_apply_t<P, STIFF, double>(pv, (const double *)C, rs, x, y, s, lz, tiled);
    if (prec == Prec::F16S) return launch_apply_t<P, STIFF, __half>(pv, (const __half *)C, rs, x, y, s, lz, tiled);
    return launch_apply_t<P, STIFF, float>(pv, (const float *)C, rs, x, y, s, lz, tiled);
}

template <int P>
static hipError_t launch_apply_p(const PatchView &pv, int op, Prec prec, const void *C, const float *rs,
                                 const double *x, double *y, hipStream_t s, int lz, bool tiled)
{
    return op == 2 ? launch_apply_o<P, true>(pv, prec, C, rs, x, y, s, lz, tiled)
                   : launch_apply_o<P, false>(pv, prec, C, rs, x, y, s, lz, tiled);
}

hipError_t launch_apply(const PatchView &pv, int op, Prec prec, const void *C, const double *x, double *y,
                        hipStream_t s, int lz, const float *rs, bool tiled)
{
    hipError_t e = launch_fill(y, pv.N, 0.0, s);
    if (e != hipSuccess) return e;
    switch (pv.P) {
    case 2: return launch_apply_p<2>(pv, op, prec, C, rs, x, y, s, lz, tiled);
    case 3: return launch_apply_p<3>(pv, op, prec, C, rs, x, y, s, lz, tiled);
    case 4: return launch_apply_p<4>(pv, op, prec, C, rs, x, y, s, lz, tiled);
    case 5: return launch_apply_p<5>(pv, op, prec, C, rs, x, y, s, lz, tiled);
    case 6: return launch_apply_p<6>(pv, op, prec, C, rs, x, y, s, lz, tiled);
    case 7: return launch_apply_p<7>(pv, op, prec, C, rs, x, y, s, lz, tiled);
    case 8: return launch_apply_p<8>(pv, op, prec, C, rs, x, y, s, lz, tiled);
    case 9: return launch_apply_p<9>(pv, op, prec, C, rs, x, y, s, lz, tiled);
    default: return hipErrorInvalidValue;
    }
}

bool apply_tiled_layout(int P, int op, Prec prec)
{
    if (P < 2 || P > kMaxOrder || prec == Prec::F16S || prec == Prec::BF16X3) return false;
    const ApplyShape sh = apply_shape(P, prec == Prec::F64 ? 0 : 1, op == 2);
    return sh.ROWS != 0 && sh.ALAY != 0;
}

}  // namespace sfiga
