// Global sum-factorized assembly (Sec. 3, Algorithm 1), d = 3, FP64, with
// every level as a small dense product on the FP64 matrix cores
// (v_mfma_f64_16x16x4).  Same ownership as the vector kernel: a workgroup
// owns rows m1 (one), m2 in [a2, a2+B2), m3 in [a3, a3+L) with all their
// columns, so each CSR value is written exactly once, without atomics.
//
// For each quadrature plane x3 of the elements that touch those rows:
//   level 1  A1[x2][(i,j)][n1] = sum_{x1 in supp m1} T1[(i,j),n1][x1] C_ij[x1][x2]
//            (rows: the pairs sharing a coefficient component x band offset,
//            inner dimension: the p^2 points of supp m1, columns: x2);
//   level 2  element by element along direction 2: the element matrix
//            T2^e[(m2,n2)][g2] (p^2 x p) times A1[(e,g2)][(pair, n1)];
//   level 3  element by element along direction 3: T3^e[(m3,n3)][group]
//            (p^2 x 4 groups BB BD DB DD, Sec. 3.1 splitting) times the
//            pair sums of A2 for one quadrature plane.
// Levels 2 and 3 accumulate the element matrices of consecutive elements in
// the matrix-core accumulators: row (m, n) of the element product lives in
// "slot" (m mod p, n mod p), which keeps its index while consecutive
// elements add to the same (m, n).  When element e starts, the slots of
// row e-1 and of column e-1 change owner: their sums are complete and are
// written out (level 2 into LDS, level 3 into the CSR values) and reset.
#include "kernels.h"

namespace sfiga {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int P> struct MCfg;                  // rows m2 per workgroup, threads
template <> struct MCfg<2> { static constexpr int B2 = 16, NT = 512; };
template <> struct MCfg<3> { static constexpr int B2 = 12, NT = 512; };
template <> struct MCfg<4> { static constexpr int B2 = 8, NT = 512; };
template <> struct MCfg<5> { static constexpr int B2 = 4, NT = 512; };
template <> struct MCfg<6> { static constexpr int B2 = 4, NT = 512; };

constexpr int ceil16(int x) { return (x + 15) / 16; }
constexpr int cmaxi(int a, int b) { return a > b ? a : b; }

template <int P, bool STIFF>
struct MShape {
    static constexpr int W = 2 * P - 1;
    static constexpr int NP = STIFF ? 9 : 1;          // (i, j) pairs, pid = 3 i + j
    static constexpr int NCOMP = STIFF ? 6 : 1;
    static constexpr int X1 = P * P;
    static constexpr int B2 = MCfg<P>::B2;
    static constexpr int NT = MCfg<P>::NT;
    static constexpr int NW = NT / 64;
    static constexpr int LSEG = 16;
    static constexpr int X2 = (B2 + P - 1) * P;
    static constexpr int X2P = X2 | 1;
    static constexpr int NSLOT = P * P;                // (m mod p, n mod p)
    static constexpr int MTS = ceil16(NSLOT);          // accumulator tiles over slots
    static constexpr int KS1 = (X1 + 3) / 4;           // level-1 k steps
    static constexpr int NT1 = ceil16(X2);             // level-1 column tiles
    static constexpr int KS2 = (P + 3) / 4;            // level-2 k steps
    static constexpr int NENT = B2 * W * W;            // level-3 columns (m2, n2, n1)
    static constexpr int NT3 = ceil16(NENT);
    static constexpr int T3PW = (NT3 + NW - 1) / NW;   // level-3 tiles per wave
    static constexpr int NSLICE = NCOMP * X2 * X1;
    static constexpr int PF = (NSLICE + NT - 1) / NT;
    static constexpr int REGION0 = cmaxi(NCOMP * X1 * X2P, B2 * W * NP * W);
    static constexpr int REGION1 = X2 * NP * W;
    static constexpr int TAB = 2 * P * P * P + 2 * (B2 + P - 1) * P * P + 2 * (LSEG + P - 1) * P * P;
    static constexpr int LDS_DOUBLES = REGION0 + REGION1 + TAB;
};

// pairs sharing coefficient component c (order 00 11 22 01 02 12)
__device__ __forceinline__ int comp_npairs(int c) { return c < 3 ? 1 : 2; }
__device__ __forceinline__ int comp_pair(int c, int q)
{
    switch (c) {
    case 0: return 0;
    case 1: return 4;
    case 2: return 8;
    case 3: return q ? 3 : 1;
    case 4: return q ? 6 : 2;
    default: return q ? 7 : 5;
    }
}
// level-2 column groups by the direction-2 table types: BB, DB, BD, DD
__device__ __forceinline__ int g2_npairs(int g) { return g == 0 ? 4 : (g == 3 ? 1 : 2); }
__device__ __forceinline__ int g2_pair(int g, int q)
{
    switch (g) {
    case 0: return q == 0 ? 0 : (q == 1 ? 2 : (q == 2 ? 6 : 8));
    case 1: return q ? 5 : 3;
    case 2: return q ? 7 : 1;
    default: return 4;
    }
}
__device__ __forceinline__ int pmod(int a, int p) { int r = a % p; return r < 0 ? r + p : r; }

template <int P, bool STIFF>
__global__ __launch_bounds__(MCfg<P>::NT) void asm3d_mfma_kernel(PatchView pv, const double *__restrict__ C,
                                                                 double *__restrict__ vals)
{
    using S = MShape<P, STIFF>;
    constexpr int W = S::W, NP = S::NP, NCOMP = S::NCOMP, X1 = S::X1, B2 = S::B2, NT = S::NT, NW = S::NW;
    constexpr int X2 = S::X2, X2P = S::X2P, L = S::LSEG, PP = P * P;
    extern __shared__ __align__(16) double smem[];
    double *cs = smem;                       // [NCOMP][X1][X2P] coefficient slice; later A2 [B2][W][NP][W]
    double *a2s = smem;
    double *a1s = smem + S::REGION0;         // [X2][NP][W]
    double *t1B = a1s + S::REGION1, *t1D = t1B + P * PP;              // [le1][g][j]
    double *t2B = t1D + P * PP, *t2D = t2B + (B2 + P - 1) * PP;       // [le2][g][j]
    double *t3B = t2D + (B2 + P - 1) * PP, *t3D = t3B + (L + P - 1) * PP;

    const Dir &d0 = pv.dir[0], &d1 = pv.dir[1], &d2 = pv.dir[2];
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int li = lane % 16, lk = lane / 16;          // matrix-core operand row/column and k index
    const int m1 = blockIdx.x, a2 = blockIdx.y * B2, a3 = blockIdx.z * L;
    const int e2s = a2 - P + 1 > 0 ? a2 - P + 1 : 0;
    const int e2e = (a2 + B2 - 1 < d1.K - 1) ? a2 + B2 - 1 : d1.K - 1;
    const int e3s = a3 - P + 1 > 0 ? a3 - P + 1 : 0;
    const int e3e = (a3 + L - 1 < d2.K - 1) ? a3 + L - 1 : d2.K - 1;
    const int Q0 = d0.Q, Q1 = d1.Q;
    const int q0base = (m1 - P + 1) * P, q1base = (a2 - P + 1) * P;
    const int e2base = a2 - P + 1;                    // element of local x2 block 0

    // ---- tables of the workgroup's elements, zero outside the mesh; clear A2
    {
        const int e1b = m1 - P + 1;
        for (int i = tid; i < P * PP; i += NT) {
            const int e = e1b + i / PP;
            const bool ok = e >= 0 && e < d0.K;
            const int64_t src = (int64_t)(ok ? e : 0) * PP + i % PP;   // in-bounds address on every lane
            t1B[i] = ok ? d0.B[src] : 0.0;
            t1D[i] = ok ? d0.D[src] : 0.0;
        }
        for (int i = tid; i < (B2 + P - 1) * PP; i += NT) {
            const int e = e2base + i / PP;
            const bool ok = e >= 0 && e < d1.K;
            const int64_t src = (int64_t)(ok ? e : 0) * PP + i % PP;
            t2B[i] = ok ? d1.B[src] : 0.0;
            t2D[i] = ok ? d1.D[src] : 0.0;
        }
        for (int i = tid; i < (L + P - 1) * PP; i += NT) {
            const int e = e3s + i / PP;
            const bool ok = e <= e3e;
            const int64_t src = (int64_t)(ok ? e : 0) * PP + i % PP;
            t3B[i] = ok ? d2.B[src] : 0.0;
            t3D[i] = ok ? d2.D[src] : 0.0;
        }
    }

    // ---- coefficient slice of one plane q3 (global order comp, lx2, lx1 fastest)
    const int64_t plane = (int64_t)NCOMP * Q1 * Q0;
    double pf[S::PF];
    auto load_slice = [&](int q2) {
        const double *base = C + (int64_t)q2 * plane;
#pragma unroll
        for (int k = 0; k < S::PF; ++k) {
            const int idx = tid + k * NT;
            const int lx1 = idx % X1, r = idx / X1;
            const int lx2 = r % X2, comp = r / X2;
            const int q0 = q0base + lx1, q1 = q1base + lx2;
            const bool ok = idx < S::NSLICE && q0 >= 0 && q0 < Q0 && q1 >= 0 && q1 < Q1;
            const double v = base[ok ? (comp * Q1 + q1) * Q0 + q0 : 0];
            pf[k] = ok ? v : 0.0;
        }
    };
    auto store_slice = [&]() {
#pragma unroll
        for (int k = 0; k < S::PF; ++k) {
            const int idx = tid + k * NT;
            const int lx1 = idx % X1, r = idx / X1;
            const int lx2 = r % X2, comp = r / X2;
            if (idx < S::NSLICE) cs[(comp * X1 + lx1) * X2P + lx2] = pf[k];
        }
    };

    // ---- level-3 accumulators: tiles wave, wave + NW, ... of the (m2, n2, n1) columns
    d4 acc3[S::T3PW][S::MTS];
#pragma unroll
    for (int t = 0; t < S::T3PW; ++t)
#pragma unroll
        for (int mt = 0; mt < S::MTS; ++mt) acc3[t][mt] = d4{0.0, 0.0, 0.0, 0.0};

    // write (level 3) the complete slots of the tile accumulators: rows m3 and
    // columns n3 they held for element `eo`; all = every slot, else only the
    // slots whose row or column is eo
    auto flush3 = [&](int eo, bool all) {
        const int so = pmod(eo, P);
#pragma unroll
        for (int t = 0; t < S::T3PW; ++t) {
            const int col = (wave + t * NW) * 16 + li;
            if (col >= S::NENT) continue;
            const int c1 = col % W, c2 = (col / W) % W, lm2 = col / (W * W);
            const int m2 = a2 + lm2, n1 = m1 + c1 - P + 1, n2 = m2 + c2 - P + 1;
            const bool ent_ok = m2 < d1.N && n1 >= 0 && n1 < d0.N && n2 >= 0 && n2 < d1.N;
#pragma unroll
            for (int mt = 0; mt < S::MTS; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int slot = mt * 16 + lk + 4 * v;
                    if (slot >= S::NSLOT) continue;
                    const int rho = slot / P, sig = slot % P;
                    if (!all && rho != so && sig != so) continue;
                    const int m3 = eo + pmod(rho - eo, P), n3 = eo + pmod(sig - eo, P);
                    if (ent_ok && m3 >= a3 && m3 < a3 + L && m3 < d2.N) {
                        const int64_t off = row_start(pv.ri, m1, m2, m3) + col_offset(pv.ri, m1, m2, m3, n1, n2, n3);
                        vals[off] = acc3[t][mt][v];
                    }
                    acc3[t][mt][v] = 0.0;
                }
        }
    };

    for (int i = tid; i < B2 * W * NP * W; i += NT) a2s[i] = 0.0;
    __syncthreads();
    load_slice(e3s * P);
    store_slice();
    __syncthreads();

    for (int e3 = e3s; e3 <= e3e; ++e3) {
        if (e3 > e3s) flush3(e3 - 1, false);
        for (int g3 = 0; g3 < P; ++g3) {
            // ================= level 1: items (comp, mt, nt), rows (pair q, n1 offset)
            {
                constexpr int MT1 = ceil16(2 * W);
                constexpr int NITEM = NCOMP * MT1 * S::NT1;
                for (int it = wave; it < NITEM; it += NW) {
                    const int nt = it % S::NT1, mt = (it / S::NT1) % MT1, c = it / (S::NT1 * MT1);
                    const int np = STIFF ? comp_npairs(c) : 1;
                    if (mt * 16 >= np * W) continue;
                    // A operand: row li of tile mt, the k-th point of supp m1
                    const int r = mt * 16 + li;
                    const int q = r / W, c1 = r % W;
                    const int pid = STIFF ? comp_pair(c, q < np ? q : 0) : 0;
                    const int pi = pid / 3, pj = pid % 3;
                    const int x2 = nt * 16 + li;
                    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int ks = 0; ks < S::KS1; ++ks) {
                        const int k = ks * 4 + lk;
                        const int rr = k / P, g1 = k % P, le1 = P - 1 - rr, s = c1 - P + 1 + rr;
                        double a = 0.0, b = 0.0;
                        if (k < X1 && q < np && s >= 0 && s < P) {
                            const int tb = (le1 * P + g1) * P;
                            const double ta = (STIFF && pi == 0) ? t1D[tb + rr] : t1B[tb + rr];
                            const double tt = (STIFF && pj == 0) ? t1D[tb + s] : t1B[tb + s];
                            a = ta * tt;
                        }
                        if (k < X1 && x2 < X2) b = cs[(c * X1 + le1 * P + g1) * X2P + x2];
                        acc = mfma_f64(a, b, acc);
                    }
                    // D: row lk + 4 v of the tile, column li
                    const int xo = nt * 16 + li;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int ro = mt * 16 + lk + 4 * v;
                        const int qo = ro / W, co = ro % W;
                        if (qo < np && xo < X2) {
                            const int po = STIFF ? comp_pair(c, qo) : 0;
                            a1s[(xo * NP + po) * W + co] = acc[v];
                        }
                    }
                }
            }
            __syncthreads();
            const bool more = (g3 + 1 < P) || (e3 < e3e);
            if (more) load_slice(g3 + 1 < P ? e3 * P + g3 + 1 : (e3 + 1) * P);

            // ================= level 2: items (group, nt, mt), element sweep along direction 2
            {
                constexpr int NG = STIFF ? 4 : 1;
                int nitem = 0;
#pragma unroll
                for (int g = 0; g < NG; ++g) nitem += ceil16((STIFF ? g2_npairs(g) : 1) * W) * S::MTS;
                for (int it = wave; it < nitem; it += NW) {
                    // decode item -> (group, column tile, slot tile)
                    int g = 0, rem = it;
                    while (g + 1 < NG && rem >= ceil16((STIFF ? g2_npairs(g) : 1) * W) * S::MTS) {
                        rem -= ceil16((STIFF ? g2_npairs(g) : 1) * W) * S::MTS;
                        ++g;
                    }
                    const int mt = rem % S::MTS, nt = rem / S::MTS;
                    const int np = STIFF ? g2_npairs(g) : 1;
                    const bool ti = STIFF && (g == 1 || g == 3);   // test side D2
                    const bool tj = STIFF && (g == 2 || g == 3);   // trial side D2
                    // B operand column: (pair q, n1 offset)
                    const int colb = nt * 16 + li;
                    const int qb = colb / W, c1b = colb % W;
                    const bool colb_ok = qb < np;
                    const int pidb = STIFF ? g2_pair(g, colb_ok ? qb : 0) : 0;
                    // output columns of this lane's accumulator: same li
                    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
                    for (int e2 = e2s; e2 <= e2e; ++e2) {
                        if (e2 > e2s) {
                            // flush the slots of row / column e2-1
                            const int eo = e2 - 1, so = pmod(eo, P);
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                const int slot = mt * 16 + lk + 4 * v;
                                if (slot >= S::NSLOT) continue;
                                const int rho = slot / P, sig = slot % P;
                                if (rho != so && sig != so) continue;
                                const int m2 = eo + pmod(rho - eo, P), n2 = eo + pmod(sig - eo, P);
                                const int lm2 = m2 - a2;
                                if (colb_ok && lm2 >= 0 && lm2 < B2)
                                    a2s[((lm2 * W + (n2 - m2 + P - 1)) * NP + pidb) * W + c1b] = acc[v];
                                acc[v] = 0.0;
                            }
                        }
                        const int le2 = e2 - e2base;
                        // A operand row li: slot -> (r2, s2) of element e2
                        const int slot_a = mt * 16 + li;
                        const int rho = slot_a / P, sig = slot_a % P;
                        const int r2 = pmod(rho - e2, P), s2 = pmod(sig - e2, P);
#pragma unroll
                        for (int ks = 0; ks < S::KS2; ++ks) {
                            const int g2 = ks * 4 + lk;
                            double a = 0.0, b = 0.0;
                            if (g2 < P && slot_a < S::NSLOT) {
                                const int tb = (le2 * P + g2) * P;
                                a = (ti ? t2D[tb + r2] : t2B[tb + r2]) * (tj ? t2D[tb + s2] : t2B[tb + s2]);
                            }
                            if (g2 < P && colb_ok) b = a1s[((le2 * P + g2) * NP + pidb) * W + c1b];
                            acc = mfma_f64(a, b, acc);
                        }
                    }
                    {
                        // all slots hold complete sums for element e2e
                        const int eo = e2e;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int slot = mt * 16 + lk + 4 * v;
                            if (slot >= S::NSLOT) continue;
                            const int rho = slot / P, sig = slot % P;
                            const int m2 = eo + pmod(rho - eo, P), n2 = eo + pmod(sig - eo, P);
                            const int lm2 = m2 - a2;
                            if (colb_ok && lm2 >= 0 && lm2 < B2)
                                a2s[((lm2 * W + (n2 - m2 + P - 1)) * NP + pidb) * W + c1b] = acc[v];
                        }
                    }
                }
            }
            __syncthreads();

            // ================= level 3: one k step over the 4 groups BB BD DB DD
            {
                const int le3 = e3 - e3s;
                const int tb3 = (le3 * P + g3) * P;
#pragma unroll
                for (int t = 0; t < S::T3PW; ++t) {
                    const int col = (wave + t * NW) * 16 + li;
                    // B operand: group lk of column col
                    double b = 0.0;
                    if (col < S::NENT) {
                        const int c1 = col % W, c2 = (col / W) % W, lm2 = col / (W * W);
                        const double *ap = a2s + ((lm2 * W + c2) * NP) * W + c1;
                        if (STIFF) {
                            if (lk == 0) b = ap[0 * W] + ap[1 * W] + ap[3 * W] + ap[4 * W];
                            else if (lk == 1) b = ap[2 * W] + ap[5 * W];
                            else if (lk == 2) b = ap[6 * W] + ap[7 * W];
                            else b = ap[8 * W];
                        } else {
                            b = lk == 0 ? ap[0] : 0.0;
                        }
                    }
                    if ((wave + t * NW) * 16 >= S::NENT) continue;
#pragma unroll
                    for (int mt = 0; mt < S::MTS; ++mt) {
                        const int slot_a = mt * 16 + li;
                        double a = 0.0;
                        if (slot_a < S::NSLOT && (STIFF || lk == 0)) {
                            const int rho = slot_a / P, sig = slot_a % P;
                            const int r3 = pmod(rho - e3, P), s3 = pmod(sig - e3, P);
                            const bool ti = STIFF && (lk == 2 || lk == 3);   // test side D3
                            const bool tj = STIFF && (lk == 1 || lk == 3);   // trial side D3
                            a = (ti ? t3D[tb3 + r3] : t3B[tb3 + r3]) * (tj ? t3D[tb3 + s3] : t3B[tb3 + s3]);
                        }
                        acc3[t][mt] = mfma_f64(a, b, acc3[t][mt]);
                    }
                }
            }
            __syncthreads();
            if (more) {
                store_slice();
                __syncthreads();
            }
        }
    }
    flush3(e3e, true);
}

template <int P, bool STIFF>
static hipError_t launch_mfma_t(const PatchView &pv, const double *C, double *vals, hipStream_t s)
{
    using S = MShape<P, STIFF>;
    const size_t lds = sizeof(double) * (size_t)S::LDS_DOUBLES;
    static size_t lds_set = 0;
    if (lds > lds_set) {
        hipError_t e = hipFuncSetAttribute((const void *)asm3d_mfma_kernel<P, STIFF>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_set = lds;
    }
    dim3 grid(pv.dir[0].N, (pv.dir[1].N + S::B2 - 1) / S::B2, (pv.dir[2].N + S::LSEG - 1) / S::LSEG);
    hipLaunchKernelGGL((asm3d_mfma_kernel<P, STIFF>), grid, dim3(S::NT), lds, s, pv, C, vals);
    return hipGetLastError();
}

hipError_t launch_assemble_mfma(const PatchView &pv, int op, const double *C, double *vals, hipStream_t s)
{
    const bool st = op == 2;
    switch (pv.P) {
    case 2: return st ? launch_mfma_t<2, true>(pv, C, vals, s) : launch_mfma_t<2, false>(pv, C, vals, s);
    case 3: return st ? launch_mfma_t<3, true>(pv, C, vals, s) : launch_mfma_t<3, false>(pv, C, vals, s);
    case 4: return st ? launch_mfma_t<4, true>(pv, C, vals, s) : launch_mfma_t<4, false>(pv, C, vals, s);
    case 5: return st ? launch_mfma_t<5, true>(pv, C, vals, s) : launch_mfma_t<5, false>(pv, C, vals, s);
    case 6: return st ? launch_mfma_t<6, true>(pv, C, vals, s) : launch_mfma_t<6, false>(pv, C, vals, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sfiga
