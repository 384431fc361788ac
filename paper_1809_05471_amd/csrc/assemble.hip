// Global sum-factorized assembly (Sec. 3, Algorithm 1) into the structural
// CSR layout.
//
// The matrix of a (test dir i, trial dir j) pair of eq. (A-sum) is
//   A_ij[m][n] = sum_{x3} T3(m3,n3,x3) sum_{x2} T2(m2,n2,x2) sum_{x1} T1(m1,n1,x1) C_ij(x)
// with T_k(m,n,x) = a_k(m,x) b_k(n,x), a_k = D_k if i == k else B_k (test
// side), b_k = D_k if j == k else B_k (trial side); the weights are folded
// into C.  Level k of Algorithm 1 is the sum over x_k; its cost is
// p_k q_k (prod_{l>=k} #X_l) nnz(A^{k-1}) (eq. (sum factorization-nnz)).
//
// d = 3 kernel ("owner computes", deterministic, no atomics): a workgroup
// owns the rows m1 (one), m2 in [a2, a2+B2) and m3 in [a3, a3+L) with all
// their columns.  It walks the elements e3 that touch those rows in order;
// for every quadrature plane x3 it
//   1. stages the coefficient slice C(x1, x2, x3) for the x1 in the support
//      of m1 and the x2 of the box's support (prefetched into registers
//      during the previous plane),
//   2. level 1: A1[x2][(i,j)][n1] for the fixed m1,
//   3. level 2: A2[m2][n2][(i,j)][n1] for the box's rows m2,
//   4. level 3: pairs with equal direction-3 tables are summed (4 groups for
//      the stiffness: BB, BD, DB, DD; Sec. 3.1 splitting) and folded into a
//      sliding window of the p rows m3 = e3 .. e3+p-1 held in FP64 registers
//      (one thread per (m2, n2, n1) entry).
// Row m3 = e3 is complete after element e3 and is written straight into
// its CSR slots.  Rows below a3 in the first window are discarded, so each
// value is written exactly once.  Redundant work: level 1 over the x2 halo
// ((B2+p-1)/B2) and levels 1-2 over the x3 halo ((L+p-1)/L).
#include "kernels.h"

#include <cstdlib>

namespace sfiga {

template <int P> struct AsmCfg;                 // rows per workgroup in direction 2, max threads
template <> struct AsmCfg<2> { static constexpr int B2 = 16, MAXT = 1024; };
template <> struct AsmCfg<3> { static constexpr int B2 = 16, MAXT = 1024; };
template <> struct AsmCfg<4> { static constexpr int B2 = 8, MAXT = 512; };
template <> struct AsmCfg<5> { static constexpr int B2 = 4, MAXT = 512; };
template <> struct AsmCfg<6> { static constexpr int B2 = 4, MAXT = 512; };

constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <int P, bool STIFF>
struct AsmShape {
    static constexpr int W = 2 * P - 1;          // band width per direction
    static constexpr int NP = STIFF ? 9 : 1;     // (i, j) pairs
    static constexpr int NI = STIFF ? 3 : 1;     // test derivative directions
    static constexpr int NCOMP = STIFF ? 6 : 1;  // symmetric coefficient components
    static constexpr int X1 = P * P;             // x1 points in the support of one m1
    static constexpr int B2 = AsmCfg<P>::B2;     // rows m2 per workgroup
    static constexpr int X2 = (B2 + P - 1) * P;  // x2 points in the support of the rows
    static constexpr int X2P = X2 | 1;           // odd LDS stride
    static constexpr int WPM = (NP * W + 63) / 64;                 // waves per m2 row, level 2
    static constexpr int NT = (cmax(cmax(NP * X2, B2 * WPM * 64), B2 * W * W) + 63) / 64 * 64;
    static constexpr int NSLICE = NCOMP * X2 * X1;                 // coefficient slice per plane
    static constexpr int PF = (NSLICE + NT - 1) / NT;              // slice values per thread
    static constexpr int LSEG = 16;              // rows m3 per workgroup (streamed)
    static constexpr int REGION0 = cmax(NCOMP * X1 * X2P, NP * B2 * W * W);
    static constexpr int REGION1 = X2 * NP * W;
    // 1D tables of the workgroup's elements (B and D), staged once:
    // direction 1: the p elements of supp(m1); direction 2: the B2+p-1
    // elements of the rows' support; direction 3: the LSEG+p-1 elements walked
    static constexpr int T1 = 2 * P * P * P;
    static constexpr int T2 = 2 * (B2 + P - 1) * P * P;
    static constexpr int T3 = 2 * (LSEG + P - 1) * P * P;
    static_assert(NT <= AsmCfg<P>::MAXT, "thread count");
};

// LDS bytes of one workgroup: the coefficient/A2 region and A1 in the
// contraction type, the tables in double (8-byte aligned after the CT part)
template <int P, bool STIFF, typename CT>
constexpr size_t asm_lds_bytes()
{
    using S = AsmShape<P, STIFF>;
    size_t a = sizeof(CT) * (size_t)(S::REGION0 + S::REGION1);
    a = (a + 15) / 16 * 16;
    return a + sizeof(double) * (size_t)(S::T1 + S::T2 + S::T3);
}

// symmetric component of pair (i, j) in the order 00 11 22 01 02 12
__device__ __forceinline__ int comp3(int i, int j)
{
    if (i == j) return i;
    int a = i < j ? i : j, b = i < j ? j : i;
    return a == 0 ? (b == 1 ? 3 : 4) : 5;
}

template <int P, bool STIFF, typename CT>
__global__ __launch_bounds__((AsmShape<P, STIFF>::NT)) void asm3d_kernel(PatchView pv, const CT *__restrict__ C,
                                                                       double *__restrict__ vals)
{
    using S = AsmShape<P, STIFF>;
    constexpr int W = S::W, NP = S::NP, NI = S::NI, NCOMP = S::NCOMP, X1 = S::X1;
    constexpr int B2 = S::B2, X2 = S::X2, X2P = S::X2P, NT = S::NT, PF = S::PF, WPM = S::WPM;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    CT *cs = reinterpret_cast<CT *>(smem_raw);   // [NCOMP][X1][X2P]  (aliased by A2 [B2][W][NP][W])
    CT *a2s = cs;
    CT *a1s = cs + S::REGION0;                   // [X2][NP][W]
    constexpr int L = S::LSEG;
    double *tab = reinterpret_cast<double *>(smem_raw + (sizeof(CT) * (S::REGION0 + S::REGION1) + 15) / 16 * 16);
    double *t1B = tab, *t1D = t1B + P * P * P;                          // [le1][g][j]
    double *t2B = t1D + P * P * P, *t2D = t2B + (B2 + P - 1) * P * P;  // [le2][g][j]
    double *t3B = t2D + (B2 + P - 1) * P * P, *t3D = t3B + (L + P - 1) * P * P;

    const Dir &d0 = pv.dir[0], &d1 = pv.dir[1], &d2 = pv.dir[2];
    const int tid = threadIdx.x;
    const int m1 = blockIdx.x;
    const int a2 = blockIdx.y * B2;
    const int a3 = blockIdx.z * L;
    const int e3s = a3 - P + 1 > 0 ? a3 - P + 1 : 0;
    const int e3e = (a3 + L - 1 < d2.K - 1) ? a3 + L - 1 : d2.K - 1;
    const int Q0 = d0.Q, Q1 = d1.Q;
    const int q0base = (m1 - P + 1) * P;          // first x1 of the support of m1
    const int q1base = (a2 - P + 1) * P;          // first x2 of the box support

    // ---- coefficient slice of one plane of constant q3, global order (comp, lx2,
    //      lx1 fastest); this thread moves elements tid + k NT, k < PF
    const int64_t plane = (int64_t)NCOMP * Q1 * Q0;
    CT pf[PF];
    auto load_slice = [&](int q2) {
        const CT *base = C + (int64_t)q2 * plane;
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int idx = tid + k * NT;
            const int lx1 = idx % X1, r = idx / X1;
            const int lx2 = r % X2, comp = r / X2;
            const int q0 = q0base + lx1, q1 = q1base + lx2;
            const bool ok = idx < S::NSLICE && q0 >= 0 && q0 < Q0 && q1 >= 0 && q1 < Q1;
            const CT v = base[ok ? (comp * Q1 + q1) * Q0 + q0 : 0];   // in-bounds address on every lane
            pf[k] = ok ? v : CT(0);
        }
    };
    auto store_slice = [&]() {
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int idx = tid + k * NT;
            const int lx1 = idx % X1, r = idx / X1;
            const int lx2 = r % X2, comp = r / X2;
            if (idx < S::NSLICE) cs[(comp * X1 + lx1) * X2P + lx2] = pf[k];
        }
    };

    // ---- level-3 entry owned by this thread
    const int nent = B2 * W * W;
    const bool has_ent = tid < nent;
    const int ec1 = tid % W, ec2 = (tid / W) % W, elm2 = tid / (W * W);
    const int em2 = a2 + elm2;
    const int en1 = m1 + ec1 - P + 1, en2 = em2 + ec2 - P + 1;
    const bool ent_ok = has_ent && em2 < d1.N && en1 >= 0 && en1 < d0.N && en2 >= 0 && en2 < d1.N;
    double win[P][W];
#pragma unroll
    for (int r = 0; r < P; ++r)
#pragma unroll
        for (int c = 0; c < W; ++c) win[r][c] = 0.0;

    // ---- level-1 lane: (pair (i, j), lx2)
    const bool l1_ok = tid < NP * X2;
    const int l1_pair = tid / X2, l1_x2 = tid % X2;
    const int l1_i = STIFF ? l1_pair / 3 : 0, l1_j = STIFF ? l1_pair % 3 : 0;
    const int l1_comp = STIFF ? comp3(l1_i, l1_j) : 0;

    // ---- level-2 lane: wave -> m2, lane -> (pair, n1 offset)
    const int wv = tid / 64, ln = tid % 64;
    const int l2_lm2 = wv / WPM, l2_t = (wv % WPM) * 64 + ln;
    const int l2_m2 = a2 + l2_lm2;
    const bool l2_ok = l2_lm2 < B2 && l2_t < NP * W && l2_m2 < d1.N;
    const int l2_pair = l2_t / W, l2_c1 = l2_t % W;
    const int l2_i = STIFF ? l2_pair / 3 : 0, l2_j = STIFF ? l2_pair % 3 : 0;

    // stage the 1D tables of this workgroup's elements (zeros outside the mesh)
    {
        constexpr int PP = P * P;
        const int e1b = m1 - P + 1, e2b = a2 - P + 1;
        for (int i = tid; i < P * PP; i += NT) {
            const int le = i / PP, e = e1b + le;
            const bool ok = e >= 0 && e < d0.K;
            t1B[i] = ok ? d0.B[(int64_t)e * PP + i % PP] : 0.0;
            t1D[i] = ok ? d0.D[(int64_t)e * PP + i % PP] : 0.0;
        }
        for (int i = tid; i < (B2 + P - 1) * PP; i += NT) {
            const int le = i / PP, e = e2b + le;
            const bool ok = e >= 0 && e < d1.K;
            t2B[i] = ok ? d1.B[(int64_t)e * PP + i % PP] : 0.0;
            t2D[i] = ok ? d1.D[(int64_t)e * PP + i % PP] : 0.0;
        }
        for (int i = tid; i < (L + P - 1) * PP; i += NT) {
            const int le = i / PP, e = e3s + le;
            const bool ok = e <= e3e;
            t3B[i] = ok ? d2.B[(int64_t)e * PP + i % PP] : 0.0;
            t3D[i] = ok ? d2.D[(int64_t)e * PP + i % PP] : 0.0;
        }
    }
    load_slice(e3s * P);
    store_slice();
    __syncthreads();

    for (int e3 = e3s; e3 <= e3e; ++e3) {
        for (int g3 = 0; g3 < P; ++g3) {
            // ---------------- level 1: contract x1 for the fixed test row m1
            if (l1_ok) {
                CT acc[W];
#pragma unroll
                for (int c = 0; c < W; ++c) acc[c] = CT(0);
#pragma unroll
                for (int r = 0; r < P; ++r) {
                    const int e1 = m1 - r;
                    if (e1 < 0 || e1 >= d0.K) continue;
                    const int le1 = P - 1 - r;
#pragma unroll 2
                    for (int g1 = 0; g1 < P; ++g1) {
                        const double *tb = t1B + (le1 * P + g1) * P;
                        const double *td = t1D + (le1 * P + g1) * P;
                        const CT cv = cs[(l1_comp * X1 + le1 * P + g1) * X2P + l1_x2] *
                                      (CT)((STIFF && l1_i == 0) ? td[r] : tb[r]);
#pragma unroll
                        for (int s = 0; s < P; ++s)
                            acc[s - r + P - 1] += cv * (CT)((STIFF && l1_j == 0) ? td[s] : tb[s]);
                    }
                }
#pragma unroll
                for (int c = 0; c < W; ++c) a1s[(l1_x2 * NP + l1_pair) * W + c] = acc[c];
            }
            __syncthreads();
            // next plane's coefficient slice is fetched while levels 2 and 3 run
            const bool more = (g3 + 1 < P) || (e3 < e3e);
            if (more) load_slice(g3 + 1 < P ? e3 * P + g3 + 1 : (e3 + 1) * P);

            // ---------------- level 2: contract x2 for the box rows m2
            if (l2_ok) {
                CT acc[W];
#pragma unroll
                for (int c = 0; c < W; ++c) acc[c] = CT(0);
#pragma unroll
                for (int r = 0; r < P; ++r) {
                    const int e2 = l2_m2 - r;
                    if (e2 < 0 || e2 >= d1.K) continue;
                    const int lx2b = (l2_lm2 + P - 1 - r) * P;
#pragma unroll 2
                    for (int g2 = 0; g2 < P; ++g2) {
                        const double *tb = t2B + ((l2_lm2 + P - 1 - r) * P + g2) * P;
                        const double *td = t2D + ((l2_lm2 + P - 1 - r) * P + g2) * P;
                        const CT v = a1s[((lx2b + g2) * NP + l2_pair) * W + l2_c1];
                        const CT tv = (CT)(l2_i == 1 ? td[r] : tb[r]) * v;
#pragma unroll
                        for (int s = 0; s < P; ++s) acc[s - r + P - 1] += tv * (CT)(l2_j == 1 ? td[s] : tb[s]);
                    }
                }
#pragma unroll
                for (int c = 0; c < W; ++c) a2s[((l2_lm2 * W + c) * NP + l2_pair) * W + l2_c1] = acc[c];
            }
            __syncthreads();

            // ---------------- level 3: fold into the sliding window of rows m3
            if (has_ent) {
                const double *tb = t3B + ((e3 - e3s) * P + g3) * P;
                const double *td = t3D + ((e3 - e3s) * P + g3) * P;
                const CT *a2e = a2s + (elm2 * W + ec2) * NP * W + ec1;
                if constexpr (STIFF) {
                    const double gBB = (double)a2e[0 * W] + (double)a2e[1 * W] + (double)a2e[3 * W] + (double)a2e[4 * W];
                    const double gBD = (double)a2e[2 * W] + (double)a2e[5 * W];
                    const double gDB = (double)a2e[6 * W] + (double)a2e[7 * W];
                    const double gDD = (double)a2e[8 * W];
                    double uB[P], uD[P];
#pragma unroll
                    for (int s = 0; s < P; ++s) {
                        uB[s] = tb[s] * gBB + td[s] * gBD;
                        uD[s] = tb[s] * gDB + td[s] * gDD;
                    }
#pragma unroll
                    for (int r = 0; r < P; ++r)
#pragma unroll
                        for (int s = 0; s < P; ++s) win[r][s - r + P - 1] += tb[r] * uB[s] + td[r] * uD[s];
                } else {
                    const double gv = (double)a2e[0];
#pragma unroll
                    for (int r = 0; r < P; ++r)
#pragma unroll
                        for (int s = 0; s < P; ++s) win[r][s - r + P - 1] += tb[r] * tb[s] * gv;
                }
            }
            __syncthreads();
            if (more) {
                store_slice();
                __syncthreads();
            }
        }
        // ---------------- rows complete after element e3: write and slide
        const bool last = (e3 == d2.K - 1);
        if (ent_ok) {
#pragma unroll
            for (int r = 0; r < P; ++r) {
                if (r > 0 && !last) break;
                const int m3 = e3 + r;
                if (m3 < a3 || m3 >= a3 + L || m3 >= d2.N) continue;
                const int lo3 = band_lo(m3, P);
                const int64_t base = row_start(pv.ri, m1, em2, m3) + col_offset(pv.ri, m1, em2, m3, en1, en2, lo3);
                const int64_t stride3 = (int64_t)band_len(em2, P, d1.N) * band_len(m1, P, d0.N);
#pragma unroll
                for (int c = 0; c < W; ++c) {
                    const int n3 = m3 + c - P + 1;
                    if (n3 >= 0 && n3 < d2.N) vals[base + (int64_t)(n3 - lo3) * stride3] = win[r][c];
                }
            }
        }
        if (!last) {
#pragma unroll
            for (int r = 0; r + 1 < P; ++r)
#pragma unroll
                for (int c = 0; c < W; ++c) win[r][c] = win[r + 1][c];
#pragma unroll
            for (int c = 0; c < W; ++c) win[P - 1][c] = 0.0;
        }
    }
}

// ------------------------------------------------------------------ d <= 2
// One thread per (row m, direction-2 band offset): the row's level-1 sums
// are formed once per x2 and reused for every direction-1 column.
template <int DIM, int P, bool STIFF, typename CT>
__global__ void asm_small_kernel(PatchView pv, const CT *__restrict__ C, double *__restrict__ vals)
{
    constexpr int W = 2 * P - 1;
    constexpr int NCOMP = STIFF ? DIM * (DIM + 1) / 2 : 1;
    constexpr int NPAIR = STIFF ? DIM * DIM : 1;
    constexpr int NB = DIM == 2 ? W : 1;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const Dir &d0 = pv.dir[0], &d1 = pv.dir[1];
    if (t >= pv.N * NB) return;
    const int64_t m = t / NB;
    const int cb = (int)(t % NB);
    const int m0 = (int)(m % d0.N), m1 = DIM == 2 ? (int)(m / d0.N) : 0;
    const int n1 = DIM == 2 ? m1 + cb - P + 1 : 0;
    if (DIM == 2 && (n1 < 0 || n1 >= d1.N)) return;
    double acc[W];
    for (int c = 0; c < W; ++c) acc[c] = 0.0;
    // direction-2 elements common to m1 and n1 (one pass with no direction 2 for DIM == 1)
    int elo = 0, ehi = 0;
    if (DIM == 2) {
        elo = (m1 > n1 ? m1 : n1) - P + 1;
        if (elo < 0) elo = 0;
        ehi = m1 < n1 ? m1 : n1;
        if (ehi > d1.K - 1) ehi = d1.K - 1;
    }
    for (int e1 = elo; e1 <= ehi; ++e1) {
        for (int g1 = 0; g1 < (DIM == 2 ? P : 1); ++g1) {
            const int q1 = e1 * P + g1;
            // level 1 at this x2 for every pair and direction-1 column
            double L1[NPAIR][W];
            for (int a = 0; a < NPAIR; ++a)
                for (int c = 0; c < W; ++c) L1[a][c] = 0.0;
            for (int r0 = 0; r0 < P; ++r0) {
                const int e0 = m0 - r0;
                if (e0 < 0 || e0 >= d0.K) continue;
                for (int g0 = 0; g0 < P; ++g0) {
                    const int q0 = e0 * P + g0;
                    const double *b = d0.B + ((int64_t)e0 * P + g0) * P, *db = d0.D + ((int64_t)e0 * P + g0) * P;
                    double cv[NCOMP];
                    for (int k = 0; k < NCOMP; ++k) cv[k] = (double)C[coef_index(DIM, NCOMP, k, q0, q1, 0, d0.Q, d1.Q)];
                    for (int s0 = 0; s0 < P; ++s0) {
                        const int c = s0 - r0 + P - 1;
                        if (!STIFF) {
                            L1[0][c] += b[r0] * b[s0] * cv[0];
                        } else {
                            for (int i = 0; i < DIM; ++i)
                                for (int j = 0; j < DIM; ++j) {
                                    double ta = (i == 0) ? db[r0] : b[r0];
                                    double tb = (j == 0) ? db[s0] : b[s0];
                                    L1[i * DIM + j][c] += ta * tb * cv[sym_comp<DIM>(i, j)];
                                }
                        }
                    }
                }
            }
            if (DIM == 1) {
                for (int a = 0; a < NPAIR; ++a)
                    for (int c = 0; c < W; ++c) acc[c] += L1[a][c];
            } else {
                const double *b = d1.B + ((int64_t)e1 * P + g1) * P, *db = d1.D + ((int64_t)e1 * P + g1) * P;
                const int r1 = m1 - e1, s1 = n1 - e1;
                for (int i = 0; i < (STIFF ? DIM : 1); ++i)
                    for (int j = 0; j < (STIFF ? DIM : 1); ++j) {
                        double ta = (STIFF && i == 1) ? db[r1] : b[r1];
                        double tb = (STIFF && j == 1) ? db[s1] : b[s1];
                        for (int c = 0; c < W; ++c) acc[c] += ta * tb * L1[STIFF ? i * DIM + j : 0][c];
                    }
            }
        }
    }
    const int64_t base = row_start(pv.ri, m0, m1, 0);
    for (int c = 0; c < W; ++c) {
        const int n0 = m0 + c - P + 1;
        if (n0 < 0 || n0 >= d0.N) continue;
        vals[base + col_offset(pv.ri, m0, m1, 0, n0, n1, 0)] = acc[c];
    }
}

// ------------------------------------------------------------------ launch

template <int P, bool STIFF, typename CT>
static hipError_t launch_asm3d(const PatchView &pv, const CT *C, double *vals, hipStream_t s)
{
    using S = AsmShape<P, STIFF>;
    constexpr int L = S::LSEG;
    const size_t lds = asm_lds_bytes<P, STIFF, CT>();
    static size_t lds_set = 0;     // per instantiation: raise the dynamic LDS limit once
    if (lds > lds_set) {
        hipError_t e = hipFuncSetAttribute((const void *)asm3d_kernel<P, STIFF, CT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_set = lds;
    }
    dim3 grid(pv.dir[0].N, (pv.dir[1].N + S::B2 - 1) / S::B2, (pv.dir[2].N + L - 1) / L);
    hipLaunchKernelGGL((asm3d_kernel<P, STIFF, CT>), grid, dim3(S::NT), lds, s, pv, C, vals);
    return hipGetLastError();
}

template <int P, bool STIFF, typename CT>
static hipError_t launch_asm_small(const PatchView &pv, const CT *C, double *vals, hipStream_t s)
{
    constexpr int W = 2 * P - 1;
    int64_t n = pv.N * (pv.d == 2 ? W : 1);
    int64_t nb = (n + 127) / 128;
    if (pv.d == 2)
        hipLaunchKernelGGL((asm_small_kernel<2, P, STIFF, CT>), dim3((unsigned)nb), dim3(128), 0, s, pv, C, vals);
    else
        hipLaunchKernelGGL((asm_small_kernel<1, P, STIFF, CT>), dim3((unsigned)nb), dim3(128), 0, s, pv, C, vals);
    return hipGetLastError();
}

template <int P>
static hipError_t launch_asm_p(const PatchView &pv, int op, Prec prec, const void *C, double *vals, hipStream_t s)
{
    if (pv.d == 3) {
        if constexpr (P <= 6) {
            if (prec == Prec::F64)
                return op == 2 ? launch_asm3d<P, true, double>(pv, (const double *)C, vals, s)
                               : launch_asm3d<P, false, double>(pv, (const double *)C, vals, s);
            return op == 2 ? launch_asm3d<P, true, float>(pv, (const float *)C, vals, s)
                           : launch_asm3d<P, false, float>(pv, (const float *)C, vals, s);
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (prec == Prec::F64)
        return op == 2 ? launch_asm_small<P, true, double>(pv, (const double *)C, vals, s)
                       : launch_asm_small<P, false, double>(pv, (const double *)C, vals, s);
    return op == 2 ? launch_asm_small<P, true, float>(pv, (const float *)C, vals, s)
                   : launch_asm_small<P, false, float>(pv, (const float *)C, vals, s);
}

bool assemble_supported(int d, int P)
{
    if (P < 2 || P > 9) return false;
    return d < 3 || P <= 6;
}

hipError_t launch_assemble(const PatchView &pv, int op, Prec prec, const void *C, double *vals, hipStream_t s)
{
    // FP64, d = 3: the matrix-core formulation is selectable for comparison
    // (SFIGA_ASSEMBLY_MFMA=1); the vector kernel is the faster one on this chip
    static const bool use_mfma = getenv("SFIGA_ASSEMBLY_MFMA") && getenv("SFIGA_ASSEMBLY_MFMA")[0] == '1';
    if (use_mfma && pv.d == 3 && prec == Prec::F64 && pv.P <= 6)
        return launch_assemble_mfma(pv, op, (const double *)C, vals, s);
    switch (pv.P) {
    case 2: return launch_asm_p<2>(pv, op, prec, C, vals, s);
    case 3: return launch_asm_p<3>(pv, op, prec, C, vals, s);
    case 4: return launch_asm_p<4>(pv, op, prec, C, vals, s);
    case 5: return launch_asm_p<5>(pv, op, prec, C, vals, s);
    case 6: return launch_asm_p<6>(pv, op, prec, C, vals, s);
    case 7: return launch_asm_p<7>(pv, op, prec, C, vals, s);
    case 8: return launch_asm_p<8>(pv, op, prec, C, vals, s);
    case 9: return launch_asm_p<9>(pv, op, prec, C, vals, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sfiga
