// Global sum-factorized assembly (Sec. 3, Algorithm 1) into the structural
// CSR layout.
//
// The matrix of a (test derivative i, trial derivative j) pair of eq. (A-sum) is
//   A_ij[m][n] = sum_{x3} T3(m3,n3,x3) sum_{x2} T2(m2,n2,x2) sum_{x1} T1(m1,n1,x1) C_ij(x)
// with T_k(m,n,x) = a_k(m,x) b_k(n,x), a_k = D_k if i == k else B_k (test
// side), b_k = D_k if j == k else B_k (trial side); the weights are folded
// into C.  Level k of Algorithm 1 is the sum over x_k; its cost is
// p_k q_k (prod_{l>=k} #X_l) nnz(A^{k-1}) (eq. (sum factorization-nnz)).
//
// d = 3 runs as two kernels over chunks of element layers in direction 3:
//
//  asm12_kernel (levels 1 and 2): a workgroup owns one quadrature plane x3
//    and a tile of T1 rows m1.  It walks the elements e2 of direction 2 in
//    order; per element it stages the coefficient slice (x1 support of the
//    tile x the p points of e2) and forms level 1 for the tile's rows and
//    the (i, j) pairs (vector ALU; (2, 1) equals (1, 2) at this level).
//    Level 2 then adds the element's p points x2: pairs that share their
//    direction-3 tables are summed here (Sec. 3.1 splitting: 4 groups BB,
//    BD, DB, DD for the stiffness).  In FP64 at p = 4 and 8 it runs on the
//    matrix cores (rows = slots (m2 mod p, n2 mod p), columns = (m1, n1),
//    K = (pair, x2)); in BF16 split on bf16 matrix cores with hi/lo operands;
//    in FP32, and in FP64 at the other orders, on the vector ALU with a
//    sliding window of the p rows m2 over the stored entries only.  Both
//    operators are symmetric, so only the entries with n2 > m2, or n2 == m2
//    and n1 >= m1, are kept (the partial of group (a, b) at (n12, m12) is
//    that of (b, a) at (m12, n12)): ((p - 1)(2p - 1) + p of the (2p - 1)^2
//    windows).  A kept entry is written to the level-2 partial of its plane,
//      A2[g][m2][m1][kh(n1 - m1 + p - 1, n2 - m2 + p - 1)],
//    once its last element e2 has been added.
//
//  asm3_kernel (level 3): one thread per kept level-2 entry (m1, m2, n1, n2)
//    walks the elements e3 of a segment of rows m3 and keeps the p x p
//    window w[r][s] of entries (m3, n3) = (e3 + r, e3 + s).  After element
//    e3 the entries with r = 0 or s = 0 are complete and go straight to
//    their CSR slots, together with their mirrors (n, m) off the diagonal
//    m12 == n12; the window then shifts along the diagonal.  Each value is
//    written once, in FP64 (no atomics, deterministic).
//
// The level-2 partials of a chunk of element layers live in a device
// workspace; when the whole patch does not fit, chunks of at least p - 1
// layers run in order and the level-3 kernel adds the partial sums of
// entries that straddle two chunks (read-modify-write, same stream).
//
// Redundant work: none at levels 1 and 3; level 1 is formed once per
// (plane, m1 tile, e2); level 3 recomputes the p - 1 element layers before
// each row segment.
#include <map>
#include <mutex>

#include "kernels.h"

#include <cstdlib>

namespace sfiga {

template <int P> struct A12Cfg;                // threads per workgroup, max rows m1 per tile
// (T1 (2p - 1) columns fill the waves' 16-column blocks, one block per wave;
// orders 7-9 use one wave per SIMD for the larger accumulator set; at
// p = 5, 6 and 7, T1 is the largest with one stored level-2 window per
// thread, T1 ((p-1)(2p-1) + p) <= NT: two per thread cost registers, and
// spills at p = 6 in FP64; p = 8 takes 2 rows when level 2 runs on the vector
// ALU and 4 on the matrix cores, see A12Shape)
template <> struct A12Cfg<2> { static constexpr int NT = 512, T1 = 42; };
template <> struct A12Cfg<3> { static constexpr int NT = 512, T1 = 25; };
template <> struct A12Cfg<4> { static constexpr int NT = 512, T1 = 18; };
template <> struct A12Cfg<5> { static constexpr int NT = 512, T1 = 12; };
template <> struct A12Cfg<6> { static constexpr int NT = 512, T1 = 8; };
template <> struct A12Cfg<7> { static constexpr int NT = 256, T1 = 3; };
template <> struct A12Cfg<8> { static constexpr int NT = 256, T1 = 4; };
template <> struct A12Cfg<9> { static constexpr int NT = 256, T1 = 3; };

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64: A[i][k] from lane i + 16k, B[k][j] from lane j + 16k,
// D[(l / 16) + 4v][l % 16] in element v of lane l
__device__ __forceinline__ d4 mfma16x16x4(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

// v_mfma_f32_16x16x16_bf16: A[i][k] from element k % 4 of lane i + 16 (k / 4),
// B[k][j] from element k % 4 of lane j + 16 (k / 4), D[4 (l / 16) + v][l % 16]
// in element v of lane l
__device__ __forceinline__ f4 mfma16x16x16bf16(s4 a, s4 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// bf16 with round-to-nearest-even, and the split x = hi + lo (hi, lo bf16):
// hi + lo holds x to about 2^-17 relative
__device__ __forceinline__ short bf16_rne(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
__device__ __forceinline__ float bf16_float(short h) { return __uint_as_float((unsigned)(unsigned short)h << 16); }
__device__ __forceinline__ void bf16_split(float x, short &hi, short &lo)
{
    hi = bf16_rne(x);
    lo = bf16_rne(x - bf16_float(hi));
}

// Pairs (i, j), index 3 i + j, summed into one direction-3 group
// g = 2 [i == 2] + [j == 2] (BB, BD, DB, DD of Sec. 3.1).
__device__ __forceinline__ int group_pair(int g, int t)
{
    constexpr int tab[4][4] = {{0, 1, 3, 4}, {2, 5, 0, 0}, {6, 7, 0, 0}, {8, 0, 0, 0}};
    return tab[g][t];
}
__host__ __device__ constexpr int group_npairs(int g) { return g == 0 ? 4 : (g == 3 ? 1 : 2); }

// Both operators are symmetric (C_ij = C_ji), so the level-2 partial of group
// (a, b) at (m12, n12) is the partial of group (b, a) at (n12, m12): only the
// windows with n2 > m2, or n2 == m2 and n1 >= m1, are formed and stored.
// Window kh < p is (c1, c2) = (p - 1 + kh, p - 1); window kh >= p is
// c1 = (kh - p) % W, c2 = p + (kh - p) / W.
__host__ __device__ constexpr int half_windows(int P) { return (P - 1) * (2 * P - 1) + P; }
template <int P>
__device__ __forceinline__ int half_index(int c1, int c2)
{
    constexpr int W = 2 * P - 1;
    if (c2 > P - 1) return P + (c2 - P) * W + c1;
    return (c2 == P - 1 && c1 >= P - 1) ? c1 - (P - 1) : -1;
}
template <int P>
__device__ __forceinline__ void half_window(int kh, int &c1, int &c2)
{
    constexpr int W = 2 * P - 1;
    if (kh < P) {
        c1 = P - 1 + kh;
        c2 = P - 1;
    } else {
        c1 = (kh - P) % W;
        c2 = P + (kh - P) / W;
    }
}

// L2M: where level 2 runs (0 vector ALU, 1 FP64 matrix cores, 2 bf16 split)
template <int P, bool STIFF, int L2M>
struct A12Shape {
    static constexpr int W = 2 * P - 1;          // band width per direction
    static constexpr int NH = half_windows(P);    // stored level-2 windows (c1, c2) per row
    static constexpr int NP = STIFF ? 9 : 1;     // (i, j) pairs
    static constexpr int NG = STIFF ? 4 : 1;     // groups sharing the direction-3 tables
    static constexpr int NCOMP = STIFF ? 6 : 1;  // symmetric coefficient components
    static constexpr int NT = A12Cfg<P>::NT;
    static constexpr int T1 = (P == 8 && L2M == 0) ? 2 : A12Cfg<P>::T1;   // rows m1 per tile (max)
    // waves per SIMD the register allocation must allow: two workgroups per CU
    // for p <= 4 (their LDS holds two), one above
    static constexpr int WPE = P <= 4 ? 2 * NT / 256 : NT / 256;
    // completed level-2 rows go through an LDS row buffer (p <= 4; above, the
    // extra LDS and registers cost more than the waits they remove)
    static constexpr bool DEFER = P <= 4;
    static constexpr int XE = T1 + P - 1;        // direction-1 elements touching the tile
    static constexpr int NSLICE = NCOMP * P * P * XE;        // coefficient slice of one element e2
    static constexpr int PF = (NSLICE + NT - 1) / NT;        // staged slice values per thread
    static constexpr int ITEMS = (T1 * NH + NT - 1) / NT;     // level-2 entries per thread
    static constexpr int L1SZ = P * NP * T1 * W;             // level-1 results of one element
    // level 2 on the matrix cores (FP64): slots (m2 mod p, n2 mod p) as rows,
    // 16 columns (m1, c1) per wave, K = (pair of the group, x2 point)
    static constexpr int NSLOT = P * P, MB = (NSLOT + 15) / 16;
    static constexpr int NW = NT / 64;
    static constexpr int NCB = (T1 * W + 15) / 16;               // column blocks (max)
    static constexpr int NBW = (NCB + NW - 1) / NW;              // column blocks per wave
};

template <int P, bool STIFF, typename CT, int L2M>
constexpr size_t a12_lds_bytes()
{
    using S = A12Shape<P, STIFF, L2M>;
    size_t a = sizeof(CT) * (size_t)(S::NSLICE + S::L1SZ);
    a = (a + 15) / 16 * 16;
    return a + sizeof(double) * (size_t)(2 * P * P * S::XE + 2 * 2 * P * P) +
           (S::DEFER ? sizeof(CT) * (size_t)S::NG * S::T1 * S::NH : 0);
}

// symmetric component of pair (i, j) in the order 00 11 22 01 02 12
__device__ __forceinline__ int comp3(int i, int j)
{
    if (i == j) return i;
    int a = i < j ? i : j, b = i < j ? j : i;
    return a == 0 ? (b == 1 ? 3 : 4) : 5;
}

// Levels 1 and 2 of plane x3 = q3base + by for the tile bx of rows m1.
// A2 layout: [plane - q3base][g][m2][m1][kh], kh the stored window of
// (c1, c2), c = n - m + p - 1.
// L2M: level 2 on the vector ALU (0), on FP64 matrix cores (1), on bf16
// matrix cores with split operands and FP32 accumulation (2).
template <int P, bool STIFF, typename CT, int L2M, bool UNR = true>
__device__ __forceinline__ void asm12_block(const PatchView &pv, const CT *__restrict__ C, CT *__restrict__ A2,
                                            int q3base, int T1r, int bx, int by)
{
    using S = A12Shape<P, STIFF, L2M>;
    constexpr int W = S::W, NP = S::NP, NG = S::NG, NCOMP = S::NCOMP, NT = S::NT, T1 = S::T1, XE = S::XE;
    constexpr int NH = S::NH;
    constexpr int NP1 = STIFF ? 8 : 1;                  // pairs formed at level 1
    // the next element's stage loads are issued before level 1 instead of
    // after it (measured faster at p = 2 and for the FP32-stored tiles at p = 4)
    constexpr bool EARLY = P == 2 || (P == 4 && sizeof(CT) == sizeof(float));
    // x2 points per level-1 lane (a divisor of p, bounded by registers)
    constexpr int G2B = (P == 2 || P == 6 || P == 8 || (P == 4 && sizeof(CT) == sizeof(float))) ? 2 : 1;
    constexpr int NGB = P / G2B;
    // unroll counts of the x1-point loop of level 1 and the x2-point loop of
    // level 2 on the vector ALU: two iterations in flight hide one LDS
    // latency each (order 6, 128^3 elements: FP64 79.7 -> 72.3 ms, FP32 level
    // 2 only 72.1 -> 70.0 ms); elsewhere the registers cost more than that
    // (single-patch kernel only: in the persistent kernel the registers
    // cost more, batched FP64 93.2 against 89.7 ms)
    constexpr int U1 = (UNR && P == 6 && sizeof(CT) == sizeof(double)) ? 2 : 1;
    constexpr int U2 = (UNR && P == 6) ? 2 : 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    CT *cs = reinterpret_cast<CT *>(smem_raw);          // [NCOMP][g2][g1][XE]
    CT *l1 = cs + S::NSLICE;                            // [g2][pair][T1][W]
    double *t1B = reinterpret_cast<double *>(smem_raw + (sizeof(CT) * (S::NSLICE + S::L1SZ) + 15) / 16 * 16);
    double *t1D = t1B + P * P * XE;                     // [g1][j][XE]
    // direction-2 tables [B, D][g2][j] of element e2 in buffer e2 & 1: the next
    // element's are staged while level 2 still reads the current ones
    double *t2buf = t1D + P * P * XE;
    double *t2B = t2buf, *t2D = t2B + P * P;
    // row m2 = e2 of the level-2 partials ([g][m1][kh]), complete after element
    // e2; written to A2 after the next barrier, away from the loads of the
    // stage (a load's first use waits for every memory operation before it)
    CT *rowbuf = reinterpret_cast<CT *>(t2buf + 2 * 2 * P * P);

    const Dir &d0 = pv.dir[0], &d1 = pv.dir[1];
    const int tid = threadIdx.x;
    const int b1 = bx * T1r;                    // first row m1 of the tile
    const int nrow1 = min(T1r, d0.N - b1);
    const int eb1 = b1 - P + 1;                         // first direction-1 element touching the tile
    const int pl = by;
    const int q3 = q3base + pl;
    const int Q0 = d0.Q, Q1 = d1.Q, N1 = d0.N, N2 = d1.N, K1 = d0.K, K2 = d1.K;
    const int64_t rowsz = (int64_t)N1 * NH;             // one row m2 of A2
    CT *A2p = A2 + (int64_t)pl * NG * N2 * rowsz;

    // direction-1 tables of the tile's elements, [g1][j][le1] (zeros outside the mesh)
    for (int i = tid; i < P * P * XE; i += NT) {
        const int le1 = i % XE, gj = i / XE;
        const int e1 = eb1 + le1;
        const bool ok = e1 >= 0 && e1 < K1;
        t1B[i] = ok ? d0.B[(int64_t)e1 * P * P + gj] : 0.0;
        t1D[i] = ok ? d0.D[(int64_t)e1 * P * P + gj] : 0.0;
    }

    // staged values of one element e2: the coefficient slice (global order
    // comp, g2, x1 with x1 fastest) and the element's direction-2 tables.
    // The loaded values are not touched until they are stored to LDS (masking
    // included): an instruction that reads a load's result waits for it, and
    // for every memory operation issued before it, the A2 stores among them.
    static_assert(2 * P * P <= NT, "at most one table value per thread");
    CT sv[S::PF];              // coefficient slice values as loaded
    double tv = 0.0;           // table value of the first 2p^2 threads
    auto load_stage = [&](int e2) {
        const CT *base = C + (int64_t)q3 * NCOMP * Q1 * Q0;
#pragma unroll
        for (int k = 0; k < S::PF; ++k) {
            const int idx = tid + k * NT;
            if (idx < S::NSLICE) {
                const int lq1 = idx % (XE * P), r = idx / (XE * P);
                const int g2 = r % P, comp = r / P;
                const int q0 = eb1 * P + lq1, q1 = e2 * P + g2;
                const bool ok = q0 >= 0 && q0 < Q0;
                sv[k] = base[ok ? ((int64_t)comp * Q1 + q1) * Q0 + q0 : 0];
            }
        }
        if (tid < 2 * P * P) {
            // a register of its own: a table value sharing one with the slice
            // values of other lanes made the compiler wait for those loads
            // before issuing this one
            int t = tid;
            // opaque here, so that the table address is formed from the scalar
            // bases at each call instead of being kept (or spilled) in vector
            // registers across the element loop
            asm volatile("" : "+v"(t));
            tv = (t < P * P ? d1.B : d1.D)[e2 * P * P + t % (P * P)];
        }
    };
    auto store_stage = [&](int e2) {
        double *t2 = t2buf + (e2 & 1) * 2 * P * P;
#pragma unroll
        for (int k = 0; k < S::PF; ++k) {
            const int idx = tid + k * NT;
            if (idx < S::NSLICE) {
                const int lq1 = idx % (XE * P), r = idx / (XE * P);
                const int le1 = lq1 / P, g1 = lq1 % P;
                const int q0 = eb1 * P + lq1;
                cs[(r * P + g1) * XE + le1] = (q0 >= 0 && q0 < Q0) ? sv[k] : CT(0);
            }
        }
        if (tid < 2 * P * P) t2[tid] = tv;
    };

    static_assert(L2M != 1 || sizeof(CT) == sizeof(double), "FP64 matrix cores take FP64 operands");
    static_assert(L2M != 2 || sizeof(CT) == sizeof(float), "bf16 split takes FP32 operands");
    constexpr bool MFMA = L2M == 1;
    // level-2 accumulators on the matrix cores: FP64 (L2M 1) or FP32 (L2M 2)
    d4 macc[MFMA ? S::NBW : 1][NG][MFMA ? S::MB : 1];
#pragma unroll
    for (int nb = 0; nb < (MFMA ? S::NBW : 1); ++nb)
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int rb = 0; rb < (MFMA ? S::MB : 1); ++rb) macc[nb][g][rb] = d4{0.0, 0.0, 0.0, 0.0};
    f4 facc[L2M == 2 ? S::NBW : 1][NG][L2M == 2 ? S::MB : 1];
#pragma unroll
    for (int nb = 0; nb < (L2M == 2 ? S::NBW : 1); ++nb)
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int rb = 0; rb < (L2M == 2 ? S::MB : 1); ++rb) facc[nb][g][rb] = f4{0.f, 0.f, 0.f, 0.f};
    // vector ALU: level-2 entries of this thread, it = c1 + W (c2 + W lm1)
    CT acc[L2M == 0 ? S::ITEMS : 1][P][NG];
#pragma unroll
    for (int k = 0; k < (L2M == 0 ? S::ITEMS : 1); ++k)
#pragma unroll
        for (int r = 0; r < P; ++r)
#pragma unroll
            for (int g = 0; g < NG; ++g) acc[k][r][g] = CT(0);
    const int nitems = nrow1 * NH;

    auto flush_row = [&](int e) {
        const int n = nrow1 * NH;
        for (int i = tid; i < NG * n; i += NT) {
            const int g = i / n, rem = i - g * n;
            A2p[((int64_t)g * N2 + e) * rowsz + (int64_t)b1 * NH + rem] = rowbuf[i];
        }
    };

    load_stage(0);
    store_stage(0);
    __syncthreads();

    // per element: level 1 | barrier | level 2 while the next slice is stored
    // (level 2 reads no slice, and the tables are double-buffered) | barrier.
    // The stage of the next element is loaded and stored on every pass (the
    // last element reloads itself): with a condition around them, the
    // compiler's count of loads in flight is lost at the loop's back edge and
    // it waits for every earlier memory operation before the next loads.
    for (int e2 = 0; e2 < K2; ++e2) {
        t2B = t2buf + (e2 & 1) * 2 * P * P;
        t2D = t2B + P * P;
        if (S::DEFER && e2 > 0) flush_row(e2 - 1);
        const int en = e2 + 1 < K2 ? e2 + 1 : e2;
        if constexpr (EARLY) load_stage(en);
        // ---------------- level 1: contract x1 for every row of the tile.
        // One lane per (pair, row m1) forms all p x2 points of the element, so
        // the table values of each (element, x1 point) serve p x2 points.
        // Pair (2, 1) equals (1, 2) at this level (same tables and
        // coefficient component) and is not formed.
        for (int it = tid; it < NP1 * NGB * nrow1; it += NT) {
            const int lm1 = it % nrow1, rest = it / nrow1;
            const int gb = rest % NGB, pi = rest / NGB;
            const int pair = STIFF ? (pi < 7 ? pi : 8) : 0;
            const int i = STIFF ? pair / 3 : 1, j = STIFF ? pair % 3 : 1;
            const int comp = STIFF ? comp3(i, j) : 0;
            const double *ta = i == 0 ? t1D : t1B;
            const double *tb = j == 0 ? t1D : t1B;
            const CT *cg = cs + (comp * P + gb * G2B) * P * XE;
            const int m1 = b1 + lm1;
            CT a[G2B][W];
#pragma unroll
            for (int g = 0; g < G2B; ++g)
#pragma unroll
                for (int c = 0; c < W; ++c) a[g][c] = CT(0);
#pragma unroll
            for (int r = 0; r < P; ++r) {
                const int e1 = m1 - r;
                if (e1 < 0 || e1 >= K1) continue;
                const int le1 = lm1 + P - 1 - r;
#pragma unroll (U1)
                for (int g1 = 0; g1 < P; ++g1) {
                    const CT av = (CT)ta[(g1 * P + r) * XE + le1];
                    CT bv[P];
#pragma unroll
                    for (int s = 0; s < P; ++s) bv[s] = (CT)tb[(g1 * P + s) * XE + le1];
#pragma unroll
                    for (int g = 0; g < G2B; ++g) {
                        const CT cv = cg[(g * P + g1) * XE + le1] * av;
#pragma unroll
                        for (int s = 0; s < P; ++s) a[g][s - r + P - 1] += cv * bv[s];
                    }
                }
            }
#pragma unroll
            for (int g = 0; g < G2B; ++g)
#pragma unroll
                for (int c = 0; c < W; ++c) l1[(((gb * G2B + g) * NP + pair) * T1 + lm1) * W + c] = a[g][c];
        }
        __syncthreads();
        if constexpr (!EARLY) load_stage(en);

        // ---------------- level 2: fold x2 into the rows m2 = e2 + r
        const bool last = e2 == K2 - 1;
        if constexpr (MFMA) {
            // slot (ms, ns) holds entry (m2, n2) with m2 = ms, n2 = ns (mod p);
            // for element e2 (phase ph) it is (r, s) = (ms - ph, ns - ph) mod p
            const int ph = e2 % P;
            const int lane = tid & 63, wave = tid >> 6;
            const int ncols = nrow1 * W;
#pragma unroll
            for (int nb = 0; nb < S::NBW; ++nb) {
                const int cb = wave + nb * S::NW;
                if (cb * 16 >= ncols) break;
                const int col = cb * 16 + (lane & 15);
                const bool colok = col < ncols;
                const int kq = lane >> 4;
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const int nk = (STIFF ? group_npairs(g) : 1) * P;
#pragma unroll 1
                    for (int ks = 0; ks < (4 * P + 3) / 4; ++ks) {
                        if (ks * 4 >= nk) break;
                        const int k = ks * 4 + kq;
                        const bool kok = k < nk;
                        const int pair = STIFF ? group_pair(g, kok ? k / P : 0) : 0;
                        const int g2 = k % P;
                        const int pi = STIFF ? pair / 3 : 0, pj = STIFF ? pair % 3 : 0;
                        const int lp = pair == 7 ? 5 : pair;          // (2, 1) is stored as (1, 2)
                        const double b = (kok && colok) ? (double)l1[(g2 * NP + lp) * (T1 * W) + col] : 0.0;
                        const double *ta = pi == 1 ? t2D : t2B, *tb = pj == 1 ? t2D : t2B;
#pragma unroll
                        for (int rb = 0; rb < S::MB; ++rb) {
                            const int i = (lane & 15) + 16 * rb;
                            const int ms = i / P, ns = i % P;
                            const int r = (ms - ph + P) % P, sj = (ns - ph + P) % P;
                            const double a = (kok && i < S::NSLOT) ? ta[g2 * P + r] * tb[g2 * P + sj] : 0.0;
                            macc[nb][g][rb] = mfma16x16x4(a, b, macc[nb][g][rb]);
                        }
                    }
                }
                // entries whose last element is e2 (r == 0 or s == 0), all after the last element
                const int lm1 = col / W, c1 = col % W;
                CT *dst = A2p + (int64_t)(b1 + lm1) * NH;
#pragma unroll
                for (int rb = 0; rb < S::MB; ++rb)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = (lane >> 4) + 4 * v + 16 * rb;
                        const int ms = i / P, ns = i % P;
                        if (i < S::NSLOT && (last || ms == ph || ns == ph)) {
                            const int m2 = e2 + (ms - ph + P) % P, n2 = e2 + (ns - ph + P) % P;
                            const int kh = half_index<P>(c1, n2 - m2 + P - 1);
#pragma unroll
                            for (int g = 0; g < NG; ++g) {
                                if (colok && kh >= 0) {
                                    if (S::DEFER && ms == ph) rowbuf[(g * nrow1 + lm1) * NH + kh] = macc[nb][g][rb][v];
                                    else dst[((int64_t)g * N2 + m2) * rowsz + kh] = macc[nb][g][rb][v];   // last element
                                }
                                macc[nb][g][rb][v] = 0.0;
                            }
                        }
                    }
            }
        } else if constexpr (L2M == 2) {
            // as the FP64 path with K in steps of 16; every operand x = hi + lo
            // in bf16 and A B ~ Ahi Bhi + Ahi Blo + Alo Bhi, accumulated in FP32
            const int ph = e2 % P;
            const int lane = tid & 63, wave = tid >> 6;
            const int ncols = nrow1 * W;
#pragma unroll
            for (int nb = 0; nb < S::NBW; ++nb) {
                const int cb = wave + nb * S::NW;
                if (cb * 16 >= ncols) break;
                const int col = cb * 16 + (lane & 15);
                const bool colok = col < ncols;
                const int kq = lane >> 4;
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const int nk = (STIFF ? group_npairs(g) : 1) * P;
#pragma unroll 1
                    for (int ks = 0; ks < (4 * P + 15) / 16; ++ks) {
                        if (ks * 16 >= nk) break;
                        s4 bhi, blo, ahi[S::MB], alo[S::MB];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int k = ks * 16 + 4 * kq + e;
                            const bool kok = k < nk;
                            const int pair = STIFF ? group_pair(g, kok ? k / P : 0) : 0;
                            const int g2 = k % P;
                            const int pi = STIFF ? pair / 3 : 0, pj = STIFF ? pair % 3 : 0;
                            const int lp = pair == 7 ? 5 : pair;      // (2, 1) is stored as (1, 2)
                            const float b = (kok && colok) ? (float)l1[(g2 * NP + lp) * (T1 * W) + col] : 0.f;
                            short h, l;
                            bf16_split(b, h, l);
                            bhi[e] = h;
                            blo[e] = l;
                            const double *ta = pi == 1 ? t2D : t2B, *tb = pj == 1 ? t2D : t2B;
#pragma unroll
                            for (int rb = 0; rb < S::MB; ++rb) {
                                const int i = (lane & 15) + 16 * rb;
                                const int r = (i / P - ph + P) % P, sj = (i % P - ph + P) % P;
                                const float a = (kok && i < S::NSLOT) ? (float)(ta[g2 * P + r] * tb[g2 * P + sj]) : 0.f;
                                bf16_split(a, h, l);
                                ahi[rb][e] = h;
                                alo[rb][e] = l;
                            }
                        }
#pragma unroll
                        for (int rb = 0; rb < S::MB; ++rb) {
                            facc[nb][g][rb] = mfma16x16x16bf16(ahi[rb], bhi, facc[nb][g][rb]);
                            facc[nb][g][rb] = mfma16x16x16bf16(ahi[rb], blo, facc[nb][g][rb]);
                            facc[nb][g][rb] = mfma16x16x16bf16(alo[rb], bhi, facc[nb][g][rb]);
                        }
                    }
                }
                const int lm1 = col / W, c1 = col % W;
                CT *dst = A2p + (int64_t)(b1 + lm1) * NH;
#pragma unroll
                for (int rb = 0; rb < S::MB; ++rb)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = 4 * (lane >> 4) + v + 16 * rb;
                        const int ms = i / P, ns = i % P;
                        if (i < S::NSLOT && (last || ms == ph || ns == ph)) {
                            const int m2 = e2 + (ms - ph + P) % P, n2 = e2 + (ns - ph + P) % P;
                            const int kh = half_index<P>(c1, n2 - m2 + P - 1);
#pragma unroll
                            for (int g = 0; g < NG; ++g) {
                                if (colok && kh >= 0) {
                                    if (S::DEFER && ms == ph) rowbuf[(g * nrow1 + lm1) * NH + kh] = (CT)facc[nb][g][rb][v];
                                    else dst[((int64_t)g * N2 + m2) * rowsz + kh] = (CT)facc[nb][g][rb][v];   // last element
                                }
                                facc[nb][g][rb][v] = 0.f;
                            }
                        }
                    }
            }
        } else {
#pragma unroll
            for (int k = 0; k < (L2M == 0 ? S::ITEMS : 1); ++k) {
                const int it = tid + k * NT;
                if (it >= nitems) continue;
                const int lm1 = it / NH;
                int c1, c2;
                half_window<P>(it % NH, c1, c2);
#pragma unroll (U2)
                for (int g2 = 0; g2 < P; ++g2) {
                    CT L[NP];
#pragma unroll
                    for (int a = 0; a < NP; ++a) L[a] = l1[((g2 * NP + (a == 7 ? 5 : a)) * T1 + lm1) * W + c1];
#pragma unroll
                    for (int r = 0; r < P; ++r) {
                        const int s = r + c2 - (P - 1);
                        if (s < 0 || s >= P) continue;
                        const CT Br = (CT)t2B[g2 * P + r], Bs = (CT)t2B[g2 * P + s];
                        if constexpr (STIFF) {
                            const CT Dr = (CT)t2D[g2 * P + r], Ds = (CT)t2D[g2 * P + s];
                            acc[k][r][0] += Br * (Bs * L[0] + Ds * L[1]) + Dr * (Bs * L[3] + Ds * L[4]);
                            acc[k][r][1] += Bs * (Br * L[2] + Dr * L[5]);
                            acc[k][r][2] += Br * (Bs * L[6] + Ds * L[7]);
                            acc[k][r][3] += Br * Bs * L[8];
                        } else {
                            acc[k][r][0] += Br * Bs * L[0];
                        }
                    }
                }
                // row m2 = e2 is complete (and every row of the window after the last element)
                if constexpr (S::DEFER) {
#pragma unroll
                    for (int g = 0; g < NG; ++g) rowbuf[g * nrow1 * NH + it] = acc[k][0][g];
                }
                {
                    // without the row buffer row e2 goes straight to A2; the rows
                    // after it only once the last element has been added
                    CT *dst = A2p + (int64_t)b1 * NH + it;
#pragma unroll
                    for (int r = S::DEFER ? 1 : 0; r < P; ++r) {
                        if (r > 0 && !last) break;
#pragma unroll
                        for (int g = 0; g < NG; ++g) dst[((int64_t)g * N2 + e2 + r) * rowsz] = acc[k][r][g];
                    }
                }
#pragma unroll
                for (int r = 0; r + 1 < P; ++r)
#pragma unroll
                    for (int g = 0; g < NG; ++g) acc[k][r][g] = acc[k][r + 1][g];
#pragma unroll
                for (int g = 0; g < NG; ++g) acc[k][P - 1][g] = CT(0);
            }
        }
        store_stage(e2 + 1);   // into table buffer (e2 + 1) & 1, not the one level 2 reads
        __syncthreads();
    }
    if (S::DEFER) flush_row(K2 - 1);
}

template <int P, bool STIFF, typename CT, int L2M>
__global__ __launch_bounds__((A12Shape<P, STIFF, L2M>::NT), (A12Shape<P, STIFF, L2M>::WPE)) void asm12_kernel(PatchView pv, const CT *__restrict__ C,
                                                                        CT *__restrict__ A2, int q3base, int T1r)
{
    asm12_block<P, STIFF, CT, L2M>(pv, C, A2, q3base, T1r, blockIdx.x, blockIdx.y);
}

// Load of a value every lane reads at the same address from memory the kernel
// does not write (the 1D tables): a scalar load.
__device__ __forceinline__ double ld_uniform(const double *p)
{
    return *(const __attribute__((address_space(4))) double *)p;
}

// Level 3 for the chunk of elements [s0, s1) in direction 3, rows m3 of the
// segment seg0 + bz (length L).  One thread per stored level-2 window
// (m1, n1, m2 = by, n2); block bx covers 256 windows of the row m2.
//
// A thread stores its own entries (m, n) directly: consecutive threads hold
// consecutive columns of a row.  The mirrors (n, m) off the diagonal
// m12 == n12 go through LDS: the windows of a block are ordered once by
// mirror position, key (n1, c2, m1 - n1 + p - 1), with a counting sort, and
// after each element lane l stores the mirror values of the l-th window in
// that order, so a wavefront writes runs of up to 2p - 1 consecutive columns
// (for fixed n1 and c2 the mirror column advances with m1).
template <int P>
struct A3Shape {
    static constexpr int W = 2 * P - 1, NH = half_windows(P);
    static constexpr int NJ = 2 * P - 1;                        // entries per element and window
    static constexpr int NROW = 255 / NH + 2;                   // rows m1 a block touches (max)
    static constexpr int NKEY = (NROW + 2 * P - 2) * P * W;     // mirror keys (n1, c2, k)
    static_assert(NKEY <= NJ * 256 * 2, "key table fits in the mirror buffer");
};

template <int P, bool STIFF, typename CT>
__device__ __forceinline__ void asm3_block(const PatchView &pv, const CT *__restrict__ A2, double *__restrict__ vals,
                                           int s0, int s1, int L, int seg0, int bx, int by, int bz)
{
    using S3 = A3Shape<P>;
    constexpr int NH = S3::NH, NG = STIFF ? 4 : 1, NJ = S3::NJ;
    __shared__ double mv[NJ][256];          // mirror values of one element (the setup's tables first)
    __shared__ int inv[256];                // lane -> window in mirror order
    __shared__ int wsum[4];
    const Dir &d0 = pv.dir[0], &d1 = pv.dir[1], &d2 = pv.dir[2];
    const int N1 = d0.N, N2 = d1.N, N3 = d2.N;
    const int64_t rowsz = (int64_t)N1 * NH;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t it0 = (int64_t)bx * 256;
    const int a3 = (seg0 + bz) * L;
    const int ebeg = max(s0, a3 - P + 1), eend = min(s1 - 1, a3 + L - 1);
    if (ebeg > eend) return;                                    // uniform over the block

    const int64_t it = it0 + tid;
    const int m2 = by;
    const int m1 = (int)(min(it, rowsz - 1) / NH);
    int c1, c2;
    half_window<P>((int)(min(it, rowsz - 1) % NH), c1, c2);
    const int n1 = m1 + c1 - P + 1, n2 = m2 + c2 - P + 1;
    const bool active = it < rowsz && n1 >= 0 && n1 < N1 && n2 >= 0 && n2 < N2;
    const bool mirror = active && (c1 != P - 1 || c2 != P - 1);

    const RowIndex &ri = pv.ri;
    const int64_t T21 = ri.T[1] * ri.T[0];
    int64_t R12 = 0, off12 = 0, len12 = 0, mR12 = 0, moff12 = 0, mlen12 = 0;
    if (active) {
        const int64_t len1 = band_len(m1, P, N1), len2 = band_len(m2, P, N2);
        R12 = ri.S[1][m2] * ri.T[0] + len2 * ri.S[0][m1];
        off12 = (n1 - band_lo(m1, P)) + (int64_t)(n2 - band_lo(m2, P)) * len1;
        len12 = len1 * len2;
        // mirror: row (n1, n2, n3), column (m1, m2, m3)
        const int64_t ml1 = band_len(n1, P, N1), ml2 = band_len(n2, P, N2);
        mR12 = ri.S[1][n2] * ri.T[0] + ml2 * ri.S[0][n1];
        moff12 = (m1 - band_lo(n1, P)) + (int64_t)(m2 - band_lo(n2, P)) * ml1;
        mlen12 = ml1 * ml2;
    }

    // ---- mirror order: counting sort of the keys (n1 - n1min, c2 - p + 1, k)
    int *cnt = reinterpret_cast<int *>(&mv[0][0]);
    const int m1a = (int)(it0 / NH);
    const int m1b = (int)(min(it0 + 255, rowsz - 1) / NH);
    const int nkey = (m1b - m1a + 2 * P - 1) * P * S3::W;
    const int key = mirror ? ((n1 - (m1a - P + 1)) * P + (c2 - P + 1)) * S3::W + (m1 - n1 + P - 1) : -1;
    for (int i = tid; i < nkey; i += 256) cnt[i] = 0;
    __syncthreads();
    if (mirror) cnt[key] = 1;
    __syncthreads();
    const int per = (nkey + 255) / 256;
    int loc = 0;
    for (int k = 0; k < per; ++k) {
        const int i = tid * per + k;
        if (i < nkey) loc += cnt[i];
    }
    int incl = loc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int run = incl - loc;
    for (int w = 0; w < wave; ++w) run += wsum[w];
    const int nmir = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    for (int k = 0; k < per; ++k) {
        const int i = tid * per + k;
        if (i < nkey) {
            const int v = cnt[i];
            cnt[i] = run;
            run += v;
        }
    }
    __syncthreads();
    if (mirror) inv[cnt[key]] = tid;
    __syncthreads();
    int64_t *cst = reinterpret_cast<int64_t *>(&mv[0][0]);     // [3][256] mirror row constants
    cst[tid] = mR12;
    cst[256 + tid] = moff12;
    cst[512 + tid] = mlen12;
    __syncthreads();
    const int wsrc = tid < nmir ? inv[tid] : 0;                 // this lane stores the mirrors of window wsrc
    const int64_t wR12 = cst[wsrc], woff12 = cst[256 + wsrc], wlen12 = cst[512 + wsrc];
    __syncthreads();

    double w[P][P];
#pragma unroll
    for (int r = 0; r < P; ++r)
#pragma unroll
        for (int s = 0; s < P; ++s) w[r][s] = 0.0;
    const int64_t gstride = (int64_t)N2 * rowsz;         // next group of the same plane
    const CT *src = A2 + (int64_t)m2 * rowsz + (active ? it : 0) + (int64_t)(ebeg - s0) * P * NG * gstride;
    // level-2 values of the next plane are loaded one plane ahead
    CT G[NG], Gn[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) Gn[g] = active ? src[g * gstride] : CT(0);
    for (int e3 = ebeg; e3 <= eend; ++e3) {
#pragma unroll 1
        for (int g3 = 0; g3 < P; ++g3) {
#pragma unroll
            for (int g = 0; g < NG; ++g) G[g] = Gn[g];
            src += NG * gstride;
            if (active && (g3 + 1 < P || e3 < eend)) {
#pragma unroll
                for (int g = 0; g < NG; ++g) Gn[g] = src[g * gstride];
            }
            // table values of the plane: uniform, read through the scalar cache so
            // that they do not queue behind the level-2 loads in flight
            double tB[P], tD[P];
#pragma unroll
            for (int s = 0; s < P; ++s) {
                tB[s] = ld_uniform(d2.B + ((int64_t)e3 * P + g3) * P + s);
                tD[s] = STIFF ? ld_uniform(d2.D + ((int64_t)e3 * P + g3) * P + s) : 0.0;
            }
            if constexpr (STIFF) {
                double uB[P], uD[P];
#pragma unroll
                for (int s = 0; s < P; ++s) {
                    uB[s] = tB[s] * (double)G[0] + tD[s] * (double)G[1];
                    uD[s] = tB[s] * (double)G[2] + tD[s] * (double)G[3];
                }
#pragma unroll
                for (int r = 0; r < P; ++r) {
                    const double br = tB[r], dr = tD[r];
#pragma unroll
                    for (int s = 0; s < P; ++s) w[r][s] += br * uB[s] + dr * uD[s];
                }
            } else {
                double u[P];
#pragma unroll
                for (int s = 0; s < P; ++s) u[s] = tB[s] * (double)G[0];
#pragma unroll
                for (int r = 0; r < P; ++r) {
                    const double br = tB[r];
#pragma unroll
                    for (int s = 0; s < P; ++s) w[r][s] += br * u[s];
                }
            }
        }
        // entries whose last element is e3: j < p is (e3, e3 + j), j >= p is
        // (e3 + j - p + 1, e3); the row m3 must lie in the segment
        const int64_t b0 = ri.S[2][e3] * T21;
        const int64_t l0 = band_len(e3, P, N3), lo0 = band_lo(e3, P);
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int m3 = j < P ? e3 : e3 + j - P + 1, n3 = j < P ? e3 + j : e3;
            if (m3 < a3 || m3 >= a3 + L || n3 >= N3) continue;    // uniform
            if (active) {
                const int64_t pos = j < P ? b0 + l0 * R12 + off12 + (n3 - lo0) * len12
                                          : ri.S[2][m3] * T21 + band_len(m3, P, N3) * R12 + off12 +
                                                (int64_t)(n3 - band_lo(m3, P)) * len12;
                double v = j < P ? w[0][j] : w[j - P + 1][0];
                if (s0 > 0 && max(m3, n3) - P + 1 < s0) v += vals[pos];   // partial sum of the previous chunk
                vals[pos] = v;
                mv[j][tid] = v;
            }
        }
        if (e3 == s1 - 1) {
            // end of the chunk: the rest of the window is complete (last layer)
            // or partial; mirrors go straight to memory (once per chunk)
#pragma unroll
            for (int r = 1; r < P; ++r)
#pragma unroll
                for (int s = 1; s < P; ++s) {
                    const int m3 = e3 + r, n3 = e3 + s;
                    if (!active || m3 < a3 || m3 >= a3 + L || n3 >= N3) continue;
                    const int64_t pos = ri.S[2][m3] * T21 + band_len(m3, P, N3) * R12 + off12 +
                                        (int64_t)(n3 - band_lo(m3, P)) * len12;
                    double v = w[r][s];
                    if (s0 > 0 && max(m3, n3) - P + 1 < s0) v += vals[pos];
                    vals[pos] = v;
                    if (mirror)
                        vals[ri.S[2][n3] * T21 + band_len(n3, P, N3) * mR12 + moff12 +
                             (int64_t)(m3 - band_lo(n3, P)) * mlen12] = v;
                }
        }
        __syncthreads();
        if (tid < nmir) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int m3 = j < P ? e3 : e3 + j - P + 1, n3 = j < P ? e3 + j : e3;
                if (m3 < a3 || m3 >= a3 + L || n3 >= N3) continue;
                // mirror of (m3, n3): row n3, column m3
                const int64_t pos = j < P ? ri.S[2][n3] * T21 + band_len(n3, P, N3) * wR12 + woff12 +
                                                (int64_t)(m3 - band_lo(n3, P)) * wlen12
                                          : b0 + l0 * wR12 + woff12 + (m3 - lo0) * wlen12;
                vals[pos] = mv[j][wsrc];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r + 1 < P; ++r)
#pragma unroll
            for (int s = 0; s + 1 < P; ++s) w[r][s] = w[r + 1][s + 1];
#pragma unroll
        for (int k = 0; k < P; ++k) w[P - 1][k] = w[k][P - 1] = 0.0;
    }
}

template <int P, bool STIFF, typename CT>
__global__ __launch_bounds__(256) void asm3_kernel(PatchView pv, const CT *__restrict__ A2, double *__restrict__ vals,
                                                   int s0, int s1, int L, int seg0)
{
    int bx, by, bz;
    xcd_tile(bx, by, bz);
    asm3_block<P, STIFF, CT>(pv, A2, vals, s0, s1, L, seg0, bx, by, bz);
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

static size_t a2_plane_bytes(const PatchView &pv, int op, Prec prec)
{
    const int NG = op == 2 ? 4 : 1;
    return (size_t)NG * pv.dir[1].N * pv.dir[0].N * half_windows(pv.P) *
           (prec == Prec::F64 ? sizeof(double) : sizeof(float));   // BF16X3: FP32
}

// element layers per chunk for a workspace of the given size (0: too small)
static int a2_chunk(const PatchView &pv, int op, Prec prec, size_t ws_bytes)
{
    const size_t per_layer = a2_plane_bytes(pv, op, prec) * pv.P;
    const int K3 = pv.dir[2].K;
    const size_t fit = ws_bytes / per_layer;
    if (fit >= (size_t)K3) return K3;
    return (int)fit >= (pv.P - 1 > 1 ? pv.P - 1 : 1) ? (int)fit : 0;
}

size_t assemble_workspace_bytes(const PatchView &pv, int op, Prec prec, size_t cap)
{
    if (pv.d != 3) return 0;
    const size_t per_layer = a2_plane_bytes(pv, op, prec) * pv.P;
    const int K3 = pv.dir[2].K;
    const int minl = pv.P - 1 > 1 ? pv.P - 1 : 1;
    size_t layers = cap / per_layer;
    if (layers > (size_t)K3) layers = K3;
    if (layers < (size_t)(minl < K3 ? minl : K3)) layers = minl < K3 ? minl : K3;
    return layers * per_layer;
}

bool assemble_single_chunk(const PatchView &pv, int op, Prec prec, size_t ws_bytes)
{
    return pv.d == 3 && a2_chunk(pv, op, prec, ws_bytes) == pv.dir[2].K;
}

size_t assemble_min_workspace_bytes(const PatchView &pv, int op, Prec prec)
{
    if (pv.d != 3) return 0;
    const int K3 = pv.dir[2].K;
    const int minl = pv.P - 1 > 1 ? pv.P - 1 : 1;
    return a2_plane_bytes(pv, op, prec) * pv.P * (size_t)(minl < K3 ? minl : K3);
}

// Fixed device scratch for the assembly entry point that allocates nothing:
// the level-2 workspace of one chunk of element layers.  Each device the
// library runs on holds its own copy until the process ends; in host code the
// array's name is not a device address, so the address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void **ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    static std::mutex mu;
    static std::map<int, void *> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        it = addr.emplace(dev, p).first;
    }
    *ptr = it->second;
    return hipSuccess;
}

// level 2 in FP64 mode: matrix cores at p = 4 and 8, vector ALU otherwise
template <int P> constexpr int f64_level2() { return (P == 4 || P == 8) ? 1 : 0; }

template <int P> static int a12_rows(Prec prec)
{
    if (prec == Prec::F64) return A12Shape<P, true, f64_level2<P>()>::T1;
    if (prec == Prec::BF16X3) return A12Shape<P, true, 2>::T1;
    return A12Shape<P, true, 0>::T1;
}

int asm12_max_rows(int P, Prec prec)
{
    switch (P) {
    case 2: return a12_rows<2>(prec);
    case 3: return a12_rows<3>(prec);
    case 4: return a12_rows<4>(prec);
    case 5: return a12_rows<5>(prec);
    case 6: return a12_rows<6>(prec);
    case 7: return a12_rows<7>(prec);
    case 8: return a12_rows<8>(prec);
    default: return a12_rows<9>(prec);
    }
}

void asm12_blocks(const PatchView &pv, Prec prec, int t1, int &gx, int &gy, int &T1r)
{
    const int tmax = asm12_max_rows(pv.P, prec);
    if (t1 <= 0 || t1 > tmax) t1 = tmax;
    const int N1 = pv.dir[0].N;
    const int ntile = (N1 + t1 - 1) / t1;
    T1r = (N1 + ntile - 1) / ntile;                          // balanced tiles
    gx = ntile;
    gy = pv.dir[2].Q;
}

void asm3_blocks(const PatchView &pv, int seg, int &gx, int &gy, int &gz, int &L)
{
    const int N3 = pv.dir[2].N;
    const int nseg = (N3 + (seg > 0 ? seg : 16) - 1) / (seg > 0 ? seg : 16);
    L = (N3 + nseg - 1) / nseg;
    gx = (int)(((int64_t)pv.dir[0].N * half_windows(pv.P) + 255) / 256);
    gy = pv.dir[1].N;
    gz = nseg;
}

template <int P, bool STIFF, typename CT, int L2M>
static hipError_t set_asm12_lds(const void *fn)
{
    const size_t lds = a12_lds_bytes<P, STIFF, CT, L2M>();
    return allow_dynamic_lds(fn, lds);
}

template <int P, bool STIFF, typename CT, int L2M>
static hipError_t launch_asm3d(const PatchView &pv, const CT *C, double *vals, void *ws, size_t ws_bytes,
                               hipStream_t s, int t1, int seg)
{
    using S = A12Shape<P, STIFF, L2M>;
    const size_t lds = a12_lds_bytes<P, STIFF, CT, L2M>();
    {
        hipError_t e = set_asm12_lds<P, STIFF, CT, L2M>((const void *)asm12_kernel<P, STIFF, CT, L2M>);
        if (e != hipSuccess) return e;
    }
    const int op = STIFF ? 2 : 1;
    const Prec prec = sizeof(CT) == sizeof(double) ? Prec::F64 : Prec::F32;   // workspace element size
    const int chunk = a2_chunk(pv, op, prec, ws_bytes);
    if (chunk == 0 || !ws) return hipErrorInvalidValue;
    const int N3 = pv.dir[2].N, K3 = pv.dir[2].K;
    int ntile, nplane, T1r, gx3, gy3, nseg, L;
    asm12_blocks(pv, L2M == 2 ? Prec::BF16X3 : prec, t1, ntile, nplane, T1r);
    asm3_blocks(pv, seg, gx3, gy3, nseg, L);
    CT *A2 = static_cast<CT *>(ws);
    for (int s0 = 0; s0 < K3; s0 += chunk) {
        const int s1 = s0 + chunk < K3 ? s0 + chunk : K3;
        hipLaunchKernelGGL((asm12_kernel<P, STIFF, CT, L2M>), dim3(ntile, (s1 - s0) * P), dim3(S::NT), lds, s, pv, C,
                           A2, s0 * P, T1r);
        const int last_row = s1 + P - 2 < N3 - 1 ? s1 + P - 2 : N3 - 1;
        const int seg0 = s0 / L, seg1 = last_row / L;
        hipLaunchKernelGGL((asm3_kernel<P, STIFF, CT>), dim3(gx3, gy3, seg1 - seg0 + 1), dim3(256), 0, s, pv,
                           (const CT *)A2, vals, s0, s1, L, seg0);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ batched

// Persistent forms: each workgroup takes blocks it = blockIdx.x, + gridDim.x,
// ... of the concatenated per-patch grids (every patch in one chunk).
template <int P, bool STIFF, typename CT, int L2M>
__global__ __launch_bounds__((A12Shape<P, STIFF, L2M>::NT), (A12Shape<P, STIFF, L2M>::WPE)) void asm12_persistent(TaskList tl)
{
    for (int64_t it = blockIdx.x; it < tl.nitems; it += gridDim.x) {
        const int t = task_of(tl.off, tl.ntask, it);
        const BatchTask &T = tl.tasks[t];
        const int64_t l = it - tl.off[t];
        asm12_block<P, STIFF, CT, L2M, false>(T.pv, (const CT *)T.C, (CT *)T.ws, 0, T.arg, (int)(l % T.gx),
                                              (int)(l / T.gx));
        __syncthreads();   // LDS of the next block
    }
}

template <int P, bool STIFF, typename CT>
__global__ __launch_bounds__(256) void asm3_persistent(TaskList tl)
{
    for (int64_t it = blockIdx.x; it < tl.nitems; it += gridDim.x) {
        const int t = task_of(tl.off, tl.ntask, it);
        const BatchTask &T = tl.tasks[t];
        const int64_t l = it - tl.off[t];
        const int bx = (int)(l % T.gx);
        const int64_t r = l / T.gx;
        asm3_block<P, STIFF, CT>(T.pv, (const CT *)T.ws, T.out, 0, T.pv.dir[2].K, T.arg, 0, bx, (int)(r % T.gy),
                                 (int)(r / T.gy));
        __syncthreads();   // LDS of the next block
    }
}

template <int P, bool STIFF, typename CT, int L2M>
static hipError_t launch_asm12_batch_t(const TaskList &tl, int nblocks, hipStream_t s)
{
    {
        hipError_t e = set_asm12_lds<P, STIFF, CT, L2M>((const void *)asm12_persistent<P, STIFF, CT, L2M>);
        if (e != hipSuccess) return e;
    }
    constexpr int NT = A12Shape<P, STIFF, L2M>::NT;
    const size_t lds = a12_lds_bytes<P, STIFF, CT, L2M>();
    hipLaunchKernelGGL((asm12_persistent<P, STIFF, CT, L2M>), dim3(nblocks), dim3(NT), lds, s, tl);
    return hipGetLastError();
}

template <int P, bool STIFF, typename CT>
static hipError_t launch_asm3_batch_t(const TaskList &tl, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL((asm3_persistent<P, STIFF, CT>), dim3(nblocks), dim3(256), 0, s, tl);
    return hipGetLastError();
}

// Level 2 in FP64: on the matrix cores where the full slot tiles win (p = 4,
// 8), on the vector ALU over the stored windows only for the other orders
// (FP64 matrix cores and vector FMA have the same peak on this chip).

template <int P>
static hipError_t launch_batch_p(int which, const TaskList &tl, int op, Prec prec, int nblocks, hipStream_t s)
{
    if (which == 0) {
        if (prec == Prec::F64)
            return op == 2 ? launch_asm12_batch_t<P, true, double, f64_level2<P>()>(tl, nblocks, s)
                           : launch_asm12_batch_t<P, false, double, f64_level2<P>()>(tl, nblocks, s);
        if (prec == Prec::BF16X3)
            return op == 2 ? launch_asm12_batch_t<P, true, float, 2>(tl, nblocks, s)
                           : launch_asm12_batch_t<P, false, float, 2>(tl, nblocks, s);
        return op == 2 ? launch_asm12_batch_t<P, true, float, 0>(tl, nblocks, s)
                       : launch_asm12_batch_t<P, false, float, 0>(tl, nblocks, s);
    }
    if (prec == Prec::F64)
        return op == 2 ? launch_asm3_batch_t<P, true, double>(tl, nblocks, s)
                       : launch_asm3_batch_t<P, false, double>(tl, nblocks, s);
    return op == 2 ? launch_asm3_batch_t<P, true, float>(tl, nblocks, s)
                   : launch_asm3_batch_t<P, false, float>(tl, nblocks, s);
}

static hipError_t launch_batch(int which, const TaskList &tl, int P, int op, Prec prec, int nblocks, hipStream_t s)
{
    if (tl.nitems == 0) return hipSuccess;
    switch (P) {
    case 2: return launch_batch_p<2>(which, tl, op, prec, nblocks, s);
    case 3: return launch_batch_p<3>(which, tl, op, prec, nblocks, s);
    case 4: return launch_batch_p<4>(which, tl, op, prec, nblocks, s);
    case 5: return launch_batch_p<5>(which, tl, op, prec, nblocks, s);
    case 6: return launch_batch_p<6>(which, tl, op, prec, nblocks, s);
    case 7: return launch_batch_p<7>(which, tl, op, prec, nblocks, s);
    case 8: return launch_batch_p<8>(which, tl, op, prec, nblocks, s);
    case 9: return launch_batch_p<9>(which, tl, op, prec, nblocks, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_asm12_batch(const TaskList &tl, int P, int op, Prec prec, int nblocks, hipStream_t s)
{
    return launch_batch(0, tl, P, op, prec, nblocks, s);
}

hipError_t launch_asm3_batch(const TaskList &tl, int P, int op, Prec prec, int nblocks, hipStream_t s)
{
    return launch_batch(1, tl, P, op, prec, nblocks, s);
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

template <int P, typename CT, int L2M>
static hipError_t launch_asm_pt(const PatchView &pv, int op, const void *C, double *vals, void *ws,
                                size_t ws_bytes, hipStream_t s, int t1, int seg)
{
    const CT *c = static_cast<const CT *>(C);
    if (pv.d == 3)
        return op == 2 ? launch_asm3d<P, true, CT, L2M>(pv, c, vals, ws, ws_bytes, s, t1, seg)
                       : launch_asm3d<P, false, CT, L2M>(pv, c, vals, ws, ws_bytes, s, t1, seg);
    return op == 2 ? launch_asm_small<P, true, CT>(pv, c, vals, s) : launch_asm_small<P, false, CT>(pv, c, vals, s);
}

template <int P>
static hipError_t launch_asm_p(const PatchView &pv, int op, Prec prec, const void *C, double *vals, void *ws,
                               size_t ws_bytes, hipStream_t s, int t1, int seg)
{
    if (prec == Prec::F64) return launch_asm_pt<P, double, f64_level2<P>()>(pv, op, C, vals, ws, ws_bytes, s, t1, seg);
    if (prec == Prec::BF16X3) return launch_asm_pt<P, float, 2>(pv, op, C, vals, ws, ws_bytes, s, t1, seg);
    return launch_asm_pt<P, float, 0>(pv, op, C, vals, ws, ws_bytes, s, t1, seg);
}

hipError_t launch_assemble(const PatchView &pv, int op, Prec prec, const void *C, double *vals, void *ws,
                           size_t ws_bytes, hipStream_t s, int t1, int seg)
{
    switch (pv.P) {
    case 2: return launch_asm_p<2>(pv, op, prec, C, vals, ws, ws_bytes, s, t1, seg);
    case 3: return launch_asm_p<3>(pv, op, prec, C, vals, ws, ws_bytes, s, t1, seg);
    case 4: return launch_asm_p<4>(pv, op, prec, C, vals, ws, ws_bytes, s, t1, seg);
    case 5: return launch_asm_p<5>(pv, op, prec, C, vals, ws, ws_bytes, s, t1, seg);
    case 6: return launch_asm_p<6>(pv, op, prec, C, vals, ws, ws_bytes, s, t1, seg);
    case 7: return launch_asm_p<7>(pv, op, prec, C, vals, ws, ws_bytes, s, t1, seg);
    case 8: return launch_asm_p<8>(pv, op, prec, C, vals, ws, ws_bytes, s, t1, seg);
    case 9: return launch_asm_p<9>(pv, op, prec, C, vals, ws, ws_bytes, s, t1, seg);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sfiga
