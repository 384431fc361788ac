// Structural CSR pattern (Sec. 3.2): row m holds every column n whose
// support shares an element with the support of m.  For open knots with
// simple interior knots this is the tensor product of the 1D bands
// [max(0, i-p+1), min(N-1, i+p-1)], so row offsets and column indices have
// closed forms (prefix sums of the 1D band lengths, see RowIndex).
#include "kernels.h"

namespace sfiga {

__device__ __forceinline__ void row_ptr_row(const RowIndex &ri, int64_t nrows, int64_t *row_ptr, int64_t base,
                                            int64_t m)
{
    if (m > nrows) return;
    if (m == nrows) {
        row_ptr[m] = base + ri.T[0] * (ri.d >= 2 ? ri.T[1] : 1) * (ri.d >= 3 ? ri.T[2] : 1);
        return;
    }
    int m0 = (int)(m % ri.N[0]);
    int64_t r = m / ri.N[0];
    int m1 = ri.d >= 2 ? (int)(r % ri.N[1]) : 0;
    int m2 = ri.d >= 3 ? (int)(r / ri.N[1]) : 0;
    row_ptr[m] = base + row_start(ri, m0, m1, m2);
}

__global__ void row_ptr_kernel(RowIndex ri, int64_t nrows, int64_t *row_ptr, int64_t base)
{
    row_ptr_row(ri, nrows, row_ptr, base, blockIdx.x * (int64_t)blockDim.x + threadIdx.x);
}

// One wavefront per row; lanes walk the row's (2p-1)^d band entries.  Rows
// whose band is not clipped in any direction (the bulk) decompose the entry
// index with the compile-time band width; clipped rows with their own lengths.
template <int P>
__device__ __forceinline__ void col_ind_row(const RowIndex &ri, int64_t nrows, int32_t *col_ind, int64_t col_base,
                                            int64_t nnz_base, int64_t m)
{
    constexpr int W = 2 * P - 1;
    const int lane = threadIdx.x % 64;
    if (m >= nrows) return;
    int m0 = (int)(m % ri.N[0]);
    int64_t r = m / ri.N[0];
    int m1 = ri.d >= 2 ? (int)(r % ri.N[1]) : 0;
    int m2 = ri.d >= 3 ? (int)(r / ri.N[1]) : 0;
    const int lo0 = band_lo(m0, P), l0 = band_len(m0, P, ri.N[0]);
    const int lo1 = ri.d >= 2 ? band_lo(m1, P) : 0, l1 = ri.d >= 2 ? band_len(m1, P, ri.N[1]) : 1;
    const int lo2 = ri.d >= 3 ? band_lo(m2, P) : 0, l2 = ri.d >= 3 ? band_len(m2, P, ri.N[2]) : 1;
    const int64_t start = row_start(ri, m0, m1, m2);
    const int len = l0 * l1 * l2;
    int32_t *out = col_ind + nnz_base + start;
    const int64_t N0 = ri.N[0], N01 = (int64_t)ri.N[0] * ri.N[1];
    const int64_t first = col_base + lo0 + N0 * lo1 + N01 * lo2;
    if (ri.d == 3 && l0 == W && l1 == W && l2 == W) {
        for (int t = lane; t < W * W * W; t += 64) {
            const int a = t % W, b = (t / W) % W, c = t / (W * W);
            out[t] = (int32_t)(first + a + N0 * b + N01 * c);
        }
        return;
    }
    for (int t = lane; t < len; t += 64) {
        const int a = t % l0, b = (t / l0) % l1, c = t / (l0 * l1);
        out[t] = (int32_t)(first + a + N0 * b + N01 * c);
    }
}

// Rows per wavefront of the single-patch kernel.  Lane r < CI_ROWS of a
// wavefront works out the position and first column of row row0 + r (the
// prefix-sum loads of all its rows are in flight together); the wavefront then
// writes the rows one after another, taking each row's description from its
// lane by broadcast.
constexpr int CI_ROWS = 16;

template <int P>
__global__ void col_ind_kernel(RowIndex ri, int64_t nrows, int32_t *col_ind, int64_t col_base, int64_t nnz_base)
{
    constexpr int W = 2 * P - 1;
    const int lane = threadIdx.x % 64;
    const int64_t row0 = (blockIdx.x * (int64_t)(blockDim.x / 64) + threadIdx.x / 64) * CI_ROWS;
    if (row0 >= nrows) return;                                   // uniform over the wavefront
    int64_t start = 0, first = 0;
    int dims = 0;                                                // l0 | l1 << 8 | l2 << 16
    if (lane < CI_ROWS && row0 + lane < nrows) {
        const int64_t m = row0 + lane;
        const int m0 = (int)(m % ri.N[0]);
        const int64_t r = m / ri.N[0];
        const int m1 = ri.d >= 2 ? (int)(r % ri.N[1]) : 0;
        const int m2 = ri.d >= 3 ? (int)(r / ri.N[1]) : 0;
        const int lo0 = band_lo(m0, P), l0 = band_len(m0, P, ri.N[0]);
        const int lo1 = ri.d >= 2 ? band_lo(m1, P) : 0, l1 = ri.d >= 2 ? band_len(m1, P, ri.N[1]) : 1;
        const int lo2 = ri.d >= 3 ? band_lo(m2, P) : 0, l2 = ri.d >= 3 ? band_len(m2, P, ri.N[2]) : 1;
        start = nnz_base + row_start(ri, m0, m1, m2);
        first = col_base + lo0 + (int64_t)ri.N[0] * lo1 + (int64_t)ri.N[0] * ri.N[1] * lo2;
        dims = l0 | (l1 << 8) | (l2 << 16);
    }
    const int64_t N0 = ri.N[0], N01 = (int64_t)ri.N[0] * ri.N[1];
    const int nr = nrows - row0 < CI_ROWS ? (int)(nrows - row0) : CI_ROWS;
    for (int k = 0; k < nr; ++k) {
        const int64_t st = __shfl(start, k, 64), fc = __shfl(first, k, 64);
        const int dm = __shfl(dims, k, 64);
        const int l0 = dm & 255, l1 = (dm >> 8) & 255, l2 = dm >> 16;
        int32_t *out = col_ind + st;
        if (ri.d == 3 && l0 == W && l1 == W && l2 == W) {
            for (int t = lane; t < W * W * W; t += 64) {
                const int a = t % W, b = (t / W) % W, c = t / (W * W);
                out[t] = (int32_t)(fc + a + N0 * b + N01 * c);
            }
        } else {
            const int len = l0 * l1 * l2;
            for (int t = lane; t < len; t += 64) {
                const int a = t % l0, b = (t / l0) % l1, c = t / (l0 * l1);
                out[t] = (int32_t)(fc + a + N0 * b + N01 * c);
            }
        }
    }
}

// Persistent forms over the rows of a batch: block bx of a task covers rows
// [256 bx, 256 bx + 256) (row pointers) or [4 bx, 4 bx + 4) (column indices).
__global__ void row_ptr_persistent(TaskList tl)
{
    for (int64_t it = blockIdx.x; it < tl.nitems; it += gridDim.x) {
        const int t = task_of(tl.off, tl.ntask, it);
        const BatchTask &T = tl.tasks[t];
        row_ptr_row(T.pv.ri, T.pv.N, T.row_ptr, T.nnz_base, (it - tl.off[t]) * 256 + threadIdx.x);
    }
}

template <int P>
__global__ void col_ind_persistent(TaskList tl)
{
    for (int64_t it = blockIdx.x; it < tl.nitems; it += gridDim.x) {
        const int t = task_of(tl.off, tl.ntask, it);
        const BatchTask &T = tl.tasks[t];
        col_ind_row<P>(T.pv.ri, T.pv.N, T.col_ind, T.col_base, T.nnz_base, (it - tl.off[t]) * 4 + threadIdx.x / 64);
    }
}

hipError_t launch_rowptr_batch(const TaskList &tl, int nblocks, hipStream_t s)
{
    if (tl.nitems == 0) return hipSuccess;
    hipLaunchKernelGGL(row_ptr_persistent, dim3(nblocks), dim3(256), 0, s, tl);
    return hipGetLastError();
}

hipError_t launch_colind_batch(const TaskList &tl, int P, int nblocks, hipStream_t s)
{
    if (tl.nitems == 0) return hipSuccess;
    dim3 g(nblocks), b(256);
    switch (P) {
    case 2: hipLaunchKernelGGL(col_ind_persistent<2>, g, b, 0, s, tl); break;
    case 3: hipLaunchKernelGGL(col_ind_persistent<3>, g, b, 0, s, tl); break;
    case 4: hipLaunchKernelGGL(col_ind_persistent<4>, g, b, 0, s, tl); break;
    case 5: hipLaunchKernelGGL(col_ind_persistent<5>, g, b, 0, s, tl); break;
    case 6: hipLaunchKernelGGL(col_ind_persistent<6>, g, b, 0, s, tl); break;
    case 7: hipLaunchKernelGGL(col_ind_persistent<7>, g, b, 0, s, tl); break;
    case 8: hipLaunchKernelGGL(col_ind_persistent<8>, g, b, 0, s, tl); break;
    case 9: hipLaunchKernelGGL(col_ind_persistent<9>, g, b, 0, s, tl); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Values of a d = 3 matrix assembled with its directions relabelled
// cyclically (direction k of the relabelled patch is direction (k + sh) mod 3
// of this one), moved into this patch's CSR layout: entry (m, n) here is
// entry (pi(m), pi(n)) there.  One wavefront per row, lanes over its entries
// (stores contiguous, loads gathered).
__global__ __launch_bounds__(256) void gather_cyclic_kernel(RowIndex ri, RowIndex rp, int sh,
                                                            const double *__restrict__ tmp, double *__restrict__ vals,
                                                            int64_t N)
{
    const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (row >= N) return;
    const int lane = threadIdx.x % 64, P = ri.P;
    int m[3];
    m[0] = (int)(row % ri.N[0]);
    m[1] = (int)((row / ri.N[0]) % ri.N[1]);
    m[2] = (int)(row / ((int64_t)ri.N[0] * ri.N[1]));
    int lo[3], len[3], mp[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = band_lo(m[k], P);
        len[k] = band_len(m[k], P, ri.N[k]);
    }
    for (int k = 0; k < 3; ++k) mp[k] = m[(k + sh) % 3];
    const int64_t base = row_start(ri, m[0], m[1], m[2]);
    const int64_t basep = row_start(rp, mp[0], mp[1], mp[2]);
    const int total = len[0] * len[1] * len[2];
    for (int off = lane; off < total; off += 64) {
        int n[3];
        n[0] = lo[0] + off % len[0];
        n[1] = lo[1] + (off / len[0]) % len[1];
        n[2] = lo[2] + off / (len[0] * len[1]);
        const int np0 = n[sh % 3], np1 = n[(1 + sh) % 3], np2 = n[(2 + sh) % 3];
        vals[base + off] = tmp[basep + col_offset(rp, mp[0], mp[1], mp[2], np0, np1, np2)];
    }
}

hipError_t launch_gather_cyclic(const PatchView &pv, const PatchView &alt, int sh, const double *tmp, double *vals,
                                hipStream_t s)
{
    if (pv.d != 3) return hipErrorInvalidValue;
    const int64_t nb = (pv.N + 3) / 4;
    hipLaunchKernelGGL(gather_cyclic_kernel, dim3((unsigned)nb), dim3(256), 0, s, pv.ri, alt.ri, sh, tmp, vals, pv.N);
    return hipGetLastError();
}

__global__ void fill_kernel(double *y, int64_t n, double v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = v;
}

hipError_t launch_fill(double *y, int64_t n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)nb), dim3(256), 0, s, y, n, v);
    return hipGetLastError();
}

// Glued multipatch (Sec. 4, Example "Multipatch domains"): patch-local
// vectors from the global one and back, y = sum_b R_b^T (A_b R_b x).
// Map entries outside [0, ng) are not followed (the local value is 0, the
// result is dropped).
__global__ void glue_gather_kernel(const int64_t *__restrict__ map, int64_t n, int64_t ng,
                                   const double *__restrict__ xg, double *__restrict__ xl)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = map[i];
        xl[i] = (j >= 0 && j < ng) ? xg[j] : 0.0;
    }
}

__global__ void glue_scatter_kernel(const int64_t *__restrict__ map, int64_t n, int64_t ng,
                                    const double *__restrict__ yl, double *__restrict__ yg)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = map[i];
        if (j >= 0 && j < ng) atomicAdd(&yg[j], yl[i]);
    }
}

static unsigned grid_of(int64_t n)
{
    const int64_t nb = (n + 255) / 256;
    return (unsigned)(nb > 65536 ? 65536 : (nb < 1 ? 1 : nb));
}

hipError_t launch_glue_gather(const int64_t *map, int64_t n, int64_t ng, const double *xg, double *xl, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(glue_gather_kernel, dim3(grid_of(n)), dim3(256), 0, s, map, n, ng, xg, xl);
    return hipGetLastError();
}

hipError_t launch_glue_scatter(const int64_t *map, int64_t n, int64_t ng, const double *yl, double *yg, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(glue_scatter_kernel, dim3(grid_of(n)), dim3(256), 0, s, map, n, ng, yl, yg);
    return hipGetLastError();
}

hipError_t launch_pattern(const PatchView &pv, int64_t *row_ptr, int32_t *col_ind, int64_t row_base,
                          int64_t col_base, int64_t nnz_base, hipStream_t s)
{
    // row_ptr gets the entries of this patch at [row_base, row_base + N], values offset by nnz_base
    if (row_ptr) {
        int64_t nb = (pv.N + 1 + 255) / 256;
        hipLaunchKernelGGL(row_ptr_kernel, dim3((unsigned)nb), dim3(256), 0, s, pv.ri, pv.N, row_ptr + row_base,
                           nnz_base);
    }
    if (col_ind) {
        const int64_t per_block = 4 * CI_ROWS;                   // 4 wavefronts of CI_ROWS rows
        int64_t nb = (pv.N + per_block - 1) / per_block;
        dim3 g((unsigned)nb), b(256);
        switch (pv.P) {
        case 2: hipLaunchKernelGGL(col_ind_kernel<2>, g, b, 0, s, pv.ri, pv.N, col_ind, col_base, nnz_base); break;
        case 3: hipLaunchKernelGGL(col_ind_kernel<3>, g, b, 0, s, pv.ri, pv.N, col_ind, col_base, nnz_base); break;
        case 4: hipLaunchKernelGGL(col_ind_kernel<4>, g, b, 0, s, pv.ri, pv.N, col_ind, col_base, nnz_base); break;
        case 5: hipLaunchKernelGGL(col_ind_kernel<5>, g, b, 0, s, pv.ri, pv.N, col_ind, col_base, nnz_base); break;
        case 6: hipLaunchKernelGGL(col_ind_kernel<6>, g, b, 0, s, pv.ri, pv.N, col_ind, col_base, nnz_base); break;
        case 7: hipLaunchKernelGGL(col_ind_kernel<7>, g, b, 0, s, pv.ri, pv.N, col_ind, col_base, nnz_base); break;
        case 8: hipLaunchKernelGGL(col_ind_kernel<8>, g, b, 0, s, pv.ri, pv.N, col_ind, col_base, nnz_base); break;
        default: hipLaunchKernelGGL(col_ind_kernel<9>, g, b, 0, s, pv.ri, pv.N, col_ind, col_base, nnz_base); break;
        }
    }
    return hipGetLastError();
}

}  // namespace sfiga
