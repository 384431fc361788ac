// Launch descriptors shared between the host glue (sfiga.cpp) and the HIP
// kernel translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "common.h"

namespace sfiga {

// F64, F32: every contraction in that type; BF16X3: FP32 coefficients and level 1,
// level 2 of the assembly on bf16 matrix cores with hi/lo split operands and
// FP32 accumulation (level 3 and the values stay FP64); F16S: the apply with
// the coefficients stored as an FP32 reference and scale per element and an
// FP16 residual per point, contractions in FP32.
enum class Prec { F64 = 0, F32 = 1, BF16X3 = 2, F16S = 3 };

// Element tile of the d = 3 tile kernels in directions 1 and 2: about 32 x 16
// quadrature points per workgroup (one thread per quadrature column).
template <int P>
struct Tile {
    static constexpr int E1 = (32 + P - 1) / P;
    static constexpr int E2 = (16 + P - 1) / P;
    static constexpr int TX = E1 * P, TY = E2 * P;           // quadrature points
    static constexpr int NX = E1 + P - 1, NY = E2 + P - 1;   // functions
    static constexpr int NT = TX * TY;
};

// Elements per direction of the matrix-free apply's tile in directions 1 and
// 2 (about 16 x 16 quadrature columns per workgroup).
__host__ __device__ constexpr int apply_tile_elems(int P) { return (16 + P - 1) / P; }

// FP16-split storage of a coefficient tensor (used by the apply only), laid
// out tile-major so that one apply workgroup reads each of its planes as one
// contiguous block: [q3][comp][tile_y][tile_x][ty][tx], tiles of
// T = apply_tile_elems(P) * P points per direction (edge tiles padded).
__host__ __device__ inline int64_t split_index(int ncomp, int comp, int q0, int q1, int q2, int P, int K0, int K1)
{
    const int T = apply_tile_elems(P) * P;
    const int gx = (K0 * P + T - 1) / T, gy = (K1 * P + T - 1) / T;
    const int bx = q0 / T, by = q1 / T;
    return ((((int64_t)q2 * ncomp + comp) * gy + by) * gx + bx) * T * T + (q1 - by * T) * T + (q0 - bx * T);
}
__host__ __device__ inline int64_t split_size(int ncomp, int P, int K0, int K1, int K2)
{
    const int T = apply_tile_elems(P) * P;
    const int64_t gx = (K0 * P + T - 1) / T, gy = (K1 * P + T - 1) / T;
    return (int64_t)K2 * P * ncomp * gy * gx * T * T;
}

// Coefficient layout of the apply's element-row kernel (d = 3), tile by
// tile: for each tile of T x T quadrature columns (T = apply_tile_elems(P) *
// P; tiles in directions 1 and 2, direction 1 fastest), each quadrature plane
// q3 and each pair of components, the tile's columns (row ty, column tx) with
// the two components of a pair side by side (one component for the mass
// operator).  A workgroup then reads one contiguous block per layer, two
// values per load.  Columns outside the patch hold 0.
__host__ __device__ inline int apply_coef_width(int ncomp) { return ncomp > 1 ? 2 : 1; }
__host__ __device__ inline int64_t apply_coef_index(int ncomp, int comp, int q0, int q1, int q2, int P, int K0, int Q2)
{
    const int T = apply_tile_elems(P) * P, W = apply_coef_width(ncomp);
    const int gx = (K0 * P + T - 1) / T;
    const int bx = q0 / T, by = q1 / T;
    const int64_t tile = (int64_t)by * gx + bx;
    return (((tile * Q2 + q2) * (ncomp / W) + comp / W) * (T * T) + (int64_t)(q1 - by * T) * T + (q0 - bx * T)) * W +
           comp % W;
}
__host__ __device__ inline int64_t apply_coef_size(int ncomp, int P, int K0, int K1, int K2)
{
    const int T = apply_tile_elems(P) * P;
    const int64_t gx = (K0 * P + T - 1) / T, gy = (K1 * P + T - 1) / T;
    return gx * gy * (int64_t)K2 * P * ncomp * T * T;
}

// Elements per tile side of the convection kernel (d = 3): about 16
// quadrature points per side up to order 6, two elements at orders 7 and 8
// and one at order 9 (measured fastest; LDS at most about 63 KiB).
__host__ __device__ constexpr int conv_tile_elems(int P) { return P <= 6 ? (16 + P - 1) / P : (P <= 8 ? 2 : 1); }

// Convection coefficient layout (d = 3): tiles of T x T quadrature columns
// (T = conv_tile_elems(P) * P; direction 1 fastest), per tile and quadrature
// plane q3 the three components one after another, each the tile's columns
// (row ty, column tx).  Columns outside the patch hold 0.
__host__ __device__ inline int64_t conv_coef_index(int comp, int q0, int q1, int q2, int P, int K0, int Q2)
{
    const int T = conv_tile_elems(P) * P;
    const int gx = (K0 * P + T - 1) / T;
    const int bx = q0 / T, by = q1 / T;
    const int64_t tile = (int64_t)by * gx + bx;
    return ((tile * Q2 + q2) * 3 + comp) * (T * T) + (int64_t)(q1 - by * T) * T + (q0 - bx * T);
}
__host__ __device__ inline int64_t conv_coef_size(int P, int K0, int K1, int K2)
{
    const int T = conv_tile_elems(P) * P;
    const int64_t gx = (K0 * P + T - 1) / T, gy = (K1 * P + T - 1) / T;
    return gx * gy * (int64_t)K2 * P * 3 * T * T;
}

struct PatchView {
    int d, P;
    Dir dir[3];            // unused directions: K = N = Q = 1, tables null
    RowIndex ri;
    const double *ctrl;    // [N][d]
    int64_t N, Q, nnz;
};

// Geometry step output for one operator set.
struct GeomOut {
    void *c_mass;          // [Q] (layout: see coef_index), Prec element type, or null
    void *c_stiff;         // [Q][ncomp], or null
    void *ca_mass;         // the same in the apply's tiled layout (apply_coef_index, d = 3), or null
    void *ca_stiff;
    double *xyz;           // [Q][d] physical quadrature points, or null
    double *c_conv;        // convection, FP64 in the layout of conv_coef_index (d = 3), or null
    Coef coef_mass, coef_stiff, coef_conv;
    double bconv[3];       // the convection vector b (scaled by coef_conv)
    double adiff[9];       // the symmetric diffusion matrix A, row-major (stiffness: a(x) A)
    int *bad_det;          // device flag set to 1 if det J <= 0 somewhere, or null
    Prec prec;
    // evaluation of a discrete function u = sum_n u_n phi_n (Algorithm 3):
    const double *u;       // [N] coefficients, or null (no evaluation)
    double *uval;          // [Q] u at the quadrature points, or null
    double *ugrad;         // [Q][d] physical gradient J^-T grad_hat u, or null
};

// Quadrature-coefficient tensor layout: C[q_d][comp][q_{d-1}]..[q_1]
// (outermost quadrature direction, then component, then the rest with
// direction 1 fastest), so that a plane of constant q_d holds every
// component contiguously for the streaming kernels.
__host__ __device__ inline int64_t coef_index(int d, int ncomp, int comp, int q0, int q1, int q2, int Q0, int Q1)
{
    if (d == 1) return (int64_t)q0 * ncomp + comp;
    if (d == 2) return ((int64_t)q1 * ncomp + comp) * Q0 + q0;
    return (((int64_t)q2 * ncomp + comp) * Q1 + q1) * Q0 + q0;
}

// One patch's share of a batched launch: the arguments of the per-patch
// kernel and its block grid.  A persistent kernel walks the blocks of all
// tasks of one kind and order in task order (largest first).
struct BatchTask {
    PatchView pv;
    const void *C;         // coefficient tensor of the operator at the precision
    const float *rs;       // per-element reference and scale (FP16-split storage)
    void *ws;              // level-2 workspace of the assembly
    double *out;           // assembly values or y, offset to the patch
    const double *x;       // apply input, offset to the patch
    int64_t *row_ptr;      // pattern: the patch's row pointer entries
    int32_t *col_ind;      // pattern: whole column index array
    int64_t col_base, nnz_base;
    int gx, gy, gz;        // blocks of the per-patch launch
    int arg;               // rows per tile (levels 1-2), rows per segment (level 3), layers (apply)
};

struct TaskList {
    const BatchTask *tasks;    // device
    const int64_t *off;        // device, [ntask + 1] prefix sums of gx gy gz
    int ntask;
    int64_t nitems;
};

// task of block `it` (binary search in the prefix sums)
__device__ __forceinline__ int task_of(const int64_t *off, int ntask, int64_t it)
{
    int lo = 0, hi = ntask - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= it) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Raise the dynamic LDS limit of kernel `fn` to `bytes` on the current
// device, once per (device, kernel); thread safe.  Needed above 64 KiB.
hipError_t allow_dynamic_lds(const void *fn, size_t bytes);

// Workgroups are dealt to the 8 XCDs in turn (linear id mod 8), each XCD with
// its own L2.  xcd_tile gives every XCD a contiguous range of tiles instead
// (direction 1 fastest), so that neighbouring tiles, which share cache lines
// of their inputs or outputs, run on one XCD at about the same time and meet
// in its L2.
__device__ __forceinline__ void xcd_tile(int &bx, int &by, int &bz)
{
    const int gx = gridDim.x, gy = gridDim.y;
    const int nb = gx * gy * gridDim.z;
    const int b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const int q = nb / 8, r = nb % 8, x = b % 8;
    const int t = x * q + min(x, r) + b / 8;
    bx = t % gx;
    by = (t / gx) % gy;
    bz = t / (gx * gy);
}

hipError_t launch_geometry(const PatchView &pv, const GeomOut &out, hipStream_t s);
hipError_t launch_pattern(const PatchView &pv, int64_t *row_ptr, int32_t *col_ind, int64_t row_base,
                          int64_t col_base, int64_t nnz_base, hipStream_t s);
hipError_t launch_fill(double *y, int64_t n, double v, hipStream_t s);
// glued multipatch vectors: xl[i] = xg[map[i]] and yg[map[i]] += yl[i]
// (FP64 atomics), i < n, for map entries in [0, ng) (the length of xg and
// yg); other entries give xl[i] = 0 and add nothing
hipError_t launch_glue_gather(const int64_t *map, int64_t n, int64_t ng, const double *xg, double *xl, hipStream_t s);
hipError_t launch_glue_scatter(const int64_t *map, int64_t n, int64_t ng, const double *yl, double *yg, hipStream_t s);
// Values assembled on `alt`, the d = 3 patch pv with its directions relabelled
// cyclically (alt direction k = pv direction (k + sh) mod 3), moved into pv's
// CSR layout (tmp: alt's values, vals: pv's).
hipError_t launch_gather_cyclic(const PatchView &pv, const PatchView &alt, int sh, const double *tmp, double *vals,
                                hipStream_t s);
// op: 1 mass, 2 stiffness; c: coefficient tensor of that op at prec
// lz: element layers per workgroup in direction 3 (0 = default)
// rs: per-element reference and scale of the F16S storage (null otherwise)
// tiled: c is in the tiled layout of apply_coef_index (only where
// apply_tiled_layout says the kernel reads it), else in the layout of coef_index
hipError_t launch_apply(const PatchView &pv, int op, Prec prec, const void *c, const double *x, double *y,
                        hipStream_t s, int lz = 0, const float *rs = nullptr, bool tiled = false);
// true if the d = 3 apply of op at prec and order P reads its coefficients
// in the tiled layout (the geometry step then writes that copy as well)
bool apply_tiled_layout(int P, int op, Prec prec);
// Convection product y = B x (d = 3, FP64): cv the folded coefficients
// (conv_coef_index layout); y is overwritten.
hipError_t launch_conv_apply(const PatchView &pv, const double *cv, const double *x, double *y, hipStream_t s);
// F16S storage from the FP32 coefficient tensor c32 of op (d = 3): per element
// and component the reference r = (max + min) / 2 and scale s = (max - min) / 2
// of C / w over the element's points (rs [K3][K2][K1][ncomp][2]), and per point
// h = (C / w - r) / s rounded to FP16 (h16, split_index layout, split_size
// values; padding 0), w the product of the point's Gauss weights.
hipError_t launch_split_coef(const PatchView &pv, int op, const float *c32, void *h16, float *rs, hipStream_t s);
// ws: device workspace of ws_bytes for the d = 3 level-2 partials (see
// assemble_workspace_bytes; unused for d <= 2)
// t1 (rows m1 per level-1/2 tile) and seg (rows m3 per level-3 segment)
// are tile parameters (0 = default); they do not change the values.
hipError_t launch_assemble(const PatchView &pv, int op, Prec prec, const void *c, double *vals, void *ws,
                           size_t ws_bytes, hipStream_t s, int t1 = 0, int seg = 0);
// workspace of the d = 3 assembly of op at prec: whole patch if it fits in
// cap bytes, else chunks of element layers (never fewer than p - 1)
size_t assemble_workspace_bytes(const PatchView &pv, int op, Prec prec, size_t cap);
// true if the workspace holds the whole patch (one chunk)
bool assemble_single_chunk(const PatchView &pv, int op, Prec prec, size_t ws_bytes);
// smallest workspace the d = 3 assembly runs with (p - 1 element layers)
size_t assemble_min_workspace_bytes(const PatchView &pv, int op, Prec prec);
// Size of the fixed per-device scratch of the assembly entry point that
// allocates nothing, and its device address on the current device (looked up
// once per device).
constexpr size_t kNoAllocScratchBytes = size_t(256) << 20;
hipError_t noalloc_scratch(void **ptr);

// Batched (persistent) kernels of one order P; nblocks = workgroups of the
// persistent grid.  Block shapes of one task for the tunable parameter
// (0 = the single-patch default):
void asm12_blocks(const PatchView &pv, Prec prec, int t1, int &gx, int &gy, int &T1r);   // t1: rows m1 per tile
void asm3_blocks(const PatchView &pv, int seg, int &gx, int &gy, int &gz, int &L);  // seg: rows m3 per segment
void apply_blocks(const PatchView &pv, int lz, int &gx, int &gy, int &gz, int &LZ);  // lz: layers per workgroup
int asm12_max_rows(int P, Prec prec);
hipError_t launch_asm12_batch(const TaskList &tl, int P, int op, Prec prec, int nblocks, hipStream_t s);
hipError_t launch_asm3_batch(const TaskList &tl, int P, int op, Prec prec, int nblocks, hipStream_t s);
hipError_t launch_apply_batch(const TaskList &tl, int P, int op, Prec prec, int nblocks, hipStream_t s);
hipError_t launch_rowptr_batch(const TaskList &tl, int nblocks, hipStream_t s);
hipError_t launch_colind_batch(const TaskList &tl, int P, int nblocks, hipStream_t s);

}  // namespace sfiga
