// Launch descriptors shared between the host glue (sfiga.cpp) and the HIP
// kernel translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "common.h"

namespace sfiga {

enum class Prec { F64 = 0, F32 = 1 };

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
    double *xyz;           // [Q][d] physical quadrature points, or null
    Coef coef_mass, coef_stiff;
    int *bad_det;          // device flag set to 1 if det J <= 0 somewhere
    Prec prec;
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

hipError_t launch_geometry(const PatchView &pv, const GeomOut &out, hipStream_t s);
hipError_t launch_pattern(const PatchView &pv, int64_t *row_ptr, int32_t *col_ind, int64_t row_base,
                          int64_t col_base, int64_t nnz_base, hipStream_t s);
hipError_t launch_fill(double *y, int64_t n, double v, hipStream_t s);
// op: 1 mass, 2 stiffness; c: coefficient tensor of that op at prec
hipError_t launch_apply(const PatchView &pv, int op, Prec prec, const void *c, const double *x, double *y,
                        hipStream_t s);
// ws: device workspace of ws_bytes for the d = 3 level-2 partials (see
// assemble_workspace_bytes; unused for d <= 2)
hipError_t launch_assemble(const PatchView &pv, int op, Prec prec, const void *c, double *vals, void *ws,
                           size_t ws_bytes, hipStream_t s);
// workspace of the d = 3 assembly of op at prec: whole patch if it fits in
// cap bytes, else chunks of element layers (never fewer than p - 1)
size_t assemble_workspace_bytes(const PatchView &pv, int op, Prec prec, size_t cap);

}  // namespace sfiga
