/*
 * sfiga.h - sum-factorized isogeometric assembly and matrix-free apply on
 * AMD Instinct MI355X (gfx950).
 *
 * The problem statement follows Bressan & Takacs, "Sum factorization
 * techniques in Isogeometric Analysis":
 *   - tensor-product B-spline bases of order p (= degree + 1) over open knot
 *     vectors, one per direction (Sec. 3.1, eq. (prelim-tp); Corollary on
 *     #NZ for open knot vectors in Sec. 3.2);
 *   - tensor-product Gauss quadrature with p points per element and
 *     direction (Sec. 3.2, Example "Gauss quadrature");
 *   - a geometry map G = sum_n c_n phi_n given by control points (Sec. 6.3);
 *   - the mass and stiffness forms of the convection-diffusion pull-back
 *     (Sec. 2, Example 1), discretised as the quadrature sum
 *     eq. (quadrature:1):
 *        M[m][n] = sum_x w(x) c(G(x)) |det J| phi_n phi_m
 *        K[m][n] = sum_x w(x) a(G(x)) |det J| (J^-T grad phi_n).A (J^-T grad phi_m)
 *     with J_ik = dG_i/dxhat_k and A a constant symmetric matrix (default I);
 *   - the convection form of the same example, the b . grad u term of the
 *     equation tested with v (d = 3, FP64, matrix-free apply only):
 *        B[m][n] = sum_x w(x) s(G(x)) |det J| (b . J^-T grad phi_n) phi_m
 *     with a constant vector b and a scalar coefficient s; B is not
 *     symmetric (the derivative falls on the trial function n);
 *   - outputs: the matrix in CSR form (global sum factorization, Algorithm 1)
 *     or the product y = A x (matrix-free, Algorithms 2 and 3).
 *
 * Index conventions (Sec. 3.1): all multi-indices are flattened
 * lexicographically with direction 1 fastest, n = i1 + N1*(i2 + N2*i3).
 * Rows are test functions m, columns trial functions n.  The CSR pattern is
 * the structural one of Sec. 3.2 (pairs whose supports share an element),
 * explicit zeros included, columns ascending; it is shared by the mass and
 * stiffness matrices (Note after the definition of NZ).
 *
 * Supported: d = 1, 2, 3; one order p in 2..9 for all directions (the
 * descriptor carries one order per direction; unequal orders are
 * SF_EUNSUPPORTED); open knot
 * vectors with simple interior knots (maximal smoothness), any spacing.
 * Other inputs return SF_EUNSUPPORTED.
 *
 * Memory and streams.  Every pointer documented as "device" is HIP device
 * memory owned by the caller (typically a torch tensor).  The library owns
 * its internal workspace (1D tables, coefficient tensor, scratch) and frees
 * it in the matching destroy call.  All work is enqueued on the context's
 * stream and is asynchronous with respect to the host, except where a
 * function is documented to synchronise.
 *
 * Errors.  Every function returns sf_status; no C++ exception crosses the
 * ABI.  On error the outputs are unspecified, the handles stay valid and
 * sf_last_error() describes the failure.  Handles are not thread safe: one
 * host thread at a time per context.
 */
#ifndef SFIGA_H
#define SFIGA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SF_OK = 0,
    SF_EINVAL = -1,        /* bad argument: NULL pointer, size or enum out of range */
    SF_EKNOT = -2,         /* knot vector not open / not nondecreasing / too short */
    SF_EGEOM = -3,         /* det J <= 0 at some quadrature point */
    SF_ENOMEM = -4,        /* device allocation failed */
    SF_EDEVICE = -5,       /* HIP runtime error */
    SF_EUNSUPPORTED = -6   /* valid input outside the supported set listed above */
} sf_status;

typedef enum {
    SF_FP64 = 0,           /* coefficient tensor and contractions in FP64 */
    SF_FP32 = 1,           /* coefficient tensor and contractions in FP32, FP64 output */
    SF_BF16_SPLIT = 2,     /* assembly only: FP32 coefficient tensor and first contraction
                              level; the second level of the d = 3 assembly on bf16 matrix
                              cores, every operand split x = hi + lo (bf16) and the
                              products hi*hi + hi*lo + lo*hi accumulated in FP32; the
                              last level and the values in FP64 (measured error
                              < 5e-6 of max |A|); d <= 2 run FP32.  sf_apply and
                              sf_batch_apply return SF_EUNSUPPORTED. */
    SF_FP16_SPLIT = 3      /* matrix-free apply only (d = 3): the folded coefficient
                              tensor stored split, per element and component an FP32
                              reference r and scale s, per quadrature point an FP16
                              residual h, C = w (r + s h) with w the product of the
                              point's Gauss weights (2 bytes per component instead of
                              8); contractions in FP32.  Each stored coefficient is
                              within 2^-12 s w of the FP32 one.  sf_patch_prepare at
                              this precision also prepares SF_FP32; the assembly
                              entry points return SF_EUNSUPPORTED. */
} sf_precision;

/* operator bit flags (SF_CONV: the convection form, accepted by
 * sf_patch_set_coef, sf_patch_prepare and sf_apply only) */
enum { SF_MASS = 1u, SF_STIFF = 2u, SF_CONV = 4u };

typedef enum {
    SF_COEF_CONST = 0,     /* params[0] = constant value */
    SF_COEF_SINPROD = 1,   /* 1 + params[0] * prod_i sin(2 pi x_i), x = G(xhat) physical */
    SF_COEF_QPVALUES = 2   /* values at the quadrature points, device [Q], lexicographic,
                              quadrature direction 1 fastest (see sf_patch_quad_points) */
} sf_coef_kind;

typedef struct sf_ctx sf_ctx;
typedef struct sf_patch sf_patch;
typedef struct sf_batch sf_batch;

/* ------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * borrowed from the caller (NULL = the legacy default stream); it must
 * outlive the context.  *out receives the handle.  Makes `device` the calling
 * host thread's current HIP device (hipSetDevice); the library does not
 * switch devices afterwards, so calls on the context and its patches and
 * batches must be made while that device is current. */
sf_status sf_ctx_create(int device, void *hip_stream, sf_ctx **out);

/* Destroy a context.  All patches and batches created on it must have been
 * destroyed first.  NULL is accepted. */
void sf_ctx_destroy(sf_ctx *ctx);

/* Message of the last failed call on this context ("" if none).  The string
 * is owned by the context and valid until the next call on it. */
const char *sf_last_error(const sf_ctx *ctx);

/* Name of the device code object the library was built for ("gfx950"). */
const char *sf_build_target(void);

/* Host-only: the 1D tables the kernels use for one direction (Sec. 6.1),
 * without a device.  Validates the knot vector like sf_patch_create and
 * writes, for the K elements (K = n_knots - 2 order + 1), the Gauss points
 * x[K][p], weights w[K][p] (p = order points per element) and the values and
 * derivatives B[K][p][p], D[K][p][p] of the p active B-splines (element e
 * activates functions e .. e+p-1).  Host pointers; any output may be NULL;
 * *nel receives K.  Returns SF_EKNOT / SF_EUNSUPPORTED like sf_patch_create. */
sf_status sf_host_tables_1d(const double *knots, int64_t n_knots, int order, int *nel, double *x, double *w,
                            double *B, double *D);

/* --------------------------------------------------------------- patch */

/* One tensor-product patch: the inputs of Algorithms 1-3 in the IGA setting
 * of Sec. 6.3.  knots[k] (host, n_knots[k] doubles) is the open knot vector
 * of direction k+1; ctrl points to the control points c_n, [N][d] FP64,
 * lexicographic with direction 1 fastest; ctrl_on_device selects whether it
 * is a device or a host pointer.  Both are copied at create time. */
typedef struct {
    int d;                      /* 1..3 */
    int order[3];               /* p_k = degree + 1 of direction k+1, 2..9 (Sec. 3.2 lets
                                   every direction have its own order); the kernels
                                   take one order for all directions: orders that
                                   differ among the first d entries return
                                   SF_EUNSUPPORTED; entries k >= d are ignored */
    int64_t n_knots[3];
    const double *knots[3];
    const double *ctrl;
    int ctrl_on_device;
} sf_patch_desc;

/* Validate the knot vectors (SF_EKNOT), build the 1D Gauss tables (Sec. 6.1)
 * on the device and copy the control points.  Enqueues uploads on the
 * context stream and synchronises once. */
sf_status sf_patch_create(sf_ctx *ctx, const sf_patch_desc *desc, sf_patch **out);

/* Sizes needed to allocate outputs: number of basis functions N, number of
 * structural nonzeros (exactly prod_k (N_k (2p-1) - p (p-1)), Corollary on
 * #NZ), number of quadrature points Q.  Any pointer may be NULL. */
sf_status sf_patch_info(const sf_patch *patch, int64_t *ndof, int64_t *nnz, int64_t *nquad);

/* Coefficient of operator `op` (exactly one of SF_MASS, SF_STIFF, SF_CONV):
 * the reaction coefficient c for the mass form, the scalar diffusion a for
 * the stiffness form (Example 1 with A = a A0, A0 from sf_patch_set_diffusion), the scalar s of the
 * convection velocity s(x) b.  For SF_COEF_CONST and SF_COEF_SINPROD
 * `params` is a host pointer to one double; for SF_COEF_QPVALUES it is a
 * device pointer to Q doubles, which must stay valid until the next
 * sf_patch_prepare.  Default: constant 1 for all three. */
sf_status sf_patch_set_coef(sf_patch *patch, unsigned op, sf_coef_kind kind, const double *params);

/* The constant symmetric diffusion matrix A of the stiffness form (Sec. 2,
 * Example 1: the diffusion becomes a(x) A, a from sf_patch_set_coef): host
 * pointer to the d(d+1)/2 entries of its upper triangle, row by row (d = 3:
 * A11 A12 A13 A22 A23 A33).  Physical coordinates; the geometry step folds
 * w a |det J| J^-1 A J^-T.  A positive definite A gives an elliptic form
 * (not checked).  Default the identity.  Takes effect at the next
 * sf_patch_prepare of SF_STIFF (the stiffness is unprepared until then). */
sf_status sf_patch_set_diffusion(sf_patch *patch, const double *A);

/* The constant vector b of the convection form (Sec. 2, Example 1: the
 * b . grad u term), host pointer to d doubles in physical coordinates;
 * the velocity is s(x) b with s set by sf_patch_set_coef(SF_CONV).
 * Default b = 0.  Takes effect at the next sf_patch_prepare of SF_CONV. */
sf_status sf_patch_set_convection(sf_patch *patch, const double *b);

/* Physical coordinates G(x) of all quadrature points, device [Q][d],
 * lexicographic with quadrature direction 1 fastest (for SF_COEF_QPVALUES
 * users).  Asynchronous. */
sf_status sf_patch_quad_points(sf_patch *patch, double *dev_xyz);

/* Evaluation of a discrete function u = sum_n u_n phi_n at every quadrature
 * point by sum factorization (Sec. 6.2, Algorithm 3: the contractions run
 * direction by direction over the tensor grid of points, cost p^{d+1} per
 * point instead of p^{2d}), with its physical gradient J^-T grad_hat u, where
 * the Jacobian of the geometry map is evaluated in the same pass.  dev_u
 * (device, [N] FP64, lexicographic) holds the coefficients u_n; dev_val
 * (device, [Q]) receives u and dev_grad (device, [Q][d]) the gradient, both
 * lexicographic with quadrature direction 1 fastest (the point order of
 * sf_patch_quad_points); either output may be NULL, not both.  Independent of
 * sf_patch_prepare (no coefficient tensor is touched, no det J record).
 * Asynchronous. */
sf_status sf_patch_eval(sf_patch *patch, const double *dev_u, double *dev_val, double *dev_grad);

/* Geometry step (Sec. 6.3): evaluates G and its Jacobian at all quadrature
 * points by sum factorization (Algorithm 3), and folds weight, coefficient,
 * |det J| and J^-1 J^-T into the quadrature-coefficient tensor of each
 * operator in `ops`, stored at `prec` (SF_CONV: w s |det J| J^-1 b, three
 * components per point, d = 3 and SF_FP64 only, else SF_EUNSUPPORTED).
 * Synchronises once and returns SF_EGEOM if det J <= 0 anywhere.  Must
 * precede assemble/apply of an operator at a precision; repeating it is
 * allowed (recomputes). */
sf_status sf_patch_prepare(sf_patch *patch, unsigned ops, sf_precision prec);

/* sf_patch_prepare without the synchronisation (Sec. 6.3, as above): queues
 * the geometry kernel on the patch's stream and returns; the operators count
 * as prepared at once, so assemble/apply may follow on the same stream.  The
 * det J <= 0 test is still made at every quadrature point; its outcome stays
 * on the device and accumulates over calls until sf_patch_geometry_check
 * reports it (sf_patch_prepare clears it).  Argument errors are returned as
 * by sf_patch_prepare; a det J failure is not. */
sf_status sf_patch_prepare_async(sf_patch *patch, unsigned ops, sf_precision prec);

/* Outcome of the det J test of every sf_patch_prepare_async since the last
 * check: SF_OK, or SF_EGEOM if det J <= 0 was seen anywhere.  Synchronises
 * the patch's stream and clears the recorded outcome. */
sf_status sf_patch_geometry_check(sf_patch *patch);

/* Structural CSR pattern (Sec. 3.2): dev_row_ptr [N+1] int64 and
 * dev_col_ind [nnz] int32, device.  Requires N < 2^31.  Asynchronous. */
sf_status sf_csr_pattern(sf_patch *patch, int64_t *dev_row_ptr, int32_t *dev_col_ind);

/* Global sum-factorized assembly (Algorithm 1) of the operators in `ops`
 * (SF_MASS, SF_STIFF; SF_CONV returns SF_EUNSUPPORTED)
 * into the values of the sf_csr_pattern() layout: dev_val_mass and/or
 * dev_val_stiff, device [nnz] FP64 (the pointer of an operator not in ops
 * is ignored).  Needs a prior sf_patch_prepare of those operators at
 * `prec`.  Overwrites the outputs.  Deterministic: no atomics, fixed
 * summation order; the tile shapes do not change the values.
 * Asynchronous, except that for d = 3 the first call per (operator,
 * precision) times a few tile shapes on this patch (writing into the output,
 * then overwriting it) and synchronizes once.  For d = 3 the first call also
 * allocates the patch's level-2 workspace (the partial sums after the second
 * level of Algorithm 1; at most SFIGA_WORKSPACE_MB MiB if that is set, else
 * a quarter of the free device memory, at most 32 GiB; larger patches run in
 * chunks of element layers); it is freed by
 * sf_patch_destroy.  Returns SF_ENOMEM if that allocation fails. */
sf_status sf_assemble(sf_patch *patch, unsigned ops, sf_precision prec,
                      double *dev_val_mass, double *dev_val_stiff);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * assembly as sf_assemble, with the same kernels, allocating nothing.  The
 * d = 3 level-2 workspace is a fixed device array of 256 MiB that the
 * library holds on every device it runs on until the process ends (its
 * address is looked up by sf_ctx_create); patches run in chunks of element
 * layers that fit in it.  A patch whose smallest chunk (p - 1 element
 * layers of level-2 partials) exceeds 256 MiB returns SF_EUNSUPPORTED
 * (e.g. 128^3 elements at order 6 needs 1 GiB: use sf_assemble).  No
 * autotuning: tile shapes tuned by an earlier sf_assemble of the same
 * (operator, precision) are used, else the defaults; they do not change the
 * values.  Values equal sf_assemble's up to the summation order of entries
 * that straddle two chunks.  Every call on a device shares that device's
 * array, and nothing in it needs to start at zero: calls that overlap on one
 * device (two streams, two threads) race and must be serialized by the
 * caller.  Otherwise as sf_assemble: needs a prior sf_patch_prepare of the
 * operators at `prec`, overwrites the outputs, asynchronous. */
sf_status sf_assemble_noalloc(sf_patch *patch, unsigned ops, sf_precision prec,
                              double *dev_val_mass, double *dev_val_stiff);

/* Matrix-free product y = A x (Algorithm 3 forward, pointwise coefficient,
 * Algorithm 2 backward) for one operator op; dev_x, dev_y device [N] FP64,
 * y overwritten, x and y must not overlap.  Needs a prior sf_patch_prepare
 * of op at `prec`.  Accumulates through FP64 atomics, so the last bits may
 * vary between runs.  Asynchronous, except that for d = 3 the first call per
 * (operator, precision) times a few workgroup shapes on this patch (writing
 * into dev_y, then overwriting it) and synchronizes once.
 * op = SF_CONV (d = 3, SF_FP64): the convection form; Algorithm 3 forward
 * with the derivative table in one direction at a time gives the three
 * reference derivatives of x at every point, dotted with the folded
 * coefficients, then Algorithm 2 backward with value tables, in one kernel
 * (no workspace, no tuning). */
sf_status sf_apply(sf_patch *patch, unsigned op, sf_precision prec, const double *dev_x, double *dev_y);

/* Release the patch and its device workspace (synchronises its stream). */
void sf_patch_destroy(sf_patch *patch);

/* --------------------------------------------------------------- batch */

/* A set of independent patches (block-diagonal operator; Sec. 4, multipatch
 * example without interface gluing).  The patches stay owned by the caller
 * and must outlive the batch; all must belong to `ctx`. */
sf_status sf_batch_create(sf_ctx *ctx, int npatch, sf_patch *const *patches, sf_batch **out);

/* Host arrays [npatch+1]: first row (= first dof) and first nonzero of every
 * patch in the concatenated block-diagonal CSR / vectors. */
sf_status sf_batch_offsets(const sf_batch *batch, int64_t *row_off, int64_t *nnz_off);

/* Pattern and values of all patches into concatenated device arrays
 * (row_ptr [sum N + 1] int64 with global offsets, col_ind [sum nnz] int32
 * with global column indices, val_* [sum nnz]); every patch must have been
 * prepared for `ops` at `prec`.  The d = 3 patches of each order run in
 * persistent kernels that walk the per-patch work items; on a non-default
 * stream the whole call is captured into one HIP graph and replayed for
 * later calls with the same buffers.  The first call per (operator,
 * precision) times a few tile shapes and workgroups per CU on the batch
 * itself (writing into the outputs, which the call then rewrites) and
 * synchronizes; the choice does not change the values.  Task lists stay
 * allocated with the batch. */
sf_status sf_batch_assemble(sf_batch *batch, unsigned ops, sf_precision prec, int64_t *dev_row_ptr,
                            int32_t *dev_col_ind, double *dev_val_mass, double *dev_val_stiff);

/* y = blockdiag(A_b) x over the concatenated vectors; persistent kernels,
 * graph capture and first-call tuning as for sf_batch_assemble (SF_MASS,
 * SF_STIFF; SF_CONV returns SF_EUNSUPPORTED). */
sf_status sf_batch_apply(sf_batch *batch, unsigned op, sf_precision prec, const double *dev_x,
                         double *dev_y);

/* Glued multipatch (Sec. 4, Example "Multipatch domains"): conforming
 * patches identified at faces.  Host only, no context.  nfun [npatch][3]
 * (host) holds the functions per direction of each patch (entries k >= d
 * ignored); iface [ninterface][4] (host) the interfaces (patch a, face fa,
 * patch b, face fb) with face = 2 k + side for direction k+1 (side 0: the
 * functions with index 0 in that direction, side 1: the last); the other
 * directions, in increasing order, must have equal function counts on both
 * sides and are matched index by index (no flips or rotations).  Writes
 * map [sum of the patches' N] (host): the global id of every patch-local
 * function (patches in order, each lexicographic), ids numbered in order of
 * first appearance, and *n_global.  SF_EINVAL for bad arguments or a
 * non-conforming interface. */
sf_status sf_glue_map(int d, int npatch, const int32_t *nfun, int ninterface, const int32_t *iface, int64_t *map,
                      int64_t *n_global);

/* y = sum_b R_b^T A_b R_b x (Sec. 4, Example "Multipatch domains"): the
 * glued operator of the batch's patches under dev_map (device, [sum N]
 * int64, e.g. sf_glue_map's map copied to the device; an entry outside
 * [0, n_global) is not followed: its local value is 0 and its result is
 * dropped); dev_x, dev_y device [n_global] FP64, y overwritten, no
 * overlap.  Gathers the patch-local vectors, runs sf_batch_apply on them
 * and adds back with FP64 atomics (the last bits may vary between runs).
 * The patch-local vectors (2 x sum N doubles) are allocated by the first
 * call and kept with the batch.  Preparation and errors as sf_batch_apply. */
sf_status sf_batch_apply_glued(sf_batch *batch, unsigned op, sf_precision prec, const int64_t *dev_map,
                               int64_t n_global, const double *dev_x, double *dev_y);

void sf_batch_destroy(sf_batch *batch);

#ifdef __cplusplus
}
#endif
#endif /* SFIGA_H */
