// C ABI of the sfiga library (include/sfiga.h): handles, validation, device
// workspace and kernel dispatch.  No C++ exception crosses the ABI.
#include "sfiga.h"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "kernels.h"
#include "spline.h"

using namespace sfiga;

struct sf_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // device address of the fixed assembly scratch (sf_assemble_noalloc),
    // looked up at creation with the context's device current
    void *scratch = nullptr;
};

struct sf_patch {
    sf_ctx *ctx = nullptr;
    int d = 0, P = 0;
    Tables1D t[3];
    double *dB[3] = {nullptr, nullptr, nullptr}, *dD[3] = {nullptr, nullptr, nullptr};
    double *dW[3] = {nullptr, nullptr, nullptr}, *dX[3] = {nullptr, nullptr, nullptr};
    float *dBf[3] = {nullptr, nullptr, nullptr}, *dDf[3] = {nullptr, nullptr, nullptr};
    std::vector<float> Bf[3], Df[3];     // host copies of the FP32 tables (kept for the async upload)
    int64_t *dS[3] = {nullptr, nullptr, nullptr};
    double *dctrl = nullptr;
    int *dflag = nullptr;
    Coef coef[2];                 // [0] mass, [1] stiffness
    double adiff[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};   // diffusion matrix A of the stiffness form (a(x) A)
    // [op][storage: FP64, FP32, FP16 residual of the FP16 split]
    void *C[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    float *rs[2] = {nullptr, nullptr};   // [op] per-element reference and scale of the FP16 split
    // [op][storage: FP64, FP32] the coefficient tensor in the apply's tiled
    // layout (d = 3, where the apply kernel of the order reads it), written
    // by the geometry step beside C
    void *CA[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    bool assembly_only = false;          // the relabelled copy of a patch: no apply
    // convection form (d = 3, FP64, matrix-free apply only): scalar
    // coefficient s and vector b, folded coefficients w s |det J| J^-1 b
    // (conv_coef_index layout)
    Coef coef_conv{0, 1.0, nullptr};
    double bconv[3] = {0.0, 0.0, 0.0};
    double *Cv = nullptr;
    bool conv_ready = false;
    bool ready[2][4] = {};               // [op][precision mode]
    // level-2 workspace of the d = 3 assembly, sized once for the largest
    // (operator, precision) so that captured graphs never see it move
    void *ws = nullptr;
    size_t ws_bytes = 0;
    // autotuned assembly tile parameters per [op][prec] (-1: not yet tuned)
    int tune_t1[2][4] = {{-1, -1, -1, -1}, {-1, -1, -1, -1}}, tune_seg[2][4] = {{-1, -1, -1, -1}, {-1, -1, -1, -1}};
    int tune_lz[2][4] = {{-1, -1, -1, -1}, {-1, -1, -1, -1}};   // apply: layers per workgroup
    PatchView view{};
    // Contraction order of the d = 3 assembly (Algorithm 1 contracts direction
    // 1 first and direction 3 last): per [op][prec] the cyclic relabelling sh
    // chosen by the tuner (-1 untuned, 0 the given order, 1 or 2: assembled on
    // `alt`, whose direction k is direction (k + sh) mod 3 here, then gathered
    // into this layout through `tmpv`).
    std::vector<double> knots[3];
    int order_sh[2][4] = {{-1, -1, -1, -1}, {-1, -1, -1, -1}};
    sf_patch *alt = nullptr;
    int alt_sh = 0;
    double *tmpv = nullptr;
};

struct sf_batch {
    sf_ctx *ctx = nullptr;
    std::vector<sf_patch *> patches;
    std::vector<int64_t> row_off, nnz_off;
    int ncu = 256;                // compute units (persistent grid = ncu x multiplier)
    // cached graphs keyed by the launch arguments
    struct Cached {
        int kind;                 // 0 assemble, 1 apply
        unsigned ops;
        int prec;
        const void *p0, *p1, *p2, *p3;
        hipGraphExec_t exec;
    };
    std::vector<Cached> graphs;
    // autotuned launch parameters per (kernel, order, operator, precision):
    // tile parameter (see *_blocks) and workgroups per compute unit
    struct Tuned {
        int kernel, P, op, prec;
        int param, mult;
        float ms;
    };
    std::vector<Tuned> tuned;
    std::vector<void *> dev;      // device task lists referenced by the graphs
    // patch-local x and y of the glued apply (sum N each), allocated by its first call
    double *xl = nullptr, *yl = nullptr;
};

namespace sfiga {

hipError_t allow_dynamic_lds(const void *fn, size_t bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    static std::mutex mu;
    static std::set<std::pair<int, const void *>> done;
    std::lock_guard<std::mutex> lock(mu);
    if (done.count({dev, fn})) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) done.insert({dev, fn});
    return e;
}

}  // namespace sfiga

namespace {

sf_status fail(sf_ctx *ctx, sf_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return st;
}

sf_status hip_fail(sf_ctx *ctx, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(ctx, e == hipErrorOutOfMemory ? SF_ENOMEM : SF_EDEVICE, m);
}

template <typename T>
hipError_t upload(T **dst, const T *src, size_t n, hipStream_t s)
{
    hipError_t e = hipMalloc((void **)dst, sizeof(T) * (n ? n : 1));
    if (e != hipSuccess) return e;
    if (n) e = hipMemcpyAsync(*dst, src, sizeof(T) * n, hipMemcpyHostToDevice, s);
    return e;
}

// Precision modes: 0 FP64, 1 FP32, 2 BF16 split (FP32 coefficients and
// level 1, level 2 of the assembly on bf16 matrix cores with a hi/lo split;
// assembly only), 3 FP16 split (FP16 residuals of the coefficients with a
// per-element FP32 reference and scale; apply only).
bool prec_index(sf_precision prec, int &pi)
{
    if (prec == SF_FP64) { pi = 0; return true; }
    if (prec == SF_FP32) { pi = 1; return true; }
    if (prec == SF_BF16_SPLIT) { pi = 2; return true; }
    if (prec == SF_FP16_SPLIT) { pi = 3; return true; }
    return false;
}

int cidx(int pi) { return pi == 0 ? 0 : (pi == 3 ? 2 : 1); }       // coefficient tensor storage
int geom_storage(int pi) { return pi == 0 ? 0 : 1; }                // storage the geometry kernel writes
Prec asm_prec(int pi) { return pi == 0 ? Prec::F64 : (pi == 1 ? Prec::F32 : Prec::BF16X3); }
Prec apply_prec(int pi) { return pi == 0 ? Prec::F64 : (pi == 3 ? Prec::F16S : Prec::F32); }

int ncomp(int op_idx, int d) { return op_idx == 0 ? 1 : d * (d + 1) / 2; }

void free_patch_memory(sf_patch *p)
{
    for (int k = 0; k < 3; ++k) {
        (void)hipFree(p->dB[k]);
        (void)hipFree(p->dD[k]);
        (void)hipFree(p->dW[k]);
        (void)hipFree(p->dX[k]);
        (void)hipFree(p->dBf[k]);
        (void)hipFree(p->dDf[k]);
        (void)hipFree(p->dS[k]);
    }
    (void)hipFree(p->dctrl);
    (void)hipFree(p->dflag);
    (void)hipFree(p->ws);
    (void)hipFree(p->tmpv);
    for (auto &a : p->C)
        for (void *c : a) (void)hipFree(c);
    for (auto &a : p->CA)
        for (void *c : a) (void)hipFree(c);
    for (float *r : p->rs) (void)hipFree(r);
    (void)hipFree(p->Cv);
}

}  // namespace

extern "C" {

const char *sf_build_target(void) { return "gfx950"; }

sf_status sf_host_tables_1d(const double *knots, int64_t n_knots, int order, int *nel, double *x, double *w,
                            double *B, double *D)
{
    if (!knots) return SF_EINVAL;
    if (order < 2 || order > kMaxOrder) return SF_EUNSUPPORTED;
    Tables1D t;
    bool unsup = false;
    std::string why = build_tables_1d(knots, n_knots, order, t, unsup);
    if (!why.empty()) return unsup ? SF_EUNSUPPORTED : SF_EKNOT;
    if (nel) *nel = t.nel;
    if (x) std::memcpy(x, t.x.data(), sizeof(double) * t.x.size());
    if (w) std::memcpy(w, t.w.data(), sizeof(double) * t.w.size());
    if (B) std::memcpy(B, t.B.data(), sizeof(double) * t.B.size());
    if (D) std::memcpy(D, t.D.data(), sizeof(double) * t.D.size());
    return SF_OK;
}

sf_status sf_ctx_create(int device, void *hip_stream, sf_ctx **out)
{
    if (!out) return SF_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return SF_EDEVICE;
    if (device < 0 || device >= n) return SF_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return SF_EDEVICE;
    sf_ctx *c = new (std::nothrow) sf_ctx;
    if (!c) return SF_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (noalloc_scratch(&c->scratch) != hipSuccess) {
        delete c;
        return SF_EDEVICE;
    }
    *out = c;
    return SF_OK;
}

void sf_ctx_destroy(sf_ctx *ctx) { delete ctx; }

const char *sf_last_error(const sf_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

sf_status sf_patch_create(sf_ctx *ctx, const sf_patch_desc *desc, sf_patch **out)
{
    if (!ctx) return SF_EINVAL;
    if (!desc || !out) return fail(ctx, SF_EINVAL, "null argument");
    *out = nullptr;
    ctx->err.clear();
    if (desc->d < 1 || desc->d > 3) return fail(ctx, SF_EUNSUPPORTED, "dimension must be 1, 2 or 3");
    for (int k = 0; k < desc->d; ++k) {
        if (desc->order[k] < 1) return fail(ctx, SF_EINVAL, "order must be >= 1");
        if (desc->order[k] < 2 || desc->order[k] > kMaxOrder)
            return fail(ctx, SF_EUNSUPPORTED, "order must be in 2..9");
        if (desc->order[k] != desc->order[0])
            return fail(ctx, SF_EUNSUPPORTED, "per-direction orders differ: the kernels take one order for all "
                                              "directions");
    }
    if (!desc->ctrl) return fail(ctx, SF_EINVAL, "null control points");
    sf_patch *p = new (std::nothrow) sf_patch;
    if (!p) return fail(ctx, SF_ENOMEM, "host allocation failed");
    p->ctx = ctx;
    p->d = desc->d;
    p->P = desc->order[0];
    for (int k = 0; k < desc->d; ++k) {
        if (!desc->knots[k]) { delete p; return fail(ctx, SF_EINVAL, "null knot vector"); }
        if (desc->n_knots[k] > 0) p->knots[k].assign(desc->knots[k], desc->knots[k] + desc->n_knots[k]);
        bool unsup = false;
        std::string why = build_tables_1d(desc->knots[k], desc->n_knots[k], p->P, p->t[k], unsup);
        if (!why.empty()) {
            delete p;
            return fail(ctx, unsup ? SF_EUNSUPPORTED : SF_EKNOT, "direction " + std::to_string(k + 1) + ": " + why);
        }
    }
    int64_t N = 1, Q = 1, nnz = 1;
    for (int k = 0; k < p->d; ++k) {
        N *= p->t[k].nfun;
        Q *= (int64_t)p->t[k].nel * p->P;
        nnz *= (int64_t)p->t[k].nfun * (2 * p->P - 1) - (int64_t)p->P * (p->P - 1);
    }
    if (N >= (int64_t(1) << 31)) { delete p; return fail(ctx, SF_EUNSUPPORTED, "N >= 2^31 (int32 column indices)"); }

    hipStream_t s = ctx->stream;
    hipError_t e = hipSuccess;
    PatchView &v = p->view;
    std::memset(&v, 0, sizeof(v));
    v.d = p->d;
    v.P = p->P;
    v.ri.P = p->P;
    v.ri.d = p->d;
    std::vector<std::vector<int64_t>> S(3);
    for (int k = 0; k < 3 && e == hipSuccess; ++k) {
        Dir &dr = v.dir[k];
        if (k < p->d) {
            const Tables1D &t = p->t[k];
            e = upload(&p->dB[k], t.B.data(), t.B.size(), s);
            if (e == hipSuccess) e = upload(&p->dD[k], t.D.data(), t.D.size(), s);
            if (e == hipSuccess) e = upload(&p->dW[k], t.w.data(), t.w.size(), s);
            if (e == hipSuccess) e = upload(&p->dX[k], t.x.data(), t.x.size(), s);
            p->Bf[k].assign(t.B.begin(), t.B.end());
            p->Df[k].assign(t.D.begin(), t.D.end());
            if (e == hipSuccess) e = upload(&p->dBf[k], p->Bf[k].data(), p->Bf[k].size(), s);
            if (e == hipSuccess) e = upload(&p->dDf[k], p->Df[k].data(), p->Df[k].size(), s);
            dr.Bf = p->dBf[k];
            dr.Df = p->dDf[k];
            dr.B = p->dB[k];
            dr.D = p->dD[k];
            dr.W = p->dW[k];
            dr.X = p->dX[k];
            dr.K = t.nel;
            dr.N = t.nfun;
            dr.Q = t.nel * p->P;
            S[k].resize(t.nfun + 1);
            S[k][0] = 0;
            for (int i = 0; i < t.nfun; ++i) {
                int lo = i - p->P + 1 > 0 ? i - p->P + 1 : 0;
                int hi = i + p->P - 1 < t.nfun - 1 ? i + p->P - 1 : t.nfun - 1;
                S[k][i + 1] = S[k][i] + (hi - lo + 1);
            }
        } else {
            dr.K = dr.N = dr.Q = 1;
            S[k] = {0, 1};
        }
        if (e == hipSuccess) e = upload(&p->dS[k], S[k].data(), S[k].size(), s);
        v.ri.S[k] = p->dS[k];
        v.ri.T[k] = S[k].back();
        v.ri.N[k] = dr.N;
    }
    if (e == hipSuccess) {
        if (desc->ctrl_on_device) {
            e = hipMalloc((void **)&p->dctrl, sizeof(double) * N * p->d);
            if (e == hipSuccess)
                e = hipMemcpyAsync(p->dctrl, desc->ctrl, sizeof(double) * N * p->d, hipMemcpyDeviceToDevice, s);
        } else {
            e = upload(&p->dctrl, desc->ctrl, (size_t)(N * p->d), s);
        }
    }
    if (e == hipSuccess) e = hipMalloc((void **)&p->dflag, sizeof(int));
    if (e == hipSuccess) e = hipMemsetAsync(p->dflag, 0, sizeof(int), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_patch_memory(p);
        delete p;
        return hip_fail(ctx, e, "sf_patch_create");
    }
    v.ctrl = p->dctrl;
    v.N = N;
    v.Q = Q;
    v.nnz = nnz;
    for (auto &c : p->coef) c = Coef{0, 1.0, nullptr};
    *out = p;
    return SF_OK;
}

sf_status sf_patch_info(const sf_patch *p, int64_t *ndof, int64_t *nnz, int64_t *nquad)
{
    if (!p) return SF_EINVAL;
    if (ndof) *ndof = p->view.N;
    if (nnz) *nnz = p->view.nnz;
    if (nquad) *nquad = p->view.Q;
    return SF_OK;
}

sf_status sf_patch_set_coef(sf_patch *p, unsigned op, sf_coef_kind kind, const double *params)
{
    if (!p) return SF_EINVAL;
    sf_ctx *ctx = p->ctx;
    if (op != SF_MASS && op != SF_STIFF && op != SF_CONV)
        return fail(ctx, SF_EINVAL, "op must be SF_MASS, SF_STIFF or SF_CONV");
    if (!params) return fail(ctx, SF_EINVAL, "null params");
    Coef c{};
    switch (kind) {
    case SF_COEF_CONST: c = Coef{0, params[0], nullptr}; break;
    case SF_COEF_SINPROD: c = Coef{1, params[0], nullptr}; break;
    case SF_COEF_QPVALUES: c = Coef{2, 0.0, params}; break;
    default: return fail(ctx, SF_EINVAL, "unknown coefficient kind");
    }
    if (op == SF_CONV) {
        p->coef_conv = c;
        p->conv_ready = false;
        return SF_OK;
    }
    int oi = op == SF_MASS ? 0 : 1;
    p->coef[oi] = c;
    for (bool &r : p->ready[oi]) r = false;
    if (p->alt) {
        // quadrature-point values follow this patch's point order: the
        // relabelled patch cannot take them, so the given order is used
        p->alt->coef[oi] = c;
        for (bool &r : p->alt->ready[oi]) r = false;
        if (c.kind == 2)
            for (int &o : p->order_sh[oi]) o = o > 0 ? 0 : o;
    }
    return SF_OK;
}

sf_status sf_patch_set_diffusion(sf_patch *p, const double *A)
{
    if (!p) return SF_EINVAL;
    p->ctx->err.clear();
    if (!A) return fail(p->ctx, SF_EINVAL, "null matrix");
    double m[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    for (int i = 0, t = 0; i < p->d; ++i)
        for (int j = i; j < p->d; ++j, ++t) m[3 * i + j] = m[3 * j + i] = A[t];
    // the relabelled patch of a tuned contraction order has the same
    // physical coordinates, so the same A
    for (sf_patch *q : {p, p->alt}) {
        if (!q) continue;
        for (int k = 0; k < 9; ++k) q->adiff[k] = m[k];
        for (bool &r : q->ready[1]) r = false;
    }
    return SF_OK;
}

sf_status sf_patch_set_convection(sf_patch *p, const double *b)
{
    if (!p) return SF_EINVAL;
    p->ctx->err.clear();
    if (!b) return fail(p->ctx, SF_EINVAL, "null vector");
    for (int k = 0; k < 3; ++k) p->bconv[k] = k < p->d ? b[k] : 0.0;
    p->conv_ready = false;
    return SF_OK;
}

sf_status sf_patch_quad_points(sf_patch *p, double *dev_xyz)
{
    if (!p) return SF_EINVAL;
    if (!dev_xyz) return fail(p->ctx, SF_EINVAL, "null output");
    GeomOut o{};
    o.xyz = dev_xyz;
    o.bad_det = nullptr;          // G only: the det J record belongs to the prepares
    o.prec = Prec::F64;
    o.coef_mass = o.coef_stiff = Coef{0, 1.0, nullptr};
    hipError_t e = launch_geometry(p->view, o, p->ctx->stream);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "geometry kernel");
    return SF_OK;
}

sf_status sf_patch_eval(sf_patch *p, const double *dev_u, double *dev_val, double *dev_grad)
{
    if (!p) return SF_EINVAL;
    p->ctx->err.clear();
    if (!dev_u || (!dev_val && !dev_grad)) return fail(p->ctx, SF_EINVAL, "null input or no output");
    GeomOut o{};
    o.bad_det = nullptr;          // the det J record belongs to the prepares
    o.prec = Prec::F64;
    o.coef_mass = o.coef_stiff = Coef{0, 1.0, nullptr};
    o.u = dev_u;
    o.uval = dev_val;
    o.ugrad = dev_grad;
    hipError_t e = launch_geometry(p->view, o, p->ctx->stream);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "evaluation kernel");
    return SF_OK;
}

// Geometry step.  sync: clear the det J flag, run, read the flag back and
// report it.  Otherwise only the kernel is queued; the flag keeps any det J <= 0
// seen since the last sf_patch_geometry_check, which reads and clears it.
static sf_status prepare_impl(sf_patch *p, unsigned ops, sf_precision prec, bool sync)
{
    if (!p) return SF_EINVAL;
    sf_ctx *ctx = p->ctx;
    ctx->err.clear();
    if (ops == 0 || (ops & ~(unsigned)(SF_MASS | SF_STIFF | SF_CONV))) return fail(ctx, SF_EINVAL, "bad operator flags");
    int pi;
    if (!prec_index(prec, pi)) return fail(ctx, SF_EINVAL, "bad precision");
    if (pi == 3 && p->d != 3) return fail(ctx, SF_EUNSUPPORTED, "the FP16-split storage is built for d = 3");
    if ((ops & SF_CONV) && (p->d != 3 || pi != 0 || p->assembly_only))
        return fail(ctx, SF_EUNSUPPORTED, "the convection form is built for d = 3 at SF_FP64");
    if ((ops & SF_CONV) && p->coef_conv.kind == 2 && !p->coef_conv.qp)
        return fail(ctx, SF_EINVAL, "missing quadrature values");
    hipStream_t s = ctx->stream;
    const int gi = geom_storage(pi);
    const size_t esz = gi == 0 ? sizeof(double) : sizeof(float);
    const int64_t nel = (int64_t)p->view.dir[0].K * p->view.dir[1].K * p->view.dir[2].K;
    GeomOut o{};
    o.prec = gi == 0 ? Prec::F64 : Prec::F32;
    o.bad_det = p->dflag;
    o.coef_mass = p->coef[0];
    o.coef_stiff = p->coef[1];
    for (int k = 0; k < 9; ++k) o.adiff[k] = p->adiff[k];
    auto alloc = [&](void **ptr, size_t bytes) -> sf_status {
        if (*ptr) return SF_OK;
        hipError_t e = hipMalloc(ptr, bytes);
        if (e != hipSuccess) {
            *ptr = nullptr;
            return hip_fail(ctx, e, "coefficient tensor allocation");
        }
        return SF_OK;
    };
    for (int oi = 0; oi < 2; ++oi) {
        unsigned bit = oi == 0 ? SF_MASS : SF_STIFF;
        if (!(ops & bit)) continue;
        if (p->coef[oi].kind == 2 && !p->coef[oi].qp) return fail(ctx, SF_EINVAL, "missing quadrature values");
        const size_t nq = (size_t)p->view.Q * ncomp(oi, p->d);
        sf_status st = alloc(&p->C[oi][gi], esz * nq);
        if (st == SF_OK && pi == 3)
            st = alloc(&p->C[oi][2], 2 * (size_t)split_size(ncomp(oi, p->d), p->P, p->view.dir[0].K,
                                                              p->view.dir[1].K, p->view.dir[2].K));
        const bool tiled = p->d == 3 && !p->assembly_only &&
                           apply_tiled_layout(p->P, oi + 1, gi == 0 ? Prec::F64 : Prec::F32);
        if (st == SF_OK && tiled && !p->CA[oi][gi]) {
            // columns outside the patch are never written: cleared once here
            const size_t bytes = esz * (size_t)apply_coef_size(ncomp(oi, p->d), p->P, p->view.dir[0].K,
                                                                 p->view.dir[1].K, p->view.dir[2].K);
            st = alloc(&p->CA[oi][gi], bytes);
            if (st == SF_OK) {
                hipError_t e0 = hipMemsetAsync(p->CA[oi][gi], 0, bytes, s);
                if (e0 != hipSuccess) st = hip_fail(ctx, e0, "apply coefficient layout");
            }
        }
        if (st == SF_OK && pi == 3) st = alloc((void **)&p->rs[oi], sizeof(float) * 2 * ncomp(oi, p->d) * nel);
        if (st != SF_OK) return st;
        // the modes stored in what this call rewrites are stale until it is done
        for (int m = 0; m < 4; ++m)
            if (geom_storage(m) == gi) p->ready[oi][m] = false;
        if (oi == 0) o.c_mass = p->C[oi][gi]; else o.c_stiff = p->C[oi][gi];
        if (tiled) (oi == 0 ? o.ca_mass : o.ca_stiff) = p->CA[oi][gi];
    }
    if (ops & SF_CONV) {
        if (!p->Cv) {
            // columns outside the patch are never written: cleared once here
            const size_t bytes = sizeof(double) * (size_t)conv_coef_size(p->P, p->view.dir[0].K, p->view.dir[1].K,
                                                                         p->view.dir[2].K);
            sf_status st = alloc((void **)&p->Cv, bytes);
            if (st != SF_OK) return st;
            hipError_t e0 = hipMemsetAsync(p->Cv, 0, bytes, s);
            if (e0 != hipSuccess) return hip_fail(ctx, e0, "convection coefficients");
        }
        p->conv_ready = false;
        o.c_conv = p->Cv;
        o.coef_conv = p->coef_conv;
        for (int k = 0; k < 3; ++k) o.bconv[k] = p->bconv[k];
    }
    hipError_t e = sync ? hipMemsetAsync(p->dflag, 0, sizeof(int), s) : hipSuccess;
    if (e == hipSuccess) e = launch_geometry(p->view, o, s);
    if (pi == 3)
        for (int oi = 0; oi < 2 && e == hipSuccess; ++oi)
            if (ops & (oi == 0 ? SF_MASS : SF_STIFF))
                e = launch_split_coef(p->view, oi + 1, (const float *)p->C[oi][1], p->C[oi][2], p->rs[oi], s);
    int flag = 0;
    if (sync) {
        if (e == hipSuccess) e = hipMemcpyAsync(&flag, p->dflag, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "geometry step");
    if (flag) return fail(ctx, SF_EGEOM, "det J <= 0 at some quadrature point");
    if (ops & SF_CONV) p->conv_ready = true;
    for (int oi = 0; oi < 2; ++oi)
        if (ops & (oi == 0 ? SF_MASS : SF_STIFF)) {
            // FP32 storage serves FP32 and BF16 split; the FP16 split needs its own pass
            for (int m = 0; m < 3; ++m)
                if (geom_storage(m) == gi) p->ready[oi][m] = true;
            if (pi == 3) p->ready[oi][3] = true;
        }
    // the relabelled patch of a tuned contraction order follows every prepare
    if (p->alt && pi != 3) {
        unsigned aops = 0;
        for (int oi = 0; oi < 2; ++oi)
            if ((ops & (oi == 0 ? SF_MASS : SF_STIFF)) && p->coef[oi].kind != 2) aops |= oi == 0 ? SF_MASS : SF_STIFF;
        if (aops) return prepare_impl(p->alt, aops, prec, sync);
    }
    return SF_OK;
}

sf_status sf_patch_prepare(sf_patch *p, unsigned ops, sf_precision prec)
{
    return prepare_impl(p, ops, prec, true);
}

sf_status sf_patch_prepare_async(sf_patch *p, unsigned ops, sf_precision prec)
{
    return prepare_impl(p, ops, prec, false);
}

sf_status sf_patch_geometry_check(sf_patch *p)
{
    if (!p) return SF_EINVAL;
    sf_ctx *ctx = p->ctx;
    ctx->err.clear();
    hipStream_t s = ctx->stream;
    int flag = 0;
    hipError_t e = hipMemcpyAsync(&flag, p->dflag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemsetAsync(p->dflag, 0, sizeof(int), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(ctx, e, "geometry check");
    if (flag) return fail(ctx, SF_EGEOM, "det J <= 0 at some quadrature point");
    return SF_OK;
}

sf_status sf_csr_pattern(sf_patch *p, int64_t *row_ptr, int32_t *col_ind)
{
    if (!p) return SF_EINVAL;
    if (!row_ptr || !col_ind) return fail(p->ctx, SF_EINVAL, "null output");
    hipError_t e = launch_pattern(p->view, row_ptr, col_ind, 0, 0, 0, p->ctx->stream);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "pattern kernels");
    return SF_OK;
}

// for_apply: the matrix-free apply (the FP16 split is its mode; the BF16 split
// is a mode of the assembly only)
static sf_status check_ready(sf_patch *p, unsigned ops, sf_precision prec, int &pi, bool for_apply)
{
    sf_ctx *ctx = p->ctx;
    if (ops & SF_CONV)
        return fail(ctx, SF_EUNSUPPORTED, "the convection form is built for the single-patch matrix-free "
                                          "apply (sf_apply) only");
    if (ops == 0 || (ops & ~(unsigned)(SF_MASS | SF_STIFF))) return fail(ctx, SF_EINVAL, "bad operator flags");
    if (!prec_index(prec, pi)) return fail(ctx, SF_EINVAL, "bad precision");
    if (for_apply && pi == 2)
        return fail(ctx, SF_EUNSUPPORTED, "BF16 split is a mode of the assembly; the reduced-storage apply is "
                                          "SF_FP16_SPLIT");
    if (!for_apply && pi == 3)
        return fail(ctx, SF_EUNSUPPORTED, "FP16 split is a storage of the matrix-free apply; assemble at FP64, FP32 "
                                          "or BF16 split");
    for (int oi = 0; oi < 2; ++oi)
        if ((ops & (oi == 0 ? SF_MASS : SF_STIFF)) && !p->ready[oi][pi])
            return fail(ctx, SF_EINVAL, "operator not prepared at this precision (call sf_patch_prepare)");
    return SF_OK;
}

// Upper bound of the assembly workspace: SFIGA_WORKSPACE_MB, else a quarter
// of the device memory free when the workspace is sized, at most 32 GiB.
// Patches whose level-2 partials exceed it are assembled in chunks of
// element layers (128^3 at order 6, 26.5 GB of partials: 84 ms per call in
// 7 chunks under a 4 GiB cap, 77.5 ms in one).
static size_t workspace_cap()
{
    const char *v = getenv("SFIGA_WORKSPACE_MB");
    long mb = v ? atol(v) : 0;
    if (mb > 0) return (size_t)mb << 20;
    size_t free_b = 0, total_b = 0;
    size_t cap = size_t(4096) << 20;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b / 4 > cap) cap = free_b / 4;
    const size_t most = size_t(32) << 30;
    return cap < most ? cap : most;
}

static sf_status ensure_workspace(sf_patch *p)
{
    if (p->ws || p->d != 3) return SF_OK;
    const size_t need = assemble_workspace_bytes(p->view, 2, Prec::F64, workspace_cap());
    hipError_t e = hipMalloc(&p->ws, need);
    if (e != hipSuccess) {
        p->ws = nullptr;
        return hip_fail(p->ctx, e, "assembly workspace allocation");
    }
    p->ws_bytes = need;
    return SF_OK;
}

// Autotuner of the single-patch d = 3 assembly: rows m1 per level-1/2 tile
// (which sets the workgroup count against the resident slots of the chip)
// and rows m3 per level-3 segment, timed with HIP events on this patch
// into its own output buffer (rewritten by the call that follows).  Runs
// once per (operator, precision) and synchronizes the stream.
static sf_status tune_assembly(sf_patch *p, int oi, int pi, double *dst)
{
    if (p->d != 3) {
        p->tune_t1[oi][pi] = p->tune_seg[oi][pi] = 0;
        return SF_OK;
    }
    hipStream_t s = p->ctx->stream;
    const Prec prec = asm_prec(pi);
    const int tmax = asm12_max_rows(p->P, prec);
    std::vector<int> t1s;
    for (int t : {tmax, (3 * tmax + 3) / 4, (tmax + 1) / 2, (tmax + 2) / 3})
        if (t >= 1 && std::find(t1s.begin(), t1s.end(), t) == t1s.end()) t1s.push_back(t);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    auto run = [&](int t1, int seg) {
        return launch_assemble(p->view, oi + 1, prec, p->C[oi][cidx(pi)], dst, p->ws, p->ws_bytes, s, t1, seg);
    };
    auto timed = [&](int t1, int seg, float &ms) {
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = run(t1, seg);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    };
    if (e == hipSuccess) e = run(0, 0);          // warm-up (first launch of the kernels)
    float best = 1e30f, ms = 0.f;
    int bt1 = 0, bseg = 0;
    for (int t1 : t1s) {
        timed(t1, 0, ms);
        if (e == hipSuccess && ms < best) { best = ms; bt1 = t1; }
    }
    for (int seg : {8, 32}) {                    // 16 is the default just timed
        timed(bt1, seg, ms);
        if (e == hipSuccess && ms < best) { best = ms; bseg = seg; }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "assembly autotuning");
    p->tune_t1[oi][pi] = bt1;
    p->tune_seg[oi][pi] = bseg;
    return SF_OK;
}

// One operator in the given order (sh = 0) or on the relabelled patch and
// gathered back (sh > 0).
static hipError_t assemble_op(sf_patch *p, int oi, int pi, double *dst, hipStream_t s, int sh)
{
    sf_patch *q = sh > 0 ? p->alt : p;
    const int t1 = q->tune_t1[oi][pi] > 0 ? q->tune_t1[oi][pi] : 0;
    const int seg = q->tune_seg[oi][pi] > 0 ? q->tune_seg[oi][pi] : 0;
    hipError_t e = launch_assemble(q->view, oi + 1, asm_prec(pi), q->C[oi][cidx(pi)], sh > 0 ? p->tmpv : dst, q->ws,
                                   q->ws_bytes, s, t1, seg);
    if (e == hipSuccess && sh > 0) e = launch_gather_cyclic(p->view, q->view, sh, p->tmpv, dst, s);
    return e;
}

static sf_status assemble_into(sf_patch *p, unsigned ops, int pi, double *vm, double *vs, hipStream_t s)
{
    for (int oi = 0; oi < 2; ++oi) {
        if (!(ops & (oi == 0 ? SF_MASS : SF_STIFF))) continue;
        const int sh = p->order_sh[oi][pi] > 0 && p->alt ? p->order_sh[oi][pi] : 0;
        hipError_t e = assemble_op(p, oi, pi, oi == 0 ? vm : vs, s, sh);
        if (e != hipSuccess) return hip_fail(p->ctx, e, "assembly kernel");
    }
    return SF_OK;
}

// The patch with its directions relabelled cyclically by sh (direction k of
// the new patch is direction (k + sh) mod 3 here): knots and control points
// reordered, coordinates unchanged.  A cyclic relabelling is an even
// permutation of the reference axes, so det J keeps its sign.
static sf_status make_alt(sf_patch *p, int sh)
{
    if (p->alt) return p->alt_sh == sh ? SF_OK : fail(p->ctx, SF_EINVAL, "another contraction order exists");
    sf_ctx *ctx = p->ctx;
    const int64_t N = p->view.N;
    std::vector<double> c(N * 3), ca(N * 3);
    hipError_t e = hipMemcpyAsync(c.data(), p->dctrl, sizeof(double) * N * 3, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "control points for the relabelled patch");
    int na[3];
    for (int k = 0; k < 3; ++k) na[k] = p->t[(k + sh) % 3].nfun;
    for (int64_t n = 0; n < N; ++n) {
        const int i[3] = {(int)(n % p->t[0].nfun), (int)((n / p->t[0].nfun) % p->t[1].nfun),
                          (int)(n / ((int64_t)p->t[0].nfun * p->t[1].nfun))};
        const int64_t na_idx = i[sh % 3] + (int64_t)na[0] * (i[(1 + sh) % 3] + (int64_t)na[1] * i[(2 + sh) % 3]);
        for (int x = 0; x < 3; ++x) ca[na_idx * 3 + x] = c[n * 3 + x];
    }
    sf_patch_desc d{};
    d.d = 3;
    for (int k = 0; k < 3; ++k) {
        d.order[k] = p->P;
        d.n_knots[k] = (int64_t)p->knots[(k + sh) % 3].size();
        d.knots[k] = p->knots[(k + sh) % 3].data();
    }
    d.ctrl = ca.data();
    d.ctrl_on_device = 0;
    sf_patch *a = nullptr;
    sf_status st = sf_patch_create(ctx, &d, &a);
    if (st != SF_OK) return st;
    a->assembly_only = true;
    a->coef[0] = p->coef[0];
    a->coef[1] = p->coef[1];
    for (int k = 0; k < 9; ++k) a->adiff[k] = p->adiff[k];
    e = hipMalloc((void **)&p->tmpv, sizeof(double) * (size_t)p->view.nnz);
    if (e != hipSuccess) {
        p->tmpv = nullptr;
        sf_patch_destroy(a);
        return hip_fail(ctx, e, "values of the relabelled patch");
    }
    p->alt = a;
    p->alt_sh = sh;
    return SF_OK;
}

// SFIGA_ASSEMBLY_ORDER: "given" keeps direction 3 last, "relabelled" always
// takes the relabelled order, anything else (default) times both.
static int order_policy()
{
    const char *v = getenv("SFIGA_ASSEMBLY_ORDER");
    if (v && !strcmp(v, "given")) return 0;
    if (v && !strcmp(v, "relabelled")) return 1;
    return 2;
}

// Contraction-order autotuning (the narrow direction contracted last, Sec.
// 4.2): the level-2 and level-3 costs of Algorithm 1 multiply the 1D band
// sizes of the directions contracted first, and a direction with few elements
// has a large band per point (nnz1(N)/Q is p for one element, about 2 - 1/p
// for many).  Candidates: the given order and the cyclic relabelling that
// puts the direction with the fewest elements last; each timed (with the
// gather) on this patch into dst, the faster kept.
static sf_status tune_order(sf_patch *p, int oi, int pi, double *dst)
{
    p->order_sh[oi][pi] = 0;
    if (p->d != 3 || p->coef[oi].kind == 2 || order_policy() == 0) return SF_OK;
    int kmin = 2;
    for (int k = 0; k < 3; ++k)
        if (p->t[k].nel < p->t[kmin].nel) kmin = k;
    const int sh = (kmin + 1) % 3;          // relabelled direction 2 is direction kmin
    if (sh == 0) return SF_OK;
    if (p->alt && p->alt_sh != sh) return SF_OK;
    sf_status st = make_alt(p, sh);
    if (st != SF_OK) return st;
    sf_patch *a = p->alt;
    const unsigned bit = oi == 0 ? SF_MASS : SF_STIFF;
    if (!a->ready[oi][pi]) {
        st = prepare_impl(a, bit, pi == 0 ? SF_FP64 : (pi == 1 ? SF_FP32 : SF_BF16_SPLIT), true);
        if (st != SF_OK) return st;
    }
    st = ensure_workspace(a);
    if (st == SF_OK && a->tune_t1[oi][pi] < 0) st = tune_assembly(a, oi, pi, p->tmpv);
    if (st != SF_OK) return st;
    if (order_policy() == 1) {
        p->order_sh[oi][pi] = sh;
        return SF_OK;
    }
    hipStream_t s = p->ctx->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float ms[2] = {0.f, 0.f};
    for (int c = 0; c < 2 && e == hipSuccess; ++c) {
        const int shc = c == 0 ? 0 : sh;
        e = assemble_op(p, oi, pi, dst, s, shc);            // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < 2 && e == hipSuccess; ++r) e = assemble_op(p, oi, pi, dst, s, shc);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms[c], e0, e1);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "contraction-order autotuning");
    p->order_sh[oi][pi] = ms[1] < ms[0] ? sh : 0;
    return SF_OK;
}

sf_status sf_assemble(sf_patch *p, unsigned ops, sf_precision prec, double *vm, double *vs)
{
    if (!p) return SF_EINVAL;
    p->ctx->err.clear();
    int pi;
    sf_status st = check_ready(p, ops, prec, pi, false);
    if (st != SF_OK) return st;
    if (((ops & SF_MASS) && !vm) || ((ops & SF_STIFF) && !vs)) return fail(p->ctx, SF_EINVAL, "null output");
    st = ensure_workspace(p);
    if (st != SF_OK) return st;
    for (int oi = 0; oi < 2; ++oi)
        if ((ops & (oi == 0 ? SF_MASS : SF_STIFF)) && p->tune_t1[oi][pi] < 0) {
            st = tune_assembly(p, oi, pi, oi == 0 ? vm : vs);
            if (st == SF_OK) st = tune_order(p, oi, pi, oi == 0 ? vm : vs);
            if (st != SF_OK) return st;
        }
    return assemble_into(p, ops, pi, vm, vs, p->ctx->stream);
}

sf_status sf_assemble_noalloc(sf_patch *p, unsigned ops, sf_precision prec, double *vm, double *vs)
{
    if (!p) return SF_EINVAL;
    sf_ctx *ctx = p->ctx;
    ctx->err.clear();
    int pi;
    sf_status st = check_ready(p, ops, prec, pi, false);
    if (st != SF_OK) return st;
    if (((ops & SF_MASS) && !vm) || ((ops & SF_STIFF) && !vs)) return fail(ctx, SF_EINVAL, "null output");
    if (p->d == 3) {
        for (int oi = 0; oi < 2; ++oi) {
            if (!(ops & (oi == 0 ? SF_MASS : SF_STIFF))) continue;
            const size_t need = assemble_min_workspace_bytes(p->view, oi + 1, asm_prec(pi));
            if (need > kNoAllocScratchBytes)
                return fail(ctx, SF_EUNSUPPORTED,
                            "patch too large for the fixed scratch: " + std::to_string(need >> 20) +
                                " MiB of level-2 partials for the smallest chunk, scratch " +
                                std::to_string(kNoAllocScratchBytes >> 20) + " MiB (use sf_assemble)");
        }
    }
    for (int oi = 0; oi < 2; ++oi) {
        if (!(ops & (oi == 0 ? SF_MASS : SF_STIFF))) continue;
        double *dst = oi == 0 ? vm : vs;
        // tile shapes tuned by an earlier sf_assemble if any (they do not
        // change the values); no tuning here
        const int t1 = p->tune_t1[oi][pi] > 0 ? p->tune_t1[oi][pi] : 0;
        const int seg = p->tune_seg[oi][pi] > 0 ? p->tune_seg[oi][pi] : 0;
        hipError_t e = launch_assemble(p->view, oi + 1, asm_prec(pi), p->C[oi][cidx(pi)], dst, ctx->scratch,
                                       kNoAllocScratchBytes, ctx->stream, t1, seg);
        if (e != hipSuccess) return hip_fail(ctx, e, "assembly kernel");
    }
    return SF_OK;
}

// Apply autotuner: element layers per workgroup of the d = 3 apply, timed
// on the patch into y (which the caller's launch then rewrites); once per
// (operator, precision).  Outside any graph capture.
static sf_status tune_apply_lz(sf_patch *p, int oi, int pi, const void *C, bool tiled, const double *x, double *y)
{
    const Prec pr = apply_prec(pi);
    hipStream_t s = p->ctx->stream;
    p->tune_lz[oi][pi] = 0;
    if (p->d == 3) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hipError_t e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e == hipSuccess) e = launch_apply(p->view, oi + 1, pr, C, x, y, s, 0, p->rs[oi], tiled);   // warm-up
        float best = 1e30f;
        for (int lz : {1, 2, 3, 4, 6, 8, 12, 16}) {
            if (e != hipSuccess || lz > p->view.dir[2].K) break;
            float ms = 1e30f;
            for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {     // best of two
                float t = 0.f;
                e = hipEventRecord(e0, s);
                if (e == hipSuccess) e = launch_apply(p->view, oi + 1, pr, C, x, y, s, lz, p->rs[oi], tiled);
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
                ms = t < ms ? t : ms;
            }
            if (e == hipSuccess && ms < best) {
                best = ms;
                p->tune_lz[oi][pi] = lz;
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (e != hipSuccess) return hip_fail(p->ctx, e, "apply autotuning");
    }
    return SF_OK;
}

sf_status sf_apply(sf_patch *p, unsigned op, sf_precision prec, const double *x, double *y)
{
    if (!p) return SF_EINVAL;
    p->ctx->err.clear();
    if (op == SF_CONV) {
        if (prec != SF_FP64 || p->d != 3 || p->assembly_only)
            return fail(p->ctx, SF_EUNSUPPORTED, "the convection form is built for d = 3 at SF_FP64");
        if (!p->conv_ready)
            return fail(p->ctx, SF_EINVAL, "operator not prepared at this precision (call sf_patch_prepare)");
        if (!x || !y) return fail(p->ctx, SF_EINVAL, "null vector");
        if (x == y) return fail(p->ctx, SF_EINVAL, "x and y must not overlap");
        hipError_t e = launch_conv_apply(p->view, p->Cv, x, y, p->ctx->stream);
        if (e != hipSuccess) return hip_fail(p->ctx, e, "convection kernel");
        return SF_OK;
    }
    if (op != SF_MASS && op != SF_STIFF) return fail(p->ctx, SF_EINVAL, "op must be SF_MASS, SF_STIFF or SF_CONV");
    int pi;
    sf_status st = check_ready(p, op, prec, pi, true);
    if (st != SF_OK) return st;
    if (!x || !y) return fail(p->ctx, SF_EINVAL, "null vector");
    if (x == y) return fail(p->ctx, SF_EINVAL, "x and y must not overlap");
    int oi = op == SF_MASS ? 0 : 1;
    const Prec pr = apply_prec(pi);
    const bool tiled = pi != 3 && p->CA[oi][geom_storage(pi)] != nullptr;
    const void *C = tiled ? p->CA[oi][geom_storage(pi)] : p->C[oi][cidx(pi)];
    hipStream_t s = p->ctx->stream;
    if (p->tune_lz[oi][pi] < 0) {
        sf_status st2 = tune_apply_lz(p, oi, pi, C, tiled, x, y);
        if (st2 != SF_OK) return st2;
    }
    hipError_t e = launch_apply(p->view, oi + 1, pr, C, x, y, s, p->tune_lz[oi][pi], p->rs[oi], tiled);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "apply kernel");
    return SF_OK;
}

void sf_patch_destroy(sf_patch *p)
{
    if (!p) return;
    (void)hipStreamSynchronize(p->ctx->stream);
    sf_patch_destroy(p->alt);
    free_patch_memory(p);
    delete p;
}

// ------------------------------------------------------------------ batch

sf_status sf_batch_create(sf_ctx *ctx, int npatch, sf_patch *const *patches, sf_batch **out)
{
    if (!ctx) return SF_EINVAL;
    if (!out || !patches || npatch < 1) return fail(ctx, SF_EINVAL, "bad batch arguments");
    *out = nullptr;
    sf_batch *b = new (std::nothrow) sf_batch;
    if (!b) return fail(ctx, SF_ENOMEM, "host allocation failed");
    b->ctx = ctx;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) == hipSuccess && ncu > 0)
        b->ncu = ncu;
    b->row_off.push_back(0);
    b->nnz_off.push_back(0);
    for (int i = 0; i < npatch; ++i) {
        sf_patch *p = patches[i];
        if (!p || p->ctx != ctx) { delete b; return fail(ctx, SF_EINVAL, "patch missing or from another context"); }
        b->patches.push_back(p);
        b->row_off.push_back(b->row_off.back() + p->view.N);
        b->nnz_off.push_back(b->nnz_off.back() + p->view.nnz);
    }
    if (b->row_off.back() >= (int64_t(1) << 31)) {
        delete b;
        return fail(ctx, SF_EUNSUPPORTED, "total N >= 2^31 (int32 column indices)");
    }
    *out = b;
    return SF_OK;
}

sf_status sf_batch_offsets(const sf_batch *b, int64_t *row_off, int64_t *nnz_off)
{
    if (!b) return SF_EINVAL;
    size_t n = b->row_off.size();
    if (row_off) std::memcpy(row_off, b->row_off.data(), n * sizeof(int64_t));
    if (nnz_off) std::memcpy(nnz_off, b->nnz_off.data(), n * sizeof(int64_t));
    return SF_OK;
}

// ---- batched launches: persistent kernels over per-patch tasks

enum { KASM12 = 0, KASM3 = 1, KAPPLY = 2, KROWPTR = 3, KCOLIND = 4 };

struct HostTasks {
    std::vector<BatchTask> t;
    std::vector<int64_t> off;
};

// Pointers of one batched call.
struct BatchIO {
    int64_t *rp = nullptr;
    int32_t *ci = nullptr;
    double *vals[2] = {nullptr, nullptr};   // assembly outputs: mass, stiffness
    const double *x = nullptr;
    double *y = nullptr;
};

// A d = 3 patch whose own apply launch fills the chip many times over (at
// least 8 workgroups per compute unit) gains nothing from the shared
// persistent grid, and its single-patch kernel reads the tiled coefficient
// copy where the patch has one (8 patches of 64^3 elements at order 6, FP64:
// 8.87 ms in the persistent kernel).
static bool apply_alone(const sf_patch *p, int oi, int pi)
{
    if (p->d != 3 || pi == 3 || !p->CA[oi][geom_storage(pi)]) return false;
    int gx, gy, gz, LZ;
    apply_blocks(p->view, 0, gx, gy, gz, LZ);
    return (int64_t)gx * gy * gz >= 8 * 256;
}

static bool persistent_ok(const sf_patch *p, int kernel, int oi, int pi)
{
    if (kernel == KROWPTR || kernel == KCOLIND) return true;
    if (p->d != 3) return false;
    if (kernel == KAPPLY) return !apply_alone(p, oi, pi);
    return assemble_single_chunk(p->view, oi + 1, asm_prec(pi), p->ws_bytes);
}

// Tasks of one kernel for the patches of order P (P = 0: all orders), largest
// block count first so that the persistent grid ends evenly.
static HostTasks build_tasks(const sf_batch *b, int kernel, int P, int oi, int pi, int param, const BatchIO &io)
{
    HostTasks h;
    for (size_t i = 0; i < b->patches.size(); ++i) {
        const sf_patch *p = b->patches[i];
        if ((P && p->P != P) || !persistent_ok(p, kernel, oi, pi)) continue;
        BatchTask T{};
        T.pv = p->view;
        T.C = p->C[oi][cidx(pi)];
        T.rs = p->rs[oi];
        T.ws = p->ws;
        const int64_t r0 = b->row_off[i], z0 = b->nnz_off[i];
        T.gy = T.gz = 1;
        switch (kernel) {
        case KASM12: asm12_blocks(p->view, asm_prec(pi), param, T.gx, T.gy, T.arg); break;
        case KASM3:
            asm3_blocks(p->view, param, T.gx, T.gy, T.gz, T.arg);
            T.out = io.vals[oi] + z0;
            break;
        case KAPPLY:
            apply_blocks(p->view, param, T.gx, T.gy, T.gz, T.arg);
            T.x = io.x + r0;
            T.out = io.y + r0;
            break;
        case KROWPTR:
            T.gx = (int)((p->view.N + 1 + 255) / 256);
            T.row_ptr = io.rp + r0;
            T.nnz_base = z0;
            break;
        default:
            T.gx = (int)((p->view.N + 3) / 4);
            T.col_ind = io.ci;
            T.col_base = r0;
            T.nnz_base = z0;
            break;
        }
        h.t.push_back(T);
    }
    std::stable_sort(h.t.begin(), h.t.end(), [](const BatchTask &a, const BatchTask &c) {
        return (int64_t)a.gx * a.gy * a.gz > (int64_t)c.gx * c.gy * c.gz;
    });
    h.off.push_back(0);
    for (const BatchTask &T : h.t) h.off.push_back(h.off.back() + (int64_t)T.gx * T.gy * T.gz);
    return h;
}

static hipError_t upload_tasks(const HostTasks &h, TaskList &tl, void **mem)
{
    tl.ntask = (int)h.t.size();
    tl.nitems = h.off.back();
    const size_t tb = sizeof(BatchTask) * h.t.size(), ob = sizeof(int64_t) * h.off.size();
    *mem = nullptr;
    hipError_t e = hipMalloc(mem, tb + ob + 16);
    if (e != hipSuccess) return e;
    char *base = static_cast<char *>(*mem);
    if (tb) e = hipMemcpy(base, h.t.data(), tb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(base + tb, h.off.data(), ob, hipMemcpyHostToDevice);
    tl.tasks = reinterpret_cast<const BatchTask *>(base);
    tl.off = reinterpret_cast<const int64_t *>(base + tb);
    return e;
}

static hipError_t launch_kernel(int kernel, const TaskList &tl, int P, int oi, int pi, int nblocks, hipStream_t s)
{
    switch (kernel) {
    case KASM12: return launch_asm12_batch(tl, P, oi + 1, asm_prec(pi), nblocks, s);
    case KASM3: return launch_asm3_batch(tl, P, oi + 1, asm_prec(pi), nblocks, s);
    case KAPPLY: return launch_apply_batch(tl, P, oi + 1, apply_prec(pi), nblocks, s);
    case KROWPTR: return launch_rowptr_batch(tl, nblocks, s);
    default: return launch_colind_batch(tl, P, nblocks, s);
    }
}

// Autotuner: time every candidate (tile parameter x workgroups per CU) of one
// kernel on this batch's own patches and keep the fastest.  Runs once per
// (kernel, order, operator, precision), outside any capture; its outputs are
// scratch (the real launch rewrites them).
static sf_status tune(sf_batch *b, int kernel, int P, int oi, int pi, const BatchIO &io, int &param, int &mult)
{
    for (const sf_batch::Tuned &t : b->tuned)
        if (t.kernel == kernel && t.P == P && t.op == oi && t.prec == pi) {
            param = t.param;
            mult = t.mult;
            return SF_OK;
        }
    std::vector<int> params, mults = {1, 2};
    if (kernel == KASM12) {
        const int tmax = asm12_max_rows(P, asm_prec(pi));
        for (int t : {tmax, (3 * tmax + 3) / 4, (tmax + 1) / 2, (tmax + 2) / 3})
            if (t >= 1 && std::find(params.begin(), params.end(), t) == params.end()) params.push_back(t);
    } else if (kernel == KASM3) {
        params = {8, 16, 32};
        mults = {1, 2, 4};
    } else if (kernel == KAPPLY) {
        params = {1, 2, 4, 8};
    } else {
        param = 0;
        mult = 4;
        return SF_OK;
    }
    hipStream_t s = b->ctx->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 1e30f;
    param = params[0];
    mult = mults[0];
    for (int prm : params) {
        HostTasks h = build_tasks(b, kernel, P, oi, pi, prm, io);
        if (h.t.empty()) break;
        TaskList tl{};
        void *mem = nullptr;
        if (e == hipSuccess) e = upload_tasks(h, tl, &mem);
        for (int m : mults) {
            if (e != hipSuccess) break;
            e = launch_kernel(kernel, tl, P, oi, pi, b->ncu * m, s);      // warm-up
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            for (int r = 0; r < 2 && e == hipSuccess; ++r) e = launch_kernel(kernel, tl, P, oi, pi, b->ncu * m, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && ms < best) {
                best = ms;
                param = prm;
                mult = m;
            }
        }
        (void)hipStreamSynchronize(s);
        (void)hipFree(mem);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(b->ctx, e, "autotuning batched kernels");
    b->tuned.push_back(sf_batch::Tuned{kernel, P, oi, pi, param, mult, best / 2});
    return SF_OK;
}

struct Plan {
    int kernel, P, oi, param, mult;
    TaskList tl;                  // device task list (owned by the batch)
};

// Task list of one planned launch, uploaded before any capture; it stays
// alive with the batch because captured graphs reference it.
static sf_status prepare_launch(sf_batch *b, Plan &pl, int pi, const BatchIO &io)
{
    HostTasks h = build_tasks(b, pl.kernel, pl.P, pl.oi, pi, pl.param, io);
    pl.tl = TaskList{};
    if (h.t.empty()) return SF_OK;
    void *mem = nullptr;
    hipError_t e = upload_tasks(h, pl.tl, &mem);
    if (mem) b->dev.push_back(mem);
    return e == hipSuccess ? SF_OK : hip_fail(b->ctx, e, "batch task list");
}

// The launches of one batched call, tuned (before any capture).
static sf_status plan_call(sf_batch *b, int kind, unsigned ops, int pi, const BatchIO &io_in, std::vector<Plan> &plan)
{
    std::vector<int> orders;
    for (sf_patch *p : b->patches)
        if (std::find(orders.begin(), orders.end(), p->P) == orders.end()) orders.push_back(p->P);
    std::sort(orders.begin(), orders.end());
    int param, mult;
    if (kind == 0) {
        plan.push_back(Plan{KROWPTR, 0, 0, 0, 4, {}});
        for (int P : orders) plan.push_back(Plan{KCOLIND, P, 0, 0, 4, {}});
        for (int oi = 0; oi < 2; ++oi) {
            if (!(ops & (oi == 0 ? SF_MASS : SF_STIFF))) continue;
            for (int P : orders) {
                for (int k : {KASM12, KASM3}) {
                    sf_status st = tune(b, k, P, oi, pi, io_in, param, mult);
                    if (st != SF_OK) return st;
                    plan.push_back(Plan{k, P, oi, param, mult, {}});
                }
            }
        }
    } else {
        const int oi = ops == SF_MASS ? 0 : 1;
        for (int P : orders) {
            sf_status st = tune(b, KAPPLY, P, oi, pi, io_in, param, mult);
            if (st != SF_OK) return st;
            plan.push_back(Plan{KAPPLY, P, oi, param, mult, {}});
        }
        // patches applied alone: their layers per workgroup, tuned on their
        // share of the call's vectors
        for (size_t i = 0; i < b->patches.size(); ++i) {
            sf_patch *p = b->patches[i];
            if (!apply_alone(p, oi, pi) || p->tune_lz[oi][pi] >= 0) continue;
            const int64_t r0 = b->row_off[i];
            sf_status st = tune_apply_lz(p, oi, pi, p->CA[oi][geom_storage(pi)], true, io_in.x + r0, io_in.y + r0);
            if (st != SF_OK) return st;
        }
    }
    for (Plan &pl : plan) {
        sf_status st = prepare_launch(b, pl, pi, io_in);
        if (st != SF_OK) return st;
    }
    return SF_OK;
}

// Record (or run, on the null stream) the launches of a batched call.
static sf_status record_call(sf_batch *b, int kind, unsigned ops, int pi, const BatchIO &io_in,
                             const std::vector<Plan> &plan, hipStream_t s)
{
    if (kind == 1) {
        hipError_t e = launch_fill(io_in.y, b->row_off.back(), 0.0, s);
        if (e != hipSuccess) return hip_fail(b->ctx, e, "fill");
    }
    for (const Plan &pl : plan) {
        if (pl.tl.nitems == 0) continue;
        hipError_t e = launch_kernel(pl.kernel, pl.tl, pl.P, pl.oi, pi, b->ncu * pl.mult, s);
        if (e != hipSuccess) return hip_fail(b->ctx, e, "batched kernel");
    }
    // patches the persistent kernels do not take (d < 3, assembled in chunks,
    // or applied alone)
    for (size_t i = 0; i < b->patches.size(); ++i) {
        sf_patch *p = b->patches[i];
        const int64_t r0 = b->row_off[i], z0 = b->nnz_off[i];
        for (int oi = 0; oi < 2; ++oi) {
            if (kind == 0 && !(ops & (oi == 0 ? SF_MASS : SF_STIFF))) continue;
            if (kind == 1 && oi != (ops == SF_MASS ? 0 : 1)) continue;
            const int kernel = kind == 0 ? KASM12 : KAPPLY;
            if (persistent_ok(p, kernel, oi, pi)) continue;
            hipError_t e;
            if (kind == 0) {
                double *dst = io_in.vals[oi] + z0;
                e = launch_assemble(p->view, oi + 1, asm_prec(pi), p->C[oi][cidx(pi)], dst, p->ws, p->ws_bytes, s);
            } else {
                const bool tiled = apply_alone(p, oi, pi);
                const void *C = tiled ? p->CA[oi][geom_storage(pi)] : p->C[oi][cidx(pi)];
                const int lz = p->tune_lz[oi][pi] > 0 ? p->tune_lz[oi][pi] : 0;
                e = launch_apply(p->view, oi + 1, apply_prec(pi), C, io_in.x + r0, io_in.y + r0, s, lz, p->rs[oi],
                                 tiled);
            }
            if (e != hipSuccess) return hip_fail(b->ctx, e, "per-patch kernel");
        }
    }
    return SF_OK;
}

static sf_status run_call(sf_batch *b, int kind, unsigned ops, int pi, const BatchIO &io, const void *k0,
                          const void *k1, const void *k2, const void *k3)
{
    sf_ctx *ctx = b->ctx;
    hipStream_t s = ctx->stream;
    for (auto &c : b->graphs)
        if (c.kind == kind && c.ops == ops && c.prec == pi && c.p0 == k0 && c.p1 == k1 && c.p2 == k2 && c.p3 == k3) {
            hipError_t e = hipGraphLaunch(c.exec, s);
            return e == hipSuccess ? SF_OK : hip_fail(ctx, e, "graph launch");
        }
    std::vector<Plan> plan;
    sf_status st = plan_call(b, kind, ops, pi, io, plan);
    if (st != SF_OK) return st;
    // a capture needs a non-default stream
    if (!s) return record_call(b, kind, ops, pi, io, plan, s);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(ctx, e, "begin capture");
    st = record_call(b, kind, ops, pi, io, plan, s);
    e = hipStreamEndCapture(s, &graph);
    if (st != SF_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "end capture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(ctx, e, "graph instantiate");
    b->graphs.push_back(sf_batch::Cached{kind, ops, pi, k0, k1, k2, k3, exec});
    e = hipGraphLaunch(exec, s);
    return e == hipSuccess ? SF_OK : hip_fail(ctx, e, "graph launch");
}

sf_status sf_batch_assemble(sf_batch *b, unsigned ops, sf_precision prec, int64_t *rp, int32_t *ci, double *vm,
                            double *vs)
{
    if (!b) return SF_EINVAL;
    b->ctx->err.clear();
    if (!rp || !ci) return fail(b->ctx, SF_EINVAL, "null pattern output");
    if (((ops & SF_MASS) && !vm) || ((ops & SF_STIFF) && !vs)) return fail(b->ctx, SF_EINVAL, "null output");
    int pi = 0;
    for (sf_patch *p : b->patches) {
        sf_status st = check_ready(p, ops, prec, pi, false);
        if (st != SF_OK) return st;
        st = ensure_workspace(p);
        if (st != SF_OK) return st;
    }
    BatchIO io;
    io.rp = rp;
    io.ci = ci;
    io.vals[0] = (ops & SF_MASS) ? vm : nullptr;
    io.vals[1] = (ops & SF_STIFF) ? vs : nullptr;
    return run_call(b, 0, ops, pi, io, rp, ci, io.vals[0], io.vals[1]);
}

sf_status sf_batch_apply(sf_batch *b, unsigned op, sf_precision prec, const double *x, double *y)
{
    if (!b) return SF_EINVAL;
    b->ctx->err.clear();
    if (op != SF_MASS && op != SF_STIFF) return fail(b->ctx, SF_EINVAL, "op must be SF_MASS or SF_STIFF");
    if (!x || !y || x == y) return fail(b->ctx, SF_EINVAL, "bad vectors");
    int pi = 0;
    for (sf_patch *p : b->patches) {
        sf_status st = check_ready(p, op, prec, pi, true);
        if (st != SF_OK) return st;
    }
    BatchIO io;
    io.x = x;
    io.y = y;
    return run_call(b, 1, op, pi, io, x, y, nullptr, nullptr);
}

void sf_batch_destroy(sf_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->ctx->stream);
    for (auto &c : b->graphs) (void)hipGraphExecDestroy(c.exec);
    for (void *m : b->dev) (void)hipFree(m);
    (void)hipFree(b->xl);
    (void)hipFree(b->yl);
    delete b;
}

sf_status sf_glue_map(int d, int npatch, const int32_t *nfun, int ninterface, const int32_t *iface, int64_t *map,
                      int64_t *n_global)
{
    if (d < 1 || d > 3 || npatch < 1 || ninterface < 0 || !nfun || !map || !n_global || (ninterface > 0 && !iface))
        return SF_EINVAL;
    std::vector<int64_t> off(npatch + 1, 0);
    for (int b = 0; b < npatch; ++b) {
        int64_t n = 1;
        for (int k = 0; k < d; ++k) {
            if (nfun[3 * b + k] < 1) return SF_EINVAL;
            n *= nfun[3 * b + k];
        }
        off[b + 1] = off[b] + n;
    }
    // union-find over the patch-local functions; roots are the smallest index
    std::vector<int64_t> parent(off[npatch]);
    for (int64_t i = 0; i < off[npatch]; ++i) parent[i] = i;
    auto find = [&](int64_t i) {
        int64_t r = i;
        while (parent[r] != r) r = parent[r];
        while (parent[i] != r) {
            const int64_t n = parent[i];
            parent[i] = r;
            i = n;
        }
        return r;
    };
    auto lin = [&](int b, const int *idx) {
        int64_t m = 0, stride = 1;
        for (int k = 0; k < d; ++k) {
            m += idx[k] * stride;
            stride *= nfun[3 * b + k];
        }
        return off[b] + m;
    };
    for (int f = 0; f < ninterface; ++f) {
        const int a = iface[4 * f], fa = iface[4 * f + 1], b = iface[4 * f + 2], fb = iface[4 * f + 3];
        if (a < 0 || a >= npatch || b < 0 || b >= npatch || fa < 0 || fa >= 2 * d || fb < 0 || fb >= 2 * d)
            return SF_EINVAL;
        const int ka = fa / 2, kb = fb / 2;
        int ta[2], tb[2], nt = 0;
        for (int k = 0, ia = 0, ib = 0; k < d; ++k) {
            if (k != ka) ta[ia++] = k;
            if (k != kb) tb[ib++] = k;
        }
        nt = d - 1;
        int cnt[2] = {1, 1};
        for (int j = 0; j < nt; ++j) {
            if (nfun[3 * a + ta[j]] != nfun[3 * b + tb[j]]) return SF_EINVAL;   // not conforming
            cnt[j] = nfun[3 * a + ta[j]];
        }
        for (int t1 = 0; t1 < cnt[1]; ++t1)
            for (int t0 = 0; t0 < cnt[0]; ++t0) {
                int ia[3] = {0, 0, 0}, ib[3] = {0, 0, 0};
                ia[ka] = fa % 2 ? nfun[3 * a + ka] - 1 : 0;
                ib[kb] = fb % 2 ? nfun[3 * b + kb] - 1 : 0;
                const int t[2] = {t0, t1};
                for (int j = 0; j < nt; ++j) {
                    ia[ta[j]] = t[j];
                    ib[tb[j]] = t[j];
                }
                const int64_t ra = find(lin(a, ia)), rb = find(lin(b, ib));
                if (ra != rb) parent[ra > rb ? ra : rb] = ra < rb ? ra : rb;
            }
    }
    // global ids in the order of first appearance (patch order, lexicographic)
    std::vector<int64_t> gid(off[npatch], -1);
    int64_t next = 0;
    for (int64_t i = 0; i < off[npatch]; ++i) {
        const int64_t r = find(i);
        if (gid[r] < 0) gid[r] = next++;
        map[i] = gid[r];
    }
    *n_global = next;
    return SF_OK;
}

sf_status sf_batch_apply_glued(sf_batch *b, unsigned op, sf_precision prec, const int64_t *dev_map, int64_t n_global,
                               const double *x, double *y)
{
    if (!b) return SF_EINVAL;
    sf_ctx *ctx = b->ctx;
    ctx->err.clear();
    if (!dev_map || !x || !y || x == y || n_global < 1) return fail(ctx, SF_EINVAL, "bad map or vectors");
    const int64_t nloc = b->row_off.back();
    hipStream_t s = ctx->stream;
    for (double **v : {&b->xl, &b->yl})
        if (!*v) {
            hipError_t e = hipMalloc((void **)v, sizeof(double) * (size_t)nloc);
            if (e != hipSuccess) {
                *v = nullptr;
                return hip_fail(ctx, e, "patch-local vectors of the glued apply");
            }
        }
    hipError_t e = launch_glue_gather(dev_map, nloc, n_global, x, b->xl, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "glued gather");
    sf_status st = sf_batch_apply(b, op, prec, b->xl, b->yl);
    if (st != SF_OK) return st;
    e = launch_fill(y, n_global, 0.0, s);
    if (e == hipSuccess) e = launch_glue_scatter(dev_map, nloc, n_global, b->yl, y, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "glued scatter");
    return SF_OK;
}

}  // extern "C"
