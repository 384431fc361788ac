#!/usr/bin/env python3
"""Benchmark of the sum-factorized IGA hot path on one MI355X.

Default workload (``--workload large``): d = 3, 128^3 elements, order p = 6
(N = 2,352,637 functions, 2,942,649,737 nonzeros, 452,984,832 quadrature
points), perturbed-Greville geometry, a(x) = 1 + 0.5 sin(2 pi x1) sin(2 pi x2)
sin(2 pi x3), stiffness, FP64.  One step = the whole hot path on inputs
resident in HBM:
  geometry step (Jacobian, inverse and determinant folded into the
  coefficient tensor, FP64) -> CSR pattern -> global sum-factorized assembly
  -> 100 matrix-free applies y = K x.
The same step then runs in the reduced-precision modes (FP32 contractions,
BF16 split) for a few steps each, with their errors against the oracle on the
same sampled rows ("mixed vs FP64 at stated error").  ``--workload single``
is the 48^3 order-4 patch with one apply per step.

Prints one JSON line.  ``value`` is the throughput of the whole step in
nonzeros per second: nnz / step time, in Gnnz/s.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "matrix-free apply GDoF/s + assembly Gnnz/s, mixed vs FP64 at stated rel. error"
PEAK_FP64_TFLOPS = 78.6          # 256 CU x 2.4 GHz x 64 FP64 FMA lanes x 2
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
COPY_BYTES = 1 << 30
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1809_05471_amd", "csrc")


def measured_traffic(name, sources):
    """HBM bytes per dispatch of the kernels listed in a committed counter
    summary ``profiles/<name>`` (FETCH_SIZE and WRITE_SIZE, each scaled by
    the same counter on a plain device copy of known size); None if the file
    is missing or the kernel sources changed since the counters were taken."""
    try:
        kv = {}
        for line in open(os.path.join(PROFILES, name)):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        h = hashlib.sha256(b"".join(open(os.path.join(CSRC, s), "rb").read() for s in sources)).hexdigest()
        if kv.get("source_sha256") != h:
            return None
        cb = float(kv["copy_bytes"])
        ff = float(kv["copy_fetch_kib"]) * 1024 / cb
        wf = float(kv["copy_write_kib"]) * 1024 / cb
        fetch = sum(float(kv[k]) for k in kv if k.endswith("_fetch_kib") and not k.startswith("copy"))
        write = sum(float(kv[k]) for k in kv if k.endswith("_write_kib") and not k.startswith("copy"))
        return (fetch / ff + write / wf) * 1024
    except (OSError, KeyError, ValueError):
        return None


def nnz1(N, p):
    return N * (2 * p - 1) - p * (p - 1)


def assembly_flops(K, p, op):
    """Algorithmic flops of Algorithm 1 with exact band sizes (eq. (sum
    factorization-nnz)): level i costs p^2 (prod_{l>=i} #X_l) nnz(A^{i-1})
    per (test, trial) pair; stiffness pairs are grouped as the kernel does
    (9 pairs at levels 1-2, 4 groups at level 3)."""
    Q = [k * p for k in K]
    N = [k + p - 1 for k in K]
    npair, ngroup = (9, 4) if op == "stiff" else (1, 1)
    fma = (npair * Q[2] * Q[1] * Q[0] * p * p
           + npair * Q[2] * Q[1] * p * p * nnz1(N[0], p)
           + ngroup * Q[2] * p * p * nnz1(N[0], p) * nnz1(N[1], p))
    return 2 * fma


def apply_flops(K, p, op):
    """Sum-factorized apply (Algorithms 3 and 2): forward contractions
    3 -> 2 -> 1, pointwise 3x3 product, backward 1 -> 2 -> 3."""
    Q = [k * p for k in K]
    N = [k + p - 1 for k in K]
    if op == "stiff":
        fwd = 2 * p * (2 * Q[2] * N[1] * N[0] + 3 * Q[2] * Q[1] * N[0] + 3 * Q[2] * Q[1] * Q[0])
        return 2 * fwd + 2 * 9 * Q[0] * Q[1] * Q[2]
    fwd = 2 * p * (Q[2] * N[1] * N[0] + Q[2] * Q[1] * N[0] + Q[2] * Q[1] * Q[0])
    return 2 * fwd + 2 * Q[0] * Q[1] * Q[2]


def coef_bytes_per_point(prec_name, op="stiff", p=6):
    """Stored bytes of the folded coefficient tensor per quadrature point (FP16
    split: 2 bytes per component plus an FP32 reference and scale per element
    and component, shared by its p^3 points)."""
    nc = 6 if op == "stiff" else 1
    if prec_name == "fp16":
        return nc * (2 + 8 / p ** 3)
    return nc * {"fp64": 8, "fp32": 4, "bf16": 4}[prec_name]


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["large", "single", "sweep", "batched", "order", "conv", "glued"], default="large",
                    help="large: d=3 128^3 order 6, geometry + pattern + assembly + 100 applies per step (the "
                         "headline line); single: 48^3 order 4 with one apply; sweep: matrix-free apply at "
                         "N = 126^3 for orders 2..9; batched: 512 patches; order: stiffness assembly of "
                         "anisotropic patches in the given and the relabelled contraction order; conv: "
                         "matrix-free convection product (FP64) at 128^3 order 6 and N = 126^3 for orders 2..9; "
                         "glued: stiffness product of the unit cube as 2 x 2 x 2 glued patches of 64^3 elements, "
                         "order 6, against the same patches unglued")
    ap.add_argument("--prec", choices=["fp64", "fp32", "bf16", "fp16"], default=None,
                    help="precision of the timed step (default fp64; sweep and batched: see their help)")
    ap.add_argument("--mixed-steps", type=int, default=3,
                    help="steps timed per reduced-precision mode after the headline (0: skip)")
    ap.add_argument("--applies", type=int, default=None, help="matrix-free applies per step")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (errors and CPU timing)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain device copy of %d bytes first (scale factor for HBM counters)" % COPY_BYTES)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the sharding design is described in the design notes); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        # plain device copy of known size, for scaling the HBM counters of a profiled run
        src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "sweep":
        return run_sweep(args)
    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "order":
        return run_order(args)
    if args.workload == "conv":
        return run_conv(args)
    if args.workload == "glued":
        return run_glued(args)
    return run_patch(args)


def _sample_rows(P, p, precs_bytes):
    """Rows for the error check: first / middle / last index per direction,
    the clipped-band indices 1, p-2, N-p+1, N-2 one direction at a time, and
    rows just after every level-3 chunk boundary of the assembly (entries
    summed over two chunks)."""
    n = P.nfun
    base = [[0, v // 2, v - 1] for v in n]
    clip = [[1, p - 2, v - p + 1, v - 2] for v in n]
    idx = set()
    for j in range(4):
        axes = [clip[k] if k == j - 1 else base[k] for k in range(3)]
        for a in axes[0]:
            for b in axes[1]:
                for c in axes[2]:
                    idx.add((a, b, c))
    hw = (p - 1) * (2 * p - 1) + p
    plane = 4 * n[1] * n[0] * hw
    layers = min(max((4096 << 20) // (plane * 8 * p), p - 1), P.nel[2])
    for eb in precs_bytes:
        chunk = min(layers * 8 // eb, P.nel[2])
        for s0 in range(chunk, P.nel[2], chunk):
            for m3 in range(s0, min(s0 + p - 1, n[2])):
                idx.add((n[0] // 2, n[1] // 2, m3))
    return np.array(sorted(a + n[0] * (b + n[1] * c) for a, b, c in idx), dtype=np.int64)


def run_patch(args):
    import torch

    import paper_1809_05471_amd as sf
    from paper_1809_05471_amd import inputs
    large = args.workload == "large"
    K, p = ((128, 128, 128), 6) if large else ((48, 48, 48), 4)
    applies = args.applies if args.applies is not None else (100 if large else 1)
    head_prec = args.prec or "fp64"
    precs = {"fp64": sf.SF_FP64, "fp32": sf.SF_FP32, "bf16": sf.SF_BF16_SPLIT, "fp16": sf.SF_FP16_SPLIT}
    # precision of (geometry step, assembly, applies) per mode: BF16 split is
    # a mode of the assembly and FP16 split a storage of the apply, so those
    # steps take FP32 for the other stage
    plan = {"fp64": ("fp64", "fp64", "fp64"), "fp32": ("fp32", "fp32", "fp32"),
            "bf16": ("bf16", "bf16", "fp32"), "fp16": ("fp16", "fp32", "fp16")}
    w = inputs.workload_3d(K, p)
    stream = torch.cuda.current_stream()
    ctx = sf.sf_ctx_create(0, stream.cuda_stream)
    t_tab = time.perf_counter()
    h = sf.sf_patch_create(ctx, 3, p, w["knots"], w["ctrl"])
    t_tab = time.perf_counter() - t_tab
    N, nnz, Q = sf.sf_patch_info(h)
    sf.sf_patch_set_coef(ctx, h, sf.SF_STIFF, sf.SF_COEF_SINPROD, 0.5)
    rp = torch.empty(N + 1, dtype=torch.int64, device="cuda")
    ci = torch.empty(nnz, dtype=torch.int32, device="cuda")
    vals = torch.empty(nnz, dtype=torch.float64, device="cuda")
    x = torch.as_tensor(w["x"]).cuda()
    y = torch.empty(N, dtype=torch.float64, device="cuda")

    def step(mode, ev):
        pg, pa, py = (precs[m] for m in plan[mode])
        if ev:
            ev[0].record(stream)
        # geometry step queued without a host round trip; its det J test is
        # read back once, after the timed steps (sf_patch_geometry_check)
        sf.sf_patch_prepare_async(ctx, h, sf.SF_STIFF, pg)
        if ev:
            ev[1].record(stream)
        sf.sf_csr_pattern(ctx, h, rp, ci)
        if ev:
            ev[2].record(stream)
        sf.sf_assemble(ctx, h, sf.SF_STIFF, pa, val_stiff=vals)
        if ev:
            ev[3].record(stream)
        for _ in range(applies):
            sf.sf_apply(ctx, h, sf.SF_STIFF, py, x, y)
        if ev:
            ev[4].record(stream)

    def timed(prec, steps, warmup):
        for _ in range(warmup):
            step(prec, None)
        # HIP events on the library's stream (torch's current stream, handed to the context)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            step(prec, evs[k])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sf.sf_patch_geometry_check(ctx, h)             # raises SfError(SF_EGEOM) on det J <= 0
        st = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(4)] for e in evs]).mean(axis=0)
        return (t1 - t0) / steps * 1e3, st.tolist()

    def device_rows(rows):
        rpn = rp.cpu().numpy()
        segs = [np.arange(rpn[r], rpn[r + 1]) for r in rows]
        gidx = torch.as_tensor(np.concatenate(segs)).cuda()
        vg, cg = vals[gidx].cpu().numpy(), ci[gidx].cpu().numpy()
        out, o = [], 0
        for sg in segs:
            out.append((cg[o:o + len(sg)].astype(np.int64), vg[o:o + len(sg)]))
            o += len(sg)
        return out, y.cpu().numpy()[rows]

    ms_step, (geom_ms, pat_ms, asm_ms, app_ms) = timed(head_prec, args.steps, args.warmup)
    app_ms /= applies
    # sampled rows of every mode's results, for the error check against the oracle
    got = {}
    oracle_rows = None
    if not args.no_cpu_baseline:
        import oracle
        P = oracle.Problem(w["knots"], p, w["ctrl"], w["coef"])
        oracle_rows = _sample_rows(P, p, (8, 4))
        got[head_prec] = device_rows(oracle_rows)

    # reduced-precision modes of the same step ("mixed vs FP64")
    modes = {}
    if args.mixed_steps > 0:
        for name in ("fp64", "fp32", "bf16", "fp16"):
            if name == head_prec:
                continue
            try:
                ms, (g_ms, p_ms, a_ms, y_ms) = timed(name, args.mixed_steps, 1)
            except sf.SfError as e:          # a mode the library does not build
                modes[name] = {"status": str(e)}
                continue
            modes[name] = {"precision_geometry_assembly_apply": list(plan[name]),
                           "ms_per_step": ms, "value_gnnz_s": nnz / (ms * 1e-3) / 1e9,
                           "stages_ms": {"geometry": g_ms, "pattern": p_ms, "assembly": a_ms,
                                         "apply": y_ms / applies},
                           "assembly_gnnz_s": nnz / (a_ms * 1e-3) / 1e9,
                           "apply_gdof_s": N / (y_ms / applies * 1e-3) / 1e9,
                           "apply_hbm_frac": (Q * coef_bytes_per_point(plan[name][2], p=p) + 16 * N)
                           / (y_ms / applies * 1e-3) / 1e9 / PEAK_HBM_GBS}
            if oracle_rows is not None:
                got[name] = device_rows(oracle_rows)

    fl_asm = assembly_flops(K, p, "stiff")
    fl_app = apply_flops(K, p, "stiff")
    asm_bytes = Q * coef_bytes_per_point(plan[head_prec][1], p=p) + nnz * 8
    app_bytes = Q * coef_bytes_per_point(plan[head_prec][2], p=p) + 2 * N * 8
    asm_tflops = fl_asm / (asm_ms * 1e-3) / 1e12
    asm_peak = PEAK_FP64_TFLOPS if head_prec == "fp64" else PEAK_FP32_TFLOPS
    tag = "d3_128_p6" if large else "d3_48_p4"
    asm_traffic = measured_traffic(f"traffic_assembly_{tag}_{head_prec}.txt", ["assemble.hip"])
    app_traffic = measured_traffic(f"traffic_apply_{tag}_{head_prec}.txt", ["apply.hip"])
    roof_asm = {"kernel": "assembly (asm12_kernel levels 1-2 + asm3_kernel level 3, one sf_assemble call)",
                "bound": "alu", "achieved": asm_tflops, "peak": asm_peak, "unit": "TFLOP/s",
                "frac": asm_tflops / asm_peak, "traffic": asm_traffic, "algorithmic_flops": fl_asm,
                "algorithmic_bytes": asm_bytes, "achieved_GBs": asm_bytes / (asm_ms * 1e-3) / 1e9}
    app_gbs = app_bytes / (app_ms * 1e-3) / 1e9
    roof_app = {"kernel": "apply3d_kernel (one sf_apply: y cleared by a fill kernel, then the apply)",
                "bound": "hbm", "achieved": app_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": app_gbs / PEAK_HBM_GBS, "traffic": app_traffic, "algorithmic_bytes": app_bytes,
                "algorithmic_flops": fl_app, "achieved_TFLOPs": fl_app / (app_ms * 1e-3) / 1e12}
    # the dominant kernel of the step: the applies at 128^3 (100 per step), else the assembly
    dominant = roof_app if applies * app_ms > asm_ms else roof_asm
    out = {
        "metric": METRIC,
        "value": nnz / (ms_step * 1e-3) / 1e9,
        "unit": "Gnnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16x3+f32", "fp16": "f16split+f32"}[head_prec],
        "data": "synthetic",
        "config": {"workload": f"d3_{K[0]}x{K[1]}x{K[2]}_p{p}_perturbed_stiffness_geometry_pattern_assembly_"
                               f"plus_{applies}_applies",
                   "d": 3, "elements": list(K), "order": p, "ndof": N, "nnz": nnz, "nquad": Q,
                   "coefficient": "1+0.5*sin(2pi x1)sin(2pi x2)sin(2pi x3)",
                   "precision": head_prec, "applies_per_step": applies},
        "stages_ms": {"geometry": geom_ms, "pattern": pat_ms, "assembly": asm_ms, "apply": app_ms,
                      "applies_total": app_ms * applies, "tables_host_once": t_tab * 1e3},
        "assembly_gnnz_s": nnz / (asm_ms * 1e-3) / 1e9,
        "apply_gdof_s": N / (app_ms * 1e-3) / 1e9,
        "apply_hbm_frac": app_gbs / PEAK_HBM_GBS,
        "roofline": dominant,
        "roofline_assembly": roof_asm,
        "roofline_apply": roof_app,
        "modes": modes,
    }
    sf.sf_patch_destroy(h)
    sf.sf_ctx_destroy(ctx)
    del vals, ci, rp, x, y
    torch.cuda.empty_cache()
    if oracle_rows is not None:
        out.update(cpu_leg(P, w, p, K, N, nnz, applies, oracle_rows, got, head_prec, modes))
    print(json.dumps(out), flush=True)


def cpu_leg(P, w, p, K, N, nnz, applies, rows, got, head_prec, modes):
    """Oracle leg: errors of every mode's GPU results on the sampled rows, and
    the oracle's own throughput on sub-boxes of the same recipe, scaled to the
    full patch by element count (its cost is the same per element)."""
    import oracle
    from paper_1809_05471_amd import inputs
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    x = w["x"]
    ref = P.rows(oracle.STIFF, rows, threads)
    vmax = max(np.abs(v).max() for _, v in ref)
    yref = np.array([v @ x[c] for c, v in ref])
    scale = max(np.abs(v) @ np.abs(x[c]) for c, v in ref)
    errs = {}
    for name, (rws, yg) in got.items():
        for (c, v), (cg, vg) in zip(ref, rws):
            assert np.array_equal(c, cg), "pattern differs from the oracle's"
        eA = max(np.abs(vg - v).max() for (_, v), (_, vg) in zip(ref, rws)) / vmax
        ey = np.abs(yg - yref).max() / scale
        errs[name] = (float(eA), float(ey))
    for name in modes:
        if name in errs:
            modes[name]["err_A"], modes[name]["err_y"] = errs[name]

    # oracle timing on sub-boxes: all threads on ks^3 elements, one thread on k1^3
    ks, k1 = (10, 4) if p >= 6 else (24, 8)
    ws = inputs.workload_3d((ks,) * 3, p)
    Ps = oracle.Problem(ws["knots"], p, ws["ctrl"], ws["coef"])
    pat = Ps.pattern()
    t0 = time.perf_counter()
    Ps.assemble(oracle.STIFF, threads, pattern=pat)
    t_asm = time.perf_counter() - t0
    t0 = time.perf_counter()
    Ps.apply(oracle.STIFF, ws["x"], threads)
    t_app = time.perf_counter() - t0
    w1 = inputs.workload_3d((k1,) * 3, p)
    P1 = oracle.Problem(w1["knots"], p, w1["ctrl"], w1["coef"])
    pat1 = P1.pattern()
    t0 = time.perf_counter()
    P1.assemble(oracle.STIFF, 1, pattern=pat1)
    t_asm1 = time.perf_counter() - t0
    nel_full = K[0] * K[1] * K[2]
    f, f1 = nel_full / ks ** 3, nel_full / k1 ** 3
    t_step = t_asm * f + applies * t_app * f
    return {
        "err_A": errs[head_prec][0], "err_y": errs[head_prec][1], "err_rows_sampled": int(len(rows)),
        "cpu_baseline": {
            "value": nnz / t_step / 1e9, "unit": "Gnnz/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"extrapolated: the oracle's element-by-element stiffness assembly (cost N p^3d) and "
                      f"matrix-free apply of the {ks}^3-element order-{p} patch of the same recipe on {threads} "
                      f"threads ({t_asm:.2f} s and {t_app:.2f} s), scaled by element count ({f:.0f}x) to the "
                      f"{K[0]}^3 step of one assembly and {applies} applies",
            "assembly_s_extrapolated": t_asm * f, "apply_s_extrapolated": t_app * f,
            "apply_gdof_s": N / (t_app * f) / 1e9,
            "one_thread": {"sample": f"assembly of the {k1}^3-element patch on 1 thread: {t_asm1:.2f} s",
                           "assembly_s_extrapolated": t_asm1 * f1,
                           "assembly_gnnz_s": nnz / (t_asm1 * f1) / 1e9},
            "seconds": t_asm + t_app + t_asm1},
    }


def _prec_list(args, sf):
    allp = {"fp64": sf.SF_FP64, "fp32": sf.SF_FP32, "fp16": sf.SF_FP16_SPLIT}
    return list(allp.items()) if args.prec is None else [(args.prec, allp[args.prec])]


def run_sweep(args):
    """Matrix-free stiffness apply, d = 3, K = 127 - p per direction (N = 126^3),
    orders 2..9, one JSON line per (order, precision)."""
    import torch

    import paper_1809_05471_amd as sf
    from paper_1809_05471_amd import inputs
    stream = torch.cuda.current_stream()
    ctx = sf.sf_ctx_create(0, stream.cuda_stream)
    for p in range(2, 10):
        w = inputs.workload_order_sweep(p)
        K = w["K"]
        h = sf.sf_patch_create(ctx, 3, p, w["knots"], w["ctrl"])
        N, nnz, Q = sf.sf_patch_info(h)
        sf.sf_patch_set_coef(ctx, h, sf.SF_STIFF, sf.SF_COEF_SINPROD, 0.5)
        x = torch.as_tensor(w["x"]).cuda()
        y = torch.empty(N, dtype=torch.float64, device="cuda")
        for name, prec in _prec_list(args, sf):
            sf.sf_patch_prepare(ctx, h, sf.SF_STIFF, prec)
            for _ in range(args.warmup):
                sf.sf_apply(ctx, h, sf.SF_STIFF, prec, x, y)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                sf.sf_apply(ctx, h, sf.SF_STIFF, prec, x, y)
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            byts = Q * coef_bytes_per_point(name, p=p) + 16 * N
            print(json.dumps({
                "metric": "matrix-free apply GDoF/s", "value": N / (ms * 1e-3) / 1e9, "unit": "GDoF/s",
                "ms": ms, "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f16split+f32"}[name],
                "config": {"workload": f"d3_{K[0]}^3_p{p}_stiffness_apply", "order": p, "ndof": N, "nquad": Q},
                "roofline": {"bound": "hbm", "achieved": byts / (ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
                             "unit": "GB/s", "frac": byts / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                             "algorithmic_bytes": byts, "algorithmic_flops": apply_flops(K, p, "stiff")}}),
                flush=True)
        sf.sf_patch_destroy(h)
        del x, y
        torch.cuda.empty_cache()
    sf.sf_ctx_destroy(ctx)


def run_conv(args):
    """Matrix-free convection product (b . grad u, FP64), d = 3: 128^3 order 6
    (with err_y on sampled rows against the oracle unless --no-cpu-baseline)
    and K = 127 - p per direction for orders 2..9; one JSON line each.
    Algorithmic bytes: the three folded coefficients per point, x read and y
    written once."""
    import torch

    import paper_1809_05471_amd as sf
    from paper_1809_05471_amd import inputs
    stream = torch.cuda.current_stream()
    ctx = sf.sf_ctx_create(0, stream.cuda_stream)
    b, alpha = (0.6, -0.9, 1.1), 0.5
    cases = [((128, 128, 128), 6, inputs.workload_3d((128, 128, 128), 6))]
    cases += [(w["K"], p, w) for p, w in ((p, inputs.workload_order_sweep(p)) for p in range(2, 10))]
    for K, p, w in cases:
        h = sf.sf_patch_create(ctx, 3, p, w["knots"], w["ctrl"])
        N, nnz, Q = sf.sf_patch_info(h)
        sf.sf_patch_set_coef(ctx, h, sf.SF_CONV, sf.SF_COEF_SINPROD, alpha)
        sf.sf_patch_set_convection(ctx, h, b)
        sf.sf_patch_prepare(ctx, h, sf.SF_CONV, sf.SF_FP64)
        x = torch.as_tensor(w["x"]).cuda()
        y = torch.empty(N, dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            sf.sf_apply(ctx, h, sf.SF_CONV, sf.SF_FP64, x, y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            sf.sf_apply(ctx, h, sf.SF_CONV, sf.SF_FP64, x, y)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        byts = 24 * Q + 16 * N
        line = {
            "metric": "matrix-free apply GDoF/s", "value": N / (ms * 1e-3) / 1e9, "unit": "GDoF/s", "ms": ms,
            "dtype": "f64", "config": {"workload": f"d3_{K[0]}^3_p{p}_convection_apply", "order": p, "ndof": N,
                                       "nquad": Q},
            "roofline": {"bound": "hbm", "achieved": byts / (ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": byts / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                         "traffic": (measured_traffic("traffic_conv_d3_128_p6_fp64.txt", ["conv.hip"])
                                     if K[0] == 128 else None),
                         "algorithmic_bytes": byts}}
        if K[0] == 128 and not args.no_cpu_baseline:
            import oracle
            P = oracle.Problem(w["knots"], p, w["ctrl"], ("sinprod", alpha), conv_b=b)
            rows = _sample_rows(P, p, [])
            xh = np.asarray(w["x"], dtype=np.float64)
            yref = P.apply_rows_by_elements(oracle.CONV, xh, rows)
            den = max(float(np.abs(v) @ np.abs(xh[c])) for c, v in P.rows(oracle.CONV, rows))
            line["err_y"] = float(np.abs(y.cpu().numpy()[rows] - yref).max() / den)
            line["err_rows"] = int(len(rows))
        print(json.dumps(line), flush=True)
        sf.sf_patch_destroy(h)
        del x, y
        torch.cuda.empty_cache()
    sf.sf_ctx_destroy(ctx)


def run_glued(args):
    """The unit cube as 2 x 2 x 2 patches of 64^3 elements at order 6 (each
    the identity map of its octant), glued at their faces: y = sum_b R_b^T
    K_b R_b x (sf_batch_apply_glued), timed beside sf_batch_apply on the
    same patches (the gather and scatter are the difference).  FP64 unless
    --prec fp32; on a side stream (captured graphs)."""
    import torch

    import paper_1809_05471_amd as sf
    from paper_1809_05471_amd import inputs
    prec = sf.SF_FP32 if args.prec == "fp32" else sf.SF_FP64
    Kp, p = 64, 6
    stream = torch.cuda.Stream()
    ctx = sf.sf_ctx_create(0, stream.cuda_stream)
    kn = inputs.open_uniform_knots(Kp, p)
    g1 = inputs.greville(kn, p) * 0.5
    hs, nf = [], []
    with torch.cuda.stream(stream):
        for c in np.ndindex(2, 2, 2):
            axes = [g1 + 0.5 * c[k] for k in range(3)]
            grid = np.meshgrid(*axes[::-1], indexing="ij")
            ctrl = np.stack([grid[2 - k].ravel() for k in range(3)], axis=1)
            h = sf.sf_patch_create(ctx, 3, p, [kn] * 3, ctrl)
            sf.sf_patch_set_coef(ctx, h, sf.SF_STIFF, sf.SF_COEF_SINPROD, 0.5)
            sf.sf_patch_prepare(ctx, h, sf.SF_STIFF, prec)
            hs.append(h)
            nf.append([Kp + p - 1] * 3)
        ids = {c: i for i, c in enumerate(np.ndindex(2, 2, 2))}
        ifc = []
        for c, i in ids.items():
            for k in range(3):
                if c[k] == 0:
                    q = list(c)
                    q[k] = 1
                    ifc.append((i, 2 * k + 1, ids[tuple(q)], 2 * k))
        m, ng = sf.sf_glue_map(3, nf, ifc)
        bt = sf.sf_batch_create(ctx, hs)
        nloc = len(m)
        dmap = torch.as_tensor(m).cuda()
        x = torch.as_tensor(inputs.random_vector(ng, 0)).cuda()
        y = torch.empty(ng, dtype=torch.float64, device="cuda")
        xl = torch.as_tensor(inputs.random_vector(nloc, 0)).cuda()
        yl = torch.empty(nloc, dtype=torch.float64, device="cuda")
        out = {}
        for name, call in (("glued", lambda: sf.sf_batch_apply_glued(ctx, bt, sf.SF_STIFF, prec, dmap, ng, x, y)),
                           ("unglued", lambda: sf.sf_batch_apply(ctx, bt, sf.SF_STIFF, prec, xl, yl))):
            for _ in range(max(args.warmup, 1)):
                call()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                call()
            e1.record(stream)
            e1.synchronize()
            out[name] = e0.elapsed_time(e1) / args.steps
        Q = 8 * (Kp * p) ** 3
        byts = Q * coef_bytes_per_point("fp64" if prec == sf.SF_FP64 else "fp32", p=p) + 16 * nloc
        ms = out["glued"]
        print(json.dumps({
            "metric": "matrix-free apply GDoF/s", "value": ng / (ms * 1e-3) / 1e9, "unit": "GDoF/s", "ms": ms,
            "dtype": "f64" if prec == sf.SF_FP64 else "f32",
            "config": {"workload": f"d3_glued_2x2x2_patches_{Kp}^3_p{p}_stiffness_apply", "order": p,
                       "ndof_global": ng, "ndof_local": nloc, "nquad": Q},
            "unglued_batch_apply_ms": out["unglued"],
            "roofline": {"bound": "hbm", "achieved": byts / (ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": byts / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, "algorithmic_bytes": byts}}), flush=True)
        sf.sf_batch_destroy(bt)
        for h in hs:
            sf.sf_patch_destroy(h)
    sf.sf_ctx_destroy(ctx)


def run_order(args):
    """Stiffness assembly (FP64) of anisotropic patches with the given
    contraction order (direction 3 last), with the cyclic relabelling that
    contracts the direction of fewest elements last, and with the tuner's
    choice; one JSON line per patch."""
    import torch

    import paper_1809_05471_amd as sf
    from paper_1809_05471_amd import inputs
    stream = torch.cuda.current_stream()
    ctx = sf.sf_ctx_create(0, stream.cuda_stream)
    for K, p in (((16, 128, 128), 4), ((2, 128, 128), 6), ((128, 4, 128), 4), ((128, 128, 16), 4)):
        w = inputs.workload_3d(K, p)
        res = {}
        for policy in ("given", "relabelled", "tune"):
            os.environ["SFIGA_ASSEMBLY_ORDER"] = policy
            h = sf.sf_patch_create(ctx, 3, p, w["knots"], w["ctrl"])
            N, nnz, Q = sf.sf_patch_info(h)
            sf.sf_patch_set_coef(ctx, h, sf.SF_STIFF, sf.SF_COEF_SINPROD, 0.5)
            sf.sf_patch_prepare(ctx, h, sf.SF_STIFF, sf.SF_FP64)
            v = torch.empty(nnz, dtype=torch.float64, device="cuda")
            for _ in range(args.warmup + 1):
                sf.sf_assemble(ctx, h, sf.SF_STIFF, sf.SF_FP64, val_stiff=v)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                sf.sf_assemble(ctx, h, sf.SF_STIFF, sf.SF_FP64, val_stiff=v)
            e1.record(stream)
            e1.synchronize()
            res[policy] = e0.elapsed_time(e1) / args.steps
            sf.sf_patch_destroy(h)
            del v
        os.environ.pop("SFIGA_ASSEMBLY_ORDER", None)
        kmin = min(range(3), key=lambda k: K[k])
        Kr = tuple(K[(k + (kmin + 1) % 3) % 3] for k in range(3))
        print(json.dumps({
            "metric": "assembly ms, contraction order", "unit": "ms", "dtype": "f64",
            "config": {"workload": f"d3_{K[0]}x{K[1]}x{K[2]}_p{p}_stiffness_assembly", "elements": list(K),
                       "order": p, "nnz": nnz},
            "ms_given_order": res["given"], "ms_relabelled": res["relabelled"], "ms_tuned": res["tune"],
            "relabelled_elements": list(Kr),
            "algorithmic_flops_given": assembly_flops(K, p, "stiff"),
            "algorithmic_flops_relabelled": assembly_flops(Kr, p, "stiff")}), flush=True)
        torch.cuda.empty_cache()
    sf.sf_ctx_destroy(ctx)


def run_batched(args):
    """512 independent patches (K ~ U{4..32} per direction, p ~ U{2..6}),
    mass and stiffness CSR assembly plus one stiffness apply per step, all
    in captured persistent launches."""
    import torch

    import paper_1809_05471_amd as sf
    from paper_1809_05471_amd import inputs
    prec = sf.SF_FP32 if (args.prec or "fp32") == "fp32" else sf.SF_FP64
    stream = torch.cuda.Stream()            # captured graphs need a non-default stream
    ctx = sf.sf_ctx_create(0, stream.cuda_stream)
    Ks, ps = inputs.batched_draw(512, seed=2)
    hs = []
    with torch.cuda.stream(stream):
        for b in range(512):
            kn, ctrl, _ = inputs.batched_patch(b, Ks[b], ps[b])
            h = sf.sf_patch_create(ctx, 3, int(ps[b]), kn, ctrl)
            sf.sf_patch_prepare(ctx, h, sf.SF_MASS | sf.SF_STIFF, prec)
            hs.append(h)
        bt = sf.sf_batch_create(ctx, hs)
        ro, zo = sf.sf_batch_offsets(ctx, bt, 512)
        N, Z = int(ro[-1]), int(zo[-1])
        rp = torch.empty(N + 1, dtype=torch.int64, device="cuda")
        ci = torch.empty(Z, dtype=torch.int32, device="cuda")
        vm = torch.empty(Z, dtype=torch.float64, device="cuda")
        vs = torch.empty(Z, dtype=torch.float64, device="cuda")
        x = torch.as_tensor(np.concatenate([inputs.batched_patch(b, Ks[b], ps[b])[2] for b in range(512)])).cuda()
        y = torch.empty(N, dtype=torch.float64, device="cuda")
        t0 = time.perf_counter()
        sf.sf_batch_assemble(ctx, bt, sf.SF_MASS | sf.SF_STIFF, prec, rp, ci, vm, vs)
        sf.sf_batch_apply(ctx, bt, sf.SF_STIFF, prec, x, y)
        stream.synchronize()
        t_tune = time.perf_counter() - t0
        for _ in range(args.warmup):
            sf.sf_batch_assemble(ctx, bt, sf.SF_MASS | sf.SF_STIFF, prec, rp, ci, vm, vs)
            sf.sf_batch_apply(ctx, bt, sf.SF_STIFF, prec, x, y)
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
        stream.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            ev[k][0].record(stream)
            sf.sf_batch_assemble(ctx, bt, sf.SF_MASS | sf.SF_STIFF, prec, rp, ci, vm, vs)
            ev[k][1].record(stream)
            sf.sf_batch_apply(ctx, bt, sf.SF_STIFF, prec, x, y)
            ev[k][2].record(stream)
        stream.synchronize()
        ms_step = (time.perf_counter() - t0) / args.steps * 1e3
    asm_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    app_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    print(json.dumps({
        "metric": "assembly Gnnz/s (mass + stiffness) and apply GDoF/s, batched", "value": 2 * Z / (ms_step * 1e-3) / 1e9,
        "unit": "Gnnz/s", "ms_per_step": ms_step, "steps": args.steps, "warmup": args.warmup,
        "dtype": "f64" if prec == sf.SF_FP64 else "f32",
        "config": {"workload": "batched_512_patches_K4-32_p2-6_mass_stiffness_plus_apply", "npatch": 512,
                   "ndof": N, "nnz_per_operator": Z},
        "stages_ms": {"assembly_mass_stiffness": asm_ms, "apply": app_ms, "first_call_tune_capture_s": t_tune},
        "assembly_gnnz_s": 2 * Z / (asm_ms * 1e-3) / 1e9, "apply_gdof_s": N / (app_ms * 1e-3) / 1e9}), flush=True)
    sf.sf_batch_destroy(bt)
    for h in hs:
        sf.sf_patch_destroy(h)
    sf.sf_ctx_destroy(ctx)


if __name__ == "__main__":
    main()
