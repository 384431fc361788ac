#!/usr/bin/env python3
"""Benchmark of the sum-factorized IGA hot path on one MI355X.

Default workload: d = 3, 48^3 elements, order p = 4, perturbed-Greville
geometry, a(x) = 1 + 0.5 sin(2 pi x1) sin(2 pi x2) sin(2 pi x3), stiffness,
FP64.  One step = the whole hot path on inputs resident in HBM:
  geometry step (Jacobian, inverse, determinant folded into the coefficient
  tensor) -> CSR pattern -> global sum-factorized assembly -> one
  matrix-free apply y = K x.
The 1D tables are built once at patch creation (host, cost sum p^2 #X) and
reported separately.

Prints one JSON line.  ``value`` is the assembly throughput of the whole
step: nnz / step time, in Gnnz/s.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "matrix-free apply GDoF/s + assembly Gnnz/s, mixed vs FP64 at stated rel. error"
PEAK_FP64_TFLOPS = 78.6          # 256 CU x 2.4 GHz x 64 FP64 FMA lanes x 2
PEAK_HBM_GBS = 8000.0
COPY_BYTES = 1 << 30
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_assembly_d3_48_p4_fp64.txt")


def measured_traffic(source):
    """HBM bytes of one assembly call from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE of its kernels, each scaled by the same counter
    on a plain copy of known size); None if the kernels changed since."""
    import hashlib
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        h = hashlib.sha256(open(source, "rb").read()).hexdigest()
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["single", "large", "sweep", "batched"], default="single",
                    help="single: d=3 48^3 order 4 (the headline line); large: 128^3 order 6 with 100 applies per "
                         "step; sweep: matrix-free apply at N = 126^3 for orders 2..9; batched: 512 patches")
    ap.add_argument("--prec", choices=["fp64", "fp32", "bf16"], default=None)
    ap.add_argument("--elements", type=int, default=48)
    ap.add_argument("--order", type=int, default=4)
    ap.add_argument("--applies", type=int, default=1, help="matrix-free applies per step")
    ap.add_argument("--cpu-sample-elements", type=int, default=48,
                    help="elements per direction of the patch the oracle assembles for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    import paper_1809_05471_amd as sf
    from paper_1809_05471_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "sweep":
        return run_sweep(args)
    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "large":
        args.elements, args.order = 128, 6
        args.applies = max(args.applies, 100)
        args.prec = args.prec or "fp32"
        args.no_cpu_baseline = True
    prec = {"fp64": sf.SF_FP64, "fp32": sf.SF_FP32, "bf16": sf.SF_BF16_SPLIT}[args.prec or "fp64"]
    K = (args.elements,) * 3
    p = args.order
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

    def step(ev):
        if ev:
            ev[0].record(stream)
        # geometry step queued without a host round trip; its det J test is
        # read back once, after the timed steps (sf_patch_geometry_check)
        sf.sf_patch_prepare_async(ctx, h, sf.SF_STIFF, prec)
        if ev:
            ev[1].record(stream)
        sf.sf_csr_pattern(ctx, h, rp, ci)
        if ev:
            ev[2].record(stream)
        sf.sf_assemble(ctx, h, sf.SF_STIFF, prec, val_stiff=vals)
        if ev:
            ev[3].record(stream)
        for _ in range(args.applies):
            sf.sf_apply(ctx, h, sf.SF_STIFF, prec, x, y)
        if ev:
            ev[4].record(stream)

    if args.calibrate_copy:
        # plain device copy of known size, for scaling the HBM counters of a profiled run
        src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step(None)
    # HIP events on the library's stream (torch's current stream, handed to the context)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sf.sf_patch_geometry_check(ctx, h)             # raises SfError(SF_EGEOM) on det J <= 0
    ms_per_step = (t1 - t0) / args.steps * 1e3
    stage_ms = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(4)] for e in evs]).mean(axis=0)
    geom_ms, pat_ms, asm_ms, app_ms = stage_ms.tolist()
    app_ms /= args.applies

    fl_asm = assembly_flops(K, p, "stiff")
    fl_app = apply_flops(K, p, "stiff")
    esz = 8 if prec == sf.SF_FP64 else 4
    c_bytes = 6 * Q * esz
    asm_bytes = c_bytes + nnz * 8
    app_bytes = c_bytes + 2 * N * 8
    asm_tflops = fl_asm / (asm_ms * 1e-3) / 1e12
    traffic = measured_traffic(os.path.join(ROOT, "paper_1809_05471_amd", "csrc", "assemble.hip")) \
        if (K, p, prec) == ((48, 48, 48), 4, sf.SF_FP64) else None
    roofline = {"kernel": "assembly (asm12_kernel levels 1-2 + asm3_kernel level 3, one sf_assemble call)",
                "bound": "alu", "achieved": asm_tflops,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": asm_tflops / PEAK_FP64_TFLOPS,
                "traffic": traffic,
                "algorithmic_flops": fl_asm, "algorithmic_bytes": asm_bytes,
                "achieved_GBs": asm_bytes / (asm_ms * 1e-3) / 1e9}
    out = {
        "metric": METRIC,
        "value": nnz / (ms_per_step * 1e-3) / 1e9,
        "unit": "Gnnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {sf.SF_FP64: "f64", sf.SF_FP32: "f32", sf.SF_BF16_SPLIT: "bf16x3+f32"}[prec],
        "data": "synthetic",
        "config": {"workload": f"d3_{K[0]}x{K[1]}x{K[2]}_p{p}_perturbed_stiffness_assembly_plus_"
                               f"{args.applies}_apply",
                   "d": 3, "elements": list(K), "order": p, "ndof": N, "nnz": nnz, "nquad": Q,
                   "coefficient": "1+0.5*sin(2pi x1)sin(2pi x2)sin(2pi x3)",
                   "precision": args.prec or "fp64", "applies_per_step": args.applies},
        "stages_ms": {"geometry": geom_ms, "pattern": pat_ms, "assembly": asm_ms, "apply": app_ms,
                      "tables_host_once": t_tab * 1e3},
        "assembly_gnnz_s": nnz / (asm_ms * 1e-3) / 1e9,
        "apply_gdof_s": N / (app_ms * 1e-3) / 1e9,
        "apply_hbm_frac": app_bytes / (app_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "apply_tflops": fl_app / (app_ms * 1e-3) / 1e12,
        "roofline": roofline,
    }

    if not args.no_cpu_baseline:
        out.update(cpu_leg(args, w, h, ctx, rp, ci, vals, y, K, p, prec))
    sf.sf_patch_destroy(h)
    sf.sf_ctx_destroy(ctx)
    print(json.dumps(out), flush=True)


def _prec_list(args, sf):
    return [sf.SF_FP64, sf.SF_FP32] if args.prec is None else [sf.SF_FP64 if args.prec == "fp64" else sf.SF_FP32]


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
        for prec in _prec_list(args, sf):
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
            esz = 8 if prec == sf.SF_FP64 else 4
            byts = 6 * Q * esz + 16 * N
            print(json.dumps({
                "metric": "matrix-free apply GDoF/s", "value": N / (ms * 1e-3) / 1e9, "unit": "GDoF/s",
                "ms": ms, "dtype": "f64" if prec == sf.SF_FP64 else "f32",
                "config": {"workload": f"d3_{K[0]}^3_p{p}_stiffness_apply", "order": p, "ndof": N, "nquad": Q},
                "roofline": {"bound": "hbm", "achieved": byts / (ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
                             "unit": "GB/s", "frac": byts / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                             "algorithmic_bytes": byts, "algorithmic_flops": apply_flops(K, p, "stiff")}}),
                flush=True)
        sf.sf_patch_destroy(h)
        del x, y
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


def cpu_leg(args, w, h, ctx, rp, ci, vals, y, K, p, prec):
    """Oracle leg: error of the GPU results on sampled rows, and the oracle's
    own throughput on a bounded sample of the same recipe."""
    import torch

    import oracle
    from paper_1809_05471_amd import inputs
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    torch.cuda.synchronize()
    P = oracle.Problem(w["knots"], p, w["ctrl"], w["coef"])
    rng = np.random.default_rng(7)
    rows = np.unique(np.concatenate([[0, P.N // 2, P.N - 1], rng.integers(0, P.N, 29)]))
    rpn = rp.cpu().numpy()
    vn = vals.cpu().numpy()
    yn = y.cpu().numpy()
    ref = P.rows(oracle.STIFF, rows, threads)
    vmax = max(np.abs(v).max() for _, v in ref)
    eA = max(np.abs(vn[rpn[r]:rpn[r + 1]] - v).max() for r, (_, v) in zip(rows, ref)) / vmax
    yo = P.apply_rows(oracle.STIFF, w["x"], rows, threads)
    scale = max(np.abs(v) @ np.abs(w["x"][c]) for c, v in ref)
    ey = np.abs(yn[rows] - yo).max() / scale

    ks = args.cpu_sample_elements
    ws = inputs.workload_3d((ks, ks, ks), p)
    Ps = oracle.Problem(ws["knots"], p, ws["ctrl"], ws["coef"])
    pat = Ps.pattern()
    t0 = time.perf_counter()
    Ps.assemble(oracle.STIFF, threads, pattern=pat)
    t_asm = time.perf_counter() - t0
    t0 = time.perf_counter()
    Ps.apply(oracle.STIFF, ws["x"], threads)
    t_app = time.perf_counter() - t0
    nnz_s = len(pat[1])
    return {
        "err_A": float(eA), "err_y": float(ey), "err_rows_sampled": int(len(rows)),
        "cpu_baseline": {"value": nnz_s / t_asm / 1e9, "unit": "Gnnz/s", "cores": threads, "kind": "oracle",
                         "sample": f"oracle element-by-element stiffness assembly (cost N p^3d) of the "
                                   f"{ks}^3-element order-{p} patch of the same recipe, nnz={nnz_s}, "
                                   f"{t_asm:.2f} s; matrix-free apply of it {t_app:.2f} s",
                         "apply_gdof_s": Ps.N / t_app / 1e9,
                         "seconds": t_asm + t_app},
    }


if __name__ == "__main__":
    main()
