"""Benchmark: batched ln L + gradient of the dark-siren likelihood on one MI355X.

Workload (one step): the O5-like catalogue -- 5000 events with U[1000, 8192]
posterior samples each, 32-2048 sky pixels per event with 1024-node LOS
tables (about 10 GB in HBM), 1e7 detected injections -- evaluated for a
batch of 64 hyperparameter points drawn from the prior box, returning ln L
and d ln L / d Lambda (all 16 entries) in one call of dsl_loglike_grad.

Prints one JSON line.  `value` = Lambda-evaluations (ln L + gradient) per
second; the roofline object reports the dominant kernel (the fused weight +
adjoint sweep) against the FP32 vector peak; cpu_baseline is the FP64 oracle
on a bounded sample of the same workload.  `kde_numerator` times the same
points with the paper's KDE numerator (value only) on the same handle.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per sample-weight (one sample or injection, one Lambda), in
# FP operations with FMA = 2 and each exp2/log2/rcp/rsqrt/sqrt = 1: the op graph
# of Eq. 7's weight, its Eq. 8 sums and (adjoint) its 16 log-derivatives and
# basis sums, every per-Lambda quantity hoisted, on the common path (inside the
# support, masses above the smoothing window, table redshift prior); the kernels
# execute more (rounding residuals, window branches, exponent bookkeeping), which
# the hardware counters show and the roofline does not credit.
FLOP_PER_WEIGHT_FWD = 97
FLOP_PER_WEIGHT_GRAD = 210
# KDE numerator: the weight and its sums without prior and rate (87) and the
# redshift moments (3).  Per
# (sample, grid node) kernel term on a uniform grid, with the Gaussian's node-to-
# node ratio recurrence: a multiply and an add, plus per sample and run of 16
# nodes the start term (difference, square, exp2, weight) and the ratio (a
# multiply) and the first add: 36 / 16, plus per sample and 256 nodes its own
# ratio factor (5): 2.27.  Per grid node of a (pixel, point) pair: position and
# trapezoid weight (3), prior interpolation (5), rate psi(z)/(1+z) (1+z, log2,
# two exponents, two exp2, sum, reciprocal: 9), products (2), the recurrence's
# node factor 2^(-(i S)^2) (itself by a ratio recurrence: 3), the node's
# dot-product term (2).
FLOP_PER_KDE_WEIGHT = 90
FLOP_PER_KDE_NODE = 2.27
FLOP_PER_KDE_GRID_NODE = 24
PEAK_FP32_VECTOR_TFLOPS = 157.3        # MI355X published FP32 vector (packed) peak
PEAK_FP32_UNPACKED_TFLOPS = 78.6       # 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# The paper's own speed-up, quoted with the hardware it names (Sec. III A,
# Table I): one likelihood evaluation of a 2000-event catalogue (KDE numerator,
# one Lambda per call) on an NVIDIA H100 against the legacy CPU code on 2.4 GHz
# Xeon E5-2630v3 processors.  Context only: another machine, another workload.
PAPER_CONTEXT = {
    "speedup_quoted": "~1e3",
    "table_I_total_ms": {"cpu_legacy": 103910.31, "h100_fiducial": 160.70, "h100_2500_per_pixel": 101.82},
    "table_I_speedup": {"fiducial": 646.6, "2500_samples_per_pixel": 1020.5},
    "hardware": "NVIDIA H100 (Hopper) vs legacy gwcosmo CPU code on 2.4 GHz Xeon E5-2630v3",
    "workload": "2000 simulated events, one Lambda per evaluation, KDE numerator, selection term included",
}

# HBM bytes per sweep launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (calibrated against
# an elementwise copy of known size; profiles/sweep_c4_grad_traffic.txt), valid only for
# the kernel source they were measured on.
MEASURED_TRAFFIC = {("c4", 64, True): {"kernel_sha256_16": "6b7c09ae1c142d27", "bytes": 4.678e9}}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--config", default="c4", help="workload: c1 .. c5 (c4 is the benchmark)")
    p.add_argument("--B", type=int, default=None, help="points per launch (default: the workload's)")
    p.add_argument("--precision", default=None, choices=["fp32", "fp64"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-single", action="store_true", help="skip the one-Lambda-per-launch comparison")
    p.add_argument("--no-autotune", action="store_true", help="use the default tile shape and chunk")
    p.add_argument("--forward-only", action="store_true")
    p.add_argument("--numerator", default="mc", choices=["mc", "kde"],
                   help="mc: per-sample sums (default); kde: the paper's KDE form (value only)")
    p.add_argument("--kde-bandwidth", default="scott", choices=["scott", "silverman", "biweight"])
    p.add_argument("--kde-steps", type=int, default=3,
                   help="after the main timing on c4, time this many steps of the same points with the KDE "
                        "numerator on the same handle (0: skip); reported under 'kde_numerator'")
    p.add_argument("--max-samples-per-pixel", type=int, default=0,
                   help="keep at most this many posterior samples per pixel (seeded choice; 0: all)")
    p.add_argument("--copy-calib", type=int, default=0,
                   help="after the timed steps, run one elementwise copy of this many MiB (calibrates "
                        "rocprofv3 FETCH_SIZE / WRITE_SIZE against known bytes)")
    return p.parse_args()


def kernel_sha():
    """Hash of the sweep's sources (kernel file and shared device header)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("dsl_kernels.hip", "dsl_device.h", "dsl_internal.h"):
        with open(os.path.join(ROOT, "paper_2605_23538_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(cat, lam_row, grad, kde=None):
    """The oracle on a bounded sample of the workload, scaled to one full Lambda."""
    import numpy as np
    import torch
    from oracle import dsl_oracle as O
    n_ev = 80 if kde is None else 16
    n_inj = 2_000_000
    sub = cat.subset(np.arange(n_ev), inj=slice(0, n_inj))
    t0 = time.perf_counter()
    if kde is None:
        O.loglike(sub, lam_row, grad=grad)
    else:
        O.loglike_kde(sub, lam_row, bandwidth=kde)
    dt = time.perf_counter() - t0
    w_sub = sub.n_samp + sub.n_inj
    w_full = cat.n_samp + cat.n_inj
    per_lambda_s = dt * w_full / w_sub
    what = 'KDE ln L, ' + kde + ' bandwidth' if kde else 'ln L + autograd gradient' if grad else 'ln L'
    res = {"value": 1.0 / per_lambda_s, "unit": "Lambda-evals/s", "cores": torch.get_num_threads(),
           "kind": "oracle",
           "sample": f"FP64 oracle ({what}) on the first {n_ev} events "
                     f"({sub.n_samp} samples) and first {n_inj} injections for 1 Lambda: {dt:.2f} s, "
                     f"scaled by {w_full}/{w_sub} sample-weights to one full-catalogue Lambda"}
    # the same oracle on one core, on a smaller sample
    n_ev1, n_inj1 = (20, 250_000) if kde is None else (4, 250_000)
    sub1 = cat.subset(np.arange(n_ev1), inj=slice(0, n_inj1))
    nt = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        if kde is None:
            O.loglike(sub1, lam_row, grad=grad)
        else:
            O.loglike_kde(sub1, lam_row, bandwidth=kde)
        dt1 = time.perf_counter() - t0
    finally:
        torch.set_num_threads(nt)
    w_sub1 = sub1.n_samp + sub1.n_inj
    res["one_core"] = {"value": w_sub1 / (dt1 * w_full), "unit": "Lambda-evals/s", "cores": 1,
                       "sample": f"first {n_ev1} events ({sub1.n_samp} samples) and first {n_inj1} "
                                 f"injections: {dt1:.2f} s, scaled by {w_full}/{w_sub1}"}
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import ctypes as C

    import numpy as np
    import torch

    from paper_2605_23538_amd import binding, synth

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    # workload defaults: (points per launch, precision, gradient)
    defaults = {"c1": (1, "fp64", False), "c2": (1, "fp32", False), "c3": (512, "fp32", False),
                "c4": (64, "fp32", True), "c5": (64, "fp32", True)}[args.config]
    B = args.B or defaults[0]
    precision = args.precision or defaults[1]
    kde = args.numerator == "kde"
    grad = defaults[2] and not args.forward_only and not kde
    t0 = time.time()
    cat = synth.make_catalog(args.config)
    print(f"# generated {args.config}: {cat.n_events} events, {cat.n_pix} pixels, {cat.n_samp} samples, "
          f"{cat.n_inj} injections, LOS {cat.los.nbytes / 1e9:.2f} GB in {time.time() - t0:.1f} s",
          file=sys.stderr, flush=True)
    t0 = time.time()
    lik = binding.DarkSirenLikelihood(cat, precision=precision, numerator=args.numerator,
                                      kde_bandwidth=args.kde_bandwidth,
                                      max_samples_per_pixel=args.max_samples_per_pixel)
    n_samp = int(lik.info("n_samp"))   # posterior samples kept (all of them without a cap)
    print(f"# uploaded in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    lam_np = synth.lambdas_for(args.config, B)
    lam = torch.tensor(lam_np, device="cuda:0")
    if not args.no_autotune:
        t0 = time.time()
        lik.autotune(B, grad)
        print(f"# autotuned in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    dev = lam.device
    logL = torch.empty(B, dtype=torch.float64, device=dev)
    g = torch.empty(B, 16, dtype=torch.float64, device=dev)
    flags = torch.empty(B, dtype=torch.int32, device=dev)
    lib = lik.lib

    def step(stream):
        if grad:
            rc = lib.dsl_loglike_grad(lik.h, C.c_void_p(lam.data_ptr()), B, C.c_void_p(logL.data_ptr()),
                                      C.c_void_p(g.data_ptr()), None, None, None, C.c_void_p(flags.data_ptr()),
                                      C.c_void_p(stream))
        else:
            rc = lib.dsl_loglike(lik.h, C.c_void_p(lam.data_ptr()), B, C.c_void_p(logL.data_ptr()), None, None,
                                 None, C.c_void_p(flags.data_ptr()), C.c_void_p(stream))
        if rc:
            raise RuntimeError(lib.dsl_last_error().decode())

    st = torch.cuda.current_stream().cuda_stream
    for _ in range(args.warmup):
        step(st)
    torch.cuda.synchronize()
    print("# warm-up done", file=sys.stderr, flush=True)

    # timed region: K steps as the library runs them (captured HIP graphs, no host
    # synchronisation between steps), bracketed by a device synchronisation
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step(st)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    value = B * args.steps / wall
    ms_per_step_events = ev0.elapsed_time(ev1) / args.steps

    # kernel durations: the same K steps again with HIP events recorded around
    # each kernel on the launch stream (option "timing"; launches not captured)
    lik.set_option("timing", 1)
    sweep_ms, setup_ms, comb_ms, pix_ms = [], [], [], []
    for _ in range(args.steps):
        step(st)
        a, b, c = lik.timing()
        setup_ms.append(a)
        sweep_ms.append(b)
        comb_ms.append(c)
        if kde:
            pix_ms.append(lik.info("ms_pixels"))
    torch.cuda.synchronize()
    lik.set_option("timing", 0)
    n_w = n_samp + cat.n_inj
    flags_h = flags.cpu().numpy()
    finite = int(np.isfinite(logL.cpu().numpy()).sum())

    # dominant kernel: the sweep (the KDE kernel with the KDE numerator)
    sweep_avg = float(np.mean(sweep_ms))
    F = FLOP_PER_WEIGHT_GRAD if grad else FLOP_PER_WEIGHT_FWD
    flops = F * n_w * B
    achieved = flops / (sweep_avg * 1e-3) / 1e12
    if kde:
        kde_evals = lik.info("kde_evals")
        kde_nodes = lik.info("kde_nodes")
        kde_avg = float(np.mean(pix_ms))
        flops = (FLOP_PER_KDE_WEIGHT * n_samp * B + FLOP_PER_KDE_NODE * kde_evals
                 + FLOP_PER_KDE_GRID_NODE * kde_nodes)
        achieved = flops / (kde_avg * 1e-3) / 1e12
    peak = PEAK_FP32_VECTOR_TFLOPS if precision == "fp32" else PEAK_FP64_VECTOR_TFLOPS
    traffic = None
    mt = MEASURED_TRAFFIC.get((args.config, B, grad))
    if mt and precision == "fp32" and not kde and kernel_sha() == mt["kernel_sha256_16"]:
        traffic = mt["bytes"]
    # HBM side of the roofline: the measured traffic of the launch (FETCH_SIZE +
    # WRITE_SIZE, calibrated) when it is on record for this kernel source, else
    # the algorithmic bytes (every sample and injection record once, every LOS
    # table once, the per-item partial sums written and read back once)
    if kde:   # the KDE stage: sample records, tables, one {R, T, S1, S2} record per (pixel, point)
        alg_bytes = 32 * n_samp + cat.los.nbytes + 2 * 32 * B * cat.n_pix
    else:
        alg_bytes = 32 * n_w + cat.los.nbytes + 2 * (20 if grad else 4) * 8 * B * int(lik.info("n_items"))
    kt = (kde_avg if kde else sweep_avg) * 1e-3
    hbm_bytes = traffic if traffic else alg_bytes
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
                "hbm_bytes": hbm_bytes, "hbm_bytes_kind": "measured" if traffic else "algorithmic",
                "hbm_GBs": round(hbm_bytes / kt / 1e9, 1), "hbm_frac": round(hbm_bytes / kt / 1e9 / PEAK_HBM_GBS, 4),
                "kernel": (("kde_tile_kernel<%s,%d> + kde_event_kernel"
                            % ("float" if precision == "fp32" else "double",
                               (64 if B >= 48 else 16 if B >= 12 else 4) if precision == "fp32" else 4))
                           if B >= 4 else   # fewer points: the row kernel
                           "kde_kernel<%s> + kde_event_kernel" % ("float" if precision == "fp32" else "double"))
                if kde
                else "sweep_kernel<%s,%d,%s>" % ("float" if precision == "fp32" else "double",
                                                 int(lik.info("lambda_tile_used")), "true" if grad else "false"),
                "kernel_ms": round(kde_avg if kde else sweep_avg, 4),
                "frac_of_unpacked_fp32_peak": round(achieved / PEAK_FP32_UNPACKED_TFLOPS, 4),
                **({"flop_per_kde_weight": FLOP_PER_KDE_WEIGHT, "flop_per_kde_node": FLOP_PER_KDE_NODE,
                    "flop_per_kde_grid_node": FLOP_PER_KDE_GRID_NODE,
                    "kde_node_evals_per_launch": kde_evals, "kde_grid_nodes_per_launch": kde_nodes,
                    "kde_weights_per_launch": n_samp * B}
                   if kde else {"flop_per_weight": F, "weights_per_launch": n_w * B}),
                "chunk": int(lik.info("chunk")), "items": int(lik.info("n_items"))}

    # one-Lambda-per-launch comparison (same kernels, B = 1, 64 launches)
    single = None
    if not args.no_single and B > 1:
        lam1 = lam[:1].contiguous()
        out1 = torch.empty(1, dtype=torch.float64, device=dev)
        g1 = torch.empty(1, 16, dtype=torch.float64, device=dev)

        def step1(i):
            src = lam[i:i + 1]
            lam1.copy_(src)
            if grad:
                rc = lib.dsl_loglike_grad(lik.h, C.c_void_p(lam1.data_ptr()), 1, C.c_void_p(out1.data_ptr()),
                                          C.c_void_p(g1.data_ptr()), None, None, None, None, C.c_void_p(st))
            else:
                rc = lib.dsl_loglike(lik.h, C.c_void_p(lam1.data_ptr()), 1, C.c_void_p(out1.data_ptr()), None,
                                     None, None, None, C.c_void_p(st))
            if rc:
                raise RuntimeError(lib.dsl_last_error().decode())
        for i in range(2):
            step1(i)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(B):
            step1(i)
        torch.cuda.synchronize()
        single_s = time.perf_counter() - t1
        single = {"ms_per_lambda_single_launch": round(1e3 * single_s / B, 4),
                  "ms_per_lambda_batched": round(ms_per_step / B, 4),
                  "speedup_batched_vs_single": round((single_s / B) / (ms_per_step / 1e3 / B), 2)}

    if args.copy_calib:
        n = args.copy_calib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)      # reads and writes copy_calib MiB each
        torch.cuda.synchronize()
        del src, dst

    # the paper's KDE numerator on the same catalogue and points (value only)
    kde_side = None
    if args.kde_steps > 0 and args.config == "c4" and not kde:
        lik.set_option("numerator", 1)
        lik.set_option("kde_bandwidth", {"scott": 0, "silverman": 1, "biweight": 2}[args.kde_bandwidth])
        out = torch.empty(B, dtype=torch.float64, device=dev)

        def kstep():
            rc = lib.dsl_loglike(lik.h, C.c_void_p(lam.data_ptr()), B, C.c_void_p(out.data_ptr()), None, None,
                                 None, None, C.c_void_p(st))
            if rc:
                raise RuntimeError(lib.dsl_last_error().decode())
        kstep()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.kde_steps):
            kstep()
        torch.cuda.synchronize()
        kwall = time.perf_counter() - t1
        lik.set_option("timing", 1)
        kms = []
        for _ in range(args.kde_steps):
            kstep()
            lik.timing()
            kms.append(lik.info("ms_pixels"))
        torch.cuda.synchronize()
        lik.set_option("timing", 0)
        kev = lik.info("kde_evals")
        knodes = lik.info("kde_nodes")
        kavg = float(np.mean(kms))
        kfl = FLOP_PER_KDE_WEIGHT * n_samp * B + FLOP_PER_KDE_NODE * kev + FLOP_PER_KDE_GRID_NODE * knodes
        kach = kfl / (kavg * 1e-3) / 1e12
        kde_side = {"metric": "Lambda-evaluations/sec (log L, KDE numerator (%s), %d-node grid)"
                              % (args.kde_bandwidth, int(lik.info("kde_grid"))),
                    "value": round(B * args.kde_steps / kwall, 3), "unit": "Lambda-evals/s",
                    "steps": args.kde_steps, "ms_per_step": round(1e3 * kwall / args.kde_steps, 3),
                    "finite_logL": int(np.isfinite(out.cpu().numpy()).sum()),
                    "roofline": {"bound": "alu", "achieved": round(kach, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
                                 "unit": "TFLOP/s", "frac": round(kach / PEAK_FP32_VECTOR_TFLOPS, 4),
                                 "traffic": None, "kernel": "kde_tile_kernel<float,64> + kde_event_kernel",
                                 "kernel_ms": round(kavg, 3), "kde_node_evals_per_launch": kev,
                                 "kde_grid_nodes_per_launch": knodes,
                                 "flop_per_kde_weight": FLOP_PER_KDE_WEIGHT, "flop_per_kde_node": FLOP_PER_KDE_NODE,
                                 "flop_per_kde_grid_node": FLOP_PER_KDE_GRID_NODE}}
        lik.set_option("numerator", 0)

    cpu = None
    if not args.no_cpu_baseline and args.config in ("c4", "c2") and not args.max_samples_per_pixel:
        cpu = cpu_baseline(cat, lam_np[0], grad, args.kde_bandwidth if kde else None)

    what = "log L, KDE numerator (%s)" % args.kde_bandwidth if kde else "log L + grad" if grad else "log L"
    res = {
        "metric": ("Lambda-evaluations/sec (%s) on O5-like catalogue" % what) if args.config == "c4"
        else "Lambda-evaluations/sec (%s), workload %s" % (what, args.config),
        "value": round(value, 3), "unit": "Lambda-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "ms_per_step_hip_events": round(ms_per_step_events, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %d events, %d samples%s, %d pixels x %d-node LOS tables (%.2f GB), %d injections, "
                               "%d Lambda per launch, %s"
                               % ({"c4": "O5-like batched (c4)"}.get(args.config, args.config), cat.n_events,
                                  n_samp, (" (at most %d per pixel, of %d)" % (args.max_samples_per_pixel, cat.n_samp)
                                           if args.max_samples_per_pixel else ""), cat.n_pix, cat.n_z, cat.los.nbytes / 1e9, cat.n_inj, B,
                                  "ln L + d ln L/d Lambda (16 entries)" if grad
                                  else "ln L with the KDE numerator (%s, %d-node grid)"
                                  % (args.kde_bandwidth, int(lik.info("kde_grid"))) if kde else "ln L"),
                   "B": B, "precision": "FP32 weights, FP64 sums" if precision == "fp32" else "FP64",
                   **({"max_samples_per_pixel": args.max_samples_per_pixel} if args.max_samples_per_pixel else {})},
        "gsample_weights_per_s": round(n_w * B * args.steps / wall / 1e9, 3),
        "kernel_timing": "HIP events around each kernel on the launch stream, a second pass of K steps",
        "kernel_ms": {"setup": round(float(np.mean(setup_ms)), 4), "sweep": round(sweep_avg, 4),
                      "combine": round(float(np.mean(comb_ms)), 4),
                      **({"kde": round(kde_avg, 4)} if kde else {})},
        "finite_logL": finite, "flags_nonzero": int((flags_h != 0).sum()),
        "roofline": roofline, "cpu_baseline": cpu, "single_lambda_launches": single,
        "paper_context": dict(PAPER_CONTEXT, **({"this_run_vs_oracle": round(value / cpu["value"], 1)}
                                                if cpu else {})),
    }
    if kde_side:
        res["kde_numerator"] = kde_side
    print(json.dumps(res), flush=True)
    lik.close()


if __name__ == "__main__":
    main()
