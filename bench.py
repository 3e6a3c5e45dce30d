"""Benchmark of the JK-CALS hot path on one MI355X.

One step = one complete leave-one-out jackknife of the benchmark workload on
the GPU: tensor residency and slice norms, multi-factor packing (context
init from device-resident inputs), then the fixed budget of concurrent ALS
sweeps (fused MTTKRP, slice correction, batched Gram / Cholesky / update /
normalisation, per-submodel error).  Workload: 100 x 200 x 200 float64
tensor shaped like fluorescence data (rank 5, 2 % noise), 100 leave-one-out
submodels of rank 5, 100 sweeps each (the fixed-iteration protocol).

Prints one JSON line.  `value` = submodels fitted per second with the
library's default evaluation (for 3-way float64 sweeps a shared partial
contraction serves two modes); `alg3_fused_per_mode` = the same jackknife
with the fused MTTKRP of Alg. 3 on every mode, timed separately.  The
`roofline` object is that fused MTTKRP with its split-K reduction (float64
MFMA), averaged over every mode; the shared contraction is reported on its
own (`tree_w`).  Also reported: the same jackknife done the plain way on the
same GPU (one submodel at a time on its explicitly reduced tensor), and the
CPU oracle's rate on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import shutil
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense float64 matrix peak (datasheet)
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense bfloat16 matrix peak (datasheet)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sweeps", type=int, default=100)
    ap.add_argument("--no-tune", action="store_true",
                    help="never autotune; use cached tilings or the cost model")
    ap.add_argument("--retune", action="store_true",
                    help="autotune the MTTKRP tilings (untimed) even for shapes in the shipped table")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-submodel GPU baseline")
    ap.add_argument("--no-tree", action="store_true",
                    help="fused MTTKRP on every mode (no shared partial contraction W = T x_2 U_2)")
    ap.add_argument("--plain-models", type=int, default=10)
    ap.add_argument("--cpu-models", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5"],
                    help="c2: the benchmark workload (default); c3/c4/c5: the uneven-batch, "
                         "split-precision and refinement workloads")
    ap.add_argument("--precision", default=None, choices=["fp64", "bf16x3", "bf16x6"])
    ap.add_argument("--protocol", default="fixed", choices=["fixed", "application"],
                    help="fixed: every model runs --sweeps sweeps (the paper's timing "
                         "protocol); application: tol 1e-6, at most 1000 sweeps, timed with "
                         "convergence compaction on and off")
    ap.add_argument("--delete-d", type=int, default=1,
                    help="c2 only: delete-d jackknife over groups of d consecutive samples "
                         "(I/d submodels; the baselines are skipped)")
    ap.add_argument("--gradient-path", default="default", choices=["default", "allmode", "per-mode"],
                    help="c5: the all-mode MTTKRP of the refinement's gradient -- the library's "
                         "default, the one-pass kernel (jk_cals_set_allmode 1), or the per-mode "
                         "path (shared contraction / fused MTTKRPs)")
    ap.add_argument("--efficiency-sweep", action="store_true",
                    help="instead of the benchmark: fused MTTKRP efficiency against the column "
                         "count C on a 50x200x200 tensor (the analogue of the paper's Fig. 1); "
                         "prints one JSON line per (C, mode)")
    return ap.parse_args()


def application_protocol(args, wl, T, init, precision, desc_w, prec_name):
    """The application protocol of the paper's experiments (tolerance 1e-6
    on the change of fit, at most 1000 sweeps): whole fits timed with
    convergence compaction on (value) and off."""
    import numpy as np
    import torch

    import paper_2112_03985_amd as jk

    def one(compact):
        ctx = jk.JkCals(T, wl.dims, 0, wl.ranks, wl.left_out, init, precision=precision)
        if args.no_tree and ctx.describe(len(wl.dims)):
            ctx.set_mttkrp_tree(False)
        ctx.set_compaction(compact)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters, fit, status = ctx.fit(1000, 1e-6)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, iters, fit

    one(True)                                   # warm-up (tilings, clocks)
    times = {}
    for compact in (True, False):
        best = None
        for _ in range(max(1, args.steps)):
            sec, iters, fit = one(compact)
            best = sec if best is None else min(best, sec)
        times[compact] = best
    it = np.asarray(iters)
    out = {"metric": "jackknife submodels fitted/sec (JK-CALS, tol 1e-6, at most 1000 sweeps)",
           "value": round(wl.K / times[True], 2), "unit": "submodels/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 1, "ms_per_step": round(1e3 * times[True], 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if precision == jk.JKC_FP64 else prec_name, "data": "synthetic",
           "config": {"workload": (desc_w % 1000).replace("1000 ALS sweeps", "tol 1e-6, <= 1000 sweeps"),
                      "dims": list(wl.dims), "models": wl.K, "columns": wl.C},
           "sweeps_per_model": {"min": int(it.min()), "median": int(np.median(it)), "max": int(it.max())},
           "compaction_off": {"value": round(wl.K / times[False], 2), "ms": round(1e3 * times[False], 3),
                              "speedup_from_compaction": round(times[False] / times[True], 3)},
           "fit_range": [round(float(np.min(fit)), 6), round(float(np.max(fit)), 6)]}
    print(json.dumps(out), flush=True)
    return 0


def efficiency_sweep():
    """Fused float64 MTTKRP TFLOP/s against C on 50 x 200 x 200 (Sec. 4.2's
    experiment shape): models of rank 5 (the last one narrower) side by side,
    tilings tuned per C, kernel time from HIP events on the context stream."""
    import numpy as np
    import torch

    import paper_2112_03985_amd as jk

    shape = (50, 200, 200)
    P = int(np.prod(shape))
    rng = np.random.default_rng(211203985)
    T = jk.to_device_tensor(np.asfortranarray(rng.standard_normal(shape)))
    for C in (1, 2, 5, 10, 20, 50, 100, 200, 500, 1000):
        ranks = [5] * (C // 5) + ([C % 5] if C % 5 else [])
        init = [torch.from_numpy(rng.standard_normal((I, C))).cuda() for I in shape]
        ctx = jk.JkCals(T, shape, 0, ranks, [-1] * len(ranks), init)
        ctx.tune(3)
        out = torch.empty((max(shape), C), dtype=torch.float64, device="cuda")
        for n in range(3):
            for _ in range(2):
                ctx.mttkrp(n, out[:shape[n]])
            torch.cuda.synchronize()
            ctx.profile(True)
            for _ in range(10):
                ctx.mttkrp(n, out[:shape[n]])
            cnt, ms = ctx.profile_read()
            ctx.profile(False)
            kms = float(ms[n] / max(cnt[n], 1))
            tf = 2.0 * C * P / (kms * 1e-3) / 1e12
            print(json.dumps({"experiment": "mttkrp_efficiency_vs_C", "dims": list(shape), "C": C,
                              "mode": n, "kernel_ms": round(kms, 5), "tflops": round(tf, 3),
                              "frac_fp64_peak": round(tf / PEAK_FP64_TFLOPS, 4),
                              "tiling": ctx.describe(n)}), flush=True)
        del ctx
    return 0


PROF_SWEEPS = 10


def measured_traffic(workload, prec_name, desc):
    """HBM bytes per fused MTTKRP launch with its split-K reduction, from the
    committed rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE, calibrated
    with a copy kernel), or None when there is no such record for this
    workload or when a kernel source or the tiling has changed since the
    counters were taken."""
    path = os.path.join(ROOT, "profiles", "k_mttkrp_f64_%s_traffic.md" % workload)
    if prec_name != "fp64" or not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", " ", "|")):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    try:
        paths = [x.strip() for x in rec["kernel_source"].split(";")]
        hashes = [x.strip() for x in rec["kernel_source_sha256"].split(";")]
        if len(paths) != len(hashes):
            return None
        for path, h in zip(paths, hashes):
            src = open(os.path.join(ROOT, path), "rb").read()
            if hashlib.sha256(src).hexdigest() != h:
                return None
        if [t.strip() for t in rec["tiling"].split(";")] != list(desc):
            return None
        return int(rec["traffic_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2
    import numpy as np
    import torch

    import synth
    import paper_2112_03985_amd as jk

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if args.efficiency_sweep:
        return efficiency_sweep()
    refine_steps = 0
    if args.workload == "c2" and args.delete_d > 1:
        wl = synth.config2(delete_d=args.delete_d)
        desc_w = ("c2: 100x200x200 f64 fluorescence-like tensor, rank 5, 2%%%% noise; "
                  "%d delete-%d submodels of rank 5; %%d ALS sweeps" % (wl.K, args.delete_d))
        prec_name = args.precision or "fp64"
        args.no_plain = True
        args.no_cpu = True
    elif args.workload == "c2":
        wl = synth.config2()
        desc_w = ("c2: 100x200x200 f64 fluorescence-like tensor, rank 5, 2%% noise; "
                  "100 leave-one-out submodels of rank 5; %d ALS sweeps")
        prec_name = args.precision or "fp64"
    elif args.workload == "c3":
        wl = synth.config3()
        desc_w = ("c3: 300x250x200 f64 rank-8 tensor; ranks 1..10 x 5 inits x 300 leave-one-out "
                  "= 15000 submodels (C = 82500); %d ALS sweeps")
        prec_name = args.precision or "fp64"
    elif args.workload == "c4":
        wl = synth.config4()
        desc_w = ("c4: 200x120x100x80 f64 rank-12 tensor, 1%% noise; 200 leave-one-out submodels "
                  "of rank 12; split-precision MTTKRP; %d ALS sweeps")
        # the six-product split is the one that holds the 1e-5 gate
        prec_name = args.precision or "bf16x6"
    else:
        wl = synth.config5()
        refine_steps = 200
        if args.sweeps == 100:
            args.sweeps = 20
        desc_w = ("c5: 100x150x150 rank-10 tensor stored as f32; 100 leave-one-out submodels of "
                  "rank 10; %d ALS sweeps + " + "%d gradient-refinement steps" % refine_steps)
        prec_name = args.precision or "fp64"
    precision = {"fp64": jk.JKC_FP64, "bf16x3": jk.JKC_SPLIT_BF16X3,
                 "bf16x6": jk.JKC_SPLIT_BF16X6}[prec_name]
    K, C, P = wl.K, wl.C, int(np.prod(wl.dims))
    N = len(wl.dims)
    sweeps = args.sweeps
    if args.workload in ("c3", "c5"):
        args.no_plain = True
        args.no_cpu = True
    if args.workload == "c4":
        args.no_plain = True
    T = jk.to_device_tensor(wl.T)
    init = [torch.from_numpy(np.ascontiguousarray(u)).cuda() for u in wl.init]
    torch.cuda.synchronize()

    # Tilings: the table shipped with the package holds tuned tilings for
    # known shapes; shapes it lacks are tuned here (untimed), or always with
    # --retune.  A scratch copy is used so that the shipped table is never
    # rewritten.
    if "JKC_TUNE_CACHE" not in os.environ:
        shipped = os.path.join(ROOT, "paper_2112_03985_amd", "tuned_gfx950.txt")
        scratch = os.path.join(tempfile.mkdtemp(prefix="jkc_tune_"), "tune.txt")
        if os.path.exists(shipped):
            shutil.copyfile(shipped, scratch)
        os.environ["JKC_TUNE_CACHE"] = scratch
    ldc = (C + 15) // 16 * 16
    keys = ["gfx950 p%d f32_%d N%d d%s ldc%d mode%d" % (precision, int(wl.T.dtype == np.float32), N,
                                                        "x".join(str(d) for d in wl.dims), ldc, n)
            for n in range(N)]
    try:
        have = {line.split("|", 1)[0] for line in open(os.environ["JKC_TUNE_CACHE"])}
    except OSError:
        have = set()
    tiling = None
    if args.retune or (not args.no_tune and not all(k in have for k in keys)):
        ctx = jk.JkCals(T, wl.dims, 0, wl.ranks, wl.left_out, init, precision=precision)
        ctx.tune(5)
        tiling = [ctx.describe(n) for n in range(N)]
        if ctx.describe(N):
            tiling.append(ctx.describe(N))
        del ctx

    # MTTKRP launch durations come from HIP events stamped by the dispatches
    # of the first PROF_SWEEPS sweeps of every timed step; the remaining
    # sweeps run untimed (the stamps cost about 5 % of a sweep)
    prof_sweeps = min(PROF_SWEEPS, sweeps)

    def step(profile=False, tree=True):
        ctx = jk.JkCals(T, wl.dims, 0, wl.ranks, wl.left_out, init, precision=precision)
        if not tree and ctx.describe(N):
            ctx.set_mttkrp_tree(False)
        if profile:
            ctx.profile(True)
            ctx.sweep(prof_sweeps)
            ctx.profile(False)
            if sweeps > prof_sweeps:
                ctx.sweep(sweeps - prof_sweeps)
        else:
            ctx.sweep(sweeps)
        if refine_steps:
            if args.gradient_path != "default":
                ctx.set_allmode(args.gradient_path == "allmode")
            ctx.refine(refine_steps)
        return ctx

    if args.protocol == "application":
        return application_protocol(args, wl, T, init, precision, desc_w, prec_name)

    def timed(tree):
        """Warm-up, then args.steps timed steps; (seconds, launches per
        profiling slot, milliseconds per slot, last context)."""
        for _ in range(args.warmup):
            c = step(tree=tree)
            del c
        torch.cuda.synchronize()
        launches = np.zeros(N + 1, np.int64)
        kms = np.zeros(N + 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            c = step(profile=True, tree=tree)
            n_, ms_ = c.profile_read()          # synchronises this step's stream
            launches += n_
            kms += ms_
        torch.cuda.synchronize()
        return time.perf_counter() - t0, launches, kms, c

    default_tree = not args.no_tree
    print("[bench] %d warmup + %d timed steps (default evaluation)" % (args.warmup, args.steps),
          file=sys.stderr, flush=True)
    sec, launches, kms, c = timed(default_tree)
    ms_per_step = 1000.0 * sec / args.steps
    value = K * args.steps / sec
    has_tree = bool(c.describe(N))

    # fit quality and tilings of the last step (not timed)
    fit = c.get_status()[1].cpu().numpy()
    desc = [c.describe(n) for n in range(N)]
    if has_tree:
        desc.append(c.describe(N))
    fused = {"launches": launches, "ms": kms, "sec": sec}
    alg3 = None
    if has_tree:
        # the same jackknife with the fused MTTKRP of Alg. 3 on every mode
        print("[bench] %d timed steps, fused MTTKRP on every mode" % args.steps, file=sys.stderr,
              flush=True)
        sec3, launches3, kms3, c3 = timed(False)
        del c3
        fused = {"launches": launches3, "ms": kms3, "sec": sec3}
        alg3 = {"value": round(K * args.steps / sec3, 2), "unit": "submodels/s",
                "ms_per_step": round(1000.0 * sec3 / args.steps, 3),
                "note": "Alg. 3 as printed: the fused MTTKRP of every mode (no shared contraction)"}

    flops_per_launch = 2.0 * C * P          # fused MTTKRP of one mode (Sec. 4.2)
    fl, fm = fused["launches"][:N], fused["ms"][:N]
    per_mode_ms = [float(fm[n] / fl[n]) if fl[n] else None for n in range(N)]
    avg_ms = float(fm.sum() / max(fl.sum(), 1))
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    if precision == jk.JKC_FP64:
        peak, kname, issued = PEAK_FP64_TFLOPS, "k_mttkrp_f64 + k_reduce", 1.0
    else:
        # bf16 matrix peak, counting the bf16 flops actually issued
        issued = 3.0 if precision == jk.JKC_SPLIT_BF16X3 else 6.0
        peak, kname = PEAK_BF16_TFLOPS, "k_mttkrp_bf + k_reduce"
    roofline = {"bound": "mfma", "achieved": round(achieved * issued, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved * issued / peak, 4),
                "traffic": measured_traffic(args.workload, prec_name, desc[:N]),
                "kernel": kname + " (the fused concurrent MTTKRP of Alg. 3 with its split-K "
                                  "reduction, every mode)",
                "avg_launch_ms": round(avg_ms, 5),
                "per_mode_avg_ms": [None if x is None else round(x, 5) for x in per_mode_ms],
                "timed_launches": "HIP events stamped by the MTTKRP dispatch (start) and its "
                                  "reduction's dispatch (stop), first %d sweeps of every timed step"
                                  % prof_sweeps + ("" if alg3 is None else
                                                   " of the alg3_fused_per_mode leg"),
                "flops_per_launch": flops_per_launch * issued}
    # MTTKRP TFLOP/s as defined for the metric: 2 C P N per sweep over the
    # summed MTTKRP time with its reduction
    sweep_ms = float(sum(x for x in per_mode_ms if x is not None))
    out = {"metric": "jackknife submodels fitted/sec (JK-CALS, %d sweeps each%s)"
                     % (sweeps, "" if not refine_steps else " + %d refinement steps" % refine_steps),
           "value": round(value, 2), "unit": "submodels/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if precision == jk.JKC_FP64 else "bf16x%d+f32acc+f64" % (3 if precision == 1 else 6),
           "data": "synthetic",
           "config": {"workload": desc_w % sweeps, "dims": list(wl.dims), "models": K,
                      "columns": C, "sweeps": sweeps, "precision": prec_name,
                      "delete_d": int(wl.left_out.shape[1]) if wl.left_out.ndim == 2 else 1,
                      "fused_flop_overhead": round(wl.dims[0] / (wl.dims[0] - (
                          int(wl.left_out.shape[1]) if wl.left_out.ndim == 2 else 1)), 5),
                      "evaluation": "shared partial contraction W = T x_2 U_2 for modes 0 and 1, "
                                    "fused MTTKRP for mode 2" if has_tree else
                                    "fused MTTKRP on every mode (Alg. 3)",
                      "tiling": tiling or desc},
           "mttkrp_tflops": round(N * flops_per_launch / (sweep_ms * 1e-3) / 1e12, 3) if sweep_ms else None,
           "roofline": roofline}
    if alg3 is not None:
        out["alg3_fused_per_mode"] = alg3
    if has_tree and launches[N]:
        w_ms = float(kms[N] / launches[N])
        w_tf = flops_per_launch / (w_ms * 1e-3) / 1e12
        out["tree_w"] = {"kernel": "k_mttkrp_f64 on the two-way view of T (W = T x_2 U_2, no "
                                   "Khatri-Rao products, no split-K)",
                         "avg_launch_ms": round(w_ms, 5), "achieved": round(w_tf, 3),
                         "frac": round(w_tf / PEAK_FP64_TFLOPS, 4), "launches_per_sweep": 1}

    if refine_steps:
        # loss + gradient per call (fold, all-mode MTTKRP, gradient assembly)
        # on the one-pass kernel and on the per-mode path, torch events
        lg = {}
        lbuf = torch.empty(K, dtype=torch.float64, device="cuda")
        for path in ("allmode", "per-mode"):
            try:
                c.set_allmode(path == "allmode")
            except jk.JkcError:
                continue
            c.loss_grad(lbuf)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(10):
                c.loss_grad(lbuf)
            e1.record()
            torch.cuda.synchronize()
            lg[path] = round(e0.elapsed_time(e1) / 10, 5)
        out["loss_grad_call_ms"] = dict(lg, note="jk_cals_loss_grad per call; the all-mode "
                                        "MTTKRP costs 4 C P matrix-core flops on the one-pass "
                                        "kernel, the refinement ran on the '%s' path"
                                        % args.gradient_path)

    # after the timed region: the MTTKRP with its split-K reduction (what a
    # caller of jk_cals_mttkrp gets), per mode, HIP events on the stream
    mout = torch.empty((max(wl.dims), C), dtype=torch.float64, device="cuda")
    with_reduce_ms = []
    for n in range(N):
        c.mttkrp(n, mout[:wl.dims[n]])
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            c.mttkrp(n, mout[:wl.dims[n]])
        e1.record()
        torch.cuda.synchronize()
        with_reduce_ms.append(e0.elapsed_time(e1) / 5)
    out["mttkrp_call"] = {
        "per_mode_ms": [round(x, 5) for x in with_reduce_ms],
        "tflops": round(flops_per_launch * issued / (float(np.mean(with_reduce_ms)) * 1e-3) / 1e12, 3),
        "note": "jk_cals_mttkrp (MTTKRP, reduction and copy-out into a caller buffer), "
                "torch events around 5 calls"}
    # jackknife post-processing (Alg. 2: matching, scale adjustment and the
    # standard deviations) of one set of fitted submodels: the leave-one-out
    # run after the first model, against the full model when there is one
    # (else against the first submodel), at most one per left-out sample
    def first_left(k):
        return int(np.asarray(wl.left_out[k]).ravel()[0])
    ref = 0
    s0 = 1 if first_left(0) < 0 and K > 1 else 0
    cnt = 0
    while (s0 + cnt < K and cnt < wl.dims[0] and int(wl.ranks[s0 + cnt]) == int(wl.ranks[ref])
           and first_left(s0 + cnt) >= 0):
        cnt += 1
    jk_ms = None
    if cnt > 0:
        c.jackknife_std(ref, s0, cnt)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            c.jackknife_std(ref, s0, cnt)
        e1.record()
        torch.cuda.synchronize()
        jk_ms = e0.elapsed_time(e1) / 5
    del c, mout
    # context init alone (tensor copy or split, slice norms, packing, Grams)
    torch.cuda.synchronize()
    t_i = time.perf_counter()
    for _ in range(3):
        ci = jk.JkCals(T, wl.dims, 0, wl.ranks, wl.left_out, init, precision=precision)
        torch.cuda.synchronize()
        del ci
    init_ms = 1000.0 * (time.perf_counter() - t_i) / 3
    out["init_ms"] = round(init_ms, 3)
    out["fit_range"] = [round(float(fit.min()), 6), round(float(fit.max()), 6)]
    out["jackknife_postprocess"] = {"ms": None if jk_ms is None else round(jk_ms, 4),
                                    "reference_model": ref, "submodels": cnt}

    if not args.no_plain:
        print("[bench] plain per-submodel ALS on the GPU (%d models)" % args.plain_models,
              file=sys.stderr, flush=True)
        n_plain = min(args.plain_models, K)
        dims_red = [wl.dims[0] - 1] + list(wl.dims[1:])
        buf = torch.empty(P // wl.dims[0] * dims_red[0], dtype=torch.float64, device="cuda")
        cols = np.arange(C).reshape(K, 5)
        # per-submodel inputs prepared before timing: the reduced init rows
        inits = []
        for k in range(n_plain):
            p = int(wl.left_out[k])
            keep = [i for i in range(wl.dims[0]) if i != p]
            inits.append([torch.from_numpy(np.ascontiguousarray(wl.init[0][keep][:, cols[k]])).cuda(),
                          torch.from_numpy(np.ascontiguousarray(wl.init[1][:, cols[k]])).cuda(),
                          torch.from_numpy(np.ascontiguousarray(wl.init[2][:, cols[k]])).cuda()])

        def plain_one(k, profile=False):
            # Alg. 2: the slice removed explicitly, then ALS on the reduced
            # tensor alone: every mode's MTTKRP a streaming pass over it (the
            # narrow vector-ALU tiling for the 16-column pitch of one rank-5
            # model; no shared contraction)
            jk.jk_cals_remove_slice(T, wl.dims, 0, int(wl.left_out[k]), out=buf)
            cx = jk.JkCals(buf, dims_red, 0, [5], [-1], inits[k], copy_tensor=False)
            if cx.describe(N):
                cx.set_mttkrp_tree(False)
            if profile:
                cx.profile(True)
            cx.sweep(sweeps)
            return cx

        cx = plain_one(0, profile=True)
        pl_n, pl_ms = cx.profile_read()
        plain_tilings = [cx.describe(n) for n in range(N)]
        torch.cuda.synchronize()
        del cx
        t0 = time.perf_counter()
        for k in range(n_plain):
            cx = plain_one(k)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        plain_rate = n_plain / tp
        # the per-mode MTTKRP of the plain fit (with its split-K reduction),
        # HIP events; its HBM rate counts one read of the reduced tensor
        red_bytes = P // wl.dims[0] * dims_red[0] * 8
        per_mode = [float(pl_ms[n] / pl_n[n]) if pl_n[n] else None for n in range(N)]
        avg = float(np.sum(pl_ms[:N]) / max(np.sum(pl_n[:N]), 1))
        gbps = red_bytes / (avg * 1e-3) / 1e9
        out["plain_als_gpu"] = {"value": round(plain_rate, 2), "unit": "submodels/s",
                                "sample": "%d of %d submodels, %d sweeps each" % (n_plain, K, sweeps),
                                "speedup_jk_cals": round(value / plain_rate, 2),
                                "ms_per_model_sweep": round(1000.0 * tp / n_plain / sweeps, 4),
                                "mttkrp": {"tiling": plain_tilings,
                                           "per_mode_ms": [None if x is None else round(x, 5) for x in per_mode],
                                           "hbm_gbps": round(gbps, 1),
                                           "hbm_frac": round(gbps / 8000.0, 4),
                                           "bytes_per_launch": red_bytes,
                                           "note": "one streaming read of the reduced tensor per mode "
                                                   "(the algorithmic bytes), MTTKRP plus its split-K "
                                                   "reduction, against 8 TB/s"}}

    if not args.no_cpu:
        out.update(cpu_baseline(args, wl, T, init, precision, sweeps))
    print(json.dumps(out))
    return 0


def cpu_baseline(args, wl, T, init, precision, sweeps):
    """The oracle (per-submodel float64 ALS on the reduced tensor) timed on
    the host on a bounded sample, at one thread and at up to sixteen; the
    faster run is the baseline.  For the split-precision workload the sample
    is one model for one sweep, and the GPU's result for that model is
    compared with it (every result's error stated)."""
    import numpy as np
    import torch

    import oracle
    import paper_2112_03985_amd as jk
    from threadpoolctl import threadpool_info, threadpool_limits

    print("[bench] CPU oracle on a sample", file=sys.stderr, flush=True)
    cores = min(16, os.cpu_count() or 1)
    split = precision != jk.JKC_FP64
    n_cpu = 1 if split else min(args.cpu_models, wl.K)
    n_sweeps = 1 if split else sweeps
    Th = np.asarray(wl.T)
    runs = []
    res = None
    for lim in (1, cores):
        with threadpool_limits(limits=lim):
            used = 1 if lim == 1 else max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
            t0 = time.perf_counter()
            res = oracle.jk_als(Th, 0, wl.ranks, wl.left_out, wl.init, n_sweeps,
                                models=list(range(n_cpu)), record_factors=[n_sweeps] if split else ())
            tc = time.perf_counter() - t0
        runs.append({"value": round(n_cpu * n_sweeps / sweeps / tc, 4), "unit": "submodels/s",
                     "cores": int(used), "kind": "oracle",
                     "sample": "%d of %d submodels x %d sweeps (scaled to %d sweeps per submodel), "
                               "numpy float64 per-submodel ALS" % (n_cpu, wl.K, n_sweeps, sweeps)})
    runs.sort(key=lambda r: -r["value"])
    out = {"cpu_baseline": runs[0], "cpu_baseline_other_threads": runs[1]}
    if split:
        # the GPU's split-precision run of the same sample: one sweep from
        # the same init, every result against the oracle's
        ctx = jk.JkCals(T, wl.dims, 0, wl.ranks, wl.left_out, init, precision=precision)
        Ms = [ctx.mttkrp(n).cpu().numpy() for n in range(len(wl.dims))]
        ctx.sweep(1)
        err = ctx.get_status()[0].cpu().numpy()
        facs = [ctx.get_factors(n) for n in range(len(wl.dims))]
        r = res[0]
        R = int(wl.ranks[0])
        Up = r.padded(r.U_hist[1])

        def rel(a, b):
            nb = np.linalg.norm(b)
            return float(np.linalg.norm(a - b) / nb), float(np.max(np.abs(a - b)) / np.max(np.abs(b)))

        # the init MTTKRP of model 0 by definition (reduced tensor, reduced
        # factors), padded with the left-out row
        p = int(wl.left_out[0])
        U0 = [np.array(u[:, :R]) for u in wl.init]
        U0[0] = oracle.reduce_init(U0[0], p)
        Tk = oracle.reduce_tensor(Th, 0, p)
        mt = []
        for n in range(len(wl.dims)):
            M = oracle.mttkrp(Tk, U0, n)
            if n == 0:
                M = np.insert(M, p, 0.0, axis=0)
            mt.append(rel(Ms[n][:, :R], M))
        out["split_error_vs_oracle"] = {
            "model": 0, "gate": 1e-5,
            "mttkrp_at_init": [{"normwise": round(a, 9), "elementwise": round(b, 9)} for a, b in mt],
            "factors_after_one_sweep": [
                dict(zip(("normwise", "elementwise"), (round(x, 9) for x in
                                                        rel(facs[n][0].cpu().numpy()[:, :R], Up[n]))))
                for n in range(len(wl.dims))],
            "lambda_after_one_sweep": round(rel(facs[0][1].cpu().numpy()[:R], r.lam_hist[0])[0], 9),
            "error_after_one_sweep": round(abs(float(err[0]) - r.e_hist[0]) / r.normT2, 9)}
    return out


if __name__ == "__main__":
    sys.exit(main())
