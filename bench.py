"""Benchmark: forward + adjoint of the cubic B-spline x-ray transform on a
2048 x 2048 grid over 8,847,360 lines (fan 1440 x 3072 at R = 4000 plus as many
random lines), on one MI355X.

One step = xrt_plan_forward + xrt_plan_adjoint over the whole line list (the
plan is built once, before timing; its build time is reported separately).
Inputs are device-resident when timing starts.  Prints one JSON line.

The line also carries "recon": time to relative residual 1e-3 of the
Tikhonov normal equations (lambda 1e-2) on a 512 x 512 cubic grid with
180 x 768 parallel-beam Poisson-noisy data: plain CG, flexible CG with the
trained U-Net preconditioner (training time reported separately), and CG
preconditioned by the second-difference sinogram filter.

It also carries "batch": 64 uneven problems in persistent launches (one for
the forward, two for the adjoint; with graph replay and the autotuner) against
per-problem plans, and "box3": the 3-directional box spline on the same lines
and grid.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--no-cpu-baseline] [--no-recon] [--no-batch]
                    [--no-box]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
HBM_PEAK_GBS = 8000.0


# The sources that decide what the profiled kernels do: their code and their
# launch configuration (tile split, grid sizes, layouts).
KERNEL_SOURCES = ("xrt_kernels.hip", "xrt_api.cpp", "xrt_internal.h", "xrt_geom.h")


def kernel_source_hash(paths=None) -> str:
    """SHA-256 (first 16 hex digits) of the kernel sources (KERNEL_SOURCES by
    default) with comments and whitespace removed: it changes when the code or
    a launch configuration does, not when a comment does."""
    import hashlib
    import re
    if paths is None:
        paths = [os.path.join(ROOT, "paper_2503_20907_amd", "csrc", f) for f in KERNEL_SOURCES]
    elif isinstance(paths, str):
        paths = [paths]
    h = hashlib.sha256()
    for path in paths:
        text = open(path, encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        text = re.sub(r"\s+", "", text)
        h.update(text.encode())
    return h.hexdigest()[:16]


def measured_traffic(call: str):
    """HBM bytes of one `call` ("adjoint" or "forward": every kernel the call
    launches, each as often as it launches it) from the committed rocprofv3
    summary (FETCH_SIZE and WRITE_SIZE, calibrated against a copy kernel), or
    None if the kernel sources changed since the counters were taken."""
    import re
    srcs = [os.path.join(ROOT, "paper_2503_20907_amd", "csrc", f) for f in KERNEL_SOURCES]
    summ = os.path.join(ROOT, "profiles", "hbm_traffic_2048_cubic_fan_random.md")
    if not (all(os.path.exists(f) for f in srcs) and os.path.exists(summ)):
        return None
    sha = kernel_source_hash(srcs)
    total = 0
    found = False
    pat = r"traffic call=(\w+) kernel=(\S+) count=(\d+) sha=(\w+) read_bytes=(\d+) write_bytes=(\d+)"
    for line in open(summ):
        m = re.search(pat, line)
        if m and m.group(1) == call and m.group(4) == sha:
            total += int(m.group(3)) * (int(m.group(5)) + int(m.group(6)))
            found = True
    return total if found else None


def valu_calibration(dev, iters: int = 2048, blocks_per_cu: int = 8):
    """Issue rate of the VALU measured on xrt_calib_valu: 64 * iters
    instructions per wave (FP32 FMA, INT32 add, FP64 FMA), 4 waves per
    workgroup, blocks_per_cu workgroups per compute unit.  Rate = wave
    instructions / (time x SIMDs x 2.4 GHz), i.e. instructions per cycle per
    SIMD at the published peak clock."""
    import torch

    from paper_2503_20907_amd import _lib as L
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    blocks = cus * blocks_per_cu
    out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    res = {"cus": cus, "simds": 4 * cus, "blocks": blocks, "iters": iters,
           "valu_per_wave": 64 * iters, "clock_ghz_assumed": 2.4}
    for mode, name in ((0, "fma_f32"), (1, "add_u32"), (2, "fma_f64")):
        for _ in range(2):
            assert L.xrt_calib_valu(mode, iters, blocks, out.data_ptr(), stream.cuda_stream) == 0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        reps = 5
        for _ in range(reps):
            L.xrt_calib_valu(mode, iters, blocks, out.data_ptr(), stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3 / reps
        wave_instr = blocks * 4 * 64 * iters
        rate = wave_instr / (t * 4 * cus * 2.4e9)
        res[name] = {"ms": round(t * 1e3, 4), "wave_instructions": wave_instr,
                     "instr_per_cycle_per_simd": round(rate, 4)}
        print(f"[bench] valu calibration {name}: {t * 1e3:.3f} ms, {rate:.4f} wave instructions "
              f"per cycle per SIMD at 2.4 GHz", file=sys.stderr, flush=True)
    return res


def lds_calibration(dev, iters: int = 256, blocks_per_cu: int = 5):
    """LDS cost of a wave64 32-bit integer atomic (xrt_calib_lds): for each
    address pattern the time per atomic wave instruction per compute unit,
    in cycles at 2.4 GHz (the counters of the same run give the clock)."""
    import torch

    from paper_2503_20907_amd import _lib as L
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    blocks = cus * blocks_per_cu
    out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    names = ["consecutive", "stride2", "stride32", "same_word", "hashed", "stride64", "pairs", "stride65",
             "u64_consecutive", "u64_hashed"]
    res = {"cus": cus, "blocks": blocks, "iters": iters, "atomics_per_thread": 16 * iters}
    for pat, name in enumerate(names):
        for _ in range(2):
            assert L.xrt_calib_lds(pat, iters, blocks, out.data_ptr(), stream.cuda_stream) == 0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        reps = 5
        for _ in range(reps):
            L.xrt_calib_lds(pat, iters, blocks, out.data_ptr(), stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3 / reps
        per_cu = blocks * 4 * 16 * iters / cus
        cyc = t * 2.4e9 / per_cu
        res[name] = {"ms": round(t * 1e3, 4), "cycles_per_atomic_per_cu": round(cyc, 3)}
        print(f"[bench] lds calibration {name}: {t * 1e3:.3f} ms, {cyc:.3f} cycles per wave atomic "
              f"per CU at 2.4 GHz", file=sys.stderr, flush=True)
    return res


def unet_timing(dev, applies: int = 10, steps: int = 5, batch: int = 4):
    """The reconstruction workload's preconditioner network (512 x 512, the
    linear U-Net of learn.LINEAR_RECIPE, random weights): mean time of an
    apply and of an energy-norm training step (batch 4: forward, loss through
    the normal operator, backward, Adam), for profiling the network's
    kernels."""
    import torch

    import xrt_workloads as W
    from paper_2503_20907_amd import learn, ops
    N, lam = 512, 1e-2
    rc = learn.LINEAR_RECIPE
    spec, _ = W.recon_problem(N, 180, 768)
    plan = ops.Plan(N, N, 3, ops.Lines.from_spec(spec))
    net = learn.UNet(N, N, levels=rc["levels"], base=rc["base"], max_batch=batch, seed=1,
                     max_channels=rc["max_channels"], relu=rc["relu"])
    fields = W.training_fields(batch, N, N, seed=3, device=dev)
    R = learn.make_pairs(plan, lam, fields)
    net.gain = learn.typical_gain(R, fields)
    z = torch.empty_like(R[0])
    for _ in range(2):
        net.apply(R[0], z)
        net.train_step_energy(plan, lam, R, fields, 1e-5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(applies):
        net.apply(R[0], z)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        net.train_step_energy(plan, lam, R, fields, 1e-5)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out = {"apply_ms": round((t1 - t0) / applies * 1e3, 4), "train_step_ms": round((t2 - t1) / steps * 1e3, 4),
           "batch": batch, "params": int(net.num_params)}
    net.close()
    plan.close()
    return out


def flops_per_nonzero(n: int) -> int:
    # one degree-(2n+1) polynomial evaluation (2n+1 FMAs) + one FMA, 2 flops each
    return 4 * n + 4


def cpu_baseline(spec, coeffs, degree, n_lines_total, seconds_target=15.0):
    """The FP64 oracle, as it stands, on a random sample of the same lines:
    forward + ray-major adjoint; rate scaled to lines per second."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(1234)
    lc = oracle.lines(spec)
    c64 = coeffs.astype(np.float64)
    ny, nx = coeffs.shape
    threads = oracle.max_threads()

    def run(k):
        pick = rng.choice(n_lines_total, size=k, replace=False)
        sub = tuple(v[pick] for v in lc)
        t0 = time.perf_counter()
        s = oracle.forward(degree, c64, sub)
        t1 = time.perf_counter()
        oracle.adjoint(degree, s, sub, nx, ny)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1

    # time = fixed + k * per_line (the ray-major adjoint has a fixed cost: one
    # FP64 image per thread); two sizes fix both, the third run is the sample
    k1, k2 = 1024, 8192
    t1 = sum(run(k1))
    t2 = sum(run(k2))
    per = max((t2 - t1) / (k2 - k1), 1e-9)
    fixed = max(t1 - k1 * per, 0.0)
    k3 = int(max(k2, min(400000, (seconds_target - fixed) / per)))
    tf, ta = run(k3)
    k2 = k3
    rate = k2 / (tf + ta)
    return {"value": rate / 1e9, "unit": "Gray/s", "cores": threads, "kind": "oracle",
            "sample": f"{k2} random lines of the workload, forward + ray-major adjoint "
                      f"(FP64 C/OpenMP), {tf + ta:.1f} s; rate = lines / time",
            "lines_per_s": rate, "cpu": host_cpu_model()}


def host_cpu_model() -> str:
    """The host processor's model name (from /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def recon_leg(log):
    """Metric 2: wall time to ||b - M x|| <= 1e-3 ||b|| from x = 0."""
    import numpy as np
    import torch

    import xrt_workloads as W
    from paper_2503_20907_amd import learn, ops
    dev = torch.device("cuda:0")
    N, n, lam, tol = 512, 3, 1e-2, 1e-3
    spec, c_true = W.recon_problem(N, 180, 768)
    plan = ops.Plan(N, N, n, ops.Lines.from_spec(spec))
    clean = plan.forward(torch.as_tensor(c_true, device=dev)).cpu().numpy()
    p = torch.as_tensor(W.noisy_log_data(clean, photons=1e4, peak=3.0), device=dev)
    b = plan.adjoint(p)

    def timed(reps=3, **kw):
        out = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = learn.solve(plan, b, lam, tol=tol, maxit=2000, **kw)
            torch.cuda.synchronize()
            out.append(((time.perf_counter() - t0) * 1e3, info))
        out.sort(key=lambda v: v[0])
        return out[len(out) // 2]

    cg_ms, cg = timed()
    log(f"[bench] recon CG {cg_ms:.2f} ms, {cg['iterations']} steps")
    # preconditioned CG with the second-difference sinogram filter (180 views of 768 bins)
    pc = learn.SinoPreconditioner.second_difference(180, 768, dev)
    fl_ms, fl = timed(precond=pc)
    log(f"[bench] recon filter-preconditioned {fl_ms:.2f} ms, {fl['iterations']} steps")
    fields = W.training_fields(800, N, N, seed=3, device=dev)
    net, st = learn.train_preconditioner(plan, lam, fields, **learn.LINEAR_RECIPE,
                                         val_fields=W.training_fields(8, N, N, seed=11, device=dev))
    log(f"[bench] recon training {st['train_s']:.1f} s (round {st['kept_round']} kept)")
    # the linear network proposes on every step; flexible CG keeps the last 8 directions
    window, period, net_steps = 8, 1, 0
    ln_ms, ln = timed(net=net, window=window, period=period, net_steps=net_steps)
    log(f"[bench] recon learned {ln_ms:.2f} ms, {ln['iterations']} steps")
    z = torch.empty_like(b)
    for _ in range(3):
        net.apply(b, z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        net.apply(b, z)
    torch.cuda.synchronize()
    net_ms = (time.perf_counter() - t0) * 100.0
    q = torch.empty_like(b)
    ws = torch.empty(plan.lines.n, dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    for _ in range(10):
        learn.normal_apply(plan, b, lam, out=q, sino_ws=ws)
    torch.cuda.synchronize()
    op_ms = (time.perf_counter() - t0) * 100.0
    net.close()
    plan.close()
    return {"metric": "wall ms to relative residual 1e-3: CG, learned U-Net preconditioner, "
                      "sinogram-filter preconditioner",
            "workload": "512x512 cubic B-spline, 180x768 parallel beam, Poisson I0=1e4, lambda=1e-2, x0=0",
            "cg_ms": round(cg_ms, 3), "cg_steps": cg["iterations"],
            "cg_operator_applies": cg["operator_applies"],
            "learned_ms": round(ln_ms, 3), "learned_steps": ln["iterations"],
            "learned_operator_applies": ln["operator_applies"],
            "learned_network_steps": ln["learned_accepted"], "learned_rejected": ln["learned_rejected"],
            "learned_over_cg_time": round(ln_ms / cg_ms, 3),
            "solver": f"flexible CG, window {window}, network on every step",
            "network": "linear U-Net (no activations, no biases): 6 levels of 32 channels, bf16 MFMA, "
                       f"energy-norm loss, {st['pairs']} operator-made pairs (refreshed with the solver's "
                       f"states), {st['steps']} Adam steps x batch {st['batch']}, round {st['kept_round']} of "
                       f"{len(st['val_scores'])} kept by validation on 8 held-out problems",
            "deviations": "6 levels rather than 4 (the residual keeps energy at wavelengths beyond a 4-level "
                          "receptive field); 32 channels at every level; no activations; 800 pairs refreshed "
                          "between rounds rather than 2000 fixed ones",
            "train_s": round(st["train_s"], 1), "network_apply_ms": round(net_ms, 3),
            "operator_apply_ms": round(op_ms, 3),
            "filter_ms": round(fl_ms, 3), "filter_steps": fl["iterations"],
            "filter_over_cg_time": round(fl_ms / cg_ms, 3),
            "filter": "P r = H^T (f * (H r)), f = (-1, 2, -1) along each view's 768 bins; preconditioned CG",
            "rel_residual": {"cg": cg["rel_residual"], "learned": ln["rel_residual"],
                             "filter": fl["rel_residual"]}}


def batch_leg(log):
    """64 uneven problems (sizes 128..1024, degrees 1 and 3, 60..720 views,
    parallel or fan): per-problem plans one after another vs the batch's
    persistent launches, eager and replayed as a HIP graph, before and after
    the autotuner.  Rates in lines per second over the whole batch."""
    import torch

    import xrt_workloads as W
    from paper_2503_20907_amd import batch, ops
    probs = W.batch_problems(64, phantoms=False)
    lines = [ops.Lines.from_spec(p["spec"]) for p in probs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = batch.Batch([(p["N"], p["N"], p["degree"], l) for p, l in zip(probs, lines)])
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    g = torch.Generator(device="cuda").manual_seed(0)
    for k in range(len(b)):
        b.coeffs(k).normal_(generator=g)
    plans = [ops.Plan(p["N"], p["N"], p["degree"], l) for p, l in zip(probs, lines)]
    sinos = [torch.empty(l.n, device="cuda") for l in lines]
    backs = [torch.empty(p["N"], p["N"], device="cuda") for p in probs]

    def seq():
        for k, pl in enumerate(plans):
            pl.forward(b.coeffs(k), sinos[k])
            pl.adjoint(sinos[k], backs[k])

    def timeit(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps * 1e3

    M = b.info()["lines"]
    out = {"workload": "64 problems: N in {128,256,512,1024}, degree in {1,3}, 60-720 views, "
                       "ceil(1.5N) bins, parallel or fan (seed 21)",
           "lines": int(M), "create_ms": round(create_ms, 1)}
    out["sequential_plans_ms"] = round(timeit(seq), 3)
    out["batch_ms_default"] = round(timeit(lambda: b.run(graph=False)), 3)
    t0 = time.perf_counter()
    out["autotuned_config"] = b.autotune(reps=2)
    out["autotune_s"] = round(time.perf_counter() - t0, 2)
    out["batch_ms"] = round(timeit(lambda: b.run(graph=False)), 3)
    out["batch_graph_ms"] = round(timeit(lambda: b.run(graph=True)), 3)
    out["batch_fwd_ms"] = round(timeit(b.forward), 3)
    out["batch_adj_ms"] = round(timeit(b.adjoint), 3)
    best = min(out["batch_ms"], out["batch_graph_ms"])
    out["gray_per_s"] = round(M / (best / 1e3) / 1e9, 5)
    out["speedup_vs_sequential"] = round(out["sequential_plans_ms"] / best, 3)
    log(f"[bench] batch: sequential {out['sequential_plans_ms']} ms, batched {out['batch_ms']} ms, "
        f"graph {out['batch_graph_ms']} ms, config {out['autotuned_config']}")
    for pl in plans:
        pl.close()
    b.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-recon", action="store_true", help="skip the reconstruction (learned vs CG) leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-problems leg")
    ap.add_argument("--no-box", action="store_true", help="skip the box-spline timing on the same lines")
    ap.add_argument("--n-src", type=int, default=1440)
    ap.add_argument("--n-bins", type=int, default=3072)
    ap.add_argument("--grid", type=int, default=2048)
    ap.add_argument("--degree", type=int, default=3)
    ap.add_argument("--copy-only", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device (calibrates HBM byte counters)")
    ap.add_argument("--lds-calib", action="store_true",
                    help="time xrt_calib_lds (LDS atomic cost per address pattern) and exit")
    ap.add_argument("--valu-calib", action="store_true",
                    help="only run the VALU calibration kernel (known instruction count) and print its issue rate")
    ap.add_argument("--unet-only", action="store_true",
                    help="only time the U-Net preconditioner (512x512, 6 levels, 32..256 channels): "
                         "applies and residual-space training steps (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is a design note only)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import xrt_workloads as W
    from paper_2503_20907_amd import ops

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_only:
        # a plain copy of known size: FETCH_SIZE / WRITE_SIZE of this kernel
        # give the scale between the counters and bytes moved
        nel = args.copy_only * (1 << 20) // 4
        a = torch.ones(nel, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_only, "bytes_read": nel * 4,
                          "bytes_written": nel * 4}), flush=True)
        return
    if args.valu_calib:
        print(json.dumps(valu_calibration(dev)), flush=True)
        return
    if args.lds_calib:
        print(json.dumps(lds_calibration(dev)), flush=True)
        return
    if args.unet_only:
        print(json.dumps(unet_timing(dev)), flush=True)
        return
    N, n = args.grid, args.degree
    print(f"[bench] building workload {N}^2 degree {n}", file=sys.stderr, flush=True)
    spec, nfan = W.large_lines(args.n_src, args.n_bins, None, N, n)
    coeffs = W.large_phantom(N)
    M = spec["endpoints"].shape[0]
    lines = ops.Lines.from_spec(spec)
    c = torch.as_tensor(coeffs, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = ops.Plan(N, N, n, lines)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    nnz = plan.nnz()
    _, n_cross = plan.info()
    print(f"[bench] plan {plan_ms:.1f} ms, lines {M}, crossing {n_cross}, nnz {nnz}",
          file=sys.stderr, flush=True)

    sino = torch.empty(M, dtype=torch.float32, device=dev)
    back = torch.empty((N, N), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    nsteps = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(nsteps)]

    for _ in range(args.warmup):
        plan.forward(c, sino)
        plan.adjoint(sino, back)
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for k in range(nsteps):
        ev[k][0].record(stream)
        plan.forward(c, sino)
        ev[k][1].record(stream)
        plan.adjoint(sino, back)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tf = np.array([ev[k][0].elapsed_time(ev[k][1]) for k in range(nsteps)])
    ta = np.array([ev[k][1].elapsed_time(ev[k][2]) for k in range(nsteps)])
    ms_per_step = wall * 1e3 / nsteps
    value = M / (ms_per_step / 1e3) / 1e9
    print(f"[bench] fwd {tf.mean():.3f} ms (median {np.median(tf):.3f}), adj {ta.mean():.3f} ms "
          f"(median {np.median(ta):.3f}), step {ms_per_step:.3f} ms", file=sys.stderr, flush=True)

    F = flops_per_nonzero(n)
    dominant = "adjoint" if ta.mean() >= tf.mean() else "forward"
    t_dom = max(ta.mean(), tf.mean()) / 1e3
    achieved = nnz * F / t_dom / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
                "traffic": measured_traffic(dominant),
                "kernel": ("adjoint: k_sort_sino + k_adjoint<3, 1> (vertical lines) + k_adjoint<3, 2> "
                           "(horizontal lines) + k_adj_reduce after each + k_adj_nonfinite, timed as one call"
                           if dominant == "adjoint" else
                           "forward: k_layout_v/h + k_forward_persist + k_fwd_reduce, timed as one call"),
                "frac_nonpacked_peak": round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 4),
                "work": f"nnz(H) = {nnz} basis evaluations x {F} flops per launch"}

    result = {
        "metric": "Gray/s fwd+adjoint (2048² cubic spline)",
        "value": round(value, 5),
        "unit": "Gray/s",
        "n_gpus": 1,
        "steps": nsteps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{N}x{N} B-spline degree {n}; fan {args.n_src}x{args.n_bins} "
                               f"(R=4000) + {M - nfan} random lines, as one endpoint list",
                   "grid": N, "degree": n, "lines": int(M), "lines_crossing": int(n_cross),
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "t_fwd_ms": round(float(tf.mean()), 4),
        "t_adj_ms": round(float(ta.mean()), 4),
        "t_fwd_median_ms": round(float(np.median(tf)), 4),
        "t_adj_median_ms": round(float(np.median(ta)), 4),
        "plan_ms": round(plan_ms, 2),
        "nnz_per_pass": int(nnz),
        "basis_evals_per_s": round(2 * nnz / (ms_per_step / 1e3), 1),
        "rays_per_s": round(M / (ms_per_step / 1e3), 1),
    }
    plan.close()
    if not args.no_box:
        # the 3-directional box spline (the paper's recommended basis) on the same lines
        bplan = ops.Plan(N, N, 16, lines)
        for _ in range(2):
            bplan.forward(c, sino)
            bplan.adjoint(sino, back)
        torch.cuda.synchronize()
        evb = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(5)]
        for k in range(5):
            evb[k][0].record(stream)
            bplan.forward(c, sino)
            evb[k][1].record(stream)
            bplan.adjoint(sino, back)
            evb[k][2].record(stream)
        torch.cuda.synchronize()
        bf = float(np.median([evb[k][0].elapsed_time(evb[k][1]) for k in range(5)]))
        ba = float(np.median([evb[k][1].elapsed_time(evb[k][2]) for k in range(5)]))
        bnnz = bplan.nnz()
        result["box3"] = {"basis": "3-directional box spline (e1, e2, e1+e2)", "t_fwd_ms": round(bf, 3),
                          "t_adj_ms": round(ba, 3), "gray_per_s": round(M / ((bf + ba) / 1e3) / 1e9, 5),
                          "nnz_per_pass": int(bnnz),
                          "basis_evals_per_s": round(2 * bnnz / ((bf + ba) / 1e3), 1)}
        print(f"[bench] box spline fwd {bf:.3f} ms, adj {ba:.3f} ms", file=sys.stderr, flush=True)
        bplan.close()
    del sino, back
    if not args.no_batch:
        result["batch"] = batch_leg(lambda msg: print(msg, file=sys.stderr, flush=True))
    if not args.no_recon:
        result["recon"] = recon_leg(lambda msg: print(msg, file=sys.stderr, flush=True))
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(spec, coeffs, n, M)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
