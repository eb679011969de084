"""Benchmark of the clustered spectral likelihood + adjoint on one MI355X.

Workload (default): 196608 pixels (nside-128 count), 22 bands 34-448 GHz, K = (5000, 500, 2000)
spherical K-means clusters, a batch of 64 noise realizations, FP32-bulk storage and frequency
accumulation with FP64 Cholesky and compensated FP64 reductions.  A step is one batched
likelihood + gradient evaluation of every realization (SED tables, fused per-pixel kernel,
per-cluster reductions); `value` counts evaluations (one item: -2 ln L and its full gradient)
per second with the data already resident in HBM.  The same run also reports the plain FP64
GPU path, the FP32-vs-FP64 error of every result, the once-per-clustering preparation time, the
batched on-device projected L-BFGS and AdaTopK, the per-pixel kernel against the HBM roofline (HIP events
around every launch of that kernel in the timed region), and the FP64 oracle on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-optimizer]
"""

from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pixel_stage_workload5_fp32_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2604_08463_amd", "csrc", "cs_eval.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(prob, sky, storage_bytes: int) -> float:
    """Bytes one batched evaluation must move: the packed data stream of every included
    pixel-item, the SED tables read once and the per-segment partials written once."""
    total = 0.0
    F = sky.nfreq
    for b in range(sky.nitems):
        n_incl, nseg = prob.item_info(b)
        kd, kt, ks = (int(v) for v in sky.nclusters[b])
        total += n_incl * 2 * F * storage_bytes
        total += (kd + 2 * kt + ks) * F * storage_bytes
        total += nseg * 4 * 8
    return total


def _roctx():
    """ROC-TX range API (marks the timed region for a profiler run); None if unavailable."""
    for name in ("librocprofiler-sdk-roctx.so.1", "libroctx64.so"):
        try:
            lib = ctypes.CDLL(name)
            lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
            return lib
        except OSError:
            continue
    return None


def measured_traffic(schedule):
    """HBM bytes per launch of the pixel kernel from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE scaled by a plain copy's readings), or None unless that summary was taken on the
    current kernel source and the same kernel variant (per-pixel or segment-shared sums)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
        with open(KERNEL_SOURCE, "rb") as fh:
            src = hashlib.sha256(fh.read()).hexdigest()
    except (OSError, ValueError):
        return None
    shared = int(bool(schedule and schedule.get("shared_segments")))
    if rec.get("kernel_source_sha256") != src or rec.get("shared_segments") != shared:
        return None
    return rec.get("traffic_bytes_per_launch")


def time_eval(prob, x, steps, warmup, timing=True, label=None):
    out = (torch.empty(prob.nitems, dtype=torch.float64, device="cuda"),
           torch.empty(prob.nparams, dtype=torch.float64, device="cuda"),
           torch.empty(prob.nitems, dtype=torch.int32, device="cuda"))
    for _ in range(warmup):
        prob.cs_likelihood_grad(x, out=out)
    torch.cuda.synchronize()
    prob.set_timing(timing)
    prob.kernel_time()  # reset
    tx = _roctx() if label else None
    if tx:
        tx.roctxRangePushA(label.encode())
    t0 = time.perf_counter()
    for _ in range(steps):
        prob.cs_likelihood_grad(x, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if tx:
        tx.roctxRangePop()
    kms, nl = prob.kernel_time() if timing else (0.0, 0)
    prob.set_timing(False)
    return (t1 - t0), kms, nl, out


def maps_leg(prob, x, reps=5):
    """Component maps and sigma^2_CMB of every item at x: items per second and the bytes moved
    (the stored data read once, the six FP64 maps written)."""
    prob.cs_component_maps(x)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        prob.cs_component_maps(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    pix = prob.nitems * prob.npix
    nbytes = pix * (2 * prob.nfreq * 4 + 6 * 8)
    return dict(items_per_s=prob.nitems / dt, ms_per_call=dt * 1e3, bytes_per_call=nbytes,
                achieved_gbs=nbytes / dt / 1e9)


def kmeans_leg(ntask=1024, npix=3072, iters=20, seed=2604):
    """One batched call of spherical K-means patching shaped like the configuration scan: ntask
    tasks on npix positions, latitude masks with f_sky in [0.4, 0.8], K in [10, 3000] (seeded)."""
    import paper_2604_08463_amd as cs
    import skygen
    g = np.random.default_rng(seed)
    v = skygen.sky.positions(npix, g)
    ks = g.integers(10, 3001, ntask).astype(np.int32)
    fsky = g.uniform(0.4, 0.8, ntask)
    keep = np.stack([skygen.latitude_mask(v[:, 2], f) for f in fsky])
    init = np.zeros((ntask, int(ks.max())), dtype=np.int32)
    for t in range(ntask):
        nk = int(keep[t].sum())
        if ks[t] < nk:
            init[t, :ks[t]] = g.choice(nk, size=int(ks[t]), replace=False)
    vt = torch.as_tensor(v, device="cuda")
    it = torch.as_tensor(init, device="cuda")
    kt = torch.as_tensor(keep.astype(np.uint8), device="cuda")
    cs.kmeans_batch(vt, ks[:4], it[:4], kt[:4], iters=iters)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, keff = cs.kmeans_batch(vt, ks, it, kt, iters=iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dict(tasks=ntask, npix=npix, iters=iters, k_range=[10, 3000], fsky_range=[0.4, 0.8], time_s=dt,
                tasks_per_s=ntask / dt, keff_mean=float(keff.float().mean().item()))


def cpu_baseline(sky, x_items, budget_s: float = 12.0):
    from oracle import oracle

    oracle.build(force=False)
    n = 0
    t = 0.0
    b = 0
    while t < budget_s and b < sky.nitems:
        pr = oracle.Problem.from_sky(sky, b)
        t0 = time.perf_counter()
        pr.likelihood_grad(x_items[b])
        t += time.perf_counter() - t0
        n += 1
        b += 1
    return n, t


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-optimizer", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-maps", action="store_true")
    ap.add_argument("--no-kmeans", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="kernel-profiling run: only the timed evaluations of one precision")
    ap.add_argument("--profile-optimizer", type=int, default=0, metavar="ITERS",
                    help="kernel-profiling run: only the batched optimiser, ITERS iterations, one precision")
    ap.add_argument("--precision", default="fp32_bulk", choices=["fp64", "fp32_bulk", "fp32_store"])
    ap.add_argument("--shared-segments", type=int, default=None, choices=[0, 1],
                    help="profiling run: force the per-pixel (0) or segment-shared (1) schedule")
    ap.add_argument("--schedule", default=None,
                    help="waves_per_block,blocks_per_cu,xcd_remap,shared_segments (skips the autotuner)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="HBM counter calibration: time a plain device copy of this many bytes and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X "
              "(items would be sharded across GPUs by contiguous chunks; not part of this build)", file=sys.stderr)
        sys.exit(2)

    if args.copy_bytes:
        n = args.copy_bytes // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(args.warmup + args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4, "launches": args.warmup + args.steps}), flush=True)
        return

    import paper_2604_08463_amd as cs
    import skygen

    cs.load()
    torch.cuda.init()
    t0 = time.perf_counter()
    sky = skygen.make_config(args.workload, device="cuda")
    log(f"workload {args.workload}: P={sky.npix} F={sky.nfreq} B={sky.nitems} K={sky.nclusters[0].tolist()} "
        f"generated in {time.perf_counter() - t0:.1f}s")
    x = torch.as_tensor(sky.x_packed(), device="cuda")
    # evaluation points: a seeded perturbation of the start point inside the box
    g = np.random.default_rng(7)
    lo, hi = sky.bounds_packed()
    xs = np.clip(sky.x_packed() + g.normal(0, 1, x.numel()) * np.tile(
        np.concatenate([np.full(sky.nclusters[0, 0], 0.05), np.full(sky.nclusters[0, 1], 1.0),
                        np.full(sky.nclusters[0, 2], 0.05)]), sky.nitems), lo, hi)
    x = torch.as_tensor(xs, device="cuda")
    x_items = [xs[o:e] for o, e in zip(sky.param_offsets()[:-1], sky.param_offsets()[1:])]

    fixed = None
    if args.schedule:
        w, b, xr, sh = (int(v) for v in args.schedule.split(","))
        fixed = dict(waves_per_block=w, blocks_per_cu=b, xcd_remap=xr, shared_segments=sh)

    if args.profile_optimizer:
        prob = cs.Problem.from_sky(sky, args.precision)
        if fixed:
            prob.set_schedule(**fixed)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = prob.cs_optimize_batch(lo, hi, sky.x_packed(),
                                   cs.default_opts(max_iter=args.profile_optimizer, fp64_polish=0))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        ne = int(r["nevals"].sum().item())
        print(json.dumps({"precision": args.precision, "optimizer_s": dt, "evals": ne,
                          "ms_per_step": dt / (ne / sky.nitems) * 1e3}), flush=True)
        return

    if args.profile:
        prob = cs.Problem.from_sky(sky, args.precision)
        if fixed:
            prob.set_schedule(**fixed)
        elif args.shared_segments is not None:
            prob.set_schedule(4, 0, 1, args.shared_segments)
        wall, kms, nl, _ = time_eval(prob, x, args.steps, args.warmup, label=f"bench_timed_{args.precision}")
        ab = algorithmic_bytes(prob, sky, 8 if args.precision == "fp64" else 4)
        print(json.dumps({"precision": args.precision, "ms_per_step": wall / args.steps * 1e3,
                          "kernel_ms": kms / max(nl, 1), "bytes_per_launch": ab,
                          "achieved_gbs": ab / (kms / max(nl, 1) * 1e-3) / 1e9}), flush=True)
        return

    torch.cuda.synchronize()
    tp = time.perf_counter()
    p32 = cs.Problem.from_sky(sky, "fp32_bulk", d_dtype=torch.float64)
    torch.cuda.synchronize()
    prep_ms = (time.perf_counter() - tp) * 1e3
    log(f"prepared fp32_bulk problem in {prep_ms:.1f} ms; units={p32.item_info(0)}")
    sched = fixed
    if fixed:
        p32.set_schedule(**fixed)
    elif not args.no_autotune:
        s = p32.autotune(x, reps=3)
        sched = dict(waves_per_block=s.waves_per_block, blocks_per_cu=s.blocks_per_cu, xcd_remap=s.xcd_remap,
                     shared_segments=s.shared_segments)
        log(f"autotuned schedule {sched}")
    wall, kms, nl, out32 = time_eval(p32, x, args.steps, args.warmup, label="bench_timed_fp32_bulk")
    f32 = out32[0].cpu().numpy()
    g32 = out32[1].cpu().numpy()
    evals = sky.nitems * args.steps
    value = evals / wall
    ms_per_step = wall / args.steps * 1e3
    abytes = algorithmic_bytes(p32, sky, 4)
    kavg = kms / max(nl, 1)
    achieved = abytes / (kavg * 1e-3) / 1e9
    log(f"fp32_bulk: {value:.1f} evals/s, {ms_per_step:.3f} ms/step, pixel kernel {kavg:.3f} ms, "
        f"{achieved:.0f} GB/s algorithmic ({achieved / HBM_PEAK_GBS:.1%} of peak)")

    fp64 = None
    err = None
    if not args.no_fp64:
        del p32
        torch.cuda.empty_cache()
        p64 = cs.Problem.from_sky(sky, "fp64")
        if fixed:
            p64.set_schedule(**fixed)
        elif sched:
            p64.autotune(x, reps=2)
        w64, k64, n64, out64 = time_eval(p64, x, args.steps, args.warmup)
        f64 = out64[0].cpu().numpy()
        g64 = out64[1].cpu().numpy()
        ab64 = algorithmic_bytes(p64, sky, 8)
        fp64 = dict(value=sky.nitems * args.steps / w64, ms_per_step=w64 / args.steps * 1e3,
                    kernel_ms=k64 / max(n64, 1), achieved_gbs=ab64 / (k64 / max(n64, 1) * 1e-3) / 1e9)
        off = sky.param_offsets()
        gre = max(np.max(np.abs(g32[o:e] - g64[o:e])) / np.max(np.abs(g64[o:e])) for o, e in zip(off[:-1], off[1:]))
        err = dict(max_rel_F=float(np.max(np.abs(f32 - f64) / np.abs(f64))), max_rel_grad_normwise=float(gre))
        log(f"fp64: {fp64['value']:.1f} evals/s; fp32 vs fp64 {err}")
        del p64
        torch.cuda.empty_cache()

    opt = None
    opt_ada = None
    if not args.no_optimizer:
        p32 = cs.Problem.from_sky(sky, "fp32_bulk")
        if sched:
            p32.set_schedule(**sched)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = p32.cs_optimize_batch(lo, hi, sky.x_packed(), cs.default_opts(max_iter=1000))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        st = r["status"].cpu().numpy()
        ne = r["nevals"].cpu().numpy()
        opt = dict(solver="projected L-BFGS", time_s=dt, evals=int(ne.sum()), evals_per_s=float(ne.sum() / dt),
                   iters_median=float(np.median(r["iters"].cpu().numpy())),
                   converged=int(np.sum(st & cs.CONVERGED > 0)), ls_fail=int(np.sum(st & cs.LS_FAIL > 0)),
                   maxiter=int(np.sum(st & cs.MAXITER > 0)), f_mean=float(r["f"].mean().item()))
        log(f"optimizer: {opt}")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = p32.cs_optimize_batch(lo, hi, sky.x_packed(), cs.default_opts(max_iter=1000, solver=cs.SOLVER_ADATOPK))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        st = r["status"].cpu().numpy()
        ne = r["nevals"].cpu().numpy()
        opt_ada = dict(solver="AdaTopK", time_s=dt, evals=int(ne.sum()), evals_per_s=float(ne.sum() / dt),
                       iters_median=float(np.median(r["iters"].cpu().numpy())),
                       converged=int(np.sum(st & cs.CONVERGED > 0)), ls_fail=int(np.sum(st & cs.LS_FAIL > 0)),
                       maxiter=int(np.sum(st & cs.MAXITER > 0)), f_mean=float(r["f"].mean().item()))
        log(f"optimizer (AdaTopK): {opt_ada}")

    maps = None
    if not args.no_maps:
        pm = cs.Problem.from_sky(sky, "fp32_bulk")
        if sched:
            pm.set_schedule(**sched)
        maps = maps_leg(pm, x)
        log(f"component maps: {maps}")
        del pm
        torch.cuda.empty_cache()

    km = None
    if not args.no_kmeans:
        km = kmeans_leg()
        log(f"k-means: {km}")

    cpu = None
    if not args.no_cpu_baseline:
        n, t = cpu_baseline(sky, x_items)
        cpu = dict(value=n / t, unit="evals/s", cores=1, kind="oracle",
                   sample=f"{n} single-item evaluations (F and full gradient, 196608 px, 22 bands) of the "
                          f"FP64 C oracle, one thread")
        log(f"cpu baseline: {cpu}")

    line = {
        "metric": "likelihood+gradient evals/sec and HBM GB/s, FP32-bulk vs FP64 at stated tol",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "196608 px x 22 bands x 64 noise realizations, K=(5000,500,2000), "
                               "FP32-bulk + FP64 Cholesky/reductions",
                   "npix": sky.npix, "nfreq": sky.nfreq, "items": sky.nitems,
                   "clusters": sky.nclusters[0].tolist(), "schedule": sched},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(sched),
                     "kernel": "k_pixel_stage (fused likelihood + adjoint, "
                               + ("segment-shared" if sched and sched.get("shared_segments") else "per-pixel")
                               + " sums)", "kernel_ms": kavg, "bytes_per_launch": abytes},
        "cpu_baseline": cpu,
        "fp64_path": fp64,
        "fp32_vs_fp64": err,
        "prep_ms": prep_ms,
        "optimizer": opt,
        "optimizer_adatopk": opt_ada,
        "component_maps": maps,
        "kmeans": km,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
