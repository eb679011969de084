"""Benchmark of the clustered spectral likelihood + adjoint on one MI355X.

Headline workload: 196608 pixels (nside-128 count), 22 bands 34-448 GHz, K = (5000, 500, 2000)
spherical K-means clusters, a batch of 64 noise realizations, FP32-bulk storage and frequency
accumulation with FP64 Cholesky and compensated FP64 reductions.  A step is one batched
likelihood + gradient evaluation of every realization (SED tables, per-segment sums when the
schedule shares them, the fused per-pixel kernel, per-cluster reductions); `value` counts
evaluations (one item: -2 ln L and its full gradient) per second with the data already resident
in HBM.  The same run reports:
  - the plain FP64 GPU path and the FP32-vs-FP64 error of every result;
  - the pixel kernel against the HBM roofline (HIP events around every launch of that kernel in
    the timed region) and against a plain device copy timed in the same run;
  - the batched optimiser to convergence on workload 5 (FP64 and mixed precision, with the
    parameter agreement), workload 3 (256 realizations) and the workload-4 configuration scan
    (1024 configurations, patchings by the device K-means);
  - evaluations per second of workloads 1-4 in both precisions;
  - component maps, batched K-means, and the FP64 oracle on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-optimizer] ...
"""

from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import multiprocessing as mp
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


def host_cores() -> int:
    """CPU share of this process (at most 16, the share of one GPU on the box)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def algorithmic_bytes(prob, sky, storage_bytes: int) -> float:
    """Bytes one batched evaluation must move: the data stream of every included pixel-item
    (2 F values), the three labels of every included pixel once per labelling, and one FP64
    gradient value per cluster plus F per item."""
    total = 0.0
    F = sky.nfreq
    shared_labels = sky.labels.shape[0] == 1
    for b in range(sky.nitems):
        n_incl, _ = prob.item_info(b)
        total += n_incl * 2 * F * storage_bytes + 8 * (int(sky.nclusters[b].sum()) + 1)
        if b == 0 or not shared_labels:
            total += 12 * n_incl
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
    current kernel source with the same grid form, XCD mapping and schedule mode (these decide
    which L2 fetches which SED table)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
        with open(KERNEL_SOURCE, "rb") as fh:
            src = hashlib.sha256(fh.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if not schedule or rec.get("kernel_source_sha256") != src:
        return None
    key = tuple(int(schedule.get(k, 0)) for k in ("blocks_per_cu", "xcd_remap", "shared_segments"))
    for r in rec.get("records", []):
        s = [int(v) for v in r["counter_schedule"].split(",")]
        if (s[1], s[2], s[3]) == key:
            return r["traffic_bytes_per_launch"]
    return None


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """A plain device-to-device copy of nbytes (read + write counted), GB/s."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


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


def status_counts(cs, st):
    return dict(converged=int(np.sum(st & cs.CONVERGED > 0)), ls_fail=int(np.sum(st & cs.LS_FAIL > 0)),
                maxiter=int(np.sum(st & cs.MAXITER > 0)), not_pd=int(np.sum(st & cs.NOT_PD > 0)))


def run_opt(cs, prob, lo, hi, x0, **kw):
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = prob.cs_optimize_batch(lo, hi, x0, cs.default_opts(**kw))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    h = {k: v.cpu().numpy() for k, v in r.items() if torch.is_tensor(v)}
    h["time_s"] = dt
    return h


def opt_summary(cs, h, solver="projected L-BFGS"):
    ne = h["nevals"]
    return dict(solver=solver, time_s=h["time_s"], evals=int(ne.sum()), evals_per_s=float(ne.sum() / h["time_s"]),
                iters_median=float(np.median(h["iters"])), iters_max=int(h["iters"].max()),
                **status_counts(cs, h["status"]), f_mean=float(np.mean(h["f"])))


def maps_leg(prob, x, reps=5):
    """Component maps and sigma^2_CMB of every item at x, in the caller's pixel order and in
    processing order: items per second and the bytes moved (the stored data read once, the six
    FP64 maps written)."""
    out = {}
    for name, srt in (("pixel_order", False), ("processing_order", True)):
        prob.cs_component_maps(x, sorted_order=srt)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            prob.cs_component_maps(x, sorted_order=srt)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        pix = prob.nitems * prob.npix
        nbytes = pix * (2 * prob.nfreq * 4 + 6 * 8)
        out[name] = dict(items_per_s=prob.nitems / dt, ms_per_call=dt * 1e3, bytes_per_call=nbytes,
                         achieved_gbs=nbytes / dt / 1e9)
    return out


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


def optimizer_legs(cs, sky, sched):
    """Workload 5 to convergence: FP64, then mixed precision (FP32 phase, FP64-accumulation
    polish); the parameter agreement from the common start, and the FP64 optimum of the basin
    the mixed-precision run ended in (FP64 restarted from its point)."""
    lo, hi = sky.bounds_packed()
    x0 = sky.x_packed()
    p = cs.Problem.from_sky(sky, "fp64")
    if sched:
        p.set_schedule(**sched)
    r64 = run_opt(cs, p, lo, hi, x0, max_iter=20000)
    out = dict(fp64=opt_summary(cs, r64))
    log(f"optimizer fp64: {out['fp64']}")
    p32 = cs.Problem.from_sky(sky, "fp32_bulk")
    if sched:
        p32.set_schedule(**sched)
    r32 = run_opt(cs, p32, lo, hi, x0, max_iter=20000)
    out["mixed"] = opt_summary(cs, r32)
    log(f"optimizer mixed precision: {out['mixed']}")
    rel = np.abs(r32["x"] - r64["x"]) / np.maximum(1.0, np.abs(r64["x"]))
    # the restart's own start gradient is already at the stopping scale, so it only polishes: a
    # bounded run shows how far the FP64 optimum of that basin lies
    rb = run_opt(cs, p, lo, hi, r32["x"], max_iter=200)
    relb = np.abs(r32["x"] - rb["x"]) / np.maximum(1.0, np.abs(rb["x"]))
    out["agreement"] = dict(
        from_common_start=dict(max_rel_dx=float(rel.max()), share_above_1e4=float(np.mean(rel > 1e-4)),
                               max_rel_dF=float(np.max(np.abs(r32["f"] - r64["f"]) / np.abs(r64["f"])))),
        fp64_restart_at_mixed_optimum=dict(max_rel_dx=float(relb.max()), iters_median=float(np.median(rb["iters"])),
                                           **status_counts(cs, rb["status"])))
    log(f"optimizer agreement: {out['agreement']}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r = p32.cs_optimize_batch(lo, hi, x0, cs.default_opts(max_iter=1000, solver=cs.SOLVER_ADATOPK))
    torch.cuda.synchronize()
    h = {k: v.cpu().numpy() for k, v in r.items() if torch.is_tensor(v)}
    h["time_s"] = time.perf_counter() - t1
    out["adatopk_1000_iterations"] = opt_summary(cs, h, "AdaTopK (1000 iterations)")
    log(f"optimizer AdaTopK: {out['adatopk_1000_iterations']}")
    return out


def evals_per_s(cs, sky, precision, steps=20):
    p = cs.Problem.from_sky(sky, precision)
    x = torch.as_tensor(sky.x_packed(), device="cuda")
    wall, _, _, _ = time_eval(p, x, steps, 3, timing=False)
    return sky.nitems * steps / wall


def scan_problem(cs, tasks, precision="fp64"):
    """Workload 4: the 3 x 1024 patchings by the device K-means, then the batched problem."""
    sky = tasks.sky
    C, P = len(tasks.k) // 3, sky.npix
    vecs = torch.as_tensor(sky.vecs, device="cuda")
    init = torch.as_tensor(tasks.init, device="cuda")
    keep = torch.as_tensor(tasks.keep.astype(np.uint8), device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lab, keff = cs.kmeans_batch(vecs, tasks.k, init, keep)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    keff = keff.cpu().numpy().reshape(C, 3)
    prob = cs.Problem(sky.freqs, sky.d.to("cuda"), sky.ninv, lab.view(C, 3, P).contiguous(), keff,
                      precision=precision)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return prob, keff, (t1 - t0), (t2 - t1)


def workload_legs(cs):
    """Evaluations per second of workloads 1-4 (both precisions), the optimiser on workload 3
    (256 realizations) and the workload-4 configuration scan (1024 configurations)."""
    import skygen

    out = {}
    for cid in (1, 2, 3):
        sky = skygen.make_config(cid, device="cuda")
        leg = dict(items=sky.nitems, npix=sky.npix, nfreq=sky.nfreq, clusters=sky.nclusters[0].tolist(),
                   fp32_bulk_evals_per_s=evals_per_s(cs, sky, "fp32_bulk"), fp64_evals_per_s=evals_per_s(cs, sky, "fp64"))
        if cid == 3:
            lo, hi = sky.bounds_packed()
            for prec in ("fp64", "fp32_bulk"):
                h = run_opt(cs, cs.Problem.from_sky(sky, prec), lo, hi, sky.x_packed())
                leg[f"optimizer_{prec}"] = opt_summary(cs, h)
        out[f"workload{cid}"] = leg
        log(f"workload {cid}: {leg}")
    tasks = skygen.scan_tasks(1024)
    prob, keff, t_km, t_prep = scan_problem(cs, tasks)
    C = keff.shape[0]
    x0, lo, hi = (np.concatenate(v) for v in zip(*[skygen.start_and_box(keff[c]) for c in range(C)]))
    x = torch.as_tensor(x0, device="cuda")
    w64, _, _, _ = time_eval(prob, x, 10, 2, timing=False)
    h = run_opt(cs, prob, lo, hi, x0, max_iter=20000)
    p32, _, _, _ = scan_problem(cs, tasks, "fp32_bulk")
    w32, _, _, _ = time_eval(p32, x, 10, 2, timing=False)
    del p32
    npar = keff.sum(axis=1)
    leg = dict(configurations=C, npix=tasks.sky.npix, params_per_configuration=[int(npar.min()), float(npar.mean()),
                                                                               int(npar.max())],
               kmeans_s=t_km, prepare_s=t_prep, fp64_evals_per_s=C * 10 / w64, fp32_bulk_evals_per_s=C * 10 / w32,
               optimizer_fp64=opt_summary(cs, h),
               configurations_per_s=C / (t_km + t_prep + h["time_s"]),
               min_neg2logL=dict(min=float(h["f"].min()), median=float(np.median(h["f"])), max=float(h["f"].max())))
    out["workload4"] = leg
    log(f"workload 4: {leg}")
    return out


def cpu_worker(args):
    """Oracle evaluations of one worker's contiguous chunk of items, repeated until the budget."""
    from oracle import oracle

    rank, begin, end, budget = args
    data = _CPU_DATA
    n, t0 = 0, time.perf_counter()
    probs = [oracle.Problem(data["freqs"], data["d"][b], data["ninv"], data["labels"], data["ncl"]) for b in
             range(begin, end)]
    while probs and time.perf_counter() - t0 < budget:
        for k, pr in enumerate(probs):
            pr.likelihood_grad(data["x"][begin + k])
            n += 1
    return rank, n, time.perf_counter() - t0


_CPU_DATA = {}


def cpu_baseline(cs, sky, x_items, budget_s: float = 12.0):
    """The FP64 oracle on the host cores: one process per core, worker k taking the items
    [floor(k N / P), floor((k + 1) N / P)) and evaluating them in turn until the time budget."""
    from oracle import oracle

    oracle.build(force=False)
    ncores = min(host_cores(), sky.nitems)
    _CPU_DATA.update(freqs=sky.freqs, ninv=sky.ninv, labels=sky.item_labels(0), ncl=sky.nclusters[0],
                     d=[sky.item_d(b) for b in range(sky.nitems)], x=x_items)
    jobs = [(k, *cs.item_range(k, ncores, sky.nitems), budget_s) for k in range(ncores)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(ncores) as pool:
        res = pool.map(cpu_worker, jobs)
    wall = time.perf_counter() - t0
    _CPU_DATA.clear()
    n = sum(r[1] for r in res)
    busy = max(r[2] for r in res)
    per_core = float(np.mean([r[1] / r[2] for r in res]))
    return dict(value=n / busy, unit="evals/s", cores=ncores, kind="oracle", cpu_model=cpu_model(),
                per_core_evals_per_s=per_core, wall_s=wall,
                sample=f"{n} single-item evaluations (F and full gradient, {sky.npix} px, {sky.nfreq} bands) of "
                       f"the FP64 C oracle in {ncores} processes, worker k evaluating items "
                       f"[floor(k N / P), floor((k + 1) N / P)) of the N = {sky.nitems} in turn for about "
                       f"{budget_s:.0f} s")


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
    ap.add_argument("--no-workloads", action="store_true", help="skip workloads 1-4")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="kernel-profiling run: only the timed evaluations of one precision")
    ap.add_argument("--profile-optimizer", type=int, default=0, metavar="ITERS",
                    help="kernel-profiling run: only the batched optimiser, ITERS iterations, one precision")
    ap.add_argument("--precision", default="fp32_bulk", choices=["fp64", "fp32_bulk", "fp32_store"])
    ap.add_argument("--schedule", default=None,
                    help="waves_per_block,blocks_per_cu,xcd_remap,shared_segments (skips the autotuner)")
    ap.add_argument("--profile-maps", default=None, choices=["pixel", "processing"],
                    help="kernel-profiling run: only the component maps (FP32-bulk problem), in that order")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="HBM counter calibration: time a plain device copy of this many bytes and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: items would be sharded across GPUs by contiguous chunks "
              "(cs_item_range), which this single-GPU benchmark does not run", file=sys.stderr)
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
    # evaluation points: a seeded perturbation of the start point inside the box
    g = np.random.default_rng(7)
    lo, hi = sky.bounds_packed()
    xs = np.clip(sky.x_packed() + g.normal(0, 1, lo.size) * np.tile(
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
        h = run_opt(cs, prob, lo, hi, sky.x_packed(), max_iter=args.profile_optimizer, fp64_polish=0)
        ne = int(h["nevals"].sum())
        print(json.dumps({"precision": args.precision, "optimizer_s": h["time_s"], "evals": ne,
                          "ms_per_step": h["time_s"] / (ne / sky.nitems) * 1e3}), flush=True)
        return

    if args.profile_maps:
        prob = cs.Problem.from_sky(sky, "fp32_bulk")
        srt = args.profile_maps == "processing"
        for _ in range(args.warmup):
            prob.cs_component_maps(x, sorted_order=srt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            prob.cs_component_maps(x, sorted_order=srt)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / args.steps
        print(json.dumps({"maps_order": args.profile_maps, "ms_per_call": dt * 1e3}), flush=True)
        return

    if args.profile:
        prob = cs.Problem.from_sky(sky, args.precision)
        if fixed:
            prob.set_schedule(**fixed)
        wall, kms, nl, _ = time_eval(prob, x, args.steps, args.warmup, label=f"bench_timed_{args.precision}")
        ab = algorithmic_bytes(prob, sky, 8 if args.precision == "fp64" else 4)
        print(json.dumps({"precision": args.precision, "schedule": fixed, "ms_per_step": wall / args.steps * 1e3,
                          "kernel_ms": kms / max(nl, 1), "bytes_per_launch": ab,
                          "achieved_gbs": ab / (kms / max(nl, 1) * 1e-3) / 1e9}), flush=True)
        return

    copy_gbs = copy_bandwidth()
    log(f"plain device copy: {copy_gbs:.0f} GB/s (read + write)")
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
    traffic = measured_traffic(sched)  # HBM bytes per launch from the committed counter record, or None
    log(f"fp32_bulk: {value:.1f} evals/s, {ms_per_step:.3f} ms/step, pixel kernel {kavg:.3f} ms, "
        f"{achieved:.0f} GB/s algorithmic ({achieved / HBM_PEAK_GBS:.1%} of peak, {achieved / copy_gbs:.1%} of the copy)")
    del p32
    torch.cuda.empty_cache()

    fp64 = None
    err = None
    if not args.no_fp64:
        p64 = cs.Problem.from_sky(sky, "fp64")
        if fixed:
            p64.set_schedule(**fixed)
        elif sched:
            p64.autotune(x, reps=2)
        w64, k64, n64, out64 = time_eval(p64, x, args.steps, args.warmup)
        f64 = out64[0].cpu().numpy()
        g64 = out64[1].cpu().numpy()
        ab64 = algorithmic_bytes(p64, sky, 8)
        s64 = p64.get_schedule()
        fp64 = dict(value=sky.nitems * args.steps / w64, ms_per_step=w64 / args.steps * 1e3,
                    kernel_ms=k64 / max(n64, 1), achieved_gbs=ab64 / (k64 / max(n64, 1) * 1e-3) / 1e9,
                    schedule=[s64.waves_per_block, s64.blocks_per_cu, s64.xcd_remap, s64.shared_segments])
        off = sky.param_offsets()
        gre = max(np.max(np.abs(g32[o:e] - g64[o:e])) / np.max(np.abs(g64[o:e])) for o, e in zip(off[:-1], off[1:]))
        err = dict(max_rel_F=float(np.max(np.abs(f32 - f64) / np.abs(f64))), max_rel_grad_normwise=float(gre))
        log(f"fp64: {fp64}; fp32 vs fp64 {err}")
        del p64
        torch.cuda.empty_cache()

    opt = optimizer_legs(cs, sky, sched) if not args.no_optimizer else None
    torch.cuda.empty_cache()

    maps = None
    if not args.no_maps:
        pm = cs.Problem.from_sky(sky, "fp32_bulk")
        if sched:
            pm.set_schedule(**sched)
        maps = maps_leg(pm, x)
        log(f"component maps: {maps}")
        del pm
        torch.cuda.empty_cache()

    km = kmeans_leg() if not args.no_kmeans else None
    if km:
        log(f"k-means: {km}")
    wl = workload_legs(cs) if not args.no_workloads else None
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cs, sky, x_items)
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
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_pixel_stage (fused likelihood + adjoint, schedule mode "
                               f"{sched.get('shared_segments') if sched else 'default'})",
                     "kernel_ms": kavg, "bytes_per_launch": abytes, "copy_gbs": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs,
                     # counted HBM traffic (fetch + write) over the same launch duration
                     "traffic_gbs": traffic / (kavg * 1e-3) / 1e9 if traffic else None},
        "cpu_baseline": cpu,
        "fp64_path": fp64,
        "fp32_vs_fp64": err,
        "prep_ms": prep_ms,
        "optimizer": opt,
        "component_maps": maps,
        "kmeans": km,
        "workloads": wl,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
