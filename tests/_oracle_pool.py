"""Oracle work for sampled items of the full-size workloads, run in a pool of spawned worker
processes (test code only; the workers touch no GPU)."""

from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from oracle import oracle


def workers() -> int:
    """Processes for oracle work: the host's CPU share, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def box_start(keff):
    """Start point and box of the optimiser for cluster counts keff (the generator's)."""
    import skygen

    return skygen.start_and_box(keff)


def _lbfgs(args):
    freqs, d, ninv, labels, ncl, x0, lo, hi, kw = args
    pr = oracle.Problem(freqs, d, ninv, labels, ncl)
    x, f, it, ne, st = pr.lbfgs(x0, lo, hi, **kw)
    return x, f, it, ne, st


def _eval(args):
    """F, gradient, cluster values and status of one item at x, with the per-cluster rounding
    scale of its gradient terms."""
    freqs, d, ninv, labels, ncl, nu0d, nu0s, tcmb, x = args
    pr = oracle.Problem(freqs, d, ninv, labels, ncl, nu0d, nu0s, tcmb)
    return pr.likelihood_grad(x), pr.grad_terms(x)


def _scan_item(args):
    """One configuration of the scan: its three patchings by the oracle's K-means, then the
    oracle's L-BFGS from x0 on those labels; returns (labels [3][P], keff [3], x, F, iters, status)."""
    freqs, d, ninv, vecs, tasks, kw = args
    P = vecs.shape[0]
    labels = np.full((3, P), -1, dtype=np.int32)
    keff = np.zeros(3, dtype=np.int32)
    for j, (keep, k, init) in enumerate(tasks):
        idx = np.flatnonzero(keep)
        lab, ke = oracle.kmeans(vecs[idx], k, init)
        labels[j, idx] = lab
        keff[j] = ke
    x0, lo, hi = box_start(keff)
    pr = oracle.Problem(freqs, d, ninv, labels, keff)
    x, f, it, ne, st = pr.lbfgs(x0, lo, hi, **kw)
    return labels, keff, x, f, it, st


def run(fn, jobs):
    ctx = mp.get_context("spawn")
    with ctx.Pool(min(workers(), len(jobs))) as pool:
        return pool.map(fn, jobs)


def lbfgs_many(jobs):
    return run(_lbfgs, jobs)


def eval_many(jobs):
    return run(_eval, jobs)


def scan_many(jobs):
    return run(_scan_item, jobs)
