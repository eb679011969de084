"""Helpers comparing the HIP library with the FP64 oracle (test code only)."""

from __future__ import annotations

import numpy as np
import torch

from oracle import oracle

# tolerances of the workload statement: FP64 path <= 1e-12 relative on -2 ln L and <= 1e-9
# relative on gradients; FP32-bulk <= 1e-5 relative on -2 ln L.
TOL_F = {"fp64": 1e-12, "fp32_store": 1e-6, "fp32_bulk": 1e-5}
# FP64 gradient: normwise relative error against the oracle's gradient of the item
TOL_G = {"fp64": 1e-9}
# unit roundoff of FP32
U32 = 2.0 ** -24


def fp32_grad_tol(nfreq: int, gterm: np.ndarray) -> np.ndarray:
    """Per-cluster bound on the gradient error of the FP32 precisions: each per-band sum of F terms
    carries at most about F u of the magnitude of its terms (recursive summation), and the data
    are rounded to FP32 once (u), so |dg_k| <= 2 F u gterm_k, with gterm_k the summed magnitude
    of the terms the cluster's gradient is built from (oracle grad_terms).  Unlike a normwise
    bound it holds at near-stationary points and for one-pixel clusters whose terms cancel."""
    return 2.0 * nfreq * U32 * gterm


def oracle_items(sky, items=None, x=None):
    """Oracle F, grad and cluster partials for the requested items."""
    items = range(sky.nitems) if items is None else items
    out = {}
    for b in items:
        xb = sky.x[b] if x is None else x[b]
        out[b] = oracle.Problem.from_sky(sky, b).likelihood_grad(xb)
    return out


def gpu_eval(prob, sky, x=None, cluster=True):
    xp = sky.x_packed() if x is None else np.concatenate(x)
    f, g, cf, st = prob.cs_likelihood_grad(torch.as_tensor(xp, device=prob.device), cluster=cluster)
    torch.cuda.synchronize()
    return f.cpu().numpy(), g.cpu().numpy(), (cf.cpu().numpy() if cf is not None else None), st.cpu().numpy()


def check_grad(precision, nfreq, gb, go, gterm=None):
    """Asserts the gradient bound of a precision; returns (normwise error, worst ratio to the
    per-cluster FP32 bound or 0)."""
    eg = np.max(np.abs(gb - go)) / max(np.max(np.abs(go)), 1e-300)
    if precision == "fp64":
        assert eg <= TOL_G["fp64"], eg
        return eg, 0.0
    tol = fp32_grad_tol(nfreq, gterm)
    ratio = float(np.max(np.abs(gb - go) / np.maximum(tol, 1e-300)))
    assert np.all(np.abs(gb - go) <= tol), (ratio, eg)
    return eg, ratio


def compare(sky, prob, precision, items=None, x=None, check_cluster=True):
    """Asserts parity of F, gradient and cluster partials; returns the worst relative errors
    (F, normwise gradient, cluster partials)."""
    f, g, cf, st = gpu_eval(prob, sky, x, cluster=check_cluster)
    ref = oracle_items(sky, items, x)
    off = sky.param_offsets()
    worst_f = worst_g = worst_c = worst_r = 0.0
    for b, (fo, go, co, so) in ref.items():
        assert st[b] == so, (b, st[b], so)
        ef = abs(f[b] - fo) / abs(fo)
        gb = g[off[b]:off[b + 1]]
        gt = None
        if precision != "fp64":
            xb = sky.x[b] if x is None else x[b]
            gt = oracle.Problem.from_sky(sky, b).grad_terms(xb)
        eg, r = check_grad(precision, sky.nfreq, gb, go, gt)
        worst_f, worst_g, worst_r = max(worst_f, ef), max(worst_g, eg), max(worst_r, r)
        assert ef <= TOL_F[precision], (b, f[b], fo, ef)
        if check_cluster:
            cb = cf[off[b]:off[b + 1]]
            ec = np.max(np.abs(cb - co)) / abs(fo)
            worst_c = max(worst_c, ec)
            assert ec <= TOL_F[precision], (b, ec)
    if precision != "fp64":
        print(f"  fp32 gradient: worst |dg| / (2 F u gterm) = {worst_r:.3f}, normwise {worst_g:.2e}", flush=True)
    return worst_f, worst_g, worst_c
