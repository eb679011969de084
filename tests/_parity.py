"""Helpers comparing the HIP library with the FP64 oracle (test code only)."""

from __future__ import annotations

import numpy as np
import torch

from oracle import oracle

# tolerances of the workload statement: FP64 path <= 1e-12 relative on -2 ln L and <= 1e-9
# relative on gradients; FP32-bulk <= 1e-5 relative on -2 ln L.
TOL_F = {"fp64": 1e-12, "fp32_store": 1e-6, "fp32_bulk": 1e-5}
# gradient: normwise relative error against the oracle's gradient of the item
TOL_G = {"fp64": 1e-9, "fp32_store": 1e-3, "fp32_bulk": 1e-2}


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


def compare(sky, prob, precision, items=None, x=None, check_cluster=True):
    """Asserts parity of F, gradient and cluster partials; returns the worst relative errors."""
    f, g, cf, st = gpu_eval(prob, sky, x, cluster=check_cluster)
    ref = oracle_items(sky, items, x)
    off = sky.param_offsets()
    worst_f = worst_g = worst_c = 0.0
    for b, (fo, go, co, so) in ref.items():
        assert st[b] == so, (b, st[b], so)
        ef = abs(f[b] - fo) / abs(fo)
        gb = g[off[b]:off[b + 1]]
        eg = np.max(np.abs(gb - go)) / max(np.max(np.abs(go)), 1e-300)
        worst_f, worst_g = max(worst_f, ef), max(worst_g, eg)
        assert ef <= TOL_F[precision], (b, f[b], fo, ef)
        assert eg <= TOL_G[precision], (b, eg)
        if check_cluster:
            cb = cf[off[b]:off[b + 1]]
            ec = np.max(np.abs(cb - co)) / abs(fo)
            worst_c = max(worst_c, ec)
            assert ec <= TOL_F[precision], (b, ec)
    return worst_f, worst_g, worst_c
