"""GPU parity of the component maps and the CMB map variance (cs_component_maps, and its
processing-order variant cs_component_maps_sorted) with the oracle.

The device forms the maps in FP64 from the data as stored (FP32 for the FP32 precisions); the
oracle is fed exactly those stored values, so every precision is held to the FP64 bar.  The
device solves with a Cholesky factorisation and the oracle with pivoted LU: for A^T N^-1 A of
condition number <= ~2e3 (measured on these workloads) the two agree to ~1e-14 of the pixel's
largest amplitude, so 1e-11 per pixel leaves two decades of headroom.  The variance is the
Chan-Golub-LeVeque pairwise combination of chunk moments on the device against a two-pass
compensated sum in the oracle: 1e-12 relative.
"""

import ctypes as C

import numpy as np
import pytest
import torch

import skygen
from oracle import oracle

pytestmark = pytest.mark.gpu

cs = pytest.importorskip("paper_2604_08463_amd")

TOL_MAP = 1e-11
TOL_VAR = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cs.load()


def _log(msg):
    print(msg, flush=True)


def _check_maps(sky, prob, x=None, items=None):
    xs = sky.x if x is None else x
    m, v, st = prob.cs_component_maps(torch.as_tensor(np.concatenate(xs), device=prob.device))
    torch.cuda.synchronize()
    m, v, st = m.cpu().numpy(), v.cpu().numpy(), st.cpu().numpy()
    worst_m = worst_v = 0.0
    for b in (range(sky.nitems) if items is None else items):
        so, vo, sto = oracle.Problem.from_sky(sky, b).component_maps(xs[b])
        assert st[b] == sto, (b, st[b], sto)
        nan_o = np.isnan(so)
        assert np.array_equal(np.isnan(m[b]), nan_o), b
        scale = np.nanmax(np.abs(so), axis=1, keepdims=True)  # [2][1][P]: per Stokes and pixel
        err = np.where(nan_o, 0.0, np.abs(m[b] - so) / np.where(nan_o, 1.0, scale))
        worst_m = max(worst_m, float(err.max()))
        ev = abs(v[b] - vo) / abs(vo)
        worst_v = max(worst_v, ev)
        assert err.max() <= TOL_MAP, (b, err.max())
        assert ev <= TOL_VAR, (b, v[b], vo)
    _log(f"maps worst per-pixel rel {worst_m:.3e}, variance rel {worst_v:.3e}")
    return m, v, st


def test_maps_fp64_tiny_masked_batched():
    sky = skygen.make_tiny(700, 15, (7, 3, 5), seed=21, nitems=3, mask_frac=0.1)
    _check_maps(sky, cs.Problem.from_sky(sky, "fp64"))


def test_maps_fp64_workload1():
    sky = skygen.make_config(1, device="cuda")
    _check_maps(sky, cs.Problem.from_sky(sky, "fp64"))


@pytest.mark.parametrize("precision", ["fp32_bulk", "fp32_store"])
def test_maps_fp32_storage_against_oracle_on_stored_values(precision):
    sky = skygen.make_config(2, device="cuda", nitems=3)
    prob = cs.Problem.from_sky(sky, precision)
    sky.d = sky.d.to(torch.float32).to(torch.float64)  # what the library stored
    _check_maps(sky, prob)


def test_maps_separate_stokes_and_pixel_weights():
    sky = skygen.make_tiny(400, 15, (4, 3, 2), seed=42, nitems=2, mask_frac=0.05)
    sky.ninv = sky.ninv.copy()
    sky.ninv[1] *= 1.7
    _check_maps(sky, cs.Problem.from_sky(sky, "fp64"))
    g = np.random.default_rng(5)
    wpix = sky.ninv[:, :, None] * g.uniform(0.5, 2.0, (2, sky.nfreq, sky.npix))
    prob = cs.Problem(sky.freqs, sky.d.cuda(), torch.as_tensor(wpix[None]).cuda(), sky.labels.cuda(),
                      sky.nclusters, nitems=sky.nitems, precision="fp64")
    m, v, st = prob.cs_component_maps(torch.as_tensor(sky.x_packed(), device="cuda"))
    torch.cuda.synchronize()
    for b in range(sky.nitems):
        so, vo, sto = oracle.Problem(sky.freqs, sky.item_d(b), wpix, sky.item_labels(b),
                                     sky.nclusters[b]).component_maps(sky.x[b])
        mb = m[b].cpu().numpy()
        assert np.array_equal(np.isnan(mb), np.isnan(so))
        scale = np.nanmax(np.abs(so), axis=1, keepdims=True)
        assert np.nanmax(np.abs(mb - so) / scale) <= TOL_MAP
        assert abs(v[b].item() - vo) <= TOL_VAR * abs(vo)


def test_maps_not_pd_pixel_is_nan_and_flagged():
    sky = skygen.make_tiny(200, 15, (2, 2, 2), seed=43, nitems=2)
    wpix = np.repeat(sky.ninv[:, :, None], sky.npix, axis=2)
    wpix = np.stack([wpix, wpix])
    wpix[1, :, :, 17] = 0.0
    prob = cs.Problem(sky.freqs, sky.d.cuda(), torch.as_tensor(wpix).cuda(), sky.labels.cuda(), sky.nclusters,
                      nitems=2, precision="fp64")
    m, v, st = prob.cs_component_maps(torch.as_tensor(sky.x_packed(), device="cuda"))
    torch.cuda.synchronize()
    m, v, st = m.cpu().numpy(), v.cpu().numpy(), st.cpu().numpy()
    assert st[0] == 0 and np.isfinite(v[0]) and np.all(np.isfinite(m[0]))
    assert st[1] & cs.NOT_PD and np.isnan(v[1])
    assert np.all(np.isnan(m[1, :, :, 17]))
    assert np.all(np.isfinite(np.delete(m[1], 17, axis=2)))


def test_maps_variance_only_and_item_stride():
    sky = skygen.make_tiny(300, 15, (3, 2, 2), seed=44, nitems=2, mask_frac=0.2)
    prob = cs.Problem.from_sky(sky, "fp64")
    x = torch.as_tensor(sky.x_packed(), device="cuda")
    _, v0, _ = prob.cs_component_maps(x, maps=False)
    m1, v1, _ = prob.cs_component_maps(x)
    # a caller-chosen item stride: the gap between the item blocks is left untouched
    P = sky.npix
    stride = 6 * P + 37
    buf = torch.full((sky.nitems * stride,), 7.0, dtype=torch.float64, device="cuda")
    var = torch.empty(sky.nitems, dtype=torch.float64, device="cuda")
    st = torch.empty(sky.nitems, dtype=torch.int32, device="cuda")
    rc = cs.load().cs_component_maps(prob._h, C.c_void_p(x.data_ptr()), C.c_void_p(buf.data_ptr()), stride,
                                     C.c_void_p(var.data_ptr()), C.c_void_p(st.data_ptr()),
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()
    for b in range(sky.nitems):
        blk = buf[b * stride:b * stride + 6 * P].view(2, 3, P)
        assert torch.equal(torch.nan_to_num(blk, nan=-1.0), torch.nan_to_num(m1[b], nan=-1.0))
        assert torch.all(buf[b * stride + 6 * P:(b + 1) * stride] == 7.0)
    assert torch.equal(v0, v1) and torch.equal(v1, var)
    # bad stride is rejected on the host
    rc = cs.load().cs_component_maps(prob._h, C.c_void_p(x.data_ptr()), C.c_void_p(buf.data_ptr()), 6 * P - 1,
                                     None, None, None)
    assert rc == 1


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_maps_leave_evaluations_unchanged(precision):
    # the maps reuse the evaluation's scratch (tables, partials): evaluations before and after a
    # maps call must agree bit for bit
    sky = skygen.make_config(2, device="cuda", nitems=2)
    prob = cs.Problem.from_sky(sky, precision)
    x = torch.as_tensor(sky.x_packed(), device="cuda")
    f0, g0, c0, s0 = [t.clone() for t in prob.cs_likelihood_grad(x, cluster=True)]
    prob.cs_component_maps(x)
    f1, g1, c1, s1 = prob.cs_likelihood_grad(x, cluster=True)
    torch.cuda.synchronize()
    assert torch.equal(f0, f1) and torch.equal(g0, g1) and torch.equal(c0, c1) and torch.equal(s0, s1)


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_maps_in_processing_order_match_pixel_order(precision):
    # ragged items with their own labellings and masks: the processing-order maps are the
    # pixel-order maps permuted by the exported order, bit for bit; the slots past the included
    # pixels hold NaN, as do the excluded pixels in pixel order
    sky = skygen.make_config(4, nitems=3, kmax4=(200, 30, 60))
    prob = cs.Problem.from_sky(sky, precision)
    if precision == "fp64":
        _check_maps(sky, prob)
    x = torch.as_tensor(sky.x_packed(), device="cuda")
    m, v, st = prob.cs_component_maps(x)
    ms, vs, sts = prob.cs_component_maps(x, sorted_order=True)
    torch.cuda.synchronize()
    assert torch.equal(v, vs) and torch.equal(st, sts)
    for b in range(sky.nitems):
        order = prob.pixel_order(b).long()
        n = order.numel()
        assert n == int(np.sum(sky.item_labels(b)[0] >= 0))
        assert torch.equal(ms[b][:, :, :n], m[b][:, :, order])
        assert torch.all(torch.isnan(ms[b][:, :, n:]))
        excl = torch.ones(sky.npix, dtype=torch.bool, device="cuda")
        excl[order] = False
        assert torch.all(torch.isnan(m[b][:, :, excl])) and not torch.any(torch.isnan(m[b][:, :, ~excl]))
