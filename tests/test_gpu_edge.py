"""Edge cases of the HIP path against the oracle: an item whose pixels are all excluded, a
single-pixel sky, fewer bands than components (every pixel degenerate), one cluster per pixel
(every chunk takes the direct-gather path), and non-finite data or weights (data faults set status
bits, never crash)."""

import numpy as np
import pytest
import torch

import skygen
from oracle import oracle
from tests._parity import compare, gpu_eval

pytestmark = pytest.mark.gpu

cs = pytest.importorskip("paper_2604_08463_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cs.load()


def _log(msg):
    print(msg, flush=True)


def test_item_with_every_pixel_excluded():
    sky = skygen.make_tiny(300, 15, (4, 2, 3), seed=51, nitems=2)
    lab = sky.item_labels(0)
    labels = np.stack([lab, np.full_like(lab, -1)])  # item 1 keeps no pixel
    prob = cs.Problem(sky.freqs, sky.d.cuda(), sky.ninv, torch.as_tensor(labels).cuda(), sky.nclusters,
                      nitems=2, precision="fp64")
    assert prob.item_info(1) == (0, 0)
    x = torch.as_tensor(sky.x_packed(), device="cuda")
    f, g, cf, st = prob.cs_likelihood_grad(x, cluster=True)
    torch.cuda.synchronize()
    off = sky.param_offsets()
    fo, go, co, so = oracle.Problem(sky.freqs, sky.item_d(0), sky.ninv, lab, sky.nclusters[0]).likelihood_grad(sky.x[0])
    assert abs(f[0].item() - fo) <= 1e-12 * abs(fo)
    assert f[1].item() == 0.0 and st[1].item() == 0
    assert torch.all(g[off[1]:off[2]] == 0) and torch.all(cf[off[1]:off[2]] == 0)
    # component maps: nothing included -> NaN maps and NaN variance for that item
    m, v, _ = prob.cs_component_maps(x)
    torch.cuda.synchronize()
    assert torch.all(torch.isnan(m[1])) and torch.isnan(v[1]) and torch.isfinite(v[0])
    # optimiser: a zero projected gradient converges at once, the start point unchanged
    lo, hi = sky.bounds_packed()
    r = prob.cs_optimize_batch(lo, hi, sky.x_packed(), cs.default_opts())
    torch.cuda.synchronize()
    assert r["status"][1].item() & cs.CONVERGED and r["iters"][1].item() == 0
    assert np.allclose(r["x"][off[1]:off[2]].cpu().numpy(), sky.x[1], rtol=0, atol=1e-12)


def test_single_pixel_sky():
    sky = skygen.make_tiny(1, 15, (1, 1, 1), seed=52, nitems=3)
    prob = cs.Problem.from_sky(sky, "fp64")
    compare(sky, prob, "fp64")
    prob32 = cs.Problem.from_sky(sky, "fp32_bulk")
    compare(sky, prob32, "fp32_bulk")


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_fewer_bands_than_components_is_degenerate_everywhere(precision):
    # two bands cannot separate three components: A^T N^-1 A is singular at every pixel (in
    # FP32-bulk the last pivot is then a rounding residue, whose inverse square root comes from
    # the hardware estimate; the relative pivot test must still flag it)
    sky = skygen.make_tiny(100, 2, (1, 1, 1), seed=53)
    prob = cs.Problem.from_sky(sky, precision)
    f, g, _, st = gpu_eval(prob, sky, cluster=False)
    _, _, _, so = oracle.Problem.from_sky(sky).likelihood_grad(sky.x[0])
    assert so & oracle.NOT_PD and st[0] & cs.NOT_PD and np.isnan(f[0])


def test_one_cluster_per_pixel():
    # as many beta_d clusters as pixels: every 64-pixel chunk holds 64 segments
    sky = skygen.make_tiny(200, 15, (200, 3, 2), seed=54, nitems=2)
    assert len(np.unique(sky.item_labels(0)[0])) == 200
    for precision in ("fp64", "fp32_bulk"):
        prob = cs.Problem.from_sky(sky, precision)
        for sh in (0, 1, 2):
            prob.set_schedule(4, 0, 1, sh)
            compare(sky, prob, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_non_finite_data_and_weights_set_status_like_the_oracle(precision):
    # data faults never crash: a NaN or an infinity in d, or a NaN per-pixel weight, makes F NaN
    # and sets the same status bits as the oracle; the other items of the batch are untouched
    sky = skygen.make_tiny(300, 15, (4, 3, 2), seed=61, nitems=3)
    d = sky.d.clone()
    d[1, 0, 5, 17] = float("nan")
    d[2, 1, 3, 40] = float("inf")
    sky.d = d
    prob = cs.Problem.from_sky(sky, precision)
    f, _, _, st = gpu_eval(prob, sky, cluster=False)
    for b in range(3):
        fo, _, _, so = oracle.Problem.from_sky(sky, b).likelihood_grad(sky.x[b])
        _log(f"{precision} band weights item {b}: status {st[b]} / oracle {so}, F {f[b]} / {fo}")
        assert st[b] == so and np.isfinite(f[b]) == np.isfinite(fo)
    assert st[0] == 0 and np.isfinite(f[0]) and st[1] & cs.NONFINITE and st[2] & cs.NONFINITE
    # per-pixel weights with a NaN in item 0
    sky.d = sky.d.clone()
    sky.d[1, 0, 5, 17] = 1.0
    sky.d[2, 1, 3, 40] = 1.0
    wpix = np.repeat(sky.ninv[:, :, None], sky.npix, axis=2)
    wpix = np.stack([wpix] * 3)
    wpix[0, 1, 7, 99] = np.nan
    dt = torch.float64 if precision == "fp64" else torch.float32
    prob2 = cs.Problem(sky.freqs, sky.d.to("cuda", dt), torch.as_tensor(wpix, dtype=dt).cuda(), sky.labels.cuda(),
                       sky.nclusters, nitems=3, precision=precision)
    f2, _, _, st2 = gpu_eval(prob2, sky, cluster=False)
    for b in range(3):
        pr = oracle.Problem(sky.freqs, sky.item_d(b), wpix[b], sky.item_labels(b), sky.nclusters[b])
        fo, _, _, so = pr.likelihood_grad(sky.x[b])
        _log(f"{precision} pixel weights item {b}: status {st2[b]} / oracle {so}, F {f2[b]} / {fo}")
        assert st2[b] == so and np.isfinite(f2[b]) == np.isfinite(fo)
    assert np.isnan(f2[0]) and st2[0] & cs.NOT_PD and st2[1] == 0 and st2[2] == 0
