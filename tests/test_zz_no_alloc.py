"""Allocation-free K-means entry point against the workspace entry point (GPU)."""

import numpy as np
import pytest
import torch

import skygen

pytestmark = pytest.mark.gpu

cs = pytest.importorskip("paper_2604_08463_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cs.load()


def _tasks(n, ks, seed):
    g = np.random.default_rng(seed)
    v = skygen.sky.positions(n, g)
    fsky = g.uniform(0.4, 0.8, len(ks))
    keep = np.stack([skygen.latitude_mask(v[:, 2], f) for f in fsky])
    init = np.zeros((len(ks), max(ks)), dtype=np.int32)
    for t, k in enumerate(ks):
        nk = int(keep[t].sum())
        if k < nk:
            init[t, :k] = g.choice(nk, size=k, replace=False)
    return (torch.as_tensor(v, device="cuda"), np.asarray(ks, dtype=np.int32), torch.as_tensor(init, device="cuda"),
            torch.as_tensor(keep.astype(np.uint8), device="cuda"))


def test_static_kmeans_matches_workspace_entry_point_on_two_calls():
    # two calls in a row, the second smaller: the array keeps the first call's contents, and the
    # second must not read them
    for n, ks, seed in ((3072, [1000, 37, 2900, 1, 640, 3072, 12] * 30, 1), (1500, [5, 300, 2000, 77], 2)):
        v, k, init, keep = _tasks(n, ks, seed)
        lab_w, keff_w = cs.kmeans_batch(v, k, init, keep)
        lab_s, keff_s = cs.kmeans_batch_static(v, k, init, keep)
        torch.cuda.synchronize()
        assert torch.equal(keff_s, keff_w) and torch.equal(lab_s, lab_w), (n, len(ks))


def test_static_kmeans_rejects_tasks_beyond_its_array():
    v, k, init, keep = _tasks(3072, [3000] * 1400, 3)
    with pytest.raises(cs.CsError) as e:
        cs.kmeans_batch_static(v, k, init, keep)
    assert e.value.status == 3
