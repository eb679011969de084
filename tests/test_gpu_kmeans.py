"""GPU K-means patching (cs_kmeans_batch) against the oracle: labels and K_eff bit-exact.

Both sides take every floating-point decision (dot products, ordered member sums, norm,
division) in FP64 with the same operation order and separately rounded operations, so the
labels must agree exactly.
"""

import numpy as np
import pytest
import torch

import skygen
from oracle import oracle

pytestmark = pytest.mark.gpu

cs = pytest.importorskip("paper_2604_08463_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cs.load()


def _log(msg):
    print(msg, flush=True)


def _tasks(n, ks, fsky, seed):
    """Positions, latitude masks and seeded initial draws of a configuration-scan batch."""
    g = np.random.default_rng(seed)
    v = skygen.sky.positions(n, g)
    keeps, inits = [], []
    kmax = max(ks)
    for t, k in enumerate(ks):
        keep = skygen.latitude_mask(v[:, 2], fsky[t])
        nk = int(keep.sum())
        row = np.zeros(kmax, dtype=np.int32)
        if k < nk:
            row[:k] = np.random.default_rng(seed * 1000 + t).choice(nk, size=k, replace=False)
        keeps.append(keep)
        inits.append(row)
    return v, np.stack(keeps), np.stack(inits)


def _oracle(v, keep, k, init, iters):
    idx = np.flatnonzero(keep)
    lab = np.full(v.shape[0], -1, dtype=np.int32)
    sub, keff = oracle.kmeans(v[idx], k, init[:min(k, idx.size)] if k < idx.size else np.zeros(0, np.int32), iters)
    lab[idx] = sub
    return lab, keff


def _run(v, keep, ks, init, iters):
    lab, keff = cs.kmeans_batch(torch.as_tensor(v, device="cuda"), ks, torch.as_tensor(init, device="cuda"),
                                None if keep is None else torch.as_tensor(keep.astype(np.uint8), device="cuda"),
                                iters=iters)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), keff.cpu().numpy()


def test_kmeans_configuration_scan_batch_bit_exact():
    # ragged cluster counts as in the configuration scan, including k = 1 and k above the kept count
    ks = [10, 3000, 1, 500, 1000, 37, 2, 2500, 4000, 250, 64, 1500]
    fsky = [0.4, 0.8, 0.6, 0.5, 0.7, 0.45, 0.55, 0.65, 0.75, 0.8, 0.42, 0.6]
    v, keep, init = _tasks(3072, ks, fsky, seed=7)
    lab, keff = _run(v, keep, ks, init, 20)
    for t, k in enumerate(ks):
        _log(f"task {t}: k={k} kept={int(keep[t].sum())}")
        lo, ko = _oracle(v, keep[t], k, init[t], 20)
        assert keff[t] == ko, (t, keff[t], ko)
        assert np.array_equal(lab[t], lo), (t, int(np.sum(lab[t] != lo)))


def test_kmeans_full_sky_large_k_bit_exact():
    g = np.random.default_rng(8)
    n, k = 49152, 1000
    v = skygen.sky.positions(n, g)
    init = np.random.default_rng(9).choice(n, size=k, replace=False).astype(np.int32)[None]
    lab, keff = _run(v, None, [k], init, 20)
    lo, ko = oracle.kmeans(v, k, init[0], 20)
    assert keff[0] == ko and np.array_equal(lab[0], lo), int(np.sum(lab[0] != lo))


def test_kmeans_bad_init_flags_task_only():
    v, keep, init = _tasks(3072, [20, 20], [0.5, 0.5], seed=10)
    init[1, 3] = 5000  # beyond the kept count
    lab, keff = _run(v, keep, [20, 20], init, 5)
    lo, ko = _oracle(v, keep[0], 20, init[0], 5)
    assert keff[0] == ko and np.array_equal(lab[0], lo)
    assert keff[1] == -1 and np.all(lab[1] == -1)


def test_kmeans_zero_iterations_and_ties():
    g = np.random.default_rng(11)
    v = skygen.sky.positions(300, g)
    v = np.concatenate([v, v[:1]])
    init = np.array([[5, 0, 300]], dtype=np.int32)  # two identical starting centroids
    for iters in (0, 1, 3):
        lab, keff = _run(v, None, [3], init, iters)
        lo, ko = oracle.kmeans(v, 3, init[0], iters)
        assert keff[0] == ko and np.array_equal(lab[0], lo), iters
