"""GPU checks of the resumable optimiser (checkpoint / restore of the complete state) and of the
contiguous item chunking (paper Sec. 3.1: batches of a campaign run in chunks, each checkpointed
and resumed)."""

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


def _log(msg):
    print(msg, flush=True)


def _host(r):
    return {k: r[k].cpu().numpy() for k in ("x", "f", "iters", "status", "nevals")}


def _same(a, b):
    for k in ("x", "f", "iters", "status", "nevals"):
        assert np.array_equal(a[k], b[k]), (k, a[k], b[k])


@pytest.mark.parametrize("precision,solver", [("fp32_bulk", cs.SOLVER_LBFGS), ("fp64", cs.SOLVER_LBFGS),
                                              ("fp64", cs.SOLVER_ADATOPK)])
def test_checkpoint_restore_in_fresh_problem_is_bit_identical(precision, solver):
    # an uninterrupted run against one paused every few replays: after each pause the state is
    # copied to the host, the problem is destroyed, and a problem prepared from the same inputs
    # continues from the copy.  FP32-bulk crosses from the FP32 phase into the FP64-accumulation
    # phase on the way.
    sky = skygen.make_config(2, npix=6000, nitems=3, k=(120, 12, 40))
    lo, hi = sky.bounds_packed()
    opts = cs.default_opts(max_iter=300, solver=solver, iters_per_graph=4)
    full = _host(cs.Problem.from_sky(sky, precision).cs_optimize_batch(lo, hi, sky.x_packed(), opts))
    _log(f"{precision} solver {solver}: uninterrupted status {full['status'].tolist()} iters {full['iters'].tolist()}")
    prob = cs.Problem.from_sky(sky, precision)
    st = prob.optimizer_state(opts.m)
    r = prob.cs_optimize_batch(lo, hi, sky.x_packed(), opts, state=st, max_replays=5)
    pauses = 0
    while r["running"] > 0:
        pauses += 1
        assert np.all((r["status"].cpu().numpy() & cs.RUNNING > 0) == (r["status"].cpu().numpy() & 0x1F == 0))
        saved = st.to_host()
        del prob, st
        torch.cuda.empty_cache()
        prob = cs.Problem.from_sky(sky, precision)
        st = cs.OptState.from_host(saved, prob.device)
        r = prob.cs_optimize_batch(lo, hi, None, opts, state=st, resume=True, max_replays=5 + pauses % 3)
    _log(f"  {pauses} pauses")
    assert pauses >= 3
    _same(_host(r), full)


def test_resume_rejects_foreign_state():
    sky = skygen.make_config(2, npix=3000, nitems=2, k=(40, 6, 12))
    lo, hi = sky.bounds_packed()
    prob = cs.Problem.from_sky(sky, "fp64")
    st = prob.optimizer_state(10)
    prob.cs_optimize_batch(lo, hi, sky.x_packed(), cs.default_opts(), state=st, max_replays=1)
    with pytest.raises(cs.CsError) as e:  # the state was written with m = 10
        prob.cs_optimize_batch(lo, hi, None, cs.default_opts(m=5), state=st, resume=True)
    assert e.value.status == 6
    st2 = prob.optimizer_state(10)
    st2.view.zero_()
    with pytest.raises(cs.CsError):  # no state at all
        prob.cs_optimize_batch(lo, hi, None, cs.default_opts(), state=st2, resume=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_item_chunks_match_whole_batch_bit_for_bit(precision):
    # per-item results do not depend on the other items of a batch, so every chunk of the
    # contiguous chunking reproduces its items of the whole batch exactly: evaluation and optimiser
    sky = skygen.make_config(4, nitems=7, kmax4=(200, 30, 60))
    lo, hi = sky.bounds_packed()
    whole = cs.Problem.from_sky(sky, precision)
    x = torch.as_tensor(sky.x_packed(), device="cuda")
    f, g, _, st = whole.cs_likelihood_grad(x)
    opts = cs.default_opts(max_iter=200)
    rw = _host(whole.cs_optimize_batch(lo, hi, sky.x_packed(), opts))
    off = sky.param_offsets()
    seen = 0
    for rank in range(3):
        sub = whole.chunk(rank, 3)
        b0, b1 = cs.item_range(rank, 3, sky.nitems)
        assert sub.nitems == b1 - b0 and sub.item_begin == b0
        xs = x[off[b0]:off[b1]].contiguous()
        fs, gs, _, sts = sub.cs_likelihood_grad(xs)
        assert torch.equal(fs, f[b0:b1]) and torch.equal(gs, g[off[b0]:off[b1]]) and torch.equal(sts, st[b0:b1])
        rs = _host(sub.cs_optimize_batch(lo[off[b0]:off[b1]], hi[off[b0]:off[b1]], xs, opts))
        for k in ("f", "iters", "status", "nevals"):
            assert np.array_equal(rs[k], rw[k][b0:b1]), k
        assert np.array_equal(rs["x"], rw["x"][off[b0]:off[b1]])
        seen += sub.nitems
    assert seen == sky.nitems
