"""eprop_simulate_batch_noalloc, through the C ABI: the same results as
eprop_simulate_batch on the same batches, two calls in a row with the second
smaller, and no device allocation through the handle's allocator during the
calls; oversized batches and the schedules that need buffers are refused."""
import numpy as np
import pytest

from paper_2511_21674_amd import eprop as E
from paper_2511_21674_amd import workloads as W
from tests.helpers import small_net, batch_from

pytestmark = pytest.mark.gpu
KEYS = ("w_in", "w_rec", "w_out")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


def _outcome(net, b, r):
    return {"loss": r.loss.copy(), "pred": r.predicted.copy(), "grads": net.grads(),
            "spikes": [net.read(E.EPROP_STATE_SPIKES, i) for i in range(b.n_trials)],
            "events": (r.n_syn_events, r.n_rec_spikes, r.n_flush_updates)}


def _same(a, b, what):
    assert np.array_equal(a["loss"], b["loss"]), (what, "loss")
    assert np.array_equal(a["pred"], b["pred"]), (what, "pred")
    assert a["events"] == b["events"], (what, "counts")
    for k in KEYS:
        assert np.array_equal(a["grads"][k], b["grads"][k]), (what, k)
    for x, y in zip(a["spikes"], b["spikes"]):
        assert np.array_equal(x, y), (what, "spikes")


def _batches(kind):
    if kind == "c2":       # uneven lengths, ALIF, learning window, labels; host memory
        wl = W.c2_evidence(batch_size=4)
        return wl, [wl.make_batch(0, 0, 4), wl.make_batch(1, 0, 2)]
    wl = W.c4_sparse(n_rec=3000, n_steps=300, batch_size=2, n_in=300)   # several tiles, delays, forced spikes
    b1 = W.forced_poisson(wl.make_batch(0, 0, 2), wl.network.n_rec, 10.0, 1.0, seed=3, n_ref=2)
    b2 = wl.make_batch(1, 0, 1)
    return wl, [b1, b2]


@pytest.mark.parametrize("precision,kind", [("fp64", "c2"), ("fp32", "c2"), ("fp32", "c4twin")])
def test_noalloc_equals_simulate_batch(precision, kind):
    """Two training calls with an update between them, the second batch
    smaller (fewer trials, fewer spikes): eprop_simulate_batch_noalloc gives
    bit for bit the losses, predictions, counts, spikes and gradients of
    eprop_simulate_batch (both FP32 and FP64 paths are deterministic), on a
    fresh handle (no HIP graph yet: kernel by kernel) and on a handle whose
    graph an earlier eprop_simulate_batch built; the handle's allocator sees
    no allocation during the no-allocation calls."""
    wl, bs = _batches(kind)
    T = max(int(b.n_steps.max()) for b in bs)
    ntr = max(b.n_trials for b in bs)
    ref = []
    net = E.Network(wl.network, precision, max_trials=ntr, max_steps=T)
    for b in bs:
        ref.append(_outcome(net, b, net.simulate(b)))
        net.apply()
    net.close()
    net = E.Network(wl.network, precision, max_trials=ntr, max_steps=T, torch_alloc=True)
    for i, b in enumerate(bs):
        before = sorted(net.allocator.blocks)
        got = _outcome(net, b, net.simulate(b, noalloc=True))
        assert sorted(net.allocator.blocks) == before, "the no-allocation call allocated"
        _same(got, ref[i], f"fresh handle, call {i}")
        net.apply()
    net.close()
    net = E.Network(wl.network, precision, max_trials=ntr, max_steps=T, torch_alloc=True)
    net.simulate(bs[0])          # builds the graph and the staging buffers
    net.apply()
    before = sorted(net.allocator.blocks)
    got = _outcome(net, bs[1], net.simulate(bs[1], noalloc=True))
    assert sorted(net.allocator.blocks) == before
    _same(got, ref[1], "handle with a graph")
    net.close()


def test_noalloc_refuses_what_needs_memory():
    """Host arrays beyond the static staging array (here a 64-readout target
    of 9 trials x 16000 steps, 73.7 MB) are refused with CAPACITY before any
    device work, the online and time-driven schedules with UNSUPPORTED; the
    handle stays usable."""
    K, T, B = 64, 16000, 9
    wnet = small_net(1, 2, K, [(0, 0, 0.5, 1)], [(0, 1, 0.5, 1)], w_out=np.full((K, 2), 0.1), fb=np.full((2, K), 0.1))
    net = E.Network(wnet, "fp32", max_trials=B, max_steps=T)
    big = batch_from(T, [(5, 0)], K, target=np.zeros((T, K)))
    big.n_steps = np.full(B, T, np.uint32)
    big.in_ptr = np.array([0] + [1] * B, np.uint64)
    big.target = np.zeros((B, T, K))
    big.label = np.zeros(B, np.uint32)
    assert 8 * B * T * K > E.EPROP_NOALLOC_SCRATCH_BYTES
    with pytest.raises(E.EpropError) as ei:
        net.simulate(big, noalloc=True)
    assert ei.value.status == E.EPROP_ERR_CAPACITY
    small = batch_from(50, [(5, 0)], K, target=np.zeros((50, K)))
    for kw in (dict(time_driven=True), dict(online=True)):
        with pytest.raises(E.EpropError) as ei:
            net.simulate(small, noalloc=True, **kw)
        assert ei.value.status == E.EPROP_ERR_UNSUPPORTED
    r = net.simulate(small, noalloc=True)
    assert np.isfinite(r.loss).all() and r.n_syn_events == 1
    net.close()
