"""Parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances (relative, normwise and per entry with a floor, see
tests/helpers.rel_close):
  * FP64: spike trains identical, gradients and weights within 1e-10;
  * FP32 with teacher-forced spike trains: per-iteration weight update
    within 1e-4 normwise, and per entry for entries above 1% of the largest
    (smaller entries sit in cancellations that FP32 weights, rounded after
    each update, shift by more than their own size allows);
  * FP32 free running: mean loss over the last iterations within 2% of the
    oracle's, averaged over seeds (single runs diverge by spike flips).
"""
import numpy as np
import pytest

from paper_2511_21674_amd import eprop as E
from paper_2511_21674_amd import workloads as W
import oracle as O
from tests.helpers import rel_close, small_net, batch_from, prediction_case

pytestmark = pytest.mark.gpu
KEYS = ("w_in", "w_rec", "w_out")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


def log(*a):
    print(*a, flush=True)


def gpu_train(wl, precision, iterations, bs, delivery="auto", forced_rate=None, device=False,
              max_steps=None, record=True):
    T = max_steps or max(int(wl.make_batch(it, 0, bs).n_steps.max()) for it in range(iterations))
    net = E.Network(wl.network, precision, max_trials=bs, max_steps=T, delivery=delivery)
    hist = {"loss": [], "pred": [], "spikes": [], "grads": [], "weights": [], "dw": []}
    w_prev = net.weights()
    for it in range(iterations):
        b = wl.make_batch(it, 0, bs)
        if forced_rate:
            b = W.forced_poisson(b, wl.network.n_rec, forced_rate, wl.network.params.dt, seed=99,
                                 iteration=it, n_ref=2)
        r = net.simulate(b, train=True, device=device)
        hist["loss"].append(r.loss.copy())
        hist["pred"].append(r.predicted.copy())
        if record:
            hist["spikes"].append([net.spikes(i, int(b.n_steps[i])) for i in range(b.n_trials)])
            hist["grads"].append(net.grads())
        net.apply()
        w = net.weights()
        hist["weights"].append(w)
        hist["dw"].append({k: w[k] - w_prev[k] for k in KEYS})
        w_prev = w
    net.close()
    return hist


def oracle_train(wl, iterations, bs, forced_rate=None, grad_mode=2):
    on = O.OracleNet(wl.network)
    hist = {"loss": [], "pred": [], "spikes": [], "grads": [], "weights": [], "dw": []}
    w_prev = {k: getattr(on, k).copy() for k in KEYS}
    for it in range(iterations):
        b = wl.make_batch(it, 0, bs)
        if forced_rate:
            b = W.forced_poisson(b, wl.network.n_rec, forced_rate, wl.network.params.dt, seed=99,
                                 iteration=it, n_ref=2)
        g = O.zero_grads(on)
        losses, spikes, preds = [], [], []
        for i in range(b.n_trials):
            r = O.run_trial(on, b, i, grad_mode, g, trace=True)
            losses.append(r.loss)
            spikes.append(r.trace["z"])
            preds.append(r.pred)
        hist["loss"].append(np.array(losses))
        hist["pred"].append(np.array(preds, np.uint32))
        hist["spikes"].append(spikes)
        hist["grads"].append({k: v.copy() for k, v in g.items()})
        O.apply(on, g, b.n_trials)
        w = {k: getattr(on, k).copy() for k in KEYS}
        hist["weights"].append(w)
        hist["dw"].append({k: w[k] - w_prev[k] for k in KEYS})
        w_prev = w
    return hist


def assert_fp64_parity(gh, oh, name):
    for it in range(len(oh["loss"])):
        for i, (zg, zo) in enumerate(zip(gh["spikes"][it], oh["spikes"][it])):
            assert np.array_equal(zg, zo), f"{name}: iteration {it} trial {i} spike trains differ"
        ok, e, _ = rel_close(gh["loss"][it], oh["loss"][it], 1e-12)
        assert ok, (name, it, "loss", e)
        # the predicted class (arg max of the window-summed softmax or readout)
        assert np.array_equal(gh["pred"][it], oh["pred"][it]), (name, it, gh["pred"][it], oh["pred"][it])
        for k in KEYS:
            ok, e, ent = rel_close(gh["grads"][it][k], oh["grads"][it][k], 1e-10)
            assert ok, (name, it, "grad", k, e, ent)
            ok, e, ent = rel_close(gh["weights"][it][k], oh["weights"][it][k], 1e-10)
            assert ok, (name, it, "weights", k, e, ent)
        log(f"{name} it {it}: spikes identical, max grad err "
            f"{max(rel_close(gh['grads'][it][k], oh['grads'][it][k], 1)[1] for k in KEYS):.2e}")


# ----------------------------------------------------------------- FP64: exact reproduction

@pytest.mark.parametrize("loss,surrogate", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_fp64_tiny_exact(loss, surrogate):
    wl = W.tiny(loss=loss, surrogate=surrogate)
    gh = gpu_train(wl, "fp64", 3, 2)
    oh = oracle_train(wl, 3, 2)
    assert_fp64_parity(gh, oh, f"tiny loss={loss} sg={surrogate}")


def test_fp64_c1_pattern_generation():
    """Pattern generation as configured (GD 1e-3, 10 iterations, batch 1)."""
    wl = W.c1_pattern()
    gh = gpu_train(wl, "fp64", 10, 1)
    oh = oracle_train(wl, 10, 1)
    assert_fp64_parity(gh, oh, "c1")


def test_fp64_c2_evidence_uneven_adam():
    """Evidence accumulation: LIF + ALIF, softmax, learning window, Adam,
    four trials of uneven lengths per batch."""
    wl = W.c2_evidence(batch_size=4)
    assert len(set(wl.make_batch(0, 0, 4).n_steps.tolist())) > 1
    gh = gpu_train(wl, "fp64", 2, 4)
    oh = oracle_train(wl, 2, 4)
    assert_fp64_parity(gh, oh, "c2")


def test_fp64_c3_events():
    wl = W.c3_events(batch_size=4)
    gh = gpu_train(wl, "fp64", 2, 4)
    oh = oracle_train(wl, 2, 4)
    assert_fp64_parity(gh, oh, "c3")


@pytest.mark.parametrize("delivery", ["gather", "scatter"])
def test_fp64_sparse_twin_with_delays(delivery):
    """Twin of the 1e5-neuron network (fixed in-degree 1000, delays 1..5:
    the delay ring wraps around); scatter adds in a free order, so spikes are
    compared exactly only where they are reproducible (gather)."""
    wl = W.c4_sparse(n_rec=2000, n_steps=200, batch_size=2, n_in=300)
    gh = gpu_train(wl, "fp64", 2, 2, delivery=delivery)
    oh = oracle_train(wl, 2, 2)
    if delivery == "gather":
        assert_fp64_parity(gh, oh, "c4twin gather")
    else:
        for it in range(2):
            for k in KEYS:
                ok, e, ent = rel_close(gh["weights"][it][k], oh["weights"][it][k], 1e-10)
                assert ok, ("scatter weights", it, k, e, ent)


def test_fp64_deterministic_and_batch_invariant():
    """Two runs are bitwise equal; a trial run alone equals the same trial
    inside a batch (parallel copies equal sequential samples)."""
    wl = W.c2_evidence(batch_size=4)
    b = wl.make_batch(0, 0, 4)
    T = int(b.n_steps.max())
    runs = []
    for _ in range(2):
        net = E.Network(wl.network, "fp64", max_trials=4, max_steps=T)
        r = net.simulate(b)
        runs.append((r.loss.copy(), net.grads(), [net.spikes(i, int(b.n_steps[i])) for i in range(4)]))
        net.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    for k in KEYS:
        assert np.array_equal(runs[0][1][k], runs[1][1][k])
    net = E.Network(wl.network, "fp64", max_trials=4, max_steps=T)
    gsum = {k: 0.0 for k in KEYS}
    for i in range(4):
        r = net.simulate(b.trial(i))
        assert r.loss[0] == runs[0][0][i]
        assert np.array_equal(net.spikes(0, int(b.n_steps[i])), runs[0][2][i])
    g = net.grads()
    for k in KEYS:
        assert rel_close(g[k], runs[0][1][k], 1e-13)[0]
    net.close()


def test_device_memory_batch_equals_host_batch():
    wl = W.c3_events(batch_size=3)
    b = W.forced_poisson(wl.make_batch(0, 0, 3), wl.network.n_rec, 15.0, 1.0, seed=5, n_ref=2)
    out = []
    for device in (False, True):
        net = E.Network(wl.network, "fp64", max_trials=3, max_steps=300)
        r = net.simulate(b, device=device)
        out.append((r.loss.copy(), net.grads()))
        net.close()
    assert np.array_equal(out[0][0], out[1][0])
    for k in KEYS:
        assert np.array_equal(out[0][1][k], out[1][1][k])


@pytest.mark.parametrize("precision,delivery", [("fp64", "gather"), ("fp32", "scatter")])
@pytest.mark.parametrize("loss", [1, 2])
def test_class_prediction_constructed_case(precision, delivery, loss):
    """The predicted class of the constructed trials whose answer is fixed by
    construction (tests.helpers.prediction_case: a readout dominating before
    the learning window, a tall short peak and a flat signal inside it, a
    silent network, an exact tie): the GPU's prediction equals the known
    class and the oracle's, and the loss matches the oracle's."""
    for variant in ("main", "silent", "tie"):
        net_w, b, expected = prediction_case(loss, variant)
        net = E.Network(net_w, precision, max_trials=1, max_steps=int(b.n_steps[0]), delivery=delivery)
        r = net.simulate(b, train=True)
        net.close()
        ro = O.run_trial(O.OracleNet(net_w), b, 0, 0)
        log(f"{precision} loss {loss} {variant}: predicted {int(r.predicted[0])}, expected {expected}")
        assert int(r.predicted[0]) == expected == ro.pred, (variant, int(r.predicted[0]), expected, ro.pred)
        assert rel_close(r.loss, [ro.loss], 1e-12 if precision == "fp64" else 1e-5)[0]


# ----------------------------------------------------------------- FP32

@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4twin", "tiny"])
def test_fp32_teacher_forced_weight_updates(name):
    """FP32 with the oracle's (teacher-forced) spike trains: each
    iteration's computed update (the batch-summed gradient that the
    optimiser receives) within 1e-4 relative of the FP64 oracle's; the stored
    FP32 weights within that plus FP32 rounding of the weights themselves."""
    if name == "c1":
        # as configured (GD 1e-3) the loss grows to 1e9 by the third iteration;
        # the check runs in the trained regime instead
        wl, bs, it = W.c1_pattern(), 1, 3
        wl.network.params.eta = 2e-5
    elif name == "c2":
        wl, bs, it = W.c2_evidence(batch_size=4), 4, 2
    elif name == "c3":
        wl, bs, it = W.c3_events(batch_size=4), 4, 2
    elif name == "c4twin":
        wl, bs, it = W.c4_sparse(n_rec=2000, n_steps=200, batch_size=2, n_in=300), 2, 2
    else:
        wl, bs, it = W.tiny(), 2, 3
    gh = gpu_train(wl, "fp32", it, bs, forced_rate=20.0)
    oh = oracle_train(wl, it, bs, forced_rate=20.0)
    u = 2.0 ** -24
    bound = {k: 0.0 for k in KEYS}
    for i in range(it):
        for k in KEYS:
            ok, e, ent = rel_close(gh["grads"][i][k], oh["grads"][i][k], 1e-4, floor_frac=1e-2)
            log(f"{name} it {i} update {k}: normwise {e:.2e} worst entry {ent:.2e}")
            assert ok, (name, i, k, e, ent)
            # stored weights: this and earlier updates' tolerance plus FP32 rounding of w
            dw_o = np.abs(oh["dw"][i][k])
            bound[k] = bound[k] + 1e-4 * np.maximum(dw_o, 1e-2 * dw_o.max()) + 4 * u * np.abs(oh["weights"][i][k])
            assert np.all(np.abs(gh["weights"][i][k] - oh["weights"][i][k]) <= bound[k]), (name, i, k)
        assert rel_close(gh["loss"][i], oh["loss"][i], 1e-4)[0]


def test_fp32_free_running_final_loss():
    """Trained pattern-generation runs (learning rate 1e-6, where gradient
    descent on the summed loss converges): FP32 final loss within 2% of the
    FP64 oracle's, as the mean over the last 20 of 40 iterations and over 5
    seeds (single runs decorrelate through spike flips)."""
    g_final, o_final, first = [], [], []
    for s in range(5):
        wl = W.c1_pattern(seed=W.SEED_BASE + 100 + s)
        wl.network.params.eta = 1e-6
        gh = gpu_train(wl, "fp32", 40, 1, record=False)
        oh = oracle_train(wl, 40, 1)
        g_final.append(np.mean([l.mean() for l in gh["loss"][20:]]))
        o_final.append(np.mean([l.mean() for l in oh["loss"][20:]]))
        first.append(oh["loss"][0][0])
        log(f"seed {s}: first loss {first[-1]:.1f}, final gpu {g_final[-1]:.2f} oracle {o_final[-1]:.2f}")
        assert o_final[-1] < first[-1]          # training reduced the loss
    assert np.mean(o_final) < 0.8 * np.mean(first)
    rel = abs(np.mean(g_final) - np.mean(o_final)) / np.mean(o_final)
    log(f"mean final loss gpu {np.mean(g_final):.3f} oracle {np.mean(o_final):.3f} rel {rel:.3e}")
    assert rel < 0.02


# ----------------------------------------------------------------- edge cases

def test_silent_network_and_single_step_trial():
    """No input spikes: no recurrent spikes, all gradients of plastic synapses
    exactly zero, loss 1/2 sum y*^2; a one-step trial runs."""
    net_w = small_net(3, 4, 2, [(0, 1, 0.5, 1), (2, 3, 0.1, 1)], [(1, 2, 0.3, 1), (3, 0, -0.2, 2)])
    tg = np.random.default_rng(1).normal(size=(50, 2))
    b = batch_from(50, [], 2, target=tg)
    net = E.Network(net_w, "fp32", max_trials=1, max_steps=50)
    r = net.simulate(b)
    assert r.n_rec_spikes == 0 and r.n_syn_events == 0
    assert r.loss[0] == pytest.approx(0.5 * (tg ** 2).sum(), rel=1e-12)
    g = net.grads()
    assert np.all(g["w_in"] == 0) and np.all(g["w_rec"] == 0) and np.all(g["w_out"] == 0)
    # one-step trial: the input spike emitted at step 0 reaches neuron 1 at step 1
    # (one event, below threshold), nothing else arrives within the trial
    r = net.simulate(batch_from(1, [(0, 0)], 2, target=tg[:1]))
    assert r.n_rec_spikes == 0 and r.n_syn_events == 1
    assert net.read(E.EPROP_STATE_V, 0)[1] == pytest.approx(0.5, rel=1e-7)
    # a strong input makes neuron 1 spike at step 1; its spike would arrive at step 2 > T
    net_w.in_rec.w[:] = 5.0
    net2 = E.Network(net_w, "fp32", max_trials=1, max_steps=50)
    r = net2.simulate(batch_from(1, [(0, 0)], 2, target=tg[:1]))
    assert r.n_rec_spikes == 1 and r.n_syn_events == 1
    net2.close()
    net.close()


def test_errors_are_reported():
    wl = W.tiny()
    b = wl.make_batch(0, 0, 2)
    net = E.Network(wl.network, "fp32", max_trials=2, max_steps=100)
    with pytest.raises(E.EpropError) as ei:
        net.simulate(b)                               # 200-step trials > max_steps
    assert ei.value.status == E.EPROP_ERR_CAPACITY
    with pytest.raises(E.EpropError) as ei:
        net.apply()                                   # nothing trained yet
    assert ei.value.status == E.EPROP_ERR_STATE
    with pytest.raises(E.EpropError) as ei:
        net.read(E.EPROP_STATE_PSI, 0)                # no batch yet
    assert ei.value.status == E.EPROP_ERR_STATE
    net.close()
    net = E.Network(wl.network, "fp32", max_trials=2, max_steps=200)
    bad = wl.make_batch(0, 0, 2)
    bad.in_step = bad.in_step[::-1].copy()            # unsorted (host memory: host check)
    with pytest.raises(E.EpropError) as ei:
        net.simulate(bad)
    assert ei.value.status == E.EPROP_ERR_INVALID_ARGUMENT
    bad = wl.make_batch(0, 0, 2)
    bad.in_src = bad.in_src.copy()
    bad.in_src[3] = 1000                              # out of range (device memory: kernel check)
    with pytest.raises(E.EpropError) as ei:
        net.simulate(bad, device=True)
    assert ei.value.status == E.EPROP_ERR_INVALID_ARGUMENT
    r = net.simulate(wl.make_batch(0, 0, 2))          # the handle is still usable
    assert np.all(np.isfinite(r.loss))
    net.apply()
    assert net.read(E.EPROP_STATE_ADAM_STEP)[0] == 1
    net.close()


# ----------------------------------------------------------------- full size, sampled

def test_full_size_sparse_network_sampled():
    """1e5 neurons, in-degree 1000, delays 1..5, 4 trials per batch, FP32
    scatter (the benchmark's launch configuration), teacher-forced at 10 Hz:
    the gradients of every incoming synapse of 24 sampled neurons, summed
    over the 4 trials, within 1e-4 of the oracle's per-neuron evaluation, and
    the per-trial losses within 1e-6."""
    wl = W.c4_sparse()
    b = W.forced_poisson(wl.make_batch(0, 0, 4), wl.network.n_rec, 10.0, 1.0, seed=7, n_ref=2)
    net = E.Network(wl.network, "fp32", max_trials=4, max_steps=1000)
    r = net.simulate(b, train=True)
    g = net.grads()
    net.close()
    log(f"gpu done: {r.n_rec_spikes} spikes, {r.n_syn_events} events")
    on = O.OracleNet(wl.network)
    rng = np.random.default_rng(0)
    targets = np.sort(rng.choice(wl.network.n_rec, 24, replace=False))
    gi = np.zeros_like(on.w_in)
    gr = np.zeros_like(on.w_rec)
    for i in range(4):
        loss, psi, a, c = O.forced_sampled(on, b, i, targets)
        assert abs(r.loss[i] - loss) <= 1e-6 * abs(loss), (i, r.loss[i], loss)
        mi, mr = ~np.isnan(a), ~np.isnan(c)
        gi[mi] += a[mi]
        gr[mr] += c[mr]
    for name, gg, ref, m in (("w_in", g["w_in"], gi, mi), ("w_rec", g["w_rec"], gr, mr)):
        ok, e, ent = rel_close(gg[m], ref[m], 1e-4, floor_frac=1e-2)
        log(f"full size {name}: {m.sum()} synapses, normwise {e:.2e} worst {ent:.2e}")
        assert ok, (name, e, ent)


# ----------------------------------------------------------------- recordings, counters, allocator

@pytest.mark.parametrize("loss", [0, 1])
def test_recorded_traces_match_oracle(loss):
    """FP64: the recorded psi, readout y, error E, learning signal L
    (eq. final-gradient) and final membrane potential of every trial equal
    the oracle's recordings."""
    wl = W.tiny(loss=loss)
    b = wl.make_batch(0, 0, 2)
    net = E.Network(wl.network, "fp64", max_trials=2, max_steps=int(b.n_steps.max()))
    net.simulate(b)
    on = O.OracleNet(wl.network)
    for i in range(2):
        T = int(b.n_steps[i])
        tr = O.run_trial(on, b, i, 0, trace=True).trace
        J, K = wl.network.n_rec, wl.network.n_out
        for what, ref, shape in ((E.EPROP_STATE_PSI, tr["psi"], (T, J)), (E.EPROP_STATE_Y, tr["y"], (T, K)),
                                 (E.EPROP_STATE_ERR, tr["err"], (T, K)), (E.EPROP_STATE_L, tr["learn"], (T, J))):
            got = net.read(what, i).reshape(shape)
            ok, e, ent = rel_close(got, ref, 1e-12)
            assert ok, (what, i, e, ent)
        assert rel_close(net.read(E.EPROP_STATE_V, i), tr["v"][T - 1], 1e-12)[0]
    net.close()


def _counts_from_spikes(wnet, b, spikes):
    """Synaptic events and trial-end evaluations counted on the host from the
    recorded spike trains and the graph: every delivery that arrives within
    its trial, and every (synapse, trial) pair with at least one."""
    events, flushes = 0, 0
    for i in range(b.n_trials):
        T = int(b.n_steps[i])
        lo, hi = int(b.in_ptr[i]), int(b.in_ptr[i + 1])
        src_times = [(wnet.in_rec, b.in_src[lo:hi], b.in_step[lo:hi]),
                     (wnet.rec_rec, spikes[i][:, 1], spikes[i][:, 0])]
        for proj, srcs, steps in src_times:
            rp = proj.row_ptr.astype(np.int64)
            per_src = {}
            for s, t in zip(srcs.tolist(), steps.tolist()):
                per_src.setdefault(s, []).append(t)
            for s, ts in per_src.items():
                d = proj.delay[rp[s]:rp[s + 1]].astype(np.int64)
                ts = np.asarray(ts, np.int64)
                arr = ts[None, :] + d[:, None] <= T
                events += int(arr.sum())
                flushes += int(arr.any(axis=1).sum())
    return events, flushes


def test_event_and_flush_counters_match_recorded_spikes():
    """The library's event and trial-end counters equal the counts derived on
    the host from the recorded spikes and the graph (uneven trials, ALIF)."""
    wl = W.c2_evidence(batch_size=4)
    b = wl.make_batch(0, 0, 4)
    net = E.Network(wl.network, "fp32", max_trials=4, max_steps=int(b.n_steps.max()))
    r = net.simulate(b, train=True)
    spikes = [net.read(E.EPROP_STATE_SPIKES, i) for i in range(4)]
    net.close()
    ev, fl = _counts_from_spikes(wl.network, b, spikes)
    assert r.n_rec_spikes == sum(len(s) for s in spikes)
    assert r.n_syn_events == ev and r.n_eprop_updates == ev
    assert r.n_flush_updates == fl
    log(f"c2: {ev} events, {fl} trial-end evaluations")


def test_torch_allocator_gives_identical_results():
    """Device buffers from PyTorch's caching allocator (the optional
    allocator callbacks) change nothing: FP32 results are bitwise equal."""
    wl = W.c3_events(batch_size=2)
    b = wl.make_batch(0, 0, 2)
    out = []
    for torch_alloc in (False, True):
        net = E.Network(wl.network, "fp32", max_trials=2, max_steps=300, torch_alloc=torch_alloc)
        r = net.simulate(b)
        net.apply()
        out.append((r.loss.copy(), net.weights()))
        if torch_alloc:
            assert len(net.allocator.blocks) > 10
        net.close()
        if torch_alloc:
            assert len(net.allocator.blocks) == 0
    assert np.array_equal(out[0][0], out[1][0])
    for k in KEYS:
        assert np.array_equal(out[0][1][k], out[1][1][k])


def test_fp32_multi_tile_runs_are_deterministic():
    """FP32 scatter over several tiles per trial (spike lists exchanged
    between workgroups): input currents are exact fixed-point sums, so two
    runs agree bit for bit, spikes, losses and gradients."""
    wl = W.c4_sparse(n_rec=3000, n_steps=300, batch_size=2, n_in=300)
    b = wl.make_batch(0, 0, 2)
    runs = []
    for _ in range(2):
        net = E.Network(wl.network, "fp32", max_trials=2, max_steps=300)
        assert net.layout()["tiles"] > 1
        r = net.simulate(b)
        runs.append((r.loss.copy(), net.grads(), [net.read(E.EPROP_STATE_SPIKES, i) for i in range(2)]))
        net.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    for i in range(2):
        assert np.array_equal(runs[0][2][i], runs[1][2][i])
    for k in KEYS:
        assert np.array_equal(runs[0][1][k], runs[1][1][k])


def test_gradients_restart_after_an_update():
    """After an update the accumulated gradient reads as zero, and the next
    training batch's gradient is that batch's alone (the first batch after an
    update writes the gradient pairs instead of adding to them): checked
    against the time-driven gradient of the same batch on the same updated
    weights, in the blocked-update layout."""
    wl = W.c4_sparse(n_rec=3000, n_steps=300, batch_size=2, n_in=300)
    b0, b1 = wl.make_batch(0, 0, 2), wl.make_batch(1, 0, 2)
    grads = []
    for time_driven in (False, True):
        net = E.Network(wl.network, "fp32", max_trials=2, max_steps=300)
        net.simulate(b0)
        g0 = net.grads()
        assert all(np.abs(g0[k]).max() > 0 for k in KEYS)
        net.apply()
        gz = net.grads()
        for k in ("w_in", "w_rec"):
            assert not np.any(gz[k]), k
        net.simulate(b1, time_driven=time_driven)
        grads.append(net.grads())
        net.close()
    for k in ("w_in", "w_rec"):
        ok, e, ent = rel_close(grads[0][k], grads[1][k], 1e-4, floor_frac=1e-2)
        log(f"restart {k}: normwise {e:.2e} worst {ent:.2e}")
        assert ok, (k, e, ent)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_autotuner_changes_shapes_not_results(precision):
    """With EPROP_AUTOTUNE the first training batch times the candidate
    launch shapes and keeps the fastest; two training iterations give the
    same losses and weights, bit for bit, as the default shapes."""
    wl = W.c4_sparse(n_rec=3000, n_steps=300, batch_size=2, n_in=300)
    out = []
    for autotune in (False, True):
        net = E.Network(wl.network, precision, max_trials=2, max_steps=300, autotune=autotune)
        losses = []
        for it in range(2):
            r = net.simulate(wl.make_batch(it, 0, 2))
            net.apply()
            losses.append(r.loss.copy())
        lay = net.layout()
        out.append((losses, net.weights(), lay))
        net.close()
    lay = out[1][2]
    log(f"{precision} tuned layout: {lay}")
    assert out[0][2]["autotuned"] == 0 and lay["autotuned"] == 1
    assert lay["piece"] in (4, 8, 16) and lay["adjoint_threads"] in (64, 128, 256)
    assert lay["synapse_threads"] in (64, 128, 256)
    for it in range(2):
        assert np.array_equal(out[0][0][it], out[1][0][it])
    for k in KEYS:
        assert np.array_equal(out[0][1][k], out[1][1][k])


# ----------------------------------------------------------------- time-driven baseline

def _train_mode(wl, precision, iterations, bs, time_driven, forced_rate=None):
    T = max(int(wl.make_batch(it, 0, bs).n_steps.max()) for it in range(iterations))
    net = E.Network(wl.network, precision, max_trials=bs, max_steps=T)
    out = []
    for it in range(iterations):
        b = wl.make_batch(it, 0, bs)
        if forced_rate:
            b = W.forced_poisson(b, wl.network.n_rec, forced_rate, wl.network.params.dt, seed=99,
                                 iteration=it, n_ref=2)
        r = net.simulate(b, train=True, time_driven=time_driven)
        out.append((r, net.grads()))
        net.apply()
    net.close()
    return out


@pytest.mark.parametrize("name", ["tiny", "c2", "c4twin"])
def test_time_driven_baseline_fp64_matches_oracle(name):
    """FP64 time-driven GPU gradient (every synapse, every step) against the
    oracle's time-driven mode: spike trains identical, gradients within
    1e-10, event and trial-end counts equal to the event-driven path's."""
    if name == "tiny":
        wl, bs, it = W.tiny(), 2, 2
    elif name == "c2":
        wl, bs, it = W.c2_evidence(batch_size=3), 3, 2
    else:
        wl, bs, it = W.c4_sparse(n_rec=2000, n_steps=150, batch_size=2, n_in=300), 2, 1
    td = _train_mode(wl, "fp64", it, bs, True)
    ed = _train_mode(wl, "fp64", it, bs, False)
    oh = oracle_train(wl, it, bs, grad_mode=1)
    for i in range(it):
        for k in KEYS:
            ok, e, ent = rel_close(td[i][1][k], oh["grads"][i][k], 1e-10)
            assert ok, (name, i, k, e, ent)
        assert td[i][0].n_syn_events == ed[i][0].n_syn_events
        assert td[i][0].n_flush_updates == ed[i][0].n_flush_updates
        log(f"{name} it {i}: time-driven grads match the oracle, {td[i][0].n_syn_events} events")


def test_time_driven_baseline_fp32_teacher_forced():
    """FP32 time-driven gradient with the oracle's spike trains within 1e-4."""
    wl = W.c3_events(batch_size=3)
    td = _train_mode(wl, "fp32", 1, 3, True, forced_rate=20.0)
    oh = oracle_train(wl, 1, 3, forced_rate=20.0, grad_mode=1)
    for k in KEYS:
        ok, e, ent = rel_close(td[0][1][k], oh["grads"][0][k], 1e-4, floor_frac=1e-2)
        log(f"c3 time-driven fp32 {k}: normwise {e:.2e} worst {ent:.2e}")
        assert ok, (k, e, ent)


# ----------------------------------------------------------------- generalised delays, rate regulariser

def _delayed(name, d, d_ls, c_reg, f_hz=10.0):
    if name == "tiny":
        wl, bs = W.tiny(), 2
    elif name == "c2":
        wl, bs = W.c2_evidence(batch_size=3), 3
    elif name == "c3":
        wl, bs = W.c3_events(batch_size=3), 3
    else:
        wl, bs = W.c4_sparse(n_rec=2000, n_steps=200, batch_size=2, n_in=300), 2
    p = wl.network.params
    p.d_out, p.d_ls, p.c_reg, p.f_target_hz = d, d_ls, c_reg, f_hz
    return wl, bs


@pytest.mark.parametrize("name,d,d_ls,c_reg", [("tiny", 2, 3, 1e5), ("c2", 1, 4, 1e5), ("tiny", 150, 60, 1e5),
                                               ("tiny", 0, 0, 1e5), ("c2", 3, 0, 0.0)])
def test_fp64_delays_and_rate_regulariser(name, d, d_ls, c_reg):
    """Readout delay d, learning-signal delay d^ls (Supplementary, "Generalized
    delays") and the static rate regulariser (eq. firing-rate-regularization):
    FP64 event-driven path exact against the oracle (spikes identical, loss,
    gradients and weights within 1e-10), and the time-driven baseline's
    gradient against the oracle's time-driven mode.  (150, 60) leaves no
    learning signal inside a 200-step trial: the recurrent gradient is the
    regulariser's alone."""
    wl, bs = _delayed(name, d, d_ls, c_reg)
    gh = gpu_train(wl, "fp64", 2, bs)
    oh = oracle_train(wl, 2, bs)
    assert_fp64_parity(gh, oh, f"{name} d={d} d_ls={d_ls} c_reg={c_reg}")
    td = _train_mode(wl, "fp64", 2, bs, True)
    ot = oracle_train(wl, 2, bs, grad_mode=1)
    for i in range(2):
        for k in KEYS:
            ok, e, ent = rel_close(td[i][1][k], ot["grads"][i][k], 1e-10)
            assert ok, ("time-driven", name, i, k, e, ent)


@pytest.mark.parametrize("name", ["c3", "c4twin"])
def test_fp32_teacher_forced_delays_and_rate_regulariser(name):
    """FP32 with the oracle's spike trains, d = 2, d^ls = 3, regulariser on:
    each iteration's update within 1e-4 of the FP64 oracle's (event-driven
    and time-driven paths)."""
    wl, bs = _delayed(name, 2, 3, 1e3)
    gh = gpu_train(wl, "fp32", 2, bs, forced_rate=20.0)
    oh = oracle_train(wl, 2, bs, forced_rate=20.0)
    td = _train_mode(wl, "fp32", 1, bs, True, forced_rate=20.0)
    for i in range(2):
        for k in KEYS:
            ok, e, ent = rel_close(gh["grads"][i][k], oh["grads"][i][k], 1e-4, floor_frac=1e-2)
            log(f"{name} delays+reg it {i} {k}: normwise {e:.2e} worst entry {ent:.2e}")
            assert ok, (name, i, k, e, ent)
        assert rel_close(gh["loss"][i], oh["loss"][i], 1e-4)[0]
    for k in KEYS:
        ok, e, ent = rel_close(td[0][1][k], oh["grads"][0][k], 1e-4, floor_frac=1e-2)
        assert ok, ("time-driven", name, k, e, ent)


# ----------------------------------------------------------------- the scaling network

def _scaling_twin():
    return W.scaling(n_rec=3000, indeg_rec=500, n_in=100, indeg_in=10, indeg_out=100, outdeg_fb=30, n_steps=400,
                     samples=4)


def test_scaling_twin_fp64_exact_and_fp32():
    """Twin of the scaling network (Methods, "Scaling": ignore-and-fire
    neurons at 5 Hz, fixed in-degree, sparse readout and feedback): FP64
    exact against the oracle over consecutive samples; FP32 (its spike trains
    are fixed by construction, so it is teacher-forced) within 1e-4."""
    wl = _scaling_twin()
    oh = oracle_train(wl, 2, 1)
    gh = gpu_train(wl, "fp64", 2, 1)
    assert_fp64_parity(gh, oh, "scaling twin")
    g32 = gpu_train(wl, "fp32", 2, 1)
    for i in range(2):
        for k in KEYS:
            ok, e, ent = rel_close(g32["grads"][i][k], oh["grads"][i][k], 1e-4, floor_frac=1e-2)
            log(f"scaling twin fp32 it {i} {k}: normwise {e:.2e} worst {ent:.2e}")
            assert ok, (i, k, e, ent)


def test_scaling_network_launch_configuration_sampled():
    """The scaling network at its full neuron count (128,000 ignore-and-fire
    neurons, one 1000-step sample, FP32, the tile layout of the benchmark)
    with recurrent in-degree 100 instead of 10^4 so that it builds in seconds:
    all 640,000 forced spikes are emitted, and the gradients of every
    incoming synapse of 24 sampled neurons are within 1e-4 of the oracle's
    per-neuron evaluation, the loss within 1e-6."""
    wl = W.scaling(indeg_rec=100)
    b = wl.make_batch(0, 0, 1)
    net = E.Network(wl.network, "fp32", max_trials=1, max_steps=1000)
    r = net.simulate(b, train=True)
    g = net.grads()
    lay = net.layout()
    net.close()
    log(f"gpu done: layout {lay}, {r.n_rec_spikes} spikes, {r.n_syn_events} events")
    assert r.n_rec_spikes == 640_000
    on = O.OracleNet(wl.network)
    targets = np.sort(np.random.default_rng(1).choice(wl.network.n_rec, 24, replace=False))
    loss, psi, a, c = O.forced_sampled(on, b, 0, targets)
    assert abs(r.loss[0] - loss) <= 1e-6 * abs(loss), (r.loss[0], loss)
    for name, gg, ref in (("w_in", g["w_in"], a), ("w_rec", g["w_rec"], c)):
        m = ~np.isnan(ref)
        ok, e, ent = rel_close(gg[m], ref[m], 1e-4, floor_frac=1e-2)
        log(f"scaling {name}: {m.sum()} synapses, normwise {e:.2e} worst {ent:.2e}")
        assert ok, (name, e, ent)


def test_fp32_adam_state_and_input_bound_after_updates():
    """Evidence accumulation with Adam (eq. eta-adam-fast, eq. delta-w-adam-fast),
    FP32, teacher-forced, three iterations: the optimiser's first and second
    moments read back in the caller's synapse order within 1e-4 of the
    oracle's, and the weights likewise; the per-target input bound the
    update recomputes stays above the largest sum of |w| into one target."""
    wl = W.c2_evidence(batch_size=4)
    assert wl.network.params.optimizer == 1
    on = O.OracleNet(wl.network)
    net = E.Network(wl.network, "fp32", max_trials=4, max_steps=max(int(wl.make_batch(i, 0, 4).n_steps.max())
                                                                     for i in range(3)))
    for it in range(3):
        b = W.forced_poisson(wl.make_batch(it, 0, 4), wl.network.n_rec, 20.0, 1.0, seed=99, iteration=it, n_ref=2)
        net.simulate(b, train=True)
        net.apply()
        g = O.zero_grads(on)
        for i in range(b.n_trials):
            O.run_trial(on, b, i, 2, g)
        O.apply(on, g, b.n_trials)
    for name, m_id, v_id, key in (("rec", E.EPROP_STATE_ADAM_M_REC, E.EPROP_STATE_ADAM_V_REC, "w_rec"),
                                  ("in", E.EPROP_STATE_ADAM_M_IN, E.EPROP_STATE_ADAM_V_IN, "w_in")):
        for sid, ref in ((m_id, on.m[key]), (v_id, on.v[key])):
            ok, e, ent = rel_close(net.read(sid), ref, 1e-4, floor_frac=1e-2)
            log(f"adam {name} state {sid}: normwise {e:.2e} worst {ent:.2e}")
            assert ok, (name, sid, e, ent)
    w = net.weights()
    for k in KEYS:
        ok, e, ent = rel_close(w[k], getattr(on, k), 1e-5)
        assert ok, (k, e, ent)
    # the bound: sum of |w| into each target, from the read-back weights
    pr_in, pr_rec = wl.network.in_rec, wl.network.rec_rec
    l1 = np.zeros(wl.network.n_rec)
    np.add.at(l1, pr_in.col, np.abs(w["w_in"]))
    np.add.at(l1, pr_rec.col, np.abs(w["w_rec"]))
    bound = float(net.read(E.EPROP_STATE_INPUT_BOUND)[0])
    net.close()
    log(f"input bound {bound:.6g}, largest sum of |w| into one target {l1.max():.6g}")
    indeg = np.bincount(pr_in.col, minlength=wl.network.n_rec) + np.bincount(pr_rec.col, minlength=wl.network.n_rec)
    assert l1.max() <= bound <= l1.max() * 1.001 * (1 + 1e-6) + indeg.max() * 2.0 ** -16


# ----------------------------------------------------------------- e-prop+ components

EPROP_PLUS = dict(reset_mode=1, v_reset=-0.2, etrace_filter=1, tau_e=8.0, reg_mode=1, reg_tau=50.0,
                  c_reg=30.0, f_target_hz=20.0)


def _plus(name, **extra):
    if name == "tiny":
        wl, bs = W.tiny(loss=2), 2
    elif name == "c2":
        wl, bs = W.c2_evidence(batch_size=3), 3
    elif name == "c3":
        wl, bs = W.c3_events(batch_size=3), 3
    else:
        wl, bs = W.c4_sparse(n_rec=2000, n_steps=200, batch_size=2, n_in=300), 2
    p = wl.network.params
    for k, v in dict(EPROP_PLUS, **extra).items():
        setattr(p, k, v)
    if name in ("c2", "c3"):
        p.loss = 2
    return wl, bs


@pytest.mark.parametrize("name,extra", [("tiny", {}), ("tiny", dict(etrace_filter=2, d_out=1)),
                                        ("c2", dict(d_out=2, d_ls=1)), ("c4twin", dict(loss=0))])
def test_fp64_eprop_plus_components(name, extra):
    """e-prop+ components (Results, "Event-driven e-prop with additional
    biological features"): full reset to v_reset, decoupled or removed
    eligibility filter, moving-average rate regulariser, temporal MSE, with
    delays: FP64 exact against the oracle (spikes identical, loss, gradients
    and weights within 1e-10)."""
    wl, bs = _plus(name, **extra)
    gh = gpu_train(wl, "fp64", 2, bs)
    oh = oracle_train(wl, 2, bs)
    assert_fp64_parity(gh, oh, f"e-prop+ {name} {extra}")


def test_time_driven_baseline_with_reset_filter_and_temporal_mse():
    """The time-driven baseline with the full reset, the decoupled filter and
    the temporal MSE (static regulariser): FP64 within 1e-10 of the oracle's
    time-driven mode; with the moving-average regulariser it reports
    EPROP_ERR_UNSUPPORTED."""
    wl, bs = _plus("tiny", reg_mode=0, c_reg=5.0)
    td = _train_mode(wl, "fp64", 2, bs, True)
    oh = oracle_train(wl, 2, bs, grad_mode=1)
    for i in range(2):
        for k in KEYS:
            ok, e, ent = rel_close(td[i][1][k], oh["grads"][i][k], 1e-10)
            assert ok, (i, k, e, ent)
    wl, bs = _plus("tiny")
    net = E.Network(wl.network, "fp64", max_trials=bs, max_steps=200)
    with pytest.raises(E.EpropError) as ei:
        net.simulate(wl.make_batch(0, 0, bs), train=True, time_driven=True)
    assert ei.value.status == E.EPROP_ERR_UNSUPPORTED
    net.close()


@pytest.mark.parametrize("name", ["c3", "c4twin"])
def test_fp32_teacher_forced_eprop_plus_components(name):
    """FP32 with the oracle's spike trains and every e-prop+ component on:
    each iteration's update within 1e-4 of the FP64 oracle's."""
    wl, bs = _plus(name, d_out=1)
    gh = gpu_train(wl, "fp32", 2, bs, forced_rate=20.0)
    oh = oracle_train(wl, 2, bs, forced_rate=20.0)
    for i in range(2):
        for k in KEYS:
            ok, e, ent = rel_close(gh["grads"][i][k], oh["grads"][i][k], 1e-4, floor_frac=1e-2)
            log(f"{name} e-prop+ it {i} {k}: normwise {e:.2e} worst entry {ent:.2e}")
            assert ok, (name, i, k, e, ent)
        assert rel_close(gh["loss"][i], oh["loss"][i], 1e-4)[0]


# ----------------------------------------------------------------- e-prop+ update schedule

def _online_pair(wl, precision, b, eta):
    """The GPU's and the oracle's online run of the batch's trials back to back."""
    T = int(b.n_steps.sum())
    net = E.Network(wl.network, precision, max_trials=1, max_steps=T)
    w0 = net.weights()
    r = net.simulate(b, online=True)
    g = {"loss": r.loss.copy(), "z": net.spikes(0, T), "w": net.weights(), "w0": w0, "events": r.n_syn_events}
    net.close()
    on = O.OracleNet(wl.network)
    o = O.run_online(on, b, eta, cutoff=int(wl.network.params.isi_cutoff))
    o["w"] = {k: getattr(on, k).copy() for k in KEYS}
    return g, o


@pytest.mark.parametrize("name,extra", [("tiny", {}), ("tiny", dict(d_out=1, d_ls=1)),
                                        ("tiny", dict(EPROP_PLUS, isi_cutoff=15)),
                                        ("tiny2", dict(EPROP_PLUS, d_out=2, etrace_filter=2)),
                                        ("c2", dict(d_out=1, isi_cutoff=40)), ("c4twin", dict(d_out=1))])
def test_online_schedule_fp64_matches_oracle(name, extra):
    """e-prop+ update schedule (EPROP_BATCH_ONLINE): the batch's samples run
    back to back by one network instance, every arriving spike first updating
    its synapse by gradient descent.  FP64 against the oracle's online run:
    spike trains identical, per-sample losses within 1e-12 and every weight
    (input, recurrent, readout) within 1e-10 after the run."""
    if name == "tiny":
        wl, b = W.tiny(loss=0), None
    elif name == "tiny2":
        wl, b = W.tiny(loss=2), None
    elif name == "c2":
        wl, b = W.c2_evidence(batch_size=3), None
    else:
        wl, b = W.c4_sparse(n_rec=2000, n_steps=200, batch_size=2, n_in=300), None
    p = wl.network.params
    p.optimizer = 0
    p.eta = 2e-3 if name != "c4twin" else 1e-5
    for k, v in extra.items():
        setattr(p, k, v)
    if name == "c2":
        p.loss = 2
    b = wl.make_batch(0, 0, 3 if name != "c4twin" else 2)
    g, o = _online_pair(wl, "fp64", b, p.eta)
    assert np.array_equal(g["z"], o["z"]), "spike trains differ"
    ok, e, _ = rel_close(g["loss"], o["loss"], 1e-12)
    assert ok, ("loss", e)
    for k in KEYS:
        ok, e, ent = rel_close(g["w"][k], o["w"][k], 1e-10)
        assert ok, (k, e, ent)
        assert not np.array_equal(g["w"][k], g["w0"][k]), (k, "weights did not move")
    log(f"online {name} {extra}: {g['events']} updates, loss {np.round(g['loss'], 3)}")


def test_online_schedule_fp32_ignore_and_fire():
    """FP32 online run of the scaling network's twin (ignore-and-fire spike
    trains fixed by construction, so FP32 sees the oracle's spikes): the
    weight changes within 1e-4 of the FP64 oracle's, normwise, and per entry
    within 1e-4 of max(|change|, 1% of the largest) plus the FP32 rounding of
    the weight at each of its updates (at most 32 here)."""
    wl = _scaling_twin()
    p = wl.network.params
    p.eta, p.d_out, p.isi_cutoff = 1e-4, 1, 100
    b = wl.make_batch(0, 0, 2)
    g, o = _online_pair(wl, "fp32", b, p.eta)
    assert np.array_equal(g["z"], o["z"])
    w0 = {k: getattr(O.OracleNet(wl.network), k) for k in KEYS}
    u = 2.0 ** -24
    for k in KEYS:
        dg, do = g["w"][k] - w0[k], o["w"][k] - w0[k]
        ok, e, ent = rel_close(dg, do, 1e-4, floor_frac=1e-2)
        log(f"online fp32 {k}: change normwise {e:.2e} worst {ent:.2e}")
        assert e <= 1e-4, (k, e)
        bound = 1e-4 * np.maximum(np.abs(do), 1e-2 * np.abs(do).max()) + 32 * u * np.abs(o["w"][k])
        assert np.all(np.abs(dg - do) <= bound), (k, float(np.max(np.abs(dg - do) / bound)))


def test_online_schedule_rejects_what_it_does_not_support():
    wl = W.tiny(loss=0)   # Adam
    b = wl.make_batch(0, 0, 2)
    net = E.Network(wl.network, "fp32", max_trials=1, max_steps=400)
    with pytest.raises(E.EpropError) as ei:
        net.simulate(b, online=True)
    assert ei.value.status == E.EPROP_ERR_UNSUPPORTED
    net.close()
    wl.network.params.optimizer = 0
    net = E.Network(wl.network, "fp32", max_trials=1, max_steps=300)
    with pytest.raises(E.EpropError) as ei:
        net.simulate(b, online=True)    # 400 steps > max_steps
    assert ei.value.status == E.EPROP_ERR_CAPACITY
    with pytest.raises(E.EpropError) as ei:
        net.simulate(wl.make_batch(0, 0, 1), online=True, device=True)
    assert ei.value.status == E.EPROP_ERR_UNSUPPORTED
    r = net.simulate(wl.make_batch(0, 0, 1), online=True)   # the handle still works
    assert np.isfinite(r.loss).all()
    net.close()
