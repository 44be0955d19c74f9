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


# ----------------------------------------------------------------- FP32 checks

U32 = 2.0 ** -24
FP32_TINY = 2.0 ** -126   # smallest normal FP32 number


def oracle_at(wnet, weights, m=None, v=None, step=0):
    """The oracle at the GPU's own weights (FP32 values, read back as FP64)
    and feedback weights rounded to FP32 like the library's copy; optionally
    the GPU's Adam state (m, v, step) for the optimiser check."""
    on = O.OracleNet(wnet)
    on.w_in = np.array(weights["w_in"], dtype=np.float64)
    on.w_rec = np.array(weights["w_rec"], dtype=np.float64)
    on.w_out = np.array(weights["w_out"], dtype=np.float64, order="C").reshape(wnet.n_out, wnet.n_rec)
    on.fb = np.ascontiguousarray(np.asarray(wnet.feedback, np.float64).astype(np.float32).astype(np.float64))
    if m is not None:
        on.m = {k: np.array(m[k], dtype=np.float64).reshape(on.m[k].shape) for k in KEYS}
        on.v = {k: np.array(v[k], dtype=np.float64).reshape(on.v[k].shape) for k in KEYS}
        on.step = int(step)
    return on


def read_psis(net, b, targets=None):
    """The recorded surrogate gradients of every trial of the last batch, [T, J]."""
    J = net.wnet.n_rec
    out = []
    for i in range(b.n_trials):
        T = int(b.n_steps[i])
        out.append(net.read(E.EPROP_STATE_PSI, i).reshape(T, J))
    return out


def check_fp32_batch(name, wnet, b, psis, G, weights, quantum=0.0, targets=None, downstream=1.0, keys=KEYS):
    """FP32 gradient of a teacher-forced batch, evaluated by the GPU at
    `weights` (its own FP32 values), against the FP64 oracle at the same
    weights (orc_fp32_bounds):
      (A) normwise: ||G - g|| <= 1e-4 ||g|| for each weight array (the
          tolerance of the FP32 mode);
      (C) every recorded psi within the running-error bound of an FP32
          evaluation of the neuron recursion;
      (D) every gradient entry within `downstream` times the rounding bound
          of FP32 arithmetic downstream of psi (7 u times the sum of the
          absolute values of the entry's terms) of the oracle's gradient on
          the GPU's own psi history (Alg. "time-driven gradient computation"
          takes the archived psi).  Together (C) and (D) bound every entry's
          error against the oracle's own gradient.
    Returns per-array statistics."""
    on = oracle_at(wnet, weights)
    g_own = {k: None for k in keys}
    g_giv = {k: None for k in keys}
    bnd = {k: None for k in keys}
    worst_psi = 0.0
    for i in range(b.n_trials):
        own = O.fp32_bounds(on, b, i, quantum, targets=targets)
        pg = psis[i] if targets is None else psis[i][:, targets]
        giv = O.fp32_bounds(on, b, i, quantum, psi_given=pg, targets=targets)
        err = np.abs(pg - own["psi"])
        bad = err > own["psi_bound"]
        assert not bad.any(), (name, "psi", i, int(bad.sum()), float(err[bad].max()))
        if np.any(own["psi_bound"] > 0):
            worst_psi = max(worst_psi, float((err / np.maximum(own["psi_bound"], 1e-300)).max()))
        for k in keys:
            for acc, src in ((g_own, own["g"]), (g_giv, giv["g"]), (bnd, giv["b"])):
                acc[k] = src[k].copy() if acc[k] is None else acc[k] + src[k]
    stats = {"psi_err_over_bound": worst_psi}
    for k in keys:
        gk = np.asarray(G[k], np.float64).reshape(g_own[k].shape)
        m = ~np.isnan(g_own[k])
        a, ref, giv, bd = gk[m], g_own[k][m], g_giv[k][m], bnd[k][m]
        nrm = np.linalg.norm(ref)
        nerr = float(np.linalg.norm(a - ref) / nrm) if nrm > 0 else float(np.linalg.norm(a))
        assert nerr <= 1e-4, (name, k, "normwise", nerr)
        dev = np.abs(a - giv)
        lim = downstream * bd + 1e-12 * np.abs(giv).max(initial=0.0)
        assert np.all(dev <= lim), (name, k, "entry", int((dev > lim).sum()), float((dev / np.maximum(lim, 1e-300)).max()))
        z21 = np.abs(a - ref) > 1e-4 * np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max(initial=0.0))
        stats[k] = {"normwise": nerr, "entry_over_bound": float((dev / np.maximum(lim, 1e-300)).max(initial=0.0)),
                    "beyond_z21": int(z21.sum()), "n": int(a.size)}
    log(f"{name}: psi err/bound {worst_psi:.3f}; " + "; ".join(
        f"{k} normwise {stats[k]['normwise']:.1e}, entry/bound {stats[k]['entry_over_bound']:.3f}, "
        f"{stats[k]['beyond_z21']} of {stats[k]['n']} beyond 1e-4 x max(|g|, 1e-3 |g|max)" for k in keys))
    return stats


def read_adam(net):
    ids = {"w_in": (E.EPROP_STATE_ADAM_M_IN, E.EPROP_STATE_ADAM_V_IN),
           "w_rec": (E.EPROP_STATE_ADAM_M_REC, E.EPROP_STATE_ADAM_V_REC),
           "w_out": (E.EPROP_STATE_ADAM_M_OUT, E.EPROP_STATE_ADAM_V_OUT)}
    m = {k: net.read(ids[k][0]) for k in KEYS}
    v = {k: net.read(ids[k][1]) for k in KEYS}
    return m, v, int(net.read(E.EPROP_STATE_ADAM_STEP)[0])


def check_optimizer(name, wnet, w_before, G, n_trials, w_after, adam_before=None, adam_after=None):
    """The update given the GPU's own gradient sums G: the oracle's gradient
    descent or Adam (eq. gradient-descent; eq. eta-adam-fast,
    eq. delta-w-adam-fast) from the GPU's weights (and Adam state) in FP64.
    The library may round the averaged gradient to FP32 before the step and
    stores the weights (and moments) in FP32, so each result is within
    u |x_exp| plus the change of the oracle's result when G moves by a
    relative u (evaluated at G (1 - u) and G (1 + u)), plus FP32's smallest
    normal number (a second moment of a tiny gradient underflows to zero)."""
    def step(scale):
        on = oracle_at(wnet, w_before, *adam_before) if adam_before is not None else oracle_at(wnet, w_before)
        O.apply(on, {k: np.array(G[k], np.float64).reshape(getattr(on, k).shape) * scale for k in KEYS}, n_trials)
        return on
    on, lo, hi = step(1.0), step(1.0 - U32), step(1.0 + U32)
    for k in KEYS:
        exp = getattr(on, k).ravel()
        sens = np.maximum(np.abs(getattr(lo, k).ravel() - exp), np.abs(getattr(hi, k).ravel() - exp))
        got = np.asarray(w_after[k], np.float64).ravel()
        lim = U32 * np.abs(exp) + 1.01 * sens + FP32_TINY
        dev = np.abs(got - exp)
        assert np.all(dev <= lim), (name, k, float((dev / lim).max()))
    if adam_after is not None:
        m1, v1, st = adam_after
        assert st == on.step, (name, st, on.step)
        for k in KEYS:
            for got, exp, e_lo, e_hi in ((m1[k], on.m[k], lo.m[k], hi.m[k]), (v1[k], on.v[k], lo.v[k], hi.v[k])):
                exp = exp.ravel()
                sens = np.maximum(np.abs(e_lo.ravel() - exp), np.abs(e_hi.ravel() - exp))
                lim = U32 * np.abs(exp) + 1.01 * sens + FP32_TINY
                assert np.all(np.abs(np.asarray(got).ravel() - exp) <= lim), (name, k)


def ring_quantum(net):
    """The largest rounding of one arriving weight by the delay ring: 0 for
    64-bit entries (every FP32 weight converts exactly), 2^-(F+1) for 32-bit
    entries with F = 30 - ceil(log2(input bound)) fraction bits."""
    if net.layout()["ring_bytes"] != 4:
        return 0.0
    import math
    l1 = float(net.read(E.EPROP_STATE_INPUT_BOUND)[0])
    F = 30 if l1 <= 0 else min(30, 30 - math.ceil(math.log2(l1)))
    return 2.0 ** -(F + 1)


def fp32_forced_run(name, wl, iterations, bs, rate=20.0, time_driven=False, autotune=False, T=None, max_delay=None,
                    expect_layout=None):
    """Teacher-forced FP32 training on the GPU (forced Poisson trains at
    `rate` Hz, or the batch's own forced trains with rate None); every
    iteration's gradient is checked against the oracle at the GPU's weights
    (check_fp32_batch), its loss against the oracle's (identical spikes and
    FP32 weights, FP64 readout: 1e-12), and its update against the optimiser
    given that gradient (check_optimizer).  The time-driven baseline's FP32
    eligibility recursions round at most 5 times per step, so a term that
    meets the learning signal carries at most 5 T u more than the event-driven
    path's 7 u: its entry bound is scaled by (7 + 5 T) / 7.  Returns the
    per-iteration statistics."""
    wnet = wl.network
    if T is None:
        T = max(int(wl.make_batch(it, 0, bs).n_steps.max()) for it in range(iterations))
    net = E.Network(wnet, "fp32", max_trials=bs, max_steps=T, autotune=autotune, max_delay=max_delay)
    lay = net.layout()
    for key, val in (expect_layout or {}).items():
        assert lay[key] == val, (name, key, lay[key], val)
    adam = wnet.params.optimizer == 1
    out = []
    for it in range(iterations):
        b = wl.make_batch(it, 0, bs)
        if rate is not None:
            b = W.forced_poisson(b, wnet.n_rec, rate, wnet.params.dt, seed=99, iteration=it, n_ref=2)
        w0 = net.weights()
        a0 = read_adam(net) if adam else None
        quantum = ring_quantum(net)
        r = net.simulate(b, train=True, time_driven=time_driven)
        G = net.grads()
        psis = read_psis(net, b)
        st = check_fp32_batch(f"{name} it {it}", wnet, b, psis, G, w0, quantum=quantum,
                              downstream=(7.0 + 5.0 * T) / 7.0 if time_driven else 1.0)
        on = oracle_at(wnet, w0)
        lo = [O.run_trial(on, b, i, 0).loss for i in range(b.n_trials)]
        assert rel_close(r.loss, lo, 1e-12)[0], (name, it, "loss")
        net.apply()
        check_optimizer(f"{name} it {it}", wnet, w0, G, b.n_trials, net.weights(), a0, read_adam(net) if adam else None)
        out.append(st)
    net.close()
    return out


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
    """FP32 with teacher-forced spike trains, every iteration at the GPU's own
    weights: the computed update (the batch-summed gradient the optimiser
    receives) within 1e-4 normwise of the FP64 oracle's, every recorded psi
    and every gradient entry within its derived FP32 rounding bound
    (check_fp32_batch), the loss within 1e-12, and the stored weights (and
    Adam moments, c2) the optimiser's result on that gradient rounded once
    to FP32."""
    if name == "c1":
        wl, bs, it = W.c1_pattern(), 1, 3
    elif name == "c2":
        wl, bs, it = W.c2_evidence(batch_size=4), 4, 2
    elif name == "c3":
        wl, bs, it = W.c3_events(batch_size=4), 4, 2
    elif name == "c4twin":
        wl, bs, it = W.c4_sparse(n_rec=2000, n_steps=200, batch_size=2, n_in=300), 2, 2
    else:
        wl, bs, it = W.tiny(), 2, 3
    fp32_forced_run(name, wl, it, bs)


def _free_run(run, it, bs, eta, stream):
    """One seed's free-running FP32 training (GPU), on its own stream."""
    import ctypes as C
    import torch
    with torch.cuda.stream(stream):
        wl = W.c3_events(seed=run["seed"], batch_size=bs)
        wl.network.params.eta = eta
        net = E.Network(wl.network, "fp32", max_trials=bs, max_steps=300,
                        stream=C.c_void_p(stream.cuda_stream))
        losses, acc = [], []
        for i in range(it):
            b = wl.make_batch(i, 0, bs)
            r = net.simulate(b, train=True)
            net.apply()
            losses.append(float(r.loss.mean()))
            acc.append(float(np.mean(r.predicted == b.label)))
        net.close()
    return losses, acc


def test_fp32_free_running_final_loss():
    """Free-running FP32 batched training of the event-camera classification
    task (softmax cross-entropy over the last 30 steps, gradient descent with
    eta 1e-3; 32 trials per iteration, 100 iterations, eight network seeds)
    against the FP64 oracle's training of the same batches from the same
    weights, stored by tests/golden/make_c3_training.py (which calls only the
    oracle).  Both trainings lower the loss.  A free-running spiking network
    is chaotic: one spike that flips (an FP32 rounding suffices) sends the
    trajectories apart, and FP64 training from weights perturbed by one unit
    in the last place ends as far from the unperturbed run as FP32 does, so a
    single seed's final loss is a random draw (reading Z22).  The final loss
    of a seed is the mean over its last 10 iterations; with d_s the log ratio
    of the GPU's to the oracle's for seed s, the test asks for no systematic
    difference: |mean d| within three standard errors of the mean (a paired
    test at 3 sigma), and for the seed-mean loss over the whole trained run
    to agree within 2%."""
    import json
    import os
    from concurrent.futures import ThreadPoolExecutor
    import torch
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c3_training_oracle.json")))
    it, bs, eta = ref["iterations"], ref["batch"], ref["eta"]
    runs = ref["runs"]
    streams = [torch.cuda.Stream() for _ in runs]
    with ThreadPoolExecutor(4) as ex:
        out = list(ex.map(lambda a: _free_run(a[0], it, bs, eta, a[1]), zip(runs, streams)))
    w = it // 10
    d, g_run, o_run = [], [], []
    for run, (losses, acc) in zip(runs, out):
        o = run["mean_loss"]
        assert np.mean(o[-w:]) < 0.5 * np.mean(o[:w]), "the oracle's training did not lower the loss"
        assert np.mean(losses[-w:]) < 0.5 * np.mean(losses[:w]), "the GPU's training did not lower the loss"
        d.append(np.log(np.mean(losses[-w:]) / np.mean(o[-w:])))
        g_run.append(np.mean(losses))
        o_run.append(np.mean(o))
        log(f"seed {run['seed']}: loss {np.mean(o[:w]):.1f} -> oracle {np.mean(o[-w:]):.2f}, gpu {np.mean(losses[-w:]):.2f}; "
            f"accuracy (last {w}) oracle {np.mean(run['accuracy'][-w:]):.3f}, gpu {np.mean(acc[-w:]):.3f}")
    d = np.array(d)
    se = d.std(ddof=1) / np.sqrt(len(d))
    rel_run = abs(np.mean(g_run) - np.mean(o_run)) / np.mean(o_run)
    log(f"final-loss log ratio: mean {d.mean():+.4f}, standard error {se:.4f}; "
        f"seed-mean loss over the run: gpu {np.mean(g_run):.3f}, oracle {np.mean(o_run):.3f}, relative {rel_run:.3e}")
    assert abs(d.mean()) <= 3 * se
    assert rel_run < 0.02


def _repeat_trial(b, n):
    """A batch of n copies of the single-trial batch b."""
    m = int(b.in_ptr[1])
    out = W.Batch(n_steps=np.repeat(b.n_steps, n), in_ptr=np.arange(n + 1, dtype=np.uint64) * m,
                  in_step=np.tile(b.in_step, n), in_src=np.tile(b.in_src, n))
    if b.target is not None:
        out.target = np.repeat(b.target, n, axis=0)
    if b.label is not None:
        out.label = np.repeat(b.label, n)
    if b.window is not None:
        out.window = np.repeat(b.window, n, axis=0)
    if b.forced_ptr is not None:
        f = int(b.forced_ptr[1])
        out.forced_ptr = np.arange(n + 1, dtype=np.uint64) * f
        out.forced_step = np.tile(b.forced_step, n)
        out.forced_neuron = np.tile(b.forced_neuron, n)
    return out


def test_device_kahan_accumulation_over_many_trials():
    """Compensated FP32 summation on the device against FP64 (pin P15;
    Higham, "Accuracy and Stability of Numerical Algorithms", Sec. 4.3: a
    Kahan sum of terms x_i is within 2u sum|x_i| + O(n u^2) of the exact
    sum).  256 copies of one C3 trial add the same FP32 terms 256 times (the
    forward pass is deterministic), so the exact sum is 256 times one
    trial's.  The device sums the arrivals of each chunk of 8 trials with
    Kahan (2u), stores each chunk's sum in FP32 (u) and adds the 32 chunk
    sums with Kahan (2u); one trial's gradient G_1 carries 2u of its own.
    The recurrent spikes are teacher-forced (Poisson at 20 Hz), so that the
    oracle evaluates the same spike trains.
    Hence |G_256 - 256 G_1| <= 7u * 256 * A_1 + O(u^2), with A_1 the sum of
    the absolute values of one trial's terms; the oracle's per-entry bound
    at the GPU's weights on the GPU's psi is exactly 7u A_1 (its 7u also
    count the roundings of the feedback and the archive, which are the same
    in every copy and cancel here).  Uncompensated FP32 accumulation of the same
    copies exceeds this bound on many synapses (evaluated here with numpy
    float32), so the bound tells the two apart."""
    n = 256
    wl = W.c3_events(batch_size=1)
    b1 = W.forced_poisson(wl.make_batch(0, 0, 1), wl.network.n_rec, 20.0, wl.network.params.dt, seed=7, n_ref=2)
    net = E.Network(wl.network, "fp32", max_trials=1, max_steps=300)
    net.simulate(b1, train=True)
    G1 = net.grads()
    psis = read_psis(net, b1)
    w = net.weights()
    net.close()
    net = E.Network(wl.network, "fp32", max_trials=n, max_steps=300)
    net.simulate(_repeat_trial(b1, n), train=True)
    GN = net.grads()
    assert all(np.array_equal(w[k], v) for k, v in net.weights().items())
    net.close()
    on = oracle_at(wl.network, w)
    B1 = O.fp32_bounds(on, b1, 0, psi_given=psis[0])["b"]   # 7u A_1 per entry
    tight = {}
    for k in KEYS:
        g1 = np.asarray(G1[k], np.float64).ravel()
        gn = np.asarray(GN[k], np.float64).ravel()
        b1 = np.asarray(B1[k], np.float64).ravel()
        assert b1.size == g1.size, k
        lim = 1.001 * n * b1 + 1e-300
        dev = np.abs(gn - n * g1)
        assert np.all(dev <= lim), (k, int((dev > lim).sum()), float((dev / lim).max()))
        # plain FP32 accumulation of the same n copies of one trial's sum
        x = g1.astype(np.float32)
        acc = np.zeros_like(x)
        for _ in range(n):
            acc = (acc + x).astype(np.float32)
        live = b1 > 0
        over = np.abs(acc.astype(np.float64) - n * g1) > lim
        tight[k] = (float((dev[live] / lim[live]).max(initial=0.0)), float(over[live].mean()) if live.any() else 0.0)
    log("Kahan over 256 trials: " + "; ".join(f"{k} dev/bound {tight[k][0]:.3f}, plain FP32 beyond the bound on "
                                             f"{100 * tight[k][1]:.1f}% of synapses" for k in KEYS))
    assert tight["w_in"][1] > 0.05 and tight["w_rec"][1] > 0.05


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
    scatter with the autotuner on (the benchmark's launch configuration: the
    tuner runs on this first training batch), teacher-forced at 10 Hz: the
    gradients of every incoming synapse of 24 sampled neurons and of every
    output synapse, summed over the 4 trials, against the oracle's per-neuron
    evaluation (check_fp32_batch: 1e-4 normwise, every sampled psi and every
    entry within its FP32 bound), and the per-trial losses within 1e-12."""
    wl = W.c4_sparse()
    b = W.forced_poisson(wl.make_batch(0, 0, 4), wl.network.n_rec, 10.0, 1.0, seed=7, n_ref=2)
    net = E.Network(wl.network, "fp32", max_trials=4, max_steps=1000, autotune=True)
    w0 = net.weights()
    r = net.simulate(b, train=True)
    lay = net.layout()
    assert lay["autotuned"] == 1
    G = net.grads()
    psis = read_psis(net, b)
    net.close()
    log(f"gpu done: {r.n_rec_spikes} spikes, {r.n_syn_events} events, layout {lay}")
    targets = np.sort(np.random.default_rng(0).choice(wl.network.n_rec, 24, replace=False))
    check_fp32_batch("full size", wl.network, b, psis, G, w0, targets=targets)
    on = oracle_at(wl.network, w0)
    for i in range(4):
        loss = O.forced_sampled(on, b, i, targets[:1])[0]
        assert abs(r.loss[i] - loss) <= 1e-12 * abs(loss), (i, r.loss[i], loss)


C5_TWIN_RING_STEPS = 40   # delay capacity of the twin's handle (its graph keeps delays 1..5)


def _c5_twin():
    """Twin of the million-neuron network (80/20 LIF/ALIF, fixed in-degree
    100, delays 1..5, 10 input synapses per neuron at 5 Hz, one trial) at
    40,000 neurons.  Given a delay capacity of 40 steps, 8-byte ring entries
    of 512-neuron tiles do not fit LDS, so the handle takes the 32-bit
    fixed-point ring, as the full network does; rows have under 4 synapses per
    source and tile, so the update runs in target-major order (k_apply_syn with
    k_input_bound), also as at full size."""
    return W.c5_million(n_rec=40_000, n_steps=200, batch_size=1, n_in=1000)


def test_c5_twin_fp64_exact():
    """The twin in FP64 (deterministic gather delivery): spike trains
    identical to the oracle's, loss, gradients and weights within 1e-10, over
    two iterations with an update between them."""
    wl = _c5_twin()
    assert wl.network.is_alif.sum() == 8000
    gh = gpu_train(wl, "fp64", 2, 1)
    oh = oracle_train(wl, 2, 1)
    assert_fp64_parity(gh, oh, "c5 twin")


def test_c5_twin_fp32_ring32_unblocked_alif():
    """The twin in FP32 with the paths the million-neuron network takes: the
    32-bit fixed-point delay ring (each arriving weight rounded to 2^-(F+1),
    part of the psi bound), ALIF neurons in the multi-tile forward kernel,
    and the target-major update with the input-bound pass.  Teacher-forced,
    two iterations: each gradient, loss and update checked against the oracle
    at the GPU's weights (fp32_forced_run); the input bound read back after
    each update stays above the largest sum of |w| into one target."""
    wl = _c5_twin()
    fp32_forced_run("c5 twin", wl, 2, 1, rate=5.0, max_delay=C5_TWIN_RING_STEPS,
                    expect_layout={"ring_bytes": 4, "blocked_update": 0, "gather": 0, "queues": 1})
    net = E.Network(wl.network, "fp32", max_trials=1, max_steps=200, max_delay=C5_TWIN_RING_STEPS)
    assert net.layout()["tiles"] > 1
    for it in range(2):
        net.simulate(W.forced_poisson(wl.make_batch(it, 0, 1), wl.network.n_rec, 5.0, 1.0, seed=99, iteration=it,
                                      n_ref=2))
        net.apply()
        w = net.weights()
        l1 = np.zeros(wl.network.n_rec)
        np.add.at(l1, wl.network.in_rec.col, np.abs(w["w_in"]))
        np.add.at(l1, wl.network.rec_rec.col, np.abs(w["w_rec"]))
        bound = float(net.read(E.EPROP_STATE_INPUT_BOUND)[0])
        assert l1.max() <= bound <= l1.max() * 1.001 * (1 + 1e-6), (it, bound, l1.max())
    net.close()


def _train_form(wl, form, bs, iterations, T, max_delay=None, forced_rate=None):
    """FP32 training on one handle with the given scatter form: per
    iteration the losses, every trial's spikes, the gradients and the
    weights after the update."""
    net = E.Network(wl.network, "fp32", max_trials=bs, max_steps=T, max_delay=max_delay, scatter_form=form)
    lay = net.layout()
    assert lay["queues"] == (1 if form == "queues" else 0) and lay["tiles"] > 1, (form, lay)
    h = {"loss": [], "spikes": [], "grads": [], "weights": [], "events": 0, "rec_spikes": 0}
    for it in range(iterations):
        b = wl.make_batch(it, 0, bs)
        if forced_rate:
            b = W.forced_poisson(b, wl.network.n_rec, forced_rate, wl.network.params.dt, seed=17, iteration=it,
                                 n_ref=2)
        r = net.simulate(b, train=True)
        h["events"] += r.n_syn_events
        h["rec_spikes"] += r.n_rec_spikes
        h["loss"].append(r.loss.copy())
        h["spikes"].append([net.read(E.EPROP_STATE_SPIKES, i) for i in range(bs)])
        h["grads"].append(net.grads())
        net.apply()
        h["weights"].append(net.weights())
    net.close()
    return h, lay


def _assert_same_training(a, b, what):
    assert a["events"] == b["events"] and a["rec_spikes"] == b["rec_spikes"] > 0, (what, a["events"], b["events"])
    for it in range(len(a["loss"])):
        assert np.array_equal(a["loss"][it], b["loss"][it]), (what, it)
        for i, (sa, sb) in enumerate(zip(a["spikes"][it], b["spikes"][it])):
            assert np.array_equal(sa, sb), (what, it, i)
        for k in KEYS:
            assert np.array_equal(a["grads"][it][k], b["grads"][it][k]), (what, it, k)
            assert np.array_equal(a["weights"][it][k], b["weights"][it][k]), (what, it, k)


@pytest.mark.parametrize("name", ["c5twin", "c4twin"])
def test_queues_and_lookup_deliver_the_same(name):
    """Scatter delivery through the per-tile queues (each spiking neuron's
    tile copies its synapses into one queue per target tile) against
    delivery by lookup (each tile looks up every spiking source), FP32, free
    running, three iterations with updates: the input currents are the same
    fixed-point sums however the arrivals are ordered, so spikes, losses,
    gradients and weights agree bit for bit.  The lookup form is held to
    the oracle by the other FP32 tests.  The twin of the million-neuron
    network takes the queues by default (rows sparse across tiles); the C4
    twin (rows dense within tiles) forces them."""
    if name == "c5twin":
        wl, bs, T, md = _c5_twin(), 1, 200, C5_TWIN_RING_STEPS
    else:
        wl, bs, T, md = W.c4_sparse(n_rec=2000, n_steps=200, batch_size=2, n_in=300), 2, 200, None
    hq, lay = _train_form(wl, "queues", bs, 3, T, md)
    hl, _ = _train_form(wl, "lookup", bs, 3, T, md)
    log(f"{name}: {hq['events']} events; queue layout {lay}")
    if name == "c5twin":
        net = E.Network(wl.network, "fp32", max_trials=bs, max_steps=T, max_delay=md)
        assert net.layout()["queues"] == 1
        net.close()
    _assert_same_training(hq, hl, name)


def test_queue_tags_across_many_batches():
    """The queues' step tags are 16 bits wide and every forward pass takes
    fresh ones, so after 65535 steps the library clears the queues and
    starts over.  Seventy batches of 1000 steps on a handle with the queues
    forced (four tiles) cross that point; every batch's loss and spike
    count equal those of a handle delivering by lookup."""
    wl = W.c4_sparse(n_rec=2048, n_steps=1000, batch_size=1, n_in=200)
    nets = [E.Network(wl.network, "fp32", max_trials=1, max_steps=1000, scatter_form=f) for f in ("queues", "lookup")]
    assert nets[0].layout()["queues"] == 1 and nets[0].layout()["tiles"] > 1
    assert nets[1].layout()["queues"] == 0
    for it in range(70):
        b = wl.make_batch(it, 0, 1)
        rq, rl = nets[0].simulate(b), nets[1].simulate(b)
        assert rq.n_rec_spikes == rl.n_rec_spikes > 0 and rq.n_syn_events == rl.n_syn_events, it
        assert np.array_equal(rq.loss, rl.loss), it
    assert np.array_equal(nets[0].read(E.EPROP_STATE_SPIKES, 0), nets[1].read(E.EPROP_STATE_SPIKES, 0))
    for net in nets:
        net.close()


def test_queue_form_rejected_where_it_does_not_apply():
    """EPROP_SCATTER_QUEUES needs FP32 scatter delivery with more than one
    tile per trial: FP64 and a single-tile network are refused with
    EPROP_ERR_UNSUPPORTED."""
    for wl, prec in ((W.c4_sparse(n_rec=2048, n_steps=50, batch_size=1, n_in=100), "fp64"), (W.tiny(), "fp32")):
        with pytest.raises(E.EpropError) as ex:
            E.Network(wl.network, prec, max_trials=1, max_steps=50, scatter_form="queues")
        assert ex.value.status == E.EPROP_ERR_UNSUPPORTED


def test_full_size_million_neuron_network_sampled():
    """The million-neuron network (10^6 neurons, 20% ALIF, in-degree 100,
    delays 1..5, one 2000-step trial) in the benchmark's launch configuration
    (FP32, autotuner on, 32-bit ring, target-major update), teacher-forced at
    5 Hz: the gradients of every incoming synapse of 24 sampled neurons and of
    every output synapse against the oracle's per-neuron evaluation
    (check_fp32_batch), the loss within 1e-12."""
    wl = W.c5_million()
    b = W.forced_poisson(wl.make_batch(0, 0, 1), wl.network.n_rec, 5.0, 1.0, seed=7, n_ref=2)
    net = E.Network(wl.network, "fp32", max_trials=1, max_steps=2000, autotune=True)
    lay = net.layout()
    assert lay["ring_bytes"] == 4 and lay["blocked_update"] == 0, lay
    w0 = net.weights()
    quantum = ring_quantum(net)
    r = net.simulate(b, train=True)
    G = net.grads()
    psis = read_psis(net, b)
    lay = net.layout()
    net.close()
    assert lay["autotuned"] == 1
    log(f"gpu done: {r.n_rec_spikes} spikes, {r.n_syn_events} events, layout {lay}")
    rng = np.random.default_rng(2)
    alif = np.flatnonzero(wl.network.is_alif)
    lif = np.flatnonzero(wl.network.is_alif == 0)
    targets = np.sort(np.concatenate([rng.choice(lif, 16, replace=False), rng.choice(alif, 8, replace=False)]))
    check_fp32_batch("million", wl.network, b, psis, G, w0, quantum=quantum, targets=targets)
    loss = O.forced_sampled(oracle_at(wl.network, w0), b, 0, targets[:1])[0]
    assert abs(r.loss[0] - loss) <= 1e-12 * abs(loss), (r.loss[0], loss)


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


def test_forward_launches_in_chunks_of_resident_trials():
    """A batch whose tiles do not all fit on the device at once (200 trials
    of a 6000-neuron network: 2 tiles per trial, one per CU) runs the
    forward pass in consecutive launches of as many trials as are resident
    together, so no trial waits on tiles that are not running.  Every
    trial's loss and spikes equal those of the same trial run in a batch of 8
    on a handle of the same layout, where it sits in the first launch (trials
    0..7 and 192..199, the latter in the big batch's second launch), and the
    gradient of the 200 trials equals the sum over 25 batches of 8 (FP32
    input currents are fixed-point sums, so results do not depend on the
    batch)."""
    wl = W.c4_sparse(n_rec=6000, n_steps=60, batch_size=200, n_in=300)
    big = wl.make_batch(0, 0, 200)
    net = E.Network(wl.network, "fp32", max_trials=200, max_steps=60)
    lay = net.layout()
    log(f"layout {lay}")
    assert lay["tiles"] > 1
    assert lay["forward_trials_per_launch"] < 192
    r = net.simulate(big)
    spikes = [net.read(E.EPROP_STATE_SPIKES, i) for i in range(200)]
    g = net.grads()
    net.close()
    net = E.Network(wl.network, "fp32", max_trials=200, max_steps=60)
    assert net.layout() == lay
    for c in range(0, 200, 8):     # no update between the calls: the gradient sums accumulate
        part = wl.make_batch(0, c, 8)
        rp = net.simulate(part)
        assert np.array_equal(rp.loss, r.loss[c:c + 8]), c
        for i in range(8):
            assert np.array_equal(net.read(E.EPROP_STATE_SPIKES, i), spikes[c + i]), (c, i)
    gsum = net.grads()
    net.close()
    for k in KEYS:
        ok, e, ent = rel_close(g[k], gsum[k], 1e-6)
        assert ok, (k, e, ent)


def test_gradients_restart_after_an_update():
    """After an update the accumulated gradient reads as zero, and the next
    training batch's gradient is that batch's alone (the first batch after an
    update writes the gradient pairs instead of adding to them): the
    event-driven and the time-driven gradient of the next (teacher-forced)
    batch, each checked against the oracle at the updated weights
    (check_fp32_batch), in the blocked-update layout."""
    wl = W.c4_sparse(n_rec=3000, n_steps=300, batch_size=2, n_in=300)
    forced = [W.forced_poisson(wl.make_batch(i, 0, 2), wl.network.n_rec, 10.0, 1.0, seed=11, iteration=i, n_ref=2)
              for i in range(2)]
    for time_driven in (False, True):
        net = E.Network(wl.network, "fp32", max_trials=2, max_steps=300)
        net.simulate(forced[0])
        g0 = net.grads()
        assert all(np.abs(g0[k]).max() > 0 for k in KEYS)
        net.apply()
        gz = net.grads()
        for k in ("w_in", "w_rec"):
            assert not np.any(gz[k]), k
        w1 = net.weights()
        net.simulate(forced[1], time_driven=time_driven)
        check_fp32_batch(f"restart {'time' if time_driven else 'event'}-driven", wl.network, forced[1],
                         read_psis(net, forced[1]), net.grads(), w1,
                         downstream=(7.0 + 5.0 * 300) / 7.0 if time_driven else 1.0)
        net.close()


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
    """FP32 time-driven gradient with teacher-forced spike trains against the
    oracle at the GPU's weights (check_fp32_batch with the time-driven
    recursion's rounding), its loss and its update."""
    fp32_forced_run("c3 time-driven", W.c3_events(batch_size=3), 1, 3, time_driven=True)


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
    """FP32 with teacher-forced spike trains, d = 2, d^ls = 3, regulariser on:
    every iteration's gradient, loss and update checked against the oracle at
    the GPU's weights (event-driven path, two iterations; time-driven path,
    one)."""
    wl, bs = _delayed(name, 2, 3, 1e3)
    fp32_forced_run(f"{name} delays+reg", wl, 2, bs)
    wl, bs = _delayed(name, 2, 3, 1e3)
    fp32_forced_run(f"{name} delays+reg time-driven", wl, 1, bs, time_driven=True)


# ----------------------------------------------------------------- the scaling network

def _scaling_twin():
    return W.scaling(n_rec=3000, indeg_rec=500, n_in=100, indeg_in=10, indeg_out=100, outdeg_fb=30, n_steps=400,
                     samples=4)


def test_scaling_twin_fp64_exact_and_fp32():
    """Twin of the scaling network (Methods, "Scaling": ignore-and-fire
    neurons at 5 Hz, fixed in-degree, sparse readout and feedback): FP64
    exact against the oracle over consecutive samples; FP32 (its spike trains
    are fixed by construction, so it is teacher-forced) checked against the
    oracle at the GPU's weights every sample (check_fp32_batch)."""
    wl = _scaling_twin()
    oh = oracle_train(wl, 2, 1)
    gh = gpu_train(wl, "fp64", 2, 1)
    assert_fp64_parity(gh, oh, "scaling twin")
    fp32_forced_run("scaling twin", wl, 2, 1, rate=None)


def test_scaling_network_launch_configuration_sampled():
    """The scaling network at its full neuron count (128,000 ignore-and-fire
    neurons, one 1000-step sample, FP32, the tile layout of the benchmark)
    with recurrent in-degree 100 instead of 10^4 so that it builds in seconds:
    all 640,000 forced spikes are emitted, and the gradients of every
    incoming synapse of 24 sampled neurons and of every output synapse are
    checked against the oracle's per-neuron evaluation (check_fp32_batch),
    the loss within 1e-12."""
    wl = W.scaling(indeg_rec=100)
    b = wl.make_batch(0, 0, 1)
    net = E.Network(wl.network, "fp32", max_trials=1, max_steps=1000)
    w0 = net.weights()
    r = net.simulate(b, train=True)
    G = net.grads()
    psis = read_psis(net, b)
    lay = net.layout()
    net.close()
    log(f"gpu done: layout {lay}, {r.n_rec_spikes} spikes, {r.n_syn_events} events")
    assert r.n_rec_spikes == 640_000
    targets = np.sort(np.random.default_rng(1).choice(wl.network.n_rec, 24, replace=False))
    check_fp32_batch("scaling", wl.network, b, psis, G, w0, targets=targets)
    loss = O.forced_sampled(oracle_at(wl.network, w0), b, 0, targets[:1])[0]
    assert abs(r.loss[0] - loss) <= 1e-12 * abs(loss), (r.loss[0], loss)


def test_fp32_adam_state_and_input_bound_after_updates():
    """Evidence accumulation with Adam (eq. eta-adam-fast, eq. delta-w-adam-fast),
    FP32, teacher-forced, three iterations: each iteration's gradient against
    the oracle at the GPU's weights, and the weights and both moments read
    back in the caller's synapse order equal to the oracle's Adam step from
    the GPU's gradient and state, rounded once to FP32 (fp32_forced_run);
    the per-target input bound the update recomputes stays above the largest
    sum of |w| into one target."""
    wl = W.c2_evidence(batch_size=4)
    assert wl.network.params.optimizer == 1
    fp32_forced_run("c2 adam", wl, 3, 4)
    T = max(int(wl.make_batch(i, 0, 4).n_steps.max()) for i in range(3))
    net = E.Network(wl.network, "fp32", max_trials=4, max_steps=T)
    for it in range(3):
        net.simulate(W.forced_poisson(wl.make_batch(it, 0, 4), wl.network.n_rec, 20.0, 1.0, seed=99, iteration=it,
                                      n_ref=2), train=True)
        net.apply()
    w = net.weights()
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
    """FP32 with teacher-forced spike trains and every e-prop+ component on
    (full reset, decoupled filter, moving-average regulariser, temporal MSE,
    d = 1): each iteration's gradient, loss and update checked against the
    oracle at the GPU's weights (fp32_forced_run)."""
    wl, bs = _plus(name, d_out=1)
    fp32_forced_run(f"{name} e-prop+", wl, 2, bs)


# ----------------------------------------------------------------- e-prop+ update schedule

def _online_pair(wl, precision, b, eta):
    """The GPU's and the oracle's online run of the batch's trials back to back."""
    T = int(b.n_steps.sum())
    net = E.Network(wl.network, precision, max_trials=1, max_steps=T)
    w0 = net.weights()
    r = net.simulate(b, online=True)
    g = {"loss": r.loss.copy(), "z": net.spikes(0, T), "w": net.weights(), "w0": w0, "events": r.n_syn_events}
    net.close()
    # the oracle starts from the library's initial weights (FP32 values in FP32 mode)
    on = oracle_at(wl.network, w0) if precision == "fp32" else O.OracleNet(wl.network)
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
    trains fixed by construction, so FP32 sees the oracle's spikes), both
    runs from the library's FP32 initial weights: the weight changes within
    1e-4 of the FP64 oracle's, normwise, and every entry within
    1e-4 max(|change|, 1e-3 of the largest) plus the FP32 rounding of the
    weight at each of its updates (at most 32 here) plus (7 + 5 C) u times
    the absolute term sum of its updates (the oracle's "abs"): the FP32
    eligibility recursions round at most 5 times per step and restart C
    (the cutoff) steps after an arrival at the latest, so a term carries at
    most 5 C u, and the stored learning signal, rates and sums 7 u; the
    FP32 error of psi (within 0.36 of its running bound, tens of u,
    wherever the batched tests compare it) is within that margin."""
    wl = _scaling_twin()
    p = wl.network.params
    p.eta, p.d_out, p.isi_cutoff = 1e-4, 1, 100
    b = wl.make_batch(0, 0, 2)
    g, o = _online_pair(wl, "fp32", b, p.eta)
    assert np.array_equal(g["z"], o["z"])
    w0 = g["w0"]
    for k in KEYS:
        dg = g["w"][k].ravel() - w0[k].ravel()
        do = o["w"][k].ravel() - w0[k].ravel()
        ok, e, ent = rel_close(dg, do, 1e-4)
        log(f"online fp32 {k}: change normwise {e:.2e} worst {ent:.2e}")
        assert e <= 1e-4, (k, e)
        bound = (1e-4 * np.maximum(np.abs(do), 1e-3 * np.abs(do).max()) + 32 * U32 * np.abs(o["w"][k].ravel())
                 + (7 + 5 * p.isi_cutoff) * U32 * o["abs"][k].ravel())
        dev = np.abs(dg - do)
        log(f"online fp32 {k}: entry/bound {float((dev / bound).max()):.3f}")
        assert np.all(dev <= bound), (k, float(np.max(dev / bound)))


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
