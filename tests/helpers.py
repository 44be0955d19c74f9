"""Small hand-built networks and comparison metrics shared by the tests."""
import numpy as np

from paper_2511_21674_amd import workloads as W


def proj_from_pairs(n_src, n_tgt, pairs):
    """pairs: list of (src, tgt, w, delay) -> CSR-by-source Projection."""
    if not pairs:
        return W.Projection(n_src, n_tgt, np.zeros(n_src + 1, np.uint64), np.zeros(0, np.uint32),
                            np.zeros(0), np.zeros(0, np.uint8))
    src = np.array([p[0] for p in pairs])
    tgt = np.array([p[1] for p in pairs])
    w = np.array([p[2] for p in pairs], dtype=np.float64)
    d = np.array([p[3] for p in pairs], dtype=np.uint8)
    return W._csr_from_pairs(n_src, n_tgt, src, tgt, w, d)


def small_net(n_in, n_rec, n_out, in_pairs, rec_pairs, w_out=None, fb=None, is_alif=None, **params):
    prm = W.Params(**params)
    w_out = np.ones((n_out, n_rec)) if w_out is None else np.asarray(w_out, dtype=np.float64)
    fb = np.ones((n_rec, n_out)) if fb is None else np.asarray(fb, dtype=np.float64)
    ia = np.zeros(n_rec, np.uint8) if is_alif is None else np.asarray(is_alif, np.uint8)
    return W.Network(n_in, n_rec, n_out, ia, prm, proj_from_pairs(n_in, n_rec, in_pairs),
                     proj_from_pairs(n_rec, n_rec, rec_pairs), w_out, fb)


def batch_from(n_steps, in_spikes, n_out, target=None, label=None, window=None, forced=None):
    """in_spikes: list of (emission step, src); forced: list of (step, neuron)."""
    sp = sorted(in_spikes)
    b = W.Batch(n_steps=np.array([n_steps], np.uint32),
                in_ptr=np.array([0, len(sp)], np.uint64),
                in_step=np.array([s for s, _ in sp], np.uint32),
                in_src=np.array([i for _, i in sp], np.uint32))
    b.target = np.zeros((1, n_steps, n_out)) if target is None else np.asarray(target, float).reshape(1, n_steps, n_out)
    b.label = np.array([0 if label is None else label], np.uint32)
    if window is not None:
        b.window = np.asarray(window, np.uint8).reshape(1, n_steps)
    if forced is not None:
        fs = sorted(forced)
        b.forced_ptr = np.array([0, len(fs)], np.uint64)
        b.forced_step = np.array([s for s, _ in fs], np.uint32)
        b.forced_neuron = np.array([j for _, j in fs], np.uint32)
    return b


def rel_close(a, b, tol, floor_frac=1e-3):
    """Normwise ||a-b|| <= tol ||b|| and every entry |a-b| <= tol*max(|b|, floor*||b||_inf).
    Returns (ok, normwise error, worst entry ratio)."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    if nb == 0:
        return bool(np.all(a == 0)), float(np.linalg.norm(a)), 0.0
    nerr = np.linalg.norm(a - b) / nb
    scale = np.maximum(np.abs(b), floor_frac * np.abs(b).max())
    ent = np.abs(a - b) / scale
    return bool(nerr <= tol and ent.max() <= tol), float(nerr), float(ent.max())


def prediction_case(loss, variant="main"):
    """A constructed classification trial whose predicted class is known by
    construction, with teacher-forced spikes (the readout does not feed back
    into the spikes).  Readout k sums w_out[k, j] z_j; tau_out = 1 ms, so the
    readout follows its input within a few steps.  Window: steps 301..400 of 400.

      readout 0 ("C"): neuron 41 (w 5) spikes at every step 1..250, before
          the window: it dominates every sum taken over the whole trial;
      readout 1 ("A"): neurons 0..39 (w 1 each) spike at steps 360..362: a
          tall, short peak (y up to about 60) whose window sum of y (about
          190) is the largest, while its softmax saturates at 1 for only a few
          steps;
      readout 2 ("B"): neuron 40 (w 0.63) spikes at every step 300..400: a
          flat y of about 1 over the window (window sum about 100), whose
          softmax share e/(e + 2) = 0.58 over about 93 steps makes the
          largest window sum of pi (about 54 against about 27 for A).

    Classification losses predict the arg max over k of the window-summed pi
    (softmax cross-entropy) or y (temporal MSE), lowest index on ties:
      main:   CE -> 2, temporal MSE -> 1.  A window ignored gives 0, CE
              summing y gives 1, temporal MSE summing pi gives 2;
      silent: no spikes at all, every sum equal -> 0 (first index);
      tie:    readouts 1 and 2 both receive the flat train of neuron 40
              (w 0.63) and nothing else, readout 0 nothing: 1 and 2 tie
              exactly above 0 -> 1.
    Returns (network, batch, expected class)."""
    T, K, J = 400, 3, 42
    w_out = np.zeros((K, J))
    if variant == "tie":
        w_out[1, 40] = w_out[2, 40] = 0.63
    else:
        w_out[1, :40] = 1.0
        w_out[2, 40] = 0.63
        w_out[0, 41] = 5.0
    forced = []
    if variant != "silent":
        forced += [(t, 40) for t in range(300, 401)]
        if variant == "main":
            forced += [(t, j) for t in (360, 361, 362) for j in range(40)]
            forced += [(t, 41) for t in range(1, 251)]
    window = np.zeros(T, np.uint8)
    window[300:] = 1
    net = small_net(1, J, K, [(0, 0, 1e-3, 1)], [(0, 1, 1e-3, 1)], w_out=w_out,
                    fb=np.ones((J, K)) * 0.1, tau_out=1.0, loss=loss)
    b = batch_from(T, [], K, label=0, window=window, forced=forced or [(1, 40)])
    if variant == "silent":
        b.forced_ptr = np.array([0, 0], np.uint64)
        b.forced_step = np.zeros(0, np.uint32)
        b.forced_neuron = np.zeros(0, np.uint32)
    expected = {"main": {1: 2, 2: 1}, "silent": {1: 0, 2: 0}, "tie": {1: 1, 2: 1}}[variant][loss]
    return net, b, expected
