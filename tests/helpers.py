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
