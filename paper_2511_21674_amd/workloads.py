"""Seeded synthetic workloads for event-driven e-prop.

This module holds none of the learning method's arithmetic. It only draws
random graphs, initial weights, feedback weights, Poisson spike trains,
regression targets, class labels and learning-window masks. The HIP path
and the CPU oracle both consume its arrays unchanged, so that any trial can
be regenerated alone from (seed, purpose, iteration, trial).

Shapes and statistics follow the paper's tasks (Methods, "Tasks": pattern
generation, evidence accumulation, N-MNIST; "Scaling": sparse fixed
in-degree networks) with synthetic stand-ins where the paper used data that
is not available (N-MNIST is replaced by moving-blob event-camera samples).

Conventions shared by both consumers:
  * time steps of a trial are t = 1..T; the network state at t = 0 is zero;
  * every presynaptic source (input channel or recurrent neuron) emits
    spikes at integer steps; a synapse with delay D delivers a spike emitted
    at step s at step s + D (D >= 1).  Input emission steps lie in [0, T-1];
  * projections are CSR by source: row_ptr[n_src+1] (uint64), col (uint32
    target index), w (float64), delay (uint8, >= 1);
  * w_out is [K, J] (row k holds the weights into readout k), feedback B is
    [J, K];
  * target is [B, T_max, K] float64 (entry t-1 is the target at step t),
    label is [B] uint32, window is [B, T_max] uint8 (1 = learning window
    open at that step).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Callable, Optional

import numpy as np

SEED_BASE = 2511216740

# purposes for independent random streams
_P_GRAPH_IN, _P_GRAPH_REC, _P_W_IN, _P_W_REC, _P_W_OUT, _P_FEEDBACK = 1, 2, 3, 4, 5, 6
_P_DELAY_IN, _P_DELAY_REC, _P_ALIF, _P_TEMPLATE = 7, 8, 9, 10
_P_INPUT, _P_TARGET, _P_TASK, _P_FORCED = 20, 21, 22, 23


def rng(seed: int, *path: int) -> np.random.Generator:
    """Counter-style stream: one PCG64 per (seed, purpose, iteration, trial...)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), *map(int, path)])))


@dataclass
class Params:
    """Neuron, readout and optimiser constants (times in ms)."""
    dt: float = 1.0
    tau_m: float = 20.0
    tau_out: float = 20.0
    v_th: float = 0.6
    t_ref: float = 2.0
    tau_a: float = 2000.0
    beta_a: float = 0.0
    surrogate: int = 0          # 0 piecewise linear, 1 exponential
    sg_gamma: float = 0.3 / 0.6  # gamma_original / v_th
    sg_beta: float = 1.0 / 0.6   # 1 / v_th
    loss: int = 0               # 0 mean squared error, 1 softmax cross-entropy, 2 temporal MSE on the label
    optimizer: int = 0          # 0 gradient descent, 1 Adam
    eta: float = 1e-3
    adam_beta1: float = 0.9
    adam_beta2: float = 0.999
    adam_eps_hat: float = 1e-7
    max_delay: int = 1
    d_out: int = 0              # delay from the recurrent to the output layer (steps)
    d_ls: int = 0               # delay of the learning signal (steps)
    c_reg: float = 0.0          # firing-rate regularisation strength
    f_target_hz: float = 0.0    # its target rate
    reg_mode: int = 0           # 0 static rate over the sample, 1 exponential moving average
    reg_tau: float = 0.0        # the moving average's time constant (ms)
    reset_mode: int = 0         # 0 subtract the threshold, 1 reset the membrane to v_reset
    v_reset: float = 0.0
    etrace_filter: int = 0      # eligibility filter: 0 tau_out, 1 its own tau_e, 2 none
    tau_e: float = 0.0
    isi_cutoff: int = 0         # e-prop+ schedule: eligibility steps kept after an arrival (0: all)


@dataclass
class Projection:
    n_src: int
    n_tgt: int
    row_ptr: np.ndarray   # uint64 [n_src+1]
    col: np.ndarray       # uint32 [nnz]
    w: np.ndarray         # float64 [nnz]
    delay: np.ndarray     # uint8 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


@dataclass
class Network:
    n_in: int
    n_rec: int
    n_out: int
    is_alif: np.ndarray    # uint8 [n_rec]
    params: Params
    in_rec: Projection
    rec_rec: Projection
    w_out: np.ndarray      # float64 [K, J]
    feedback: np.ndarray   # float64 [J, K]


@dataclass
class Batch:
    n_steps: np.ndarray              # uint32 [B]
    in_ptr: np.ndarray               # uint64 [B+1]
    in_step: np.ndarray              # uint32 emission steps, sorted by (step, src) per trial
    in_src: np.ndarray               # uint32
    target: Optional[np.ndarray] = None   # float64 [B, T_max, K]
    label: Optional[np.ndarray] = None    # uint32 [B]
    window: Optional[np.ndarray] = None   # uint8 [B, T_max]
    forced_ptr: Optional[np.ndarray] = None    # uint64 [B+1]
    forced_step: Optional[np.ndarray] = None   # uint32, steps 1..T, sorted by (step, neuron)
    forced_neuron: Optional[np.ndarray] = None  # uint32

    @property
    def n_trials(self) -> int:
        return int(self.n_steps.shape[0])

    @property
    def t_max(self) -> int:
        return int(self.n_steps.max()) if self.n_steps.size else 0

    def trial(self, b: int) -> "Batch":
        """The single-trial batch holding trial b of this batch."""
        lo, hi = int(self.in_ptr[b]), int(self.in_ptr[b + 1])
        t = int(self.n_steps[b])
        out = Batch(n_steps=self.n_steps[b:b + 1].copy(),
                    in_ptr=np.array([0, hi - lo], dtype=np.uint64),
                    in_step=self.in_step[lo:hi].copy(), in_src=self.in_src[lo:hi].copy())
        if self.target is not None:
            out.target = np.ascontiguousarray(self.target[b:b + 1, :t])
        if self.label is not None:
            out.label = self.label[b:b + 1].copy()
        if self.window is not None:
            out.window = np.ascontiguousarray(self.window[b:b + 1, :t])
        if self.forced_ptr is not None:
            flo, fhi = int(self.forced_ptr[b]), int(self.forced_ptr[b + 1])
            out.forced_ptr = np.array([0, fhi - flo], dtype=np.uint64)
            out.forced_step = self.forced_step[flo:fhi].copy()
            out.forced_neuron = self.forced_neuron[flo:fhi].copy()
        return out


@dataclass
class Workload:
    name: str
    network: Network
    make_batch: Callable[[int, int, int], Batch]   # (iteration, first_trial, n_trials)
    batch_size: int
    iterations: int
    description: str = ""
    info: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# graphs and weights

def _csr_from_pairs(n_src: int, n_tgt: int, src: np.ndarray, tgt: np.ndarray,
                    w: np.ndarray, delay: np.ndarray) -> Projection:
    """CSR by source; within a row, targets ascending (pairs are unique)."""
    order = np.lexsort((tgt, src))
    src_s = src[order]
    counts = np.bincount(src_s, minlength=n_src).astype(np.uint64)
    row_ptr = np.zeros(n_src + 1, dtype=np.uint64)
    np.cumsum(counts, out=row_ptr[1:])
    return Projection(n_src, n_tgt, row_ptr, tgt[order].astype(np.uint32),
                      np.ascontiguousarray(w[order], dtype=np.float64),
                      np.ascontiguousarray(delay[order], dtype=np.uint8))


def dense_projection(n_src: int, n_tgt: int, std: float, g: np.random.Generator,
                     no_self: bool = False, delay: int = 1) -> Projection:
    src, tgt = np.meshgrid(np.arange(n_src), np.arange(n_tgt), indexing="ij")
    src, tgt = src.ravel(), tgt.ravel()
    if no_self:
        keep = src != tgt
        src, tgt = src[keep], tgt[keep]
    w = g.normal(0.0, std, size=src.size)
    return _csr_from_pairs(n_src, n_tgt, src, tgt, w, np.full(src.size, delay, np.uint8))


def bernoulli_projection(n_src: int, n_tgt: int, p: float, std: float, g: np.random.Generator,
                         no_self: bool = False, delay: int = 1) -> Projection:
    mask = g.random((n_src, n_tgt)) < p
    if no_self:
        np.fill_diagonal(mask, False)
    src, tgt = np.nonzero(mask)
    w = g.normal(0.0, std, size=src.size)
    return _csr_from_pairs(n_src, n_tgt, src, tgt, w, np.full(src.size, delay, np.uint8))


def fixed_indegree_projection(n_src: int, n_tgt: int, indegree: int, std: float,
                              g_graph: np.random.Generator, g_w: np.random.Generator,
                              g_delay: np.random.Generator, no_self: bool,
                              delay_lo: int = 1, delay_hi: int = 1) -> Projection:
    """Each target draws `indegree` distinct sources (no multapses, no autapses if
    no_self).  Distinct draws: sorted uniform draws from [0, n - m] plus 0..m-1."""
    n = n_src - 1 if no_self else n_src
    m = indegree
    if m > n:
        raise ValueError("in-degree larger than the number of candidate sources")
    chunk = max(1, (1 << 24) // max(m, 1))
    srcs = np.empty((n_tgt, m), dtype=np.int64)
    for lo in range(0, n_tgt, chunk):
        hi = min(n_tgt, lo + chunk)
        d = g_graph.integers(0, n - m + 1, size=(hi - lo, m), dtype=np.int64)
        d.sort(axis=1)
        d += np.arange(m, dtype=np.int64)
        if no_self:
            tg = np.arange(lo, hi, dtype=np.int64)[:, None]
            d += (d >= tg)
        srcs[lo:hi] = d
    tgt = np.repeat(np.arange(n_tgt, dtype=np.int64), m)
    src = srcs.ravel()
    del srcs
    w = g_w.normal(0.0, std, size=src.size)
    delay = g_delay.integers(delay_lo, delay_hi + 1, size=src.size).astype(np.uint8)
    # counting sort by source; the stable order keeps targets ascending per row
    order = np.argsort(src, kind="stable")
    counts = np.bincount(src, minlength=n_src).astype(np.uint64)
    row_ptr = np.zeros(n_src + 1, dtype=np.uint64)
    np.cumsum(counts, out=row_ptr[1:])
    return Projection(n_src, n_tgt, row_ptr, tgt[order].astype(np.uint32),
                      np.ascontiguousarray(w[order]), np.ascontiguousarray(delay[order]))


def fixed_indegree_lean(n_src: int, n_tgt: int, indegree: int, std: float,
                        g_graph: np.random.Generator, g_w: np.random.Generator,
                        no_self: bool, delay: int = 1) -> Projection:
    """Fixed in-degree projection for graphs of 10^9 synapses: the same distinct
    sorted draws per target as fixed_indegree_projection, placed into CSR by
    source chunk by chunk (targets ascending within a row) without a global
    permutation; weights are drawn directly in CSR order (they are i.i.d.),
    delays are all `delay`."""
    n = n_src - 1 if no_self else n_src
    m = indegree
    if m > n:
        raise ValueError("in-degree larger than the number of candidate sources")
    chunk = max(1, (1 << 24) // max(m, 1))
    counts = np.zeros(n_src, dtype=np.int64)
    draws = []
    for lo in range(0, n_tgt, chunk):
        hi = min(n_tgt, lo + chunk)
        d = g_graph.integers(0, n - m + 1, size=(hi - lo, m), dtype=np.int64)
        d.sort(axis=1)
        d += np.arange(m, dtype=np.int64)
        if no_self:
            d += (d >= np.arange(lo, hi, dtype=np.int64)[:, None])
        d32 = d.astype(np.uint32)
        del d
        counts += np.bincount(d32.ravel(), minlength=n_src)
        draws.append(d32)
    row_ptr = np.zeros(n_src + 1, dtype=np.uint64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.empty(int(row_ptr[-1]), dtype=np.uint32)
    fill = row_ptr[:-1].astype(np.int64)
    for ci, lo in enumerate(range(0, n_tgt, chunk)):
        d32 = draws[ci]
        rows = d32.shape[0]
        key = np.sort(d32.ravel().astype(np.uint64) * np.uint64(rows)
                      + np.repeat(np.arange(rows, dtype=np.uint64), m))
        draws[ci] = None
        src = (key // np.uint64(rows)).astype(np.int64)
        tl = (key % np.uint64(rows)).astype(np.uint32)
        del key
        first = np.flatnonzero(np.r_[True, src[1:] != src[:-1]])
        cnt = np.diff(np.r_[first, src.size])
        rank = np.arange(src.size, dtype=np.int64) - np.repeat(first, cnt)
        col[fill[src] + rank] = tl + np.uint32(lo)
        fill[src[first]] += cnt
    w = np.empty(col.size, dtype=np.float64)
    step = 1 << 26
    for lo in range(0, col.size, step):
        w[lo:lo + step] = g_w.normal(0.0, std, size=min(step, col.size - lo))
    return Projection(n_src, n_tgt, row_ptr, col, w, np.full(col.size, delay, dtype=np.uint8))


# --------------------------------------------------------------------------
# spike trains and targets

def poisson_steps(g: np.random.Generator, p: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Bernoulli spikes with per-(step, channel) probability p[T, C] at emission
    steps 0..T-1; returns (steps, channels) sorted by (step, channel)."""
    hit = g.random(p.shape) < p
    s, c = np.nonzero(hit)
    return s.astype(np.uint32), c.astype(np.uint32)


def sinusoid_sum(g: np.random.Generator, n_steps: int, dt_ms: float,
                 freqs=(0.5, 1.0, 2.0, 5.0)) -> np.ndarray:
    """Sum of sinusoids with amplitudes U[0.5, 2] and phases U[0, 2pi), sampled
    at steps t = 1..T (time in seconds = t * dt / 1000)."""
    amp = g.uniform(0.5, 2.0, size=len(freqs))
    ph = g.uniform(0.0, 2 * np.pi, size=len(freqs))
    ts = np.arange(1, n_steps + 1) * dt_ms / 1000.0
    return sum(a * np.sin(2 * np.pi * f * ts + p) for a, f, p in zip(amp, freqs, ph))


def _assemble(trials: list, n_out: int, t_max: int, targets=None, labels=None, windows=None) -> Batch:
    n_steps = np.array([tr[0] for tr in trials], dtype=np.uint32)
    counts = [tr[1].size for tr in trials]
    in_ptr = np.zeros(len(trials) + 1, dtype=np.uint64)
    np.cumsum(counts, out=in_ptr[1:])
    in_step = np.concatenate([tr[1] for tr in trials]).astype(np.uint32) if trials else np.zeros(0, np.uint32)
    in_src = np.concatenate([tr[2] for tr in trials]).astype(np.uint32) if trials else np.zeros(0, np.uint32)
    b = Batch(n_steps=n_steps, in_ptr=in_ptr, in_step=in_step, in_src=in_src)
    if targets is not None:
        tg = np.zeros((len(trials), t_max, n_out), dtype=np.float64)
        for i, t in enumerate(targets):
            tg[i, :t.shape[0]] = t
        b.target = tg
    if labels is not None:
        b.label = np.asarray(labels, dtype=np.uint32)
    if windows is not None:
        wm = np.zeros((len(trials), t_max), dtype=np.uint8)
        for i, w in enumerate(windows):
            wm[i, :w.shape[0]] = w
        b.window = wm
    return b


def forced_poisson(batch: Batch, n_rec: int, rate_hz: float, dt_ms: float, seed: int,
                   iteration: int = 0, first_trial: int = 0, n_ref: int = 0) -> Batch:
    """Attach teacher-forced recurrent spike trains (steps 1..T, Bernoulli at
    rate_hz, with at least n_ref silent steps after each spike)."""
    ptr = [0]
    steps, neurons = [], []
    p = rate_hz * dt_ms / 1000.0
    for b in range(batch.n_trials):
        t = int(batch.n_steps[b])
        g = rng(seed, _P_FORCED, iteration, first_trial + b)
        hit = g.random((t, n_rec)) < p
        if n_ref > 0:
            last = np.full(n_rec, -10 ** 9)
            for s in range(t):
                ok = hit[s] & (s - last > n_ref)
                hit[s] = ok
                last[ok] = s
        s, j = np.nonzero(hit)
        steps.append((s + 1).astype(np.uint32))
        neurons.append(j.astype(np.uint32))
        ptr.append(ptr[-1] + s.size)
    out = replace(batch)
    out.forced_ptr = np.array(ptr, dtype=np.uint64)
    out.forced_step = np.concatenate(steps) if steps else np.zeros(0, np.uint32)
    out.forced_neuron = np.concatenate(neurons) if neurons else np.zeros(0, np.uint32)
    return out


# --------------------------------------------------------------------------
# the five workloads and the small brute-force network

def c1_pattern(seed: int = SEED_BASE + 1, n_steps: int = 1000, iterations: int = 10) -> Workload:
    """Pattern generation: 100 Poisson inputs at 10 Hz (frozen), 100 LIF
    neurons all-to-all without autapses, one leaky readout, MSE, GD 1e-3."""
    n_in, n_rec, n_out = 100, 100, 1
    prm = Params(loss=0, optimizer=0, eta=1e-3)
    net = Network(n_in, n_rec, n_out, np.zeros(n_rec, np.uint8), prm,
                  dense_projection(n_in, n_rec, 1 / np.sqrt(n_in), rng(seed, _P_W_IN)),
                  dense_projection(n_rec, n_rec, 1 / np.sqrt(n_rec), rng(seed, _P_W_REC), no_self=True),
                  rng(seed, _P_W_OUT).normal(0, 1 / np.sqrt(n_rec), (n_out, n_rec)),
                  rng(seed, _P_FEEDBACK).normal(0, 1 / np.sqrt(n_rec), (n_rec, n_out)))
    # frozen input pattern and target: independent of iteration and trial
    s, c = poisson_steps(rng(seed, _P_INPUT), np.full((n_steps, n_in), 10.0 * prm.dt / 1000.0))
    target = sinusoid_sum(rng(seed, _P_TARGET), n_steps, prm.dt)[:, None]

    def make_batch(iteration: int, first: int, n: int) -> Batch:
        return _assemble([(n_steps, s, c)] * n, n_out, n_steps, targets=[target] * n)
    return Workload("c1_pattern", net, make_batch, 1, iterations,
                    "pattern generation, 100 in / 100 LIF / 1 readout, FP64 plain")


def c2_evidence(seed: int = SEED_BASE + 2, batch_size: int = 256, iterations: int = 4) -> Workload:
    """Evidence accumulation: 4 input groups of 10 (left, right, recall, noise),
    50 LIF + 50 ALIF dense, 2 softmax readouts, window = recall, Adam."""
    n_in, n_rec, n_out = 40, 100, 2
    is_alif = np.zeros(n_rec, np.uint8)
    is_alif[50:] = 1
    prm = Params(beta_a=1.7, tau_a=2000.0, loss=1, optimizer=1, eta=5e-3)
    net = Network(n_in, n_rec, n_out, is_alif, prm,
                  dense_projection(n_in, n_rec, 1 / np.sqrt(n_in), rng(seed, _P_W_IN)),
                  dense_projection(n_rec, n_rec, 1 / np.sqrt(n_rec), rng(seed, _P_W_REC), no_self=True),
                  rng(seed, _P_W_OUT).normal(0, 1 / np.sqrt(n_rec), (n_out, n_rec)),
                  rng(seed, _P_FEEDBACK).normal(0, 1 / np.sqrt(n_rec), (n_rec, n_out)))
    dt = prm.dt

    def one_trial(iteration: int, trial: int):
        g = rng(seed, _P_TASK, iteration, trial)
        delta = int(g.integers(0, 601))
        t = int(round((1200 + delta) / dt))
        sides = g.integers(0, 2, size=7)
        p = np.zeros((t, n_in))
        ms = np.arange(t) * dt
        p[:, 30:40] = 10.0 * dt / 1000.0
        for k, side in enumerate(sides):
            on = (ms >= 150 * k) & (ms < 150 * k + 100)
            p[on, 10 * side:10 * side + 10] = 40.0 * dt / 1000.0
        recall = (ms >= 1050 + delta) & (ms < 1200 + delta)
        p[recall, 20:30] = 40.0 * dt / 1000.0
        s, c = poisson_steps(rng(seed, _P_INPUT, iteration, trial), p)
        label = int(sides.sum() > 3)  # 1 = right is the majority
        window = np.zeros(t, np.uint8)
        # emission step s is read at step s + 1: the window covers the recall period
        window[np.nonzero(recall)[0]] = 1
        return (t, s, c), label, window

    def make_batch(iteration: int, first: int, n: int) -> Batch:
        rows = [one_trial(iteration, first + i) for i in range(n)]
        t_max = max(r[0][0] for r in rows)
        return _assemble([r[0] for r in rows], n_out, t_max, labels=[r[1] for r in rows],
                         windows=[r[2] for r in rows])
    return Workload("c2_evidence", net, make_batch, batch_size, iterations,
                    "evidence accumulation, 40 in / 50 LIF + 50 ALIF / 2 softmax, batch 256")


def _blob_templates(seed: int, n_classes: int, n_steps: int, side: int = 34,
                    sigma: float = 3.0, travel: float = 15.0) -> np.ndarray:
    """Per-class event rates [C, T, 2*side*side]: a Gaussian blob moving in a
    random direction; ON events follow brightness increases, OFF decreases."""
    g = rng(seed, _P_TEMPLATE)
    yy, xx = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    out = np.zeros((n_classes, n_steps, 2 * side * side))
    for c in range(n_classes):
        c0 = side / 2 - 0.5 + g.uniform(-5, 5, size=2)
        th = g.uniform(0, 2 * np.pi)
        ts = np.arange(n_steps + 1) / n_steps
        cx = c0[0] + travel * ts * np.cos(th)
        cy = c0[1] + travel * ts * np.sin(th)
        img = np.exp(-((xx[None] - cx[:, None, None]) ** 2 + (yy[None] - cy[:, None, None]) ** 2)
                     / (2 * sigma ** 2))
        d = np.diff(img, axis=0).reshape(n_steps, -1)
        out[c, :, :side * side] = np.maximum(0, -d)   # OFF
        out[c, :, side * side:] = np.maximum(0, d)    # ON
    return out


def c3_events(seed: int = SEED_BASE + 3, batch_size: int = 128, iterations: int = 4,
              n_steps: int = 300) -> Workload:
    """Event-camera-shaped classification: 2312 channels, 180 LIF (p = 0.1
    recurrence), 10 softmax readouts, learning window = last 30 steps, GD."""
    side, n_classes = 34, 10
    n_in, n_rec, n_out = 2 * side * side, 180, 10
    prm = Params(loss=1, optimizer=0, eta=1e-3)
    net = Network(n_in, n_rec, n_out, np.zeros(n_rec, np.uint8), prm,
                  dense_projection(n_in, n_rec, 1 / np.sqrt(n_in), rng(seed, _P_W_IN)),
                  bernoulli_projection(n_rec, n_rec, 0.1, 1 / np.sqrt(18.0), rng(seed, _P_GRAPH_REC),
                                       no_self=True),
                  rng(seed, _P_W_OUT).normal(0, 1 / np.sqrt(n_rec), (n_out, n_rec)),
                  rng(seed, _P_FEEDBACK).normal(0, 1 / np.sqrt(n_rec), (n_rec, n_out)))
    tmpl = _blob_templates(seed, n_classes, n_steps, side)
    tmpl *= (4.0 * n_in) / tmpl.sum(axis=(1, 2), keepdims=True)   # 4 events per channel on average
    window = np.zeros(n_steps, np.uint8)
    window[-30:] = 1

    def one_trial(iteration: int, trial: int):
        g = rng(seed, _P_TASK, iteration, trial)
        label = int(g.integers(0, n_classes))
        dx, dy = g.integers(-3, 4, size=2)
        r = tmpl[label].reshape(n_steps, 2, side, side)
        r = np.roll(np.roll(r, int(dy), axis=2), int(dx), axis=3)
        if dy > 0:
            r[:, :, :dy] = 0
        elif dy < 0:
            r[:, :, dy:] = 0
        if dx > 0:
            r[:, :, :, :dx] = 0
        elif dx < 0:
            r[:, :, :, dx:] = 0
        s, c = poisson_steps(rng(seed, _P_INPUT, iteration, trial), np.minimum(1.0, r.reshape(n_steps, -1)))
        return (n_steps, s, c), label

    def make_batch(iteration: int, first: int, n: int) -> Batch:
        rows = [one_trial(iteration, first + i) for i in range(n)]
        return _assemble([r[0] for r in rows], n_out, n_steps, labels=[r[1] for r in rows],
                         windows=[window] * n)
    return Workload("c3_events", net, make_batch, batch_size, iterations,
                    "event-camera classification, 2312 in / 180 LIF / 10 softmax, batch 128")


def _large_sparse(name: str, seed: int, n_rec: int, indeg_rec: int, n_in: int, indeg_in: int,
                  rate_in_hz: float, n_steps: int, batch_size: int, gain: float, in_gain: float,
                  alif_fraction: float, iterations: int, description: str, eta: float) -> Workload:
    n_out = 10
    is_alif = np.zeros(n_rec, np.uint8)
    if alif_fraction > 0:
        perm = rng(seed, _P_ALIF).permutation(n_rec)
        is_alif[perm[n_rec - int(round(alif_fraction * n_rec)):]] = 1
    # gradient descent on a loss summed over T steps and K readouts: the
    # readout update is coherent over all J neurons, so the stable step scales
    # like 1 / (J T rate^2 tau_out^2)
    prm = Params(beta_a=1.7 if alif_fraction > 0 else 0.0, tau_a=2000.0, loss=0, optimizer=0,
                 eta=eta, max_delay=5)
    rec = fixed_indegree_projection(n_rec, n_rec, indeg_rec, gain / np.sqrt(indeg_rec),
                                    rng(seed, _P_GRAPH_REC), rng(seed, _P_W_REC),
                                    rng(seed, _P_DELAY_REC), no_self=True, delay_lo=1, delay_hi=5)
    inp = fixed_indegree_projection(n_in, n_rec, indeg_in, in_gain / np.sqrt(indeg_in),
                                    rng(seed, _P_GRAPH_IN), rng(seed, _P_W_IN),
                                    rng(seed, _P_DELAY_IN), no_self=False, delay_lo=1, delay_hi=1)
    net = Network(n_in, n_rec, n_out, is_alif, prm, inp, rec,
                  rng(seed, _P_W_OUT).normal(0, 1 / np.sqrt(n_rec), (n_out, n_rec)),
                  rng(seed, _P_FEEDBACK).normal(0, 1 / np.sqrt(n_rec), (n_rec, n_out)))
    targets = np.stack([sinusoid_sum(rng(seed, _P_TARGET, k), n_steps, prm.dt) for k in range(n_out)], axis=1)
    p_in = rate_in_hz * prm.dt / 1000.0

    def make_batch(iteration: int, first: int, n: int) -> Batch:
        trials = []
        for i in range(n):
            s, c = poisson_steps(rng(seed, _P_INPUT, iteration, first + i), np.full((n_steps, n_in), p_in))
            trials.append((n_steps, s, c))
        return _assemble(trials, n_out, n_steps, targets=[targets] * n)
    return Workload(name, net, make_batch, batch_size, iterations, description,
                    info={"gain": gain, "in_gain": in_gain, "indeg_rec": indeg_rec, "indeg_in": indeg_in})


# Recurrent gains chosen once so that the free-running recurrent rate lies near
# the configured target (about 10 Hz for the 1e5-neuron network, about 5 Hz for
# the 1e6-neuron one); measured rates are always reported next to results.
C4_GAIN, C4_IN_GAIN = 0.5, 0.75
C5_GAIN, C5_IN_GAIN = 1.1, 1.0


def c4_sparse(seed: int = SEED_BASE + 4, n_rec: int = 100_000, n_steps: int = 1000,
              batch_size: int = 4, iterations: int = 2, gain: float = None,
              n_in: int = 1000, in_gain: float = None) -> Workload:
    """Large sparse network: fixed in-degree 1000, delays 1-5, 1000 Poisson
    inputs at 20 Hz with in-degree 100, 10 readouts (MSE on sinusoid sums)."""
    return _large_sparse("c4_sparse", seed, n_rec, min(1000, n_rec - 1), n_in, min(100, n_in),
                         20.0, n_steps, batch_size, C4_GAIN if gain is None else gain,
                         C4_IN_GAIN if in_gain is None else in_gain, 0.0,
                         iterations, "1e5 LIF, in-degree 1000 (1e8 synapses), batch 4", eta=1e-7)


def c5_million(seed: int = SEED_BASE + 5, n_rec: int = 1_000_000, n_steps: int = 2000,
               batch_size: int = 1, iterations: int = 1, gain: float = None,
               n_in: int = 10_000, in_gain: float = None) -> Workload:
    """Million-neuron network: 80/20 LIF/ALIF, fixed in-degree 100, delays 1-5,
    10,000 Poisson inputs at 5 Hz with in-degree 10, 10 readouts."""
    return _large_sparse("c5_million", seed, n_rec, min(100, n_rec - 1), n_in, min(10, n_in),
                         5.0, n_steps, batch_size, C5_GAIN if gain is None else gain,
                         C5_IN_GAIN if in_gain is None else in_gain, 0.2,
                         iterations, "1e6 LIF/ALIF, in-degree 100 (1e8 synapses), batch 1", eta=1e-8)


def ignore_and_fire(batch: Batch, n_rec: int, rate_hz: float, dt_ms: float, seed: int,
                    sample0: int = 0) -> Batch:
    """Attach ignore-and-fire recurrent spike trains (Methods, "Scaling"): each
    neuron fires regularly at rate_hz with its own random phase, whatever its
    input.  Trial b is sample sample0 + b of a continuous run and covers its
    global steps (sample0 + b) * T + 1 .. + T, so consecutive samples continue
    the same regular trains."""
    period = int(round(1000.0 / (rate_hz * dt_ms)))
    phase = rng(seed, _P_FORCED).integers(0, period, size=n_rec)
    ptr = [0]
    steps, neurons = [], []
    for b in range(batch.n_trials):
        t = int(batch.n_steps[b])
        t0 = (sample0 + b) * t
        # neuron j fires at global step u with (u - phase_j) % period == 0
        first = (phase - (t0 + 1)) % period + 1           # first local step 1..period
        k = np.arange(0, t, period, dtype=np.int64)
        loc = first[None, :] + k[:, None]                  # [fires, J], may exceed t
        sj = np.broadcast_to(np.arange(n_rec), loc.shape)
        ok = loc <= t
        s, j = loc[ok], sj[ok]
        order = np.lexsort((j, s))
        steps.append(s[order].astype(np.uint32))
        neurons.append(j[order].astype(np.uint32))
        ptr.append(ptr[-1] + s.size)
    out = replace(batch)
    out.forced_ptr = np.array(ptr, dtype=np.uint64)
    out.forced_step = np.concatenate(steps)
    out.forced_neuron = np.concatenate(neurons)
    return out


def scaling(seed: int = SEED_BASE + 6, n_rec: int = 128_000, indeg_rec: int = 10_000, n_in: int = 1000,
            indeg_in: int = 100, n_out: int = 10, indeg_out: int = 1000, outdeg_fb: int = 100,
            rate_hz: float = 5.0, n_steps: int = 1000, samples: int = 20, gain: float = 1.0,
            in_gain: float = 1.0, eta: float = 1e-9) -> Workload:
    """The paper's scaling network (Methods, "Scaling"), base size: 128,000
    ignore-and-fire neurons at 5 Hz with random phases, recurrent in-degree
    10^4 without autapses or multapses (1.28e9 plastic synapses), 1000 Poisson
    inputs at 5 Hz with in-degree 100, 10 readouts with in-degree 1000 and
    feedback out-degree 100, target signals from a generator, 20 s of
    biological time in samples of n_steps steps of 1 ms.  Readout and
    feedback weights are stored dense with zeros off the drawn connections."""
    prm = Params(loss=0, optimizer=0, eta=eta, max_delay=1)
    rec = fixed_indegree_lean(n_rec, n_rec, indeg_rec, gain / np.sqrt(indeg_rec), rng(seed, _P_GRAPH_REC),
                              rng(seed, _P_W_REC), no_self=True)
    inp = fixed_indegree_lean(n_in, n_rec, indeg_in, in_gain / np.sqrt(indeg_in), rng(seed, _P_GRAPH_IN),
                              rng(seed, _P_W_IN), no_self=False)
    g_out, g_fb = rng(seed, _P_W_OUT), rng(seed, _P_FEEDBACK)
    w_out = np.zeros((n_out, n_rec))
    fb = np.zeros((n_rec, n_out))
    for k in range(n_out):
        src = g_out.choice(n_rec, size=indeg_out, replace=False)
        w_out[k, src] = g_out.normal(0.0, 1.0 / np.sqrt(indeg_out), size=indeg_out)
        tgt = g_fb.choice(n_rec, size=outdeg_fb, replace=False)
        fb[tgt, k] = g_fb.normal(0.0, 1.0 / np.sqrt(outdeg_fb), size=outdeg_fb)
    net = Network(n_in, n_rec, n_out, np.zeros(n_rec, np.uint8), prm, inp, rec, w_out, fb)
    targets = np.stack([sinusoid_sum(rng(seed, _P_TARGET, k), n_steps * samples, prm.dt)
                        for k in range(n_out)], axis=1)
    p_in = rate_hz * prm.dt / 1000.0

    def make_batch(iteration: int, first: int, n: int) -> Batch:
        trials, tg = [], []
        for i in range(n):
            s, c = poisson_steps(rng(seed, _P_INPUT, iteration, first + i), np.full((n_steps, n_in), p_in))
            trials.append((n_steps, s, c))
            u = ((iteration * n + first + i) % samples) * n_steps
            tg.append(targets[u:u + n_steps])
        b = _assemble(trials, n_out, n_steps, targets=tg)
        return ignore_and_fire(b, n_rec, rate_hz, prm.dt, seed, iteration * n + first)
    return Workload("scaling", net, make_batch, 1, samples,
                    "128k ignore-and-fire neurons at 5 Hz, in-degree 1e4 (1.28e9 synapses), 1 trial",
                    info={"indeg_rec": indeg_rec, "indeg_in": indeg_in, "rate_hz": rate_hz})


def tiny(seed: int = SEED_BASE + 11, n_steps: int = 200, loss: int = 0, n_in: int = 6,
         n_lif: int = 3, n_alif: int = 2, n_out: int = 2, max_delay: int = 2,
         rate_hz: float = 100.0, w_scale: float = 0.8, surrogate: int = 0,
         batch_size: int = 2) -> Workload:
    """Five-neuron net (3 LIF + 2 ALIF, 6 inputs, 2 readouts) with delays in
    {1, 2}, for brute-force checks of the gradient definition; with the
    default seed every neuron spikes."""
    n_rec = n_lif + n_alif
    is_alif = np.zeros(n_rec, np.uint8)
    is_alif[n_lif:] = 1
    # tau_out != tau_m so that the two filters of the eligibility trace differ
    prm = Params(beta_a=1.7, tau_a=200.0, tau_out=35.0, loss=loss, optimizer=1, eta=1e-2,
                 surrogate=surrogate, max_delay=max_delay)
    g = rng(seed, _P_DELAY_REC)
    inp = dense_projection(n_in, n_rec, w_scale, rng(seed, _P_W_IN))
    inp.delay[:] = g.integers(1, max_delay + 1, size=inp.nnz)
    rec = dense_projection(n_rec, n_rec, w_scale / 2, rng(seed, _P_W_REC), no_self=True)
    rec.delay[:] = g.integers(1, max_delay + 1, size=rec.nnz)
    net = Network(n_in, n_rec, n_out, is_alif, prm, inp, rec,
                  rng(seed, _P_W_OUT).normal(0, 1.0, (n_out, n_rec)),
                  rng(seed, _P_FEEDBACK).normal(0, 1.0, (n_rec, n_out)))
    target = np.stack([sinusoid_sum(rng(seed, _P_TARGET, k), n_steps, prm.dt) for k in range(n_out)], axis=1)

    def make_batch(iteration: int, first: int, n: int) -> Batch:
        trials, labels = [], []
        for i in range(n):
            s, c = poisson_steps(rng(seed, _P_INPUT, iteration, first + i),
                                 np.full((n_steps, n_in), rate_hz * prm.dt / 1000.0))
            trials.append((n_steps, s, c))
            labels.append(int(rng(seed, _P_TASK, iteration, first + i).integers(0, n_out)))
        window = np.ones(n_steps, np.uint8)
        window[: n_steps // 4] = 0
        return _assemble(trials, n_out, n_steps, targets=[target] * n, labels=labels,
                         windows=[window] * n)
    return Workload("tiny", net, make_batch, batch_size, 3, "5-neuron brute-force net")


WORKLOADS = {"c1_pattern": c1_pattern, "c2_evidence": c2_evidence, "c3_events": c3_events,
             "c4_sparse": c4_sparse, "c5_million": c5_million, "scaling": scaling, "tiny": tiny}
