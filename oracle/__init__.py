"""CPU FP64 oracle for event-driven e-prop -- TEST INFRASTRUCTURE ONLY.

A plain serial C implementation (``eprop_oracle.c``) of the paper's
time-driven gradient computation and its event-driven weight update,
plus forward-mode brute-force checks, driven from here through ctypes.
Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the GPU library never does, and
nothing here imports the GPU library.  Inputs come from
``paper_2511_21674_amd.workloads`` (seeded generators without method
arithmetic).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eprop_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle (serial, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Proj(C.Structure):
    _fields_ = [("n_src", C.c_int), ("n_tgt", C.c_int), ("nnz", C.c_long),
                ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("w", C.c_void_p),
                ("delay", C.c_void_p)]


class _Net(C.Structure):
    _fields_ = [("n_in", C.c_int), ("n_rec", C.c_int), ("n_out", C.c_int),
                ("is_alif", C.c_void_p),
                ("dt", C.c_double), ("tau_m", C.c_double), ("tau_out", C.c_double),
                ("v_th", C.c_double), ("t_ref", C.c_double), ("tau_a", C.c_double),
                ("beta_a", C.c_double), ("surrogate", C.c_int), ("sg_gamma", C.c_double),
                ("sg_beta", C.c_double), ("loss", C.c_int), ("inp", _Proj), ("rec", _Proj),
                ("w_out", C.c_void_p), ("fb", C.c_void_p), ("d_out", C.c_int), ("d_ls", C.c_int),
                ("c_reg", C.c_double), ("f_target", C.c_double),
                ("reset_mode", C.c_int), ("v_reset", C.c_double), ("etrace_filter", C.c_int),
                ("tau_e", C.c_double), ("reg_mode", C.c_int), ("reg_tau", C.c_double)]


class _Trial(C.Structure):
    _fields_ = [("n_steps", C.c_int), ("n_in_spikes", C.c_long), ("in_step", C.c_void_p),
                ("in_src", C.c_void_p), ("target", C.c_void_p), ("label", C.c_int),
                ("window", C.c_void_p), ("forced", C.c_int), ("n_forced", C.c_long),
                ("forced_step", C.c_void_p), ("forced_neuron", C.c_void_p)]


class _Trace(C.Structure):
    _fields_ = [("v", C.c_void_p), ("a", C.c_void_p), ("psi", C.c_void_p), ("learn", C.c_void_p),
                ("y", C.c_void_p), ("err", C.c_void_p), ("z", C.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.orc_run_trial.argtypes = [C.POINTER(_Net), C.POINTER(_Trial), C.c_int, P, P, P,
                                    C.POINTER(_Trace), C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.orc_run_trial.restype = C.c_int
        for f in (L.orc_bruteforce_eprop, L.orc_forward_mode_loss_grad):
            f.argtypes = [C.POINTER(_Net), C.POINTER(_Trial), P, P]
            f.restype = C.c_int
        L.orc_forced_sampled.argtypes = [C.POINTER(_Net), C.POINTER(_Trial), C.c_int, P, P, P, P,
                                         C.POINTER(C.c_double)]
        L.orc_forced_sampled.restype = C.c_int
        L.orc_fp32_bounds.argtypes = [C.POINTER(_Net), C.POINTER(_Trial), C.c_double, P, C.c_int, P,
                                      P, P, P, P, P, P, P, P]
        L.orc_fp32_bounds.restype = C.c_int
        L.orc_run_online.argtypes = [C.POINTER(_Net), C.c_int, C.POINTER(_Trial), C.c_double, C.c_int, C.c_int,
                                     P, P, P, P, P, P, P, P, P, P, P]
        L.orc_run_online.restype = C.c_int
        L.orc_apply.argtypes = [C.c_long, P, P, C.c_double, C.c_int, C.c_double, C.c_double,
                                C.c_double, C.c_double, C.c_long, P, P]
        L.orc_apply.restype = None
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


class OracleNet:
    """Mutable FP64 copy of a workload network (weights are trained in place)."""

    def __init__(self, net):
        self.src = net
        self.n_in, self.n_rec, self.n_out = net.n_in, net.n_rec, net.n_out
        self.params = net.params
        self.is_alif = np.ascontiguousarray(net.is_alif, dtype=np.uint8)
        self.in_row = np.ascontiguousarray(net.in_rec.row_ptr, dtype=np.uint64)
        self.in_col = np.ascontiguousarray(net.in_rec.col, dtype=np.uint32)
        self.in_delay = np.ascontiguousarray(net.in_rec.delay, dtype=np.uint8)
        self.w_in = np.array(net.in_rec.w, dtype=np.float64)
        self.rec_row = np.ascontiguousarray(net.rec_rec.row_ptr, dtype=np.uint64)
        self.rec_col = np.ascontiguousarray(net.rec_rec.col, dtype=np.uint32)
        self.rec_delay = np.ascontiguousarray(net.rec_rec.delay, dtype=np.uint8)
        self.w_rec = np.array(net.rec_rec.w, dtype=np.float64)
        self.w_out = np.array(net.w_out, dtype=np.float64, order="C")
        self.fb = np.array(net.feedback, dtype=np.float64, order="C")
        # optimiser state
        self.m = {k: np.zeros_like(getattr(self, k)) for k in ("w_in", "w_rec", "w_out")}
        self.v = {k: np.zeros_like(getattr(self, k)) for k in ("w_in", "w_rec", "w_out")}
        self.step = 0

    def cstruct(self) -> _Net:
        p = self.params
        s = _Net()
        s.n_in, s.n_rec, s.n_out = self.n_in, self.n_rec, self.n_out
        s.is_alif = _p(self.is_alif)
        s.dt, s.tau_m, s.tau_out, s.v_th = p.dt, p.tau_m, p.tau_out, p.v_th
        s.t_ref, s.tau_a, s.beta_a = p.t_ref, p.tau_a, p.beta_a
        s.surrogate, s.sg_gamma, s.sg_beta, s.loss = p.surrogate, p.sg_gamma, p.sg_beta, p.loss
        s.inp = _Proj(self.n_in, self.n_rec, int(self.in_row[-1]), _p(self.in_row), _p(self.in_col),
                      _p(self.w_in), _p(self.in_delay))
        s.rec = _Proj(self.n_rec, self.n_rec, int(self.rec_row[-1]), _p(self.rec_row),
                      _p(self.rec_col), _p(self.w_rec), _p(self.rec_delay))
        s.w_out, s.fb = _p(self.w_out), _p(self.fb)
        s.d_out, s.d_ls = int(getattr(p, "d_out", 0)), int(getattr(p, "d_ls", 0))
        # target rate in spikes per step (the rate of eq. loss-firing-rate-regularization)
        s.c_reg, s.f_target = float(getattr(p, "c_reg", 0.0)), float(getattr(p, "f_target_hz", 0.0)) * p.dt / 1000.0
        s.reset_mode, s.v_reset = int(getattr(p, "reset_mode", 0)), float(getattr(p, "v_reset", 0.0))
        s.etrace_filter, s.tau_e = int(getattr(p, "etrace_filter", 0)), float(getattr(p, "tau_e", 0.0))
        s.reg_mode, s.reg_tau = int(getattr(p, "reg_mode", 0)), float(getattr(p, "reg_tau", 0.0))
        return s


def _trial_struct(batch, b: int, keep: list) -> _Trial:
    lo, hi = int(batch.in_ptr[b]), int(batch.in_ptr[b + 1])
    T = int(batch.n_steps[b])
    st = np.ascontiguousarray(batch.in_step[lo:hi], dtype=np.uint32)
    sr = np.ascontiguousarray(batch.in_src[lo:hi], dtype=np.uint32)
    keep += [st, sr]
    tr = _Trial()
    tr.n_steps = T
    tr.n_in_spikes = hi - lo
    tr.in_step, tr.in_src = _p(st), _p(sr)
    if batch.target is not None:
        tg = np.ascontiguousarray(batch.target[b, :T], dtype=np.float64)
        keep.append(tg)
        tr.target = _p(tg)
    tr.label = int(batch.label[b]) if batch.label is not None else -1
    if batch.window is not None:
        wn = np.ascontiguousarray(batch.window[b, :T], dtype=np.uint8)
        keep.append(wn)
        tr.window = _p(wn)
    if batch.forced_ptr is not None:
        flo, fhi = int(batch.forced_ptr[b]), int(batch.forced_ptr[b + 1])
        fs = np.ascontiguousarray(batch.forced_step[flo:fhi], dtype=np.uint32)
        fn = np.ascontiguousarray(batch.forced_neuron[flo:fhi], dtype=np.uint32)
        keep += [fs, fn]
        tr.forced, tr.n_forced = 1, fhi - flo
        tr.forced_step, tr.forced_neuron = _p(fs), _p(fn)
    return tr


@dataclass
class TrialResult:
    loss: float
    pred: int
    trace: dict


def run_trial(net: OracleNet, batch, b: int, grad_mode: int = 0, grads: dict = None,
              trace: bool = False) -> TrialResult:
    """One trial; grad_mode 0 none, 1 time-driven, 2 event-driven.  Gradients
    are added into grads['w_in'|'w_rec'|'w_out'] (float64 arrays)."""
    keep: list = []
    ns = net.cstruct()
    tr = _trial_struct(batch, b, keep)
    T, J, K = int(batch.n_steps[b]), net.n_rec, net.n_out
    rec = {}
    tc = None
    if trace:
        rec = {"v": np.zeros((T, J)), "a": np.zeros((T, J)), "psi": np.zeros((T, J)),
               "learn": np.zeros((T, J)), "y": np.zeros((T, K)), "err": np.zeros((T, K)),
               "z": np.zeros((T, J), dtype=np.uint8)}
        tc = _Trace(*(_p(rec[k]) for k in ("v", "a", "psi", "learn", "y", "err", "z")))
    loss = C.c_double(0.0)
    pred = C.c_int(0)
    g = grads or {}
    rc = lib().orc_run_trial(C.byref(ns), C.byref(tr), grad_mode, _p(g.get("w_in")),
                             _p(g.get("w_rec")), _p(g.get("w_out")),
                             C.byref(tc) if tc is not None else None, C.byref(loss), C.byref(pred))
    if rc != 0:
        raise ValueError("oracle rejected the trial")
    return TrialResult(loss.value, pred.value, rec)


def run_online(net: OracleNet, batch, eta: float, cutoff: int = 0, flush: bool = False) -> dict:
    """e-prop+ update schedule over the batch's trials run back to back as one
    continuous run (weight update at every arriving spike; see
    orc_run_online).  The network's weights are trained in place.  Returns
    the per-sample losses, the recurrent spikes [T_total, J], the summed
    gradients that were applied and ("abs") |eta| times the absolute term
    sums of those gradients."""
    keep: list = []
    ns = net.cstruct()
    n = batch.n_trials
    trs = (_Trial * n)(*[_trial_struct(batch, b, keep) for b in range(n)])
    Tt = int(np.sum(batch.n_steps[:n]))
    g = zero_grads(net)
    ab = zero_grads(net)
    loss = np.zeros(n)
    z = np.zeros((Tt, net.n_rec), dtype=np.uint8)
    rc = lib().orc_run_online(C.byref(ns), n, trs, float(eta), int(cutoff), int(bool(flush)), _p(net.w_in),
                              _p(net.w_rec), _p(net.w_out), _p(g["w_in"]), _p(g["w_rec"]), _p(g["w_out"]),
                              _p(loss), _p(z), _p(ab["w_in"]), _p(ab["w_rec"]), _p(ab["w_out"]))
    if rc != 0:
        raise ValueError("oracle rejected the run")
    return {"loss": loss, "z": z, "grads": g, "abs": ab}


def zero_grads(net: OracleNet) -> dict:
    return {"w_in": np.zeros_like(net.w_in), "w_rec": np.zeros_like(net.w_rec),
            "w_out": np.zeros_like(net.w_out)}


def apply(net: OracleNet, grads: dict, n_trials: int) -> None:
    """Average over the trials of the iteration, then GD or Adam."""
    p = net.params
    net.step += 1
    for k in ("w_in", "w_rec", "w_out"):
        w = getattr(net, k)
        g = np.ascontiguousarray(grads[k], dtype=np.float64)
        lib().orc_apply(w.size, _p(w), _p(g), float(n_trials), p.optimizer, p.eta, p.adam_beta1,
                        p.adam_beta2, p.adam_eps_hat, net.step, _p(net.m[k]), _p(net.v[k]))


def bruteforce_eprop(net: OracleNet, batch, b: int) -> dict:
    keep: list = []
    ns, tr = net.cstruct(), _trial_struct(batch, b, keep)
    out = {"w_in": np.zeros_like(net.w_in), "w_rec": np.zeros_like(net.w_rec)}
    if lib().orc_bruteforce_eprop(C.byref(ns), C.byref(tr), _p(out["w_in"]), _p(out["w_rec"])):
        raise ValueError("oracle rejected the trial")
    return out


def forward_mode_loss_grad(net: OracleNet, batch, b: int) -> dict:
    keep: list = []
    ns, tr = net.cstruct(), _trial_struct(batch, b, keep)
    out = {"w_in": np.zeros_like(net.w_in), "w_rec": np.zeros_like(net.w_rec)}
    if lib().orc_forward_mode_loss_grad(C.byref(ns), C.byref(tr), _p(out["w_in"]), _p(out["w_rec"])):
        raise ValueError("oracle rejected the trial")
    return out


def forced_sampled(net: OracleNet, batch, b: int, targets) -> tuple:
    """Teacher-forced trial b: (loss, psi [n, T], g_in, g_rec) where only the
    incoming synapses of the sampled targets hold values (others NaN)."""
    keep: list = []
    ns, tr = net.cstruct(), _trial_struct(batch, b, keep)
    tg = np.ascontiguousarray(targets, dtype=np.int32)
    T = int(batch.n_steps[b])
    psi = np.zeros((tg.size, T))
    g_in = np.full(net.w_in.shape, np.nan)
    g_rec = np.full(net.w_rec.shape, np.nan)
    loss = C.c_double(0.0)
    if lib().orc_forced_sampled(C.byref(ns), C.byref(tr), tg.size, _p(tg), _p(g_in), _p(g_rec),
                                _p(psi), C.byref(loss)):
        raise ValueError("oracle rejected the trial")
    return loss.value, psi, g_in, g_rec


def fp32_bounds(net: OracleNet, batch, b: int, quantum: float = 0.0, psi_given=None, targets=None) -> dict:
    """Teacher-forced trial b (see orc_fp32_bounds): "psi" [T, n_t] the trial's
    surrogate gradient and "psi_bound" the bound of its FP32 evaluation's
    error; "g" the time-driven gradient on the psi history psi_given ([T, n_t],
    the targets' columns; None = own) and "b" the FP32 rounding bound of each
    of its entries, as dicts like zero_grads.  With targets only their
    incoming synapses hold values (others NaN) and n_t = len(targets);
    otherwise n_t = J."""
    keep: list = []
    ns, tr = net.cstruct(), _trial_struct(batch, b, keep)
    T = int(batch.n_steps[b])
    if targets is None:
        tg, n, nt = None, -1, net.n_rec
        fill = 0.0
    else:
        tg = np.ascontiguousarray(targets, dtype=np.int32)
        n = nt = tg.size
        fill = np.nan
    pg = None if psi_given is None else np.ascontiguousarray(np.asarray(psi_given, dtype=np.float64).T)
    if pg is not None and pg.shape != (nt, T):
        raise ValueError("psi_given must be [T, n_t] (the targets' columns)")
    psi, pb = np.zeros((nt, T)), np.zeros((nt, T))
    g = {"w_in": np.full(net.w_in.shape, fill), "w_rec": np.full(net.w_rec.shape, fill),
         "w_out": np.zeros_like(net.w_out)}
    bd = {"w_in": np.full(net.w_in.shape, fill), "w_rec": np.full(net.w_rec.shape, fill),
          "w_out": np.zeros_like(net.w_out)}
    if lib().orc_fp32_bounds(C.byref(ns), C.byref(tr), float(quantum), _p(pg), n, _p(tg), _p(psi), _p(pb),
                             _p(g["w_in"]), _p(g["w_rec"]), _p(g["w_out"]), _p(bd["w_in"]), _p(bd["w_rec"]),
                             _p(bd["w_out"])):
        raise ValueError("oracle rejected the trial (the bounds need forced spikes)")
    return {"psi": psi.T.copy(), "psi_bound": pb.T.copy(), "g": g, "b": bd}


def train(workload, iterations: int = None, grad_mode: int = 2, batch_size: int = None,
          record: bool = False, net: OracleNet = None) -> dict:
    """Oracle training loop: per iteration, every trial from zero state with
    shared weights, gradients summed, then averaged and applied once."""
    net = net or OracleNet(workload.network)
    iterations = workload.iterations if iterations is None else iterations
    bs = workload.batch_size if batch_size is None else batch_size
    hist = {"loss": [], "pred": [], "spikes": [], "weights": [], "grads": []}
    for it in range(iterations):
        batch = workload.make_batch(it, 0, bs)
        g = zero_grads(net)
        losses, preds, spikes = [], [], []
        for b in range(batch.n_trials):
            r = run_trial(net, batch, b, grad_mode, g, trace=record)
            losses.append(r.loss)
            preds.append(r.pred)
            if record:
                spikes.append(r.trace["z"])
        hist["loss"].append(np.array(losses))
        hist["pred"].append(np.array(preds))
        if record:
            hist["spikes"].append(spikes)
            hist["grads"].append({k: v.copy() for k, v in g.items()})
        apply(net, g, batch.n_trials)
        if record:
            hist["weights"].append({k: getattr(net, k).copy() for k in ("w_in", "w_rec", "w_out")})
    hist["net"] = net
    return hist
