"""ctypes binding of libeprop_hip.so (declared in include/eprop.h).

The functions ``eprop_*`` mirror the C entry points one to one; the
``Network`` class only marshals ``workloads`` arrays into those calls.
Every step of the computation runs in the library's HIP kernels; PyTorch
is used only to place batch arrays in device memory and to supply the
HIP stream.  If the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeprop_hip.so")

EPROP_ABI_VERSION = 4
EPROP_OK, EPROP_ERR_INVALID_ARGUMENT, EPROP_ERR_OUT_OF_MEMORY = 0, -1, -2
EPROP_ERR_DEVICE, EPROP_ERR_STATE, EPROP_ERR_CAPACITY = -3, -4, -5
EPROP_ERR_NUMERIC, EPROP_ERR_UNSUPPORTED = -6, -7
EPROP_FP32, EPROP_FP64 = 0, 1
EPROP_DELIVERY_AUTO, EPROP_DELIVERY_SCATTER, EPROP_DELIVERY_GATHER = 0, 1, 2
EPROP_FLAG_NO_GRAPH, EPROP_DETERMINISTIC, EPROP_SHARED_WEIGHTS, EPROP_AUTOTUNE = 1, 2, 4, 8
EPROP_SCATTER_LOOKUP, EPROP_SCATTER_QUEUES = 16, 32
EPROP_MEM_HOST, EPROP_MEM_DEVICE = 0, 1
EPROP_BATCH_TRAIN, EPROP_BATCH_PROFILE, EPROP_RECORD_SPIKES, EPROP_RECORD_TRACES = 1, 2, 4, 8
EPROP_BATCH_TIME_DRIVEN = 16
EPROP_BATCH_ONLINE = 32
EPROP_LOSS_MSE, EPROP_LOSS_SOFTMAX_CE, EPROP_LOSS_TEMPORAL_MSE = 0, 1, 2
EPROP_RESET_SUBTRACT, EPROP_RESET_TO_VALUE = 0, 1
EPROP_ETRACE_COUPLED, EPROP_ETRACE_DECOUPLED, EPROP_ETRACE_NONE = 0, 1, 2
EPROP_REG_STATIC, EPROP_REG_MOVING_AVERAGE = 0, 1
EPROP_TRAIN = EPROP_BATCH_TRAIN
EPROP_N_PHASES = 8
PHASES = ("stage", "forward", "readout", "adjoint", "synapse", "output")
(EPROP_STATE_W_IN, EPROP_STATE_W_REC, EPROP_STATE_W_OUT, EPROP_STATE_GRAD_IN, EPROP_STATE_GRAD_REC,
 EPROP_STATE_GRAD_OUT, EPROP_STATE_ADAM_M_IN, EPROP_STATE_ADAM_V_IN, EPROP_STATE_ADAM_M_REC,
 EPROP_STATE_ADAM_V_REC, EPROP_STATE_ADAM_M_OUT, EPROP_STATE_ADAM_V_OUT, EPROP_STATE_ADAM_STEP,
 EPROP_STATE_SPIKES, EPROP_STATE_PSI, EPROP_STATE_Y, EPROP_STATE_ERR, EPROP_STATE_V,
 EPROP_STATE_LAYOUT, EPROP_STATE_L, EPROP_STATE_INPUT_BOUND) = range(21)

EXPORTED = ("eprop_create_network", "eprop_simulate_batch", "eprop_simulate_batch_noalloc", "eprop_apply_updates",
            "eprop_read_state", "eprop_destroy_network", "eprop_status_string", "eprop_last_error")
EPROP_NOALLOC_SCRATCH_BYTES = 64 << 20

_P = C.c_void_p
DEV_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEV_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class eprop_config(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("precision", C.c_int32), ("n_in", C.c_uint32),
                ("n_rec", C.c_uint32), ("n_out", C.c_uint32), ("is_alif", _P),
                ("dt", C.c_double), ("tau_m", C.c_double), ("tau_out", C.c_double), ("v_th", C.c_double),
                ("t_ref", C.c_double), ("tau_a", C.c_double), ("beta_a", C.c_double),
                ("surrogate", C.c_int32), ("sg_gamma", C.c_double), ("sg_beta", C.c_double),
                ("loss", C.c_int32), ("optimizer", C.c_int32), ("eta", C.c_double),
                ("adam_beta1", C.c_double), ("adam_beta2", C.c_double), ("adam_eps_hat", C.c_double),
                ("max_delay", C.c_uint32), ("max_trials", C.c_uint32), ("max_steps", C.c_uint32),
                ("delivery", C.c_int32), ("flags", C.c_uint32), ("d_out", C.c_uint32), ("d_ls", C.c_uint32),
                ("history_steps", C.c_uint32), ("c_reg", C.c_double), ("f_target", C.c_double),
                ("reset_mode", C.c_int32), ("v_reset", C.c_double), ("etrace_filter", C.c_int32),
                ("tau_e", C.c_double), ("reg_mode", C.c_int32), ("reg_tau", C.c_double),
                ("isi_cutoff", C.c_uint32),
                ("dev_alloc", DEV_ALLOC_FN), ("dev_free", DEV_FREE_FN),
                ("alloc_ctx", _P)]


class eprop_projection(C.Structure):
    _fields_ = [("n_src", C.c_uint32), ("n_tgt", C.c_uint32), ("nnz", C.c_uint64), ("row_ptr", _P),
                ("col", _P), ("w", _P), ("delay", _P)]


class eprop_optimizer_state(C.Structure):
    _fields_ = [("m_in", _P), ("v_in", _P), ("m_rec", _P), ("v_rec", _P), ("m_out", _P), ("v_out", _P),
                ("step", C.c_uint64)]


class eprop_batch(C.Structure):
    _fields_ = [("n_trials", C.c_uint32), ("memory", C.c_int32), ("n_steps", _P), ("n_in_spikes", C.c_uint64),
                ("in_ptr", _P), ("in_step", _P), ("in_src", _P), ("step_stride", C.c_uint32),
                ("target", _P), ("label", _P), ("window", _P), ("n_forced", C.c_uint64),
                ("forced_ptr", _P), ("forced_step", _P), ("forced_neuron", _P), ("flags", C.c_uint32)]


class eprop_batch_result(C.Structure):
    _fields_ = [("loss", _P), ("predicted", _P), ("n_rec_spikes", C.c_uint64), ("n_in_spikes", C.c_uint64),
                ("n_syn_events", C.c_uint64), ("n_out_events", C.c_uint64), ("n_eprop_updates", C.c_uint64),
                ("n_flush_updates", C.c_uint64), ("device_seconds", C.c_double),
                ("phase_ms", C.c_double * EPROP_N_PHASES)]


_lib = None


def lib():
    """Loads libeprop_hip.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP extension not built: {LIB_PATH} is missing (run __graft_entry__.build())")
        # PyTorch ships its own HIP runtime under the same soname; loading it
        # first makes the library bind to that one runtime in this process
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        L.eprop_create_network.argtypes = [C.POINTER(eprop_config), C.POINTER(eprop_projection),
                                           C.POINTER(eprop_projection), _P, _P,
                                           C.POINTER(eprop_optimizer_state), _P, C.POINTER(_P)]
        L.eprop_create_network.restype = C.c_int32
        L.eprop_simulate_batch.argtypes = [_P, C.POINTER(eprop_batch), C.POINTER(eprop_batch_result)]
        L.eprop_simulate_batch.restype = C.c_int32
        L.eprop_simulate_batch_noalloc.argtypes = [_P, C.POINTER(eprop_batch), C.POINTER(eprop_batch_result)]
        L.eprop_simulate_batch_noalloc.restype = C.c_int32
        L.eprop_apply_updates.argtypes = [_P]
        L.eprop_apply_updates.restype = C.c_int32
        L.eprop_read_state.argtypes = [_P, C.c_int32, C.c_uint32, _P, C.c_size_t, C.POINTER(C.c_size_t)]
        L.eprop_read_state.restype = C.c_int32
        L.eprop_destroy_network.argtypes = [_P]
        L.eprop_destroy_network.restype = None
        L.eprop_status_string.argtypes = [C.c_int32]
        L.eprop_status_string.restype = C.c_char_p
        L.eprop_last_error.argtypes = [_P]
        L.eprop_last_error.restype = C.c_char_p
        _lib = L
    return _lib


# ---------------------------------------------------------------- C entry points

def eprop_create_network(cfg, in_rec, rec_rec, w_out, feedback, opt, hip_stream):
    out = _P()
    st = lib().eprop_create_network(C.byref(cfg), C.byref(in_rec), C.byref(rec_rec), w_out, feedback,
                                    C.byref(opt) if opt is not None else None, hip_stream, C.byref(out))
    return st, out


def eprop_simulate_batch(net, batch, res):
    return lib().eprop_simulate_batch(net, C.byref(batch), C.byref(res))


def eprop_simulate_batch_noalloc(net, batch, res):
    return lib().eprop_simulate_batch_noalloc(net, C.byref(batch), C.byref(res))


def eprop_apply_updates(net):
    return lib().eprop_apply_updates(net)


def eprop_read_state(net, what, trial, dst, dst_bytes):
    needed = C.c_size_t(0)
    st = lib().eprop_read_state(net, what, trial, dst, dst_bytes, C.byref(needed))
    return st, needed.value


def eprop_destroy_network(net):
    lib().eprop_destroy_network(net)


def eprop_status_string(st):
    return lib().eprop_status_string(st).decode()


def eprop_last_error(net):
    return lib().eprop_last_error(net).decode()


# ---------------------------------------------------------------- convenience wrapper

class EpropError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{eprop_status_string(status)} ({status}): {message}")
        self.status = status


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


@dataclass
class BatchResult:
    loss: np.ndarray
    predicted: np.ndarray
    n_rec_spikes: int
    n_in_spikes: int
    n_syn_events: int
    n_out_events: int
    n_eprop_updates: int
    n_flush_updates: int
    device_seconds: float
    phase_ms: dict = field(default_factory=dict)


class TorchAllocator:
    """Device allocator callbacks backed by PyTorch's caching allocator:
    each library buffer is a uint8 tensor kept alive until the library
    returns it."""

    def __init__(self):
        import torch
        self._torch = torch
        self.blocks = {}

        def alloc(nbytes, ctx):
            t = self._torch.empty(int(nbytes) + 256, dtype=self._torch.uint8, device="cuda")
            p = (t.data_ptr() + 255) & ~255
            self.blocks[p] = t
            return p

        def free(ptr, ctx):
            self.blocks.pop(ptr, None)

        self.alloc_fn = DEV_ALLOC_FN(alloc)
        self.free_fn = DEV_FREE_FN(free)


class Network:
    """One library handle built from a ``workloads.Network``."""

    def __init__(self, wnet, precision: str = "fp32", max_trials: int = 1, max_steps: int = 1000,
                 delivery: str = "auto", graph: bool = True, stream=None, max_delay: int = None,
                 torch_alloc: bool = False, deterministic: bool = False, autotune: bool = False,
                 scatter_form: str = "auto"):
        p = wnet.params
        self.wnet = wnet
        self._keep = []
        self.is_alif = _c(wnet.is_alif, np.uint8)
        md = max_delay or max(int(p.max_delay), int(wnet.in_rec.delay.max(initial=1)),
                              int(wnet.rec_rec.delay.max(initial=1)))
        cfg = eprop_config(abi_version=EPROP_ABI_VERSION,
                           precision=EPROP_FP64 if precision == "fp64" else EPROP_FP32,
                           n_in=wnet.n_in, n_rec=wnet.n_rec, n_out=wnet.n_out, is_alif=_ptr(self.is_alif),
                           dt=p.dt, tau_m=p.tau_m, tau_out=p.tau_out, v_th=p.v_th, t_ref=p.t_ref, tau_a=p.tau_a,
                           beta_a=p.beta_a, surrogate=p.surrogate, sg_gamma=p.sg_gamma, sg_beta=p.sg_beta,
                           loss=p.loss, optimizer=p.optimizer, eta=p.eta, adam_beta1=p.adam_beta1,
                           adam_beta2=p.adam_beta2, adam_eps_hat=p.adam_eps_hat, max_delay=md,
                           max_trials=max_trials, max_steps=max_steps,
                           d_out=int(getattr(p, "d_out", 0)), d_ls=int(getattr(p, "d_ls", 0)),
                           c_reg=float(getattr(p, "c_reg", 0.0)), f_target=float(getattr(p, "f_target_hz", 0.0)),
                           reset_mode=int(getattr(p, "reset_mode", 0)), v_reset=float(getattr(p, "v_reset", 0.0)),
                           etrace_filter=int(getattr(p, "etrace_filter", 0)), tau_e=float(getattr(p, "tau_e", 0.0)),
                           reg_mode=int(getattr(p, "reg_mode", 0)), reg_tau=float(getattr(p, "reg_tau", 0.0)),
                           isi_cutoff=int(getattr(p, "isi_cutoff", 0)),
                           delivery={"auto": 0, "scatter": 1, "gather": 2}[delivery],
                           flags=(0 if graph else EPROP_FLAG_NO_GRAPH) | (EPROP_DETERMINISTIC if deterministic else 0)
                           | (EPROP_AUTOTUNE if autotune else 0)
                           | {"auto": 0, "lookup": EPROP_SCATTER_LOOKUP, "queues": EPROP_SCATTER_QUEUES}[scatter_form])
        self.allocator = TorchAllocator() if torch_alloc else None
        if self.allocator is not None:
            cfg.dev_alloc, cfg.dev_free = self.allocator.alloc_fn, self.allocator.free_fn
        projs = []
        for pr in (wnet.in_rec, wnet.rec_rec):
            arrs = (_c(pr.row_ptr, np.uint64), _c(pr.col, np.uint32), _c(pr.w, np.float64), _c(pr.delay, np.uint8))
            self._keep += arrs
            projs.append(eprop_projection(pr.n_src, pr.n_tgt, pr.nnz, *(_ptr(a) for a in arrs)))
        w_out = _c(wnet.w_out, np.float64)
        fb = _c(wnet.feedback, np.float64)
        if stream is None:
            stream = _default_stream()
        self.stream = stream
        st, h = eprop_create_network(cfg, projs[0], projs[1], _ptr(w_out), _ptr(fb), None, stream)
        self._keep = []
        if st != EPROP_OK:
            raise EpropError(st, eprop_last_error(None))
        self.h = h
        self.cfg = cfg
        self.precision = precision
        self.max_trials, self.max_steps = max_trials, max_steps

    def close(self):
        if getattr(self, "h", None):
            eprop_destroy_network(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != EPROP_OK:
            raise EpropError(st, eprop_last_error(self.h))

    def simulate(self, batch, train: bool = True, device: bool = False, profile: bool = False,
                 time_driven: bool = False, online: bool = False, noalloc: bool = False) -> BatchResult:
        """Runs one batch (a ``workloads.Batch``).  device=True places the
        batch arrays in device memory (torch) before the call; time_driven
        computes the gradient by the time-driven baseline recursion; online
        runs the trials back to back with the e-prop+ per-spike schedule
        (EPROP_BATCH_ONLINE); noalloc calls eprop_simulate_batch_noalloc."""
        ntr = batch.n_trials
        n_steps = _c(batch.n_steps, np.uint32)
        stride = int(n_steps.max())
        host = {"in_ptr": _c(batch.in_ptr, np.uint64), "in_step": _c(batch.in_step, np.uint32),
                "in_src": _c(batch.in_src, np.uint32)}
        if batch.target is not None:
            host["target"] = _c(batch.target[:, :stride], np.float64)
        if batch.window is not None:
            host["window"] = _c(batch.window[:, :stride], np.uint8)
        if batch.forced_ptr is not None:
            host["forced_ptr"] = _c(batch.forced_ptr, np.uint64)
            host["forced_step"] = _c(batch.forced_step, np.uint32)
            host["forced_neuron"] = _c(batch.forced_neuron, np.uint32)
        label = _c(batch.label, np.uint32) if batch.label is not None else None
        keep = [n_steps, label]
        if device:
            ptrs, keep2 = to_device(host)
            keep += keep2
        else:
            ptrs = {k: _ptr(v) for k, v in host.items()}
            keep += list(host.values())
        b = eprop_batch(n_trials=ntr, memory=EPROP_MEM_DEVICE if device else EPROP_MEM_HOST,
                        n_steps=_ptr(n_steps), n_in_spikes=int(batch.in_ptr[-1]), in_ptr=ptrs["in_ptr"],
                        in_step=ptrs["in_step"], in_src=ptrs["in_src"], step_stride=stride,
                        target=ptrs.get("target"), label=_ptr(label), window=ptrs.get("window"),
                        n_forced=int(batch.forced_ptr[-1]) if batch.forced_ptr is not None else 0,
                        forced_ptr=ptrs.get("forced_ptr"), forced_step=ptrs.get("forced_step"),
                        forced_neuron=ptrs.get("forced_neuron"),
                        flags=(EPROP_BATCH_TRAIN if train else 0) | (EPROP_BATCH_PROFILE if profile else 0)
                        | (EPROP_BATCH_TIME_DRIVEN if time_driven else 0) | (EPROP_BATCH_ONLINE if online else 0))
        loss = np.zeros(ntr)
        pred = np.zeros(ntr, np.uint32)
        res = eprop_batch_result(loss=_ptr(loss), predicted=_ptr(pred))
        self._check((eprop_simulate_batch_noalloc if noalloc else eprop_simulate_batch)(self.h, b, res))
        del keep
        return BatchResult(loss, pred, res.n_rec_spikes, res.n_in_spikes, res.n_syn_events, res.n_out_events,
                           res.n_eprop_updates, res.n_flush_updates, res.device_seconds,
                           {k: res.phase_ms[i] for i, k in enumerate(PHASES)} if profile else {})

    def apply(self):
        self._check(eprop_apply_updates(self.h))

    def read(self, what: int, trial: int = 0) -> np.ndarray:
        st, need = eprop_read_state(self.h, what, trial, None, 0)
        self._check(st)
        if what == EPROP_STATE_SPIKES:
            buf = np.zeros(max(need // 4, 1), np.uint32)
            st, need = eprop_read_state(self.h, what, trial, _ptr(buf), buf.nbytes)
            self._check(st)
            return buf[:need // 4].reshape(-1, 2)
        if what == EPROP_STATE_LAYOUT:
            buf = np.zeros(max(need // 8, 1), np.uint64)
            self._check(eprop_read_state(self.h, what, trial, _ptr(buf), buf.nbytes)[0])
            return buf
        if what == EPROP_STATE_ADAM_STEP:
            buf = np.zeros(1, np.uint64)
            self._check(eprop_read_state(self.h, what, trial, _ptr(buf), 8)[0])
            return buf
        buf = np.zeros(max(need // 8, 1), np.float64)
        st, need = eprop_read_state(self.h, what, trial, _ptr(buf), buf.nbytes)
        self._check(st)
        return buf[:need // 8]

    def layout(self) -> dict:
        v = [int(x) for x in self.read(EPROP_STATE_LAYOUT)]
        return dict(zip(("tile_neurons", "tiles", "ring_bytes", "tile_threads", "synapse_threads",
                         "synapse_trials", "steps_per_launch", "gather", "piece", "pieces_in_flight",
                         "adjoint_threads", "autotuned", "piece_table", "synapse_prefetch", "synapse_batch",
                         "blocked_update", "forward_trials_per_launch", "queues"), v))

    def weights(self) -> dict:
        return {"w_in": self.read(EPROP_STATE_W_IN), "w_rec": self.read(EPROP_STATE_W_REC),
                "w_out": self.read(EPROP_STATE_W_OUT).reshape(self.wnet.n_out, self.wnet.n_rec)}

    def grads(self) -> dict:
        return {"w_in": self.read(EPROP_STATE_GRAD_IN), "w_rec": self.read(EPROP_STATE_GRAD_REC),
                "w_out": self.read(EPROP_STATE_GRAD_OUT).reshape(self.wnet.n_out, self.wnet.n_rec)}

    def spikes(self, trial: int, n_steps: int) -> np.ndarray:
        """Recurrent spikes of a trial of the last batch as a [T, J] 0/1 array."""
        return spikes_dense(self.read(EPROP_STATE_SPIKES, trial), n_steps, self.wnet.n_rec)


def _default_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


def to_device(host: dict):
    """Copies numpy arrays into torch device tensors; returns their pointers."""
    import torch
    ptrs, keep = {}, []
    for k, v in host.items():
        t = torch.from_numpy(np.ascontiguousarray(v).view(np.uint8).copy()).to("cuda")
        keep.append(t)
        ptrs[k] = t.data_ptr()
    torch.cuda.synchronize()
    return ptrs, keep


def spikes_dense(pairs: np.ndarray, n_steps: int, n_rec: int) -> np.ndarray:
    z = np.zeros((n_steps, n_rec), np.uint8)
    if pairs.size:
        z[pairs[:, 0] - 1, pairs[:, 1]] = 1
    return z
