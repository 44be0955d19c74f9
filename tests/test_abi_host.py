"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/eprop.h, and rejects bad arguments before it
touches a device."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2511_21674_amd import eprop as E
from paper_2511_21674_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "eprop.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(eprop_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("eprop_create_network", "eprop_simulate_batch", "eprop_apply_updates", "eprop_read_state"):
        assert n in names
    assert set(names) == set(E.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(E.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_header_constants_match_the_binding():
    """Every #define EPROP_* with an integer value in include/eprop.h equals
    the binding's constant of the same name."""
    src = open(os.path.join(ROOT, "include", "eprop.h")).read()
    found = 0
    for name, val in re.findall(r"#define\s+(EPROP_[A-Z0-9_]+)\s+\(?([0-9]+u?(?:\s*<<\s*[0-9]+)?)\)?", src):
        if not hasattr(E, name):
            continue
        parts = [int(x) for x in val.replace("u", "").split("<<")]  # a literal, or a literal shifted
        expect = parts[0] << parts[1] if len(parts) == 2 else parts[0]
        assert getattr(E, name) == expect, (name, getattr(E, name), expect)
        found += 1
    assert found >= 6, found


def test_status_strings():
    assert E.eprop_status_string(E.EPROP_OK) == "ok"
    assert "invalid" in E.eprop_status_string(E.EPROP_ERR_INVALID_ARGUMENT)
    assert E.eprop_status_string(12345) == "unknown status"


def test_struct_layout_matches_the_c_compiler(tmp_path):
    """Every field offset and struct size of the binding equals what a C
    compiler makes of include/eprop.h."""
    structs = [E.eprop_config, E.eprop_projection, E.eprop_optimizer_state, E.eprop_batch,
               E.eprop_batch_result]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "eprop.h"', "int main(void) {"]
    for st in structs:
        lines.append(f'  printf("{st.__name__} size %zu\\n", sizeof({st.__name__}));')
        for name, _ in st._fields_:
            lines.append(f'  printf("{st.__name__} {name} %zu\\n", offsetof({st.__name__}, {name}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for st in structs:
        assert got[(st.__name__, "size")] == C.sizeof(st), st.__name__
        for name, _ in st._fields_:
            assert got[(st.__name__, name)] == getattr(st, name).offset, (st.__name__, name)


def test_config_rejects_bad_delays_regulariser_and_short_history():
    cfg, projs, wo, fb, keep = _parts(W.tiny().network, d_out=70000)
    assert _create(cfg, projs, wo, fb)[0] == E.EPROP_ERR_INVALID_ARGUMENT
    cfg, projs, wo, fb, keep = _parts(W.tiny().network, d_ls=1 << 20)
    assert _create(cfg, projs, wo, fb)[0] == E.EPROP_ERR_INVALID_ARGUMENT
    cfg, projs, wo, fb, keep = _parts(W.tiny().network, c_reg=-1.0)
    assert _create(cfg, projs, wo, fb)[0] == E.EPROP_ERR_INVALID_ARGUMENT
    cfg, projs, wo, fb, keep = _parts(W.tiny().network, c_reg=float("nan"))
    assert _create(cfg, projs, wo, fb)[0] == E.EPROP_ERR_INVALID_ARGUMENT
    cfg, projs, wo, fb, keep = _parts(W.tiny().network, f_target=float("inf"))
    assert _create(cfg, projs, wo, fb)[0] == E.EPROP_ERR_INVALID_ARGUMENT
    cfg, projs, wo, fb, keep = _parts(W.tiny().network, history_steps=100)   # max_steps is 200
    assert _create(cfg, projs, wo, fb)[0] == E.EPROP_ERR_UNSUPPORTED
    cfg, projs, wo, fb, keep = _parts(W.tiny().network, flags=1 << 7)
    assert _create(cfg, projs, wo, fb)[0] == E.EPROP_ERR_INVALID_ARGUMENT
    # the two scatter forms exclude each other
    cfg, projs, wo, fb, keep = _parts(W.tiny().network, flags=E.EPROP_SCATTER_LOOKUP | E.EPROP_SCATTER_QUEUES)
    st, msg = _create(cfg, projs, wo, fb)
    assert st == E.EPROP_ERR_INVALID_ARGUMENT and "exclude" in msg, msg
    cfg, projs, wo, fb, keep = _parts(W.tiny().network, precision=E.EPROP_FP64, delivery=1,
                                      flags=E.EPROP_DETERMINISTIC)
    assert _create(cfg, projs, wo, fb)[0] == E.EPROP_ERR_INVALID_ARGUMENT
    cfg, projs, wo, fb, keep = _parts(W.tiny().network)
    cfg.dev_alloc = E.DEV_ALLOC_FN(lambda n, c: None)   # allocator without its free function
    assert _create(cfg, projs, wo, fb)[0] == E.EPROP_ERR_INVALID_ARGUMENT


def _parts(wnet, **cfg_over):
    p = wnet.params
    ia = np.ascontiguousarray(wnet.is_alif, np.uint8)
    cfg = E.eprop_config(abi_version=E.EPROP_ABI_VERSION, precision=E.EPROP_FP32, n_in=wnet.n_in,
                         n_rec=wnet.n_rec, n_out=wnet.n_out, is_alif=ia.ctypes.data, dt=p.dt, tau_m=p.tau_m,
                         tau_out=p.tau_out, v_th=p.v_th, t_ref=p.t_ref, tau_a=p.tau_a, beta_a=p.beta_a,
                         surrogate=p.surrogate, sg_gamma=p.sg_gamma, sg_beta=p.sg_beta, loss=p.loss,
                         optimizer=p.optimizer, eta=p.eta, adam_beta1=0.9, adam_beta2=0.999, adam_eps_hat=1e-7,
                         max_delay=2, max_trials=2, max_steps=200, delivery=0, flags=0)
    for k, v in cfg_over.items():
        setattr(cfg, k, v)
    keep = [ia]
    projs = []
    for pr in (wnet.in_rec, wnet.rec_rec):
        arrs = [np.array(pr.row_ptr, np.uint64), np.array(pr.col, np.uint32),
                np.array(pr.w, np.float64), np.array(pr.delay, np.uint8)]
        keep += arrs
        projs.append((E.eprop_projection(pr.n_src, pr.n_tgt, pr.nnz, *(a.ctypes.data for a in arrs)), arrs))
    wo = np.array(wnet.w_out, np.float64)
    fb = np.ascontiguousarray(wnet.feedback, np.float64)
    keep += [wo, fb]
    return cfg, projs, wo, fb, keep


def _create(cfg, projs, wo, fb):
    st, h = E.eprop_create_network(cfg, projs[0][0], projs[1][0], wo.ctypes.data, fb.ctypes.data, None, None)
    if st == E.EPROP_OK:
        E.eprop_destroy_network(h)
    return st, E.eprop_last_error(None)


@pytest.mark.parametrize("field,value,expect", [
    ("abi_version", 99, E.EPROP_ERR_UNSUPPORTED),
    ("n_out", 0, E.EPROP_ERR_INVALID_ARGUMENT),
    ("n_out", 65, E.EPROP_ERR_INVALID_ARGUMENT),
    ("precision", 7, E.EPROP_ERR_INVALID_ARGUMENT),
    ("dt", 0.0, E.EPROP_ERR_INVALID_ARGUMENT),
    ("tau_m", float("nan"), E.EPROP_ERR_INVALID_ARGUMENT),
    ("max_delay", 1, E.EPROP_ERR_INVALID_ARGUMENT),      # the network has delays of 2
    ("max_steps", 70000, E.EPROP_ERR_INVALID_ARGUMENT),
    ("max_trials", 0, E.EPROP_ERR_INVALID_ARGUMENT),
    ("t_ref", 500.0, E.EPROP_ERR_INVALID_ARGUMENT),
    ("t_ref", 1e300, E.EPROP_ERR_INVALID_ARGUMENT),
    ("surrogate", 5, E.EPROP_ERR_INVALID_ARGUMENT),
    ("delivery", 9, E.EPROP_ERR_INVALID_ARGUMENT),
])
def test_create_rejects_bad_config(field, value, expect):
    cfg, projs, wo, fb, keep = _parts(W.tiny().network, **{field: value})
    st, msg = _create(cfg, projs, wo, fb)
    assert st == expect, msg
    assert msg


def test_create_rejects_bad_graphs():
    wnet = W.tiny().network
    # self-connection in the recurrent projection
    cfg, projs, wo, fb, keep = _parts(wnet)
    arrs = projs[1][1]
    arrs[1][0] = 0          # first synapse of source 0 now targets neuron 0
    st, msg = _create(cfg, projs, wo, fb)
    assert st == E.EPROP_ERR_INVALID_ARGUMENT and "self" in msg
    # duplicate pair
    cfg, projs, wo, fb, keep = _parts(wnet)
    arrs = projs[0][1]
    arrs[1][1] = arrs[1][0]
    st, msg = _create(cfg, projs, wo, fb)
    assert st == E.EPROP_ERR_INVALID_ARGUMENT and "duplicate" in msg
    # non-finite weight
    cfg, projs, wo, fb, keep = _parts(wnet)
    projs[0][1][2][3] = np.inf
    st, msg = _create(cfg, projs, wo, fb)
    assert st == E.EPROP_ERR_INVALID_ARGUMENT and "finite" in msg
    # target out of range
    cfg, projs, wo, fb, keep = _parts(wnet)
    projs[0][1][1][0] = 99
    st, msg = _create(cfg, projs, wo, fb)
    assert st == E.EPROP_ERR_INVALID_ARGUMENT and "range" in msg
    # delay 0
    cfg, projs, wo, fb, keep = _parts(wnet)
    projs[1][1][3][0] = 0
    st, msg = _create(cfg, projs, wo, fb)
    assert st == E.EPROP_ERR_INVALID_ARGUMENT and "delay" in msg
    # non-finite readout weight
    cfg, projs, wo, fb, keep = _parts(wnet)
    wo[0, 0] = np.nan
    st, msg = _create(cfg, projs, wo, fb)
    assert st == E.EPROP_ERR_INVALID_ARGUMENT


def test_valid_network_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    cfg, projs, wo, fb, keep = _parts(W.tiny().network)
    st, msg = _create(cfg, projs, wo, fb)
    assert st == E.EPROP_ERR_DEVICE, msg


def test_null_handles_are_safe():
    E.eprop_destroy_network(None)
    assert E.lib().eprop_apply_updates(None) == E.EPROP_ERR_INVALID_ARGUMENT
    assert E.lib().eprop_simulate_batch(None, None, None) == E.EPROP_ERR_INVALID_ARGUMENT
    assert E.lib().eprop_read_state(None, 0, 0, None, 0, None) == E.EPROP_ERR_INVALID_ARGUMENT


def test_threaded_graph_build_finds_duplicates():
    """Graphs of 2^22 synapses or more are transposed by several host threads
    over ranges of sources: a repeated pair inside one source row is still
    rejected, and a clean graph of that size passes the host build (the
    call then stops at the missing device, or succeeds on a GPU)."""
    wnet = W.c4_sparse(n_rec=4500, n_steps=10, batch_size=1, n_in=100).network
    assert wnet.rec_rec.nnz >= (1 << 22)
    cfg, projs, wo, fb, keep = _parts(wnet, max_delay=5)
    st, msg = _create(cfg, projs, wo, fb)
    assert st in (E.EPROP_OK, E.EPROP_ERR_DEVICE), msg
    for src in (7, 4321):       # a row near the start and one near the end of the sources
        cfg, projs, wo, fb, keep = _parts(wnet, max_delay=5)
        row_ptr, col = projs[1][1][0], projs[1][1][1]
        lo = int(row_ptr[src])
        col[lo + 1] = col[lo]
        st, msg = _create(cfg, projs, wo, fb)
        assert st == E.EPROP_ERR_INVALID_ARGUMENT and "duplicate" in msg, (src, st, msg)


def test_create_error_message_is_per_thread():
    """eprop_last_error(NULL) gives the last failure of eprop_create_network
    in the calling thread: a failure in another thread does not replace it."""
    import threading
    wnet = W.tiny().network
    cfg, projs, wo, fb, keep = _parts(wnet, n_out=0)
    st, msg_main = _create(cfg, projs, wo, fb)
    assert st == E.EPROP_ERR_INVALID_ARGUMENT and "n_out" in msg_main
    seen = {}

    def other():
        cfg2, projs2, wo2, fb2, keep2 = _parts(wnet, max_trials=0)
        seen["st"], seen["msg"] = _create(cfg2, projs2, wo2, fb2)

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert seen["st"] == E.EPROP_ERR_INVALID_ARGUMENT and "max_trials" in seen["msg"]
    assert E.eprop_last_error(None) == msg_main
