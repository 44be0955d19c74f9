"""Benchmark of the event-driven e-prop hot path on one MI355X.

A step is one pass of the whole path over one batch: eprop_simulate_batch
(input staging, forward pass, readout and loss, archive pass, event-driven
synapse gradient, output gradient) followed by eprop_apply_updates.  The
batches are synthetic (seeded generators) and already in device memory when
the timed region starts.  Default workload: the 1e5-neuron network with
1e8 recurrent synapses (fixed in-degree 1000, delays 1-5), 4 trials of
1000 steps per batch, FP32.

Prints one JSON line:
  metric/value: synaptic events per second (input + recurrent deliveries
  that arrive within their trial), whole job; e-prop synapse updates per
  second beside it; roofline of the dominant kernel; the CPU oracle timed on
  a bounded sample of the same workload; the FP64 plain path (same kernels
  in double, one trial at a time, deterministic delivery) for comparison.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(phase, rs, counts, net, batch_T, n_trials, kt, launches):
    """Algorithmic HBM bytes of one phase (the per-unit figures are derived
    in the design doc).  counts: dict of events, rec_spikes, in_spikes."""
    J, Jp = net.n_rec, (net.n_rec + 63) // 64 * 64
    S = net.in_rec.nnz + net.rec_rec.nnz
    neuron_steps = n_trials * batch_T * Jp
    spikes = counts["rec_spikes"] + counts["in_spikes"]
    if phase == "forward":
        # per event: packed target+delay (4 B) and weight (rs); per neuron-step:
        # psi write (rs) and spike bit (1/8 B); per spike: tile offsets (8 B per
        # tile), list entry written and read per tile (4 B + 4 B per tile), spike
        # time (2 B); per launch and neuron: state and ring saved and restored.
        R = 6
        return (counts["events"] * (4 + rs) + neuron_steps * (rs + 0.125)
                + spikes * (8 * kt + 4 + 4 * kt + 2)
                + launches * n_trials * Jp * 2 * ((R + 2) * rs + 1))
    if phase == "synapse":
        # per synapse: packed source+delay (4 B), Kahan pair read and written
        # (4 rs); per trial, neuron and step: archive row read once (rs); per
        # trial and source: spike count (4 B) and spike times (2 B each).
        return S * (4 + 4 * rs) + neuron_steps * rs + n_trials * (net.n_in + J) * 4 + spikes * 2
    if phase == "adjoint":
        # per trial, neuron and step: psi read and archive written (2 rs)
        return neuron_steps * 2 * rs
    return None


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 byte
    counters (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter
    reads for a plain copy of known size), or None when there is no record
    for this workload or the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    src = os.path.join(ROOT, "paper_2511_21674_amd", "csrc", "eprop_kernels.hip")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ": " in line:
            k, v = line.strip().split(": ", 1)
            rec[k] = v
    if not rec.get("kernel", "").startswith(kernel):
        return None
    if rec.get("kernel_source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return (float(rec["fetch_kib_per_dispatch"]) * float(rec["copy_fetch_factor"])
            + float(rec["write_kib_per_dispatch"]) * float(rec["copy_write_factor"])) * 1024.0


def stage_batches(wl, n, first_iteration):
    from paper_2511_21674_amd import eprop as E
    out = []
    for i in range(n):
        b = wl.make_batch(first_iteration + i, 0, wl.batch_size)
        host = {"in_ptr": np.ascontiguousarray(b.in_ptr, np.uint64),
                "in_step": np.ascontiguousarray(b.in_step, np.uint32),
                "in_src": np.ascontiguousarray(b.in_src, np.uint32)}
        if b.target is not None:
            host["target"] = np.ascontiguousarray(b.target, np.float64)
        if b.window is not None:
            host["window"] = np.ascontiguousarray(b.window, np.uint8)
        ptrs, keep = E.to_device(host)
        out.append((b, ptrs, keep))
    return out


def run_staged(net, staged, train=True, profile=False):
    """simulate_batch on device-resident arrays (no host copies)."""
    from paper_2511_21674_amd import eprop as E
    b, ptrs, _ = staged
    n_steps = np.ascontiguousarray(b.n_steps, np.uint32)
    label = np.ascontiguousarray(b.label, np.uint32) if b.label is not None else None
    batch = E.eprop_batch(n_trials=b.n_trials, memory=E.EPROP_MEM_DEVICE, n_steps=n_steps.ctypes.data,
                          n_in_spikes=int(b.in_ptr[-1]), in_ptr=ptrs["in_ptr"], in_step=ptrs["in_step"],
                          in_src=ptrs["in_src"], step_stride=int(b.target.shape[1]) if b.target is not None
                          else int(b.window.shape[1]),
                          target=ptrs.get("target"), label=label.ctypes.data if label is not None else None,
                          window=ptrs.get("window"),
                          flags=(E.EPROP_BATCH_TRAIN if train else 0) | (E.EPROP_BATCH_PROFILE if profile else 0))
    loss = np.zeros(b.n_trials)
    res = E.eprop_batch_result(loss=loss.ctypes.data, predicted=None)
    st = E.eprop_simulate_batch(net.h, batch, res)
    if st != E.EPROP_OK:
        raise E.EpropError(st, E.eprop_last_error(net.h))
    return res, loss


def cpu_baseline(wl, n_steps_sample):
    """The FP64 oracle (event-driven gradient) on the first n steps of one
    trial of the same workload, single thread."""
    import oracle as O
    from paper_2511_21674_amd import workloads as W
    b = wl.make_batch(0, 0, 1)
    T = n_steps_sample
    keep = b.in_step < T
    lo = int(b.in_ptr[0])
    sb = W.Batch(n_steps=np.array([T], np.uint32), in_ptr=np.array([0, int(keep.sum())], np.uint64),
                 in_step=b.in_step[keep], in_src=b.in_src[keep])
    if b.target is not None:
        sb.target = np.ascontiguousarray(b.target[:1, :T])
    if b.label is not None:
        sb.label = b.label[:1]
    if b.window is not None:
        sb.window = np.ascontiguousarray(b.window[:1, :T])
    on = O.OracleNet(wl.network)
    g = O.zero_grads(on)
    t0 = time.perf_counter()
    r = O.run_trial(on, sb, 0, 2, g, trace=True)
    el = time.perf_counter() - t0
    # events: deliveries arriving within the sample (same definition as the GPU)
    net = wl.network
    ev = 0
    for proj, spikes in ((net.in_rec, [(int(s), int(i)) for s, i in zip(sb.in_step, sb.in_src)]),
                         (net.rec_rec, [(int(t) + 1, int(j)) for t, j in zip(*np.nonzero(r.trace["z"]))])):
        rp = proj.row_ptr.astype(np.int64)
        for s, i in spikes:
            d = proj.delay[rp[i]:rp[i + 1]].astype(np.int64)
            ev += int(np.count_nonzero(s + d <= T))
    return {"value": ev / el, "unit": "synaptic events/s", "cores": 1, "kind": "oracle",
            "sample": f"first {T} steps of one trial of the same network (event-driven gradient, "
                      f"{ev} events, {el:.1f} s, network construction excluded)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4_sparse")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB mebibytes three times (the reference "
                         "kernel for scaling hardware byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding of this "
              "path is a design note, not a measured configuration.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_21674_amd import eprop as E
    from paper_2511_21674_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4, "launches": 3}), flush=True)
        return
    wl = W.WORKLOADS[args.workload]()
    net_w = wl.network
    T = max(int(wl.make_batch(0, 0, 1).n_steps.max()), 1)
    if args.workload == "c2_evidence":
        T = 1800
    print(f"[bench] workload {wl.name}: J={net_w.n_rec} I={net_w.n_in} K={net_w.n_out} "
          f"synapses={net_w.in_rec.nnz + net_w.rec_rec.nnz} batch={wl.batch_size} T={T}", file=sys.stderr, flush=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        net = E.Network(net_w, "fp32", max_trials=wl.batch_size, max_steps=T,
                        stream=E.C.c_void_p(stream.cuda_stream))
        staged = stage_batches(wl, args.warmup + args.steps, 0)
        torch.cuda.synchronize()
        for i in range(args.warmup):
            run_staged(net, staged[i])
            net.apply()
        torch.cuda.synchronize()
        tot = {"events": 0, "updates": 0, "rec_spikes": 0, "in_spikes": 0}
        phases = {k: 0.0 for k in E.PHASES}
        losses = []
        t0 = time.perf_counter()
        for i in range(args.steps):
            res, loss = run_staged(net, staged[args.warmup + i], profile=True)
            net.apply()
            tot["events"] += res.n_syn_events
            tot["updates"] += res.n_eprop_updates
            tot["rec_spikes"] += res.n_rec_spikes
            tot["in_spikes"] += res.n_in_spikes
            for k, name in enumerate(E.PHASES):
                phases[name] += res.phase_ms[k]
            losses.append(float(loss.mean()))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    steps = args.steps
    n_tr = wl.batch_size
    rate_hz = tot["rec_spikes"] / (steps * n_tr * net_w.n_rec * T * net_w.params.dt / 1000.0)
    lay = net.layout()
    kt = lay["tiles"]
    launches = -(-T // lay["steps_per_launch"])
    cand = {}
    for ph in ("forward", "synapse", "adjoint"):
        ab = algorithmic_bytes(ph, 4, {k: v / steps for k, v in tot.items()}, net_w, T, n_tr, kt, launches)
        ms = phases[ph] / steps
        cand[ph] = (ms, ab)
    dom = max(cand, key=lambda k: cand[k][0])
    ms, ab = cand[dom]
    n_launch = launches if dom == "forward" else 1
    achieved = ab / (ms / 1000.0) / 1e9
    roof = {"kernel": {"forward": "k_forward_tiled", "synapse": "k_synapse", "adjoint": "k_adjoint"}[dom],
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "avg_launch_ms": round(ms / n_launch, 4), "algorithmic_bytes_per_launch": int(ab / n_launch)}
    tr = measured_traffic(wl.name, roof["kernel"])
    if tr is not None:
        roof["traffic"] = round(tr / 1e9, 3)
        roof["traffic_unit"] = "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"

    fp64 = None
    if not args.no_fp64:
        with torch.cuda.stream(stream):
            net64 = E.Network(net_w, "fp64", max_trials=1, max_steps=T, delivery="gather",
                              stream=E.C.c_void_p(stream.cuda_stream))
            b0 = staged[args.warmup][0]
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ev64, loss64 = 0, []
            for i in range(b0.n_trials):
                r = net64.simulate(b0.trial(i), train=True)
                ev64 += r.n_syn_events
                loss64.append(float(r.loss[0]))
            net64.apply()
            torch.cuda.synchronize()
            el64 = time.perf_counter() - t1
            net64.close()
        gpu32_ev_s = tot["events"] / elapsed
        fp64 = {"value": ev64 / el64, "unit": "synaptic events/s", "seconds_per_batch": el64,
                "speedup_fp32_batched": gpu32_ev_s / (ev64 / el64),
                "loss_fp64_first_batch": float(np.mean(loss64)), "loss_fp32_first_timed_batch": losses[0]}
    net.close()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, min(args.cpu_steps, T))

    out = {"metric": "synaptic events/s (event-driven e-prop training, FP32 batched)",
           "value": tot["events"] / elapsed, "unit": "synaptic events/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": elapsed / steps * 1000.0, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": f"{wl.name}: {wl.description}", "n_rec": net_w.n_rec, "n_in": net_w.n_in,
                      "n_out": net_w.n_out, "synapses": int(net_w.in_rec.nnz + net_w.rec_rec.nnz),
                      "trials_per_batch": n_tr, "steps_per_trial": T, "delivery": "scatter (LDS tiles)"},
           "eprop_updates_per_s": tot["updates"] / elapsed,
           "recurrent_rate_hz": rate_hz,
           "phase_ms_per_step": {k: round(v / steps, 3) for k, v in phases.items()},
           "mean_loss": losses,
           "layout": lay, "roofline": roof, "cpu_baseline": cpu, "fp64_plain": fp64}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
