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


# Algorithmic bytes per unit of work (FP32): what the method has to move
# at the least, whatever the implementation.
B_EVENT = 12            # synaptic event: target index 4 + weight 4 + ring add 4
B_UPDATE_LIF = 24       # e-prop update fused with its event, LIF target (trace, g, c read and written)
B_UPDATE_ALIF = 32      # ... ALIF target (adds the adaptation trace)
B_OUT_EVENT = 20        # recurrent spike to one readout: weight 4 + (g, c) read and written
B_NEURON_LIF = 34       # neuron-step: v r/w 8, refractory 2, ring slot read+clear 8, history write 8
B_NEURON_ALIF = 42      #   and history read 8 (ALIF: + a r/w 8)
B_SOURCE = 16           # spiking source: last spike time and presynaptic trace read and written
B_FWD_NEURON_LIF = 22   # forward kernel's share of a neuron-step: v 8, refractory 2, ring 8, psi 4
B_FWD_NEURON_ALIF = 30  #   (ALIF: + a r/w 8)


def path_bytes(c, net, n_trials, adam):
    """Algorithmic bytes of one batch step of the whole path (forward,
    readout, gradients, optimiser).  c: per-step counts."""
    n_alif = int(np.count_nonzero(net.is_alif)) if net.is_alif is not None else 0
    frac_alif = n_alif / net.n_rec
    S = net.in_rec.nnz + net.rec_rec.nnz
    per_iter = S * (8 * n_trials + 8 + (16 if adam else 0))
    return (c["events"] * (B_EVENT + B_UPDATE_LIF + frac_alif * (B_UPDATE_ALIF - B_UPDATE_LIF))
            + c["neuron_steps"] * (B_NEURON_LIF + frac_alif * (B_NEURON_ALIF - B_NEURON_LIF))
            + c["rec_spikes"] * net.n_out * B_OUT_EVENT
            + (c["rec_spikes"] + c["in_spikes"]) * B_SOURCE + per_iter)


def design_bytes(c, net, n_trials, adam, blocked, K):
    """Bytes this design has to move in one batch step, by kernel (the
    per-unit figures of the kernels' own algorithms rather than the
    survey's per-synapse trace model, which this design never materialises):
    forward 12 B per event + 22 B (LIF) / 30 B (ALIF) per neuron-step;
    spike-time lists 1/8 B per neuron-step + 2 B per spike; readout
    5 x 8 B per readout and trial-step; adjoint 8 B per neuron-step (psi
    read, phi written); synapse kernel 20 B per synapse (packed source 4,
    gradient pair read and written 16) + 4 B per neuron-step (phi staged)
    + 16 B per source record + 2 B per spike; output reduction
    8 B per output synapse and trial + 16; update 26 B per synapse blocked
    (10 B of target-major runs, 16 B records read and written) or 28 B in
    target-major order, + 16 B with Adam."""
    S = net.in_rec.nnz + net.rec_rec.nnz
    ns = c["neuron_steps"]
    spikes = c["rec_spikes"] + c["in_spikes"]
    trial_steps = ns / net.n_rec
    fwd = forward_bytes(c, net)
    parts = {"forward": fwd, "spike_lists": ns / 8 + 2 * spikes, "readout": 40 * K * trial_steps,
             "adjoint": 8 * ns, "synapse": 20 * S + 4 * ns + 16 * (net.n_in + net.n_rec) + 2 * spikes,
             "output": K * net.n_rec * (8 * n_trials + 16),
             "update": S * ((26 if blocked else 28) + (16 if adam else 0))}
    return parts


def forward_bytes(c, net):
    """Algorithmic bytes of the forward kernel (delivery and neuron updates)
    for one batch step."""
    n_alif = int(np.count_nonzero(net.is_alif)) if net.is_alif is not None else 0
    frac_alif = n_alif / net.n_rec
    return (c["events"] * B_EVENT
            + c["neuron_steps"] * (B_FWD_NEURON_LIF + frac_alif * (B_FWD_NEURON_ALIF - B_FWD_NEURON_LIF)))


def kernel_code_hash(path):
    """SHA-256 of a kernel source with its comments and blank space removed,
    so that the record of a measurement survives comment-only edits."""
    import hashlib
    import re
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    code = "\n".join(line.strip() for line in text.splitlines() if line.strip())
    return hashlib.sha256(code.encode()).hexdigest()


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 byte
    counters (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter
    reads for a plain copy of known size), or None when there is no record
    for this workload or the kernel source changed since it was taken.
    kernel "step": the bytes of every kernel of one batch step
    (profiles/hbm_traffic_<workload>_step.md, per-step figures)."""
    if kernel == "step":
        rec = _traffic_record(os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}_step.md"), "step")
        if rec is None:
            return None
        return (float(rec["fetch_kib_per_step"]) * float(rec["copy_fetch_factor"])
                + float(rec["write_kib_per_step"]) * float(rec["copy_write_factor"])) * 1024.0
    rec = _traffic_record(os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md"), kernel)
    if rec is None:
        return None
    return (float(rec["fetch_kib_per_dispatch"]) * float(rec["copy_fetch_factor"])
            + float(rec["write_kib_per_dispatch"]) * float(rec["copy_write_factor"])) * 1024.0


def _traffic_record(path, kernel):
    """The key: value lines of a committed counter record, if it is for
    `kernel` and for the kernel source as it is now."""
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
    if rec.get("kernel_code_sha256") != kernel_code_hash(src):
        return None
    return rec


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
        if b.forced_ptr is not None:
            host["forced_ptr"] = np.ascontiguousarray(b.forced_ptr, np.uint64)
            host["forced_step"] = np.ascontiguousarray(b.forced_step, np.uint32)
            host["forced_neuron"] = np.ascontiguousarray(b.forced_neuron, np.uint32)
        ptrs, keep = E.to_device(host)
        out.append((b, ptrs, keep))
    return out


def run_staged(net, staged, train=True, profile=False, time_driven=False):
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
                          n_forced=int(b.forced_ptr[-1]) if b.forced_ptr is not None else 0,
                          forced_ptr=ptrs.get("forced_ptr"), forced_step=ptrs.get("forced_step"),
                          forced_neuron=ptrs.get("forced_neuron"),
                          flags=(E.EPROP_BATCH_TRAIN if train else 0) | (E.EPROP_BATCH_PROFILE if profile else 0)
                          | (E.EPROP_BATCH_TIME_DRIVEN if time_driven else 0))
    loss = np.zeros(b.n_trials)
    res = E.eprop_batch_result(loss=loss.ctypes.data, predicted=None)
    st = E.eprop_simulate_batch(net.h, batch, res)
    if st != E.EPROP_OK:
        raise E.EpropError(st, E.eprop_last_error(net.h))
    return res, loss


def _events_of_trial(net, b, i, z):
    """Deliveries arriving within trial i, from its input spikes and the
    recorded recurrent spikes z ([T, J]) (same definition as the library)."""
    T = int(b.n_steps[i])
    lo, hi = int(b.in_ptr[i]), int(b.in_ptr[i + 1])
    ev = 0
    for proj, spikes in ((net.in_rec, zip(b.in_step[lo:hi].tolist(), b.in_src[lo:hi].tolist())),
                         (net.rec_rec, [(int(t) + 1, int(j)) for t, j in zip(*np.nonzero(z))])):
        rp = proj.row_ptr.astype(np.int64)
        for s, src in spikes:
            d = proj.delay[rp[src]:rp[src + 1]].astype(np.int64)
            ev += int(np.count_nonzero(s + d <= T))
    return ev


def _truncated(b, i, T):
    """Trial i of batch b cut to its first T steps."""
    from paper_2511_21674_amd import workloads as W
    lo, hi = int(b.in_ptr[i]), int(b.in_ptr[i + 1])
    keep = b.in_step[lo:hi] < T
    sb = W.Batch(n_steps=np.array([T], np.uint32), in_ptr=np.array([0, int(keep.sum())], np.uint64),
                 in_step=b.in_step[lo:hi][keep], in_src=b.in_src[lo:hi][keep])
    if b.target is not None:
        sb.target = np.ascontiguousarray(b.target[i:i + 1, :T])
    if b.label is not None:
        sb.label = b.label[i:i + 1]
    if b.window is not None:
        sb.window = np.ascontiguousarray(b.window[i:i + 1, :T])
    if b.forced_ptr is not None:
        flo, fhi = int(b.forced_ptr[i]), int(b.forced_ptr[i + 1])
        fk = b.forced_step[flo:fhi] <= T
        sb.forced_ptr = np.array([0, int(fk.sum())], np.uint64)
        sb.forced_step = b.forced_step[flo:fhi][fk]
        sb.forced_neuron = b.forced_neuron[flo:fhi][fk]
    return sb


def cpu_baseline(wl, n_steps_sample, budget_s=20.0):
    """The FP64 oracle on one host core.  Networks up to a few thousand
    neurons: whole trials of the first batch, event-driven gradient (value)
    and time-driven gradient (beside it), as many trials as fit the time
    budget.  Larger networks: the first n steps of one trial, event-driven."""
    import oracle as O
    net = wl.network
    on = O.OracleNet(net)
    b = wl.make_batch(0, 0, wl.batch_size)
    out = {"unit": "synaptic events/s", "cores": 1, "kind": "oracle"}
    if net.n_rec <= 5000:
        res = {}
        for mode, name in ((2, "event-driven"), (1, "time-driven")):
            g = O.zero_grads(on)
            ev, el, done = 0, 0.0, 0
            for i in range(b.n_trials):
                if name == "time-driven" and done >= res["event-driven"][2]:
                    break
                t0 = time.perf_counter()
                r = O.run_trial(on, b, i, mode, g, trace=True)
                el += time.perf_counter() - t0
                ev += _events_of_trial(net, b, i, r.trace["z"])
                done += 1
                if el > budget_s / 2:
                    break
            res[name] = (ev, el, done)
        ev, el, done = res["event-driven"]
        tev, tel, tdone = res["time-driven"]
        out.update(value=ev / el, time_driven_value=tev / tel,
                   sample=f"{done} whole trials of the first batch of the same workload, event-driven gradient "
                          f"({ev} events, {el:.1f} s); time-driven gradient on {tdone} of them ({tel:.1f} s); "
                          f"network construction excluded")
        return out
    T = min(n_steps_sample, int(b.n_steps[0]))
    sb = _truncated(b, 0, T)
    g = O.zero_grads(on)
    t0 = time.perf_counter()
    r = O.run_trial(on, sb, 0, 2, g, trace=True)
    el = time.perf_counter() - t0
    ev = _events_of_trial(net, sb, 0, r.trace["z"])
    out.update(value=ev / el, sample=f"first {T} steps of one trial of the same network (event-driven gradient, "
                                     f"{ev} events, {el:.1f} s including the oracle's per-trial target-major copy "
                                     f"of the graph; building the network arrays excluded)")
    return out


def _oracle_sample(job):
    """One process of the parallel oracle timing: trial `i` of the first
    batch, whole (small networks, within the time budget) or its first T
    steps; returns (events, seconds)."""
    import oracle as O
    i, T, budget = job
    wl = _oracle_sample.workload     # set before the processes are forked
    net = wl.network
    on = O.OracleNet(net)
    b = wl.make_batch(0, 0, wl.batch_size)
    ev, el = 0, 0.0
    while i < b.n_trials and el <= budget:
        sb = _truncated(b, i, min(T, int(b.n_steps[i]))) if T else b.trial(i)
        g = O.zero_grads(on)
        t0 = time.perf_counter()
        r = O.run_trial(on, sb, 0, 2, g, trace=True)
        el += time.perf_counter() - t0
        ev += _events_of_trial(net, sb, 0, r.trace["z"])
        if T:
            break
        i += _oracle_sample.stride
    return ev, el


def cpu_parallel(wl, n_steps_sample, budget_s=20.0):
    """The oracle in P independent processes, P = min(trials per batch, host
    cores, 16), one trial (or its first steps) each, forked after the
    workload is built: aggregate events over the wall-clock time."""
    import multiprocessing as mp
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    P = max(1, min(wl.batch_size, cores, 16))
    T = 0 if wl.network.n_rec <= 5000 else n_steps_sample
    _oracle_sample.stride = P
    _oracle_sample.workload = wl
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(P) as pool:
        res = pool.map(_oracle_sample, [(i, T, budget_s / 2) for i in range(P)], chunksize=1)
        pool.close()
        pool.join()  # every worker gone before the timing is reported
    wall = time.perf_counter() - t0
    ev = sum(r[0] for r in res)
    what = f"the first {T} steps of trials 0..{P - 1}" if T else f"whole trials of the first batch, trial i in process i mod {P}"
    return {"value": ev / wall, "unit": "synaptic events/s", "cores": P, "kind": "oracle",
            "sample": f"{what}, event-driven gradient, one process each ({ev} events, {wall:.1f} s wall-clock "
                      f"including each process's copy of the network; building the network arrays excluded)"}


def bench_online(args, wl, progress):
    """The e-prop+ schedule: warm-up on one sample, then `steps` samples of the
    workload run back to back as one continuous run with per-spike updates.
    The batch is host memory (the schedule joins the samples on the host), so
    the timed call includes copying its input and forced spikes."""
    import torch
    from paper_2511_21674_amd import eprop as E
    net_w = wl.network
    net_w.params.optimizer = 0   # the per-spike schedule updates by gradient descent
    if args.isi_cutoff is not None:
        net_w.params.isi_cutoff = args.isi_cutoff
    T = int(wl.make_batch(0, 0, 1).n_steps[0])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        net = E.Network(net_w, "fp32", max_trials=1, max_steps=max(args.steps, 1) * T,
                        stream=E.C.c_void_p(stream.cuda_stream))
        progress("network built")
        warm = wl.make_batch(0, 0, 1)
        run = wl.make_batch(1, 0, args.steps)
        net.simulate(warm, online=True)
        torch.cuda.synchronize()
        progress("warm-up sample done")
        t0 = time.perf_counter()
        r = net.simulate(run, online=True)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        progress(f"online run done, {elapsed / args.steps * 1000.0:.1f} ms per sample")
        net.close()
    bio_s = args.steps * T * net_w.params.dt / 1000.0
    out = {"metric": "synaptic events/s (e-prop+ per-spike schedule, FP32, one continuous run)",
           "value": r.n_syn_events / elapsed, "unit": "synaptic events/s", "n_gpus": 1, "steps": args.steps,
           "warmup": 1, "ms_per_step": elapsed / args.steps * 1000.0, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": f"{wl.name}: {wl.description}", "n_rec": net_w.n_rec, "n_in": net_w.n_in,
                      "n_out": net_w.n_out, "synapses": int(net_w.in_rec.nnz + net_w.rec_rec.nnz),
                      "samples_per_run": args.steps, "steps_per_sample": T, "isi_cutoff": int(net_w.params.isi_cutoff),
                      "gradient": "e-prop+ per-spike schedule (walk over each inter-spike interval)"},
           "eprop_updates_per_s": r.n_eprop_updates / elapsed, "recurrent_rate_hz":
               r.n_rec_spikes / (args.steps * T * net_w.n_rec * net_w.params.dt / 1000.0),
           "mean_loss": [float(x) for x in r.loss],
           "real_time_factor": bio_s / elapsed, "biological_seconds": bio_s,
           "roofline": None, "cpu_baseline": None,
           "note": "per-spike updates walk each synapse's inter-spike interval (at most isi_cutoff steps); "
                   "roofline and CPU baseline are reported for the batched path only"}
    print(json.dumps(out), flush=True)


def equal_loss(args, W, E, T, m, stream, progress):
    """FP32 batched against FP64 training over args.seeds network seeds: the
    same batches from the same initial weights, m iterations each, in FP32
    (batched) and FP64 (batched: the same arithmetic per trial as one trial
    at a time).  A free-running spiking network is chaotic (one flipped spike
    sends two runs apart), so one seed's final loss is a random draw and the
    comparison is over the seeds.  The FP64 plain path (one trial per call,
    gather delivery) is timed on the first args.plain_iters iterations of
    each seed for the speedup.  Batches are generated before the timed
    loops."""
    import inspect
    import torch
    f = W.WORKLOADS[args.workload]
    seed0 = inspect.signature(f).parameters["seed"].default
    kw = {"batch_size": args.batch} if args.batch else {}
    runs, t32, t64, tpl, npl = [], 0.0, 0.0, 0.0, 0

    def train(net, batches, plain=False):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = []
        for b in batches:
            if plain:
                lt = [float(net.simulate(b.trial(i), train=True).loss[0]) for i in range(b.n_trials)]
            else:
                lt = net.simulate(b, train=True).loss
            net.apply()
            out.append(float(np.mean(lt)))
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    for s in range(args.seed_start, args.seed_start + args.seeds):
        wl = f(seed=seed0 + 7919 * s, **kw)
        bs = wl.batch_size
        batches = [wl.make_batch(i, 0, bs) for i in range(m)]
        progress(f"equal-loss seed {s}: {m} batches generated")
        with torch.cuda.stream(stream):
            cs = E.C.c_void_p(stream.cuda_stream)
            net = E.Network(wl.network, "fp32", max_trials=bs, max_steps=T, stream=cs)
            l32, e32 = train(net, batches)
            net.close()
            progress(f"equal-loss seed {s}: FP32 batched {e32:.1f} s")
            net = E.Network(wl.network, "fp64", max_trials=bs, max_steps=T, stream=cs)
            l64, e64 = train(net, batches)
            net.close()
            progress(f"equal-loss seed {s}: FP64 batched {e64:.1f} s")
            k = min(args.plain_iters, m)
            net = E.Network(wl.network, "fp64", max_trials=1, max_steps=T, delivery="gather", stream=cs)
            lpl, epl = train(net, batches[:k], plain=True)
            net.close()
            progress(f"equal-loss seed {s}: FP64 plain {epl:.1f} s for {k} iterations")
        t32 += e32
        t64 += e64
        tpl += epl
        npl += k
        runs.append({"seed": seed0 + 7919 * s, "loss_fp32": l32, "loss_fp64": l64, "loss_fp64_plain": lpl})
    nl = max(1, m // 10)
    f32 = np.array([np.mean(r["loss_fp32"][-nl:]) for r in runs])
    f64 = np.array([np.mean(r["loss_fp64"][-nl:]) for r in runs])
    d = np.log(f32 / f64)
    r32 = np.array([np.mean(r["loss_fp32"]) for r in runs])
    r64 = np.array([np.mean(r["loss_fp64"]) for r in runs])
    n_it = m * len(runs)
    return {"iterations": m, "seeds": len(runs), "trials_per_batch": int(batches[0].n_trials),
            "seconds_per_iteration_fp32_batched": t32 / n_it, "seconds_per_iteration_fp64_batched": t64 / n_it,
            "seconds_per_iteration_fp64_plain": tpl / npl, "plain_iterations_timed": npl,
            "speedup_fp32_batched": (tpl / npl) / (t32 / n_it),
            "speedup_over_fp64_batched": (t64 / n_it) / (t32 / n_it),
            "final_loss_fp32": float(f32.mean()), "final_loss_fp64": float(f64.mean()),
            "final_loss_rel_diff": float(abs(f32.mean() - f64.mean()) / f64.mean()),
            "final_log_ratio_mean": float(d.mean()),
            "final_log_ratio_se": float(d.std(ddof=1) / np.sqrt(len(d))) if len(d) > 1 else None,
            "run_loss_fp32": float(r32.mean()), "run_loss_fp64": float(r64.mean()),
            "run_loss_rel_diff": float(abs(r32.mean() - r64.mean()) / r64.mean()),
            "per_seed_final": [[float(a), float(b)] for a, b in zip(f32, f64)],
            "plain_first_loss_rel_diff": float(max(abs(r["loss_fp64_plain"][0] - r["loss_fp64"][0])
                                                   / abs(r["loss_fp64"][0]) for r in runs)),
            "comparison": "trained: per seed, final loss = mean over the last %d of %d iterations (FP32 batched vs "
                          "FP64 batched); seed means compared, and the mean log ratio with its standard error; "
                          "run loss = mean over all iterations" % (nl, m),
            "note": "same batches and initial weights per seed; speedup = FP64 plain seconds per iteration (first "
                    "iterations of each seed) / FP32 batched seconds per iteration (host batches in both)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 5; 20 samples = 20 s of biological time for the scaling network)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4_sparse")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--time-driven", action="store_true",
                    help="gradient by the time-driven baseline recursion instead of the event-driven path")
    ap.add_argument("--online", action="store_true",
                    help="the e-prop+ schedule: the steps' samples run back to back as one continuous run, every "
                         "arriving spike updating its synapse (EPROP_BATCH_ONLINE); one warm-up sample first")
    ap.add_argument("--isi-cutoff", type=int, default=None,
                    help="with --online: eprop_isi_trace_cutoff in steps (default: the workload's, 0 = none)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes (the tuner otherwise runs in the first warm-up batch)")
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="steps of the CPU oracle's sample on large networks (default 40; 5 for the scaling network)")
    ap.add_argument("--fp64-iters", type=int, default=1,
                    help="training iterations of the FP64 plain comparison (<= warmup + steps); its final loss is "
                         "the mean over the last 10%% of them, compared with the FP32 run's over the same iterations")
    ap.add_argument("--batch", type=int, default=None, help="trials per batch (default: the workload's)")
    ap.add_argument("--plain-iters", type=int, default=5,
                    help="with --seeds: iterations of each seed timed on the FP64 plain path")
    ap.add_argument("--seed-start", type=int, default=0,
                    help="with --seeds: the first network seed's index (seed = default + 7919 * index)")
    ap.add_argument("--seeds", type=int, default=1,
                    help="with --fp64-iters: compare FP32 batched and FP64 plain training over this many network "
                         "seeds (each trained from scratch for --fp64-iters iterations)")
    ap.add_argument("--delivery", choices=("scatter", "gather"), default="scatter",
                    help="spike delivery of the FP32 run: scatter into LDS delay rings (default) or target-side "
                         "gather (one kernel per step, every target sums its arriving synapses)")
    ap.add_argument("--scatter-form", choices=("auto", "lookup", "queues"), default="auto",
                    help="scatter delivery by lookup (every tile looks up each spiking source) or through "
                         "per-tile queues (each spiking neuron's tile bins its synapses by target tile); auto: "
                         "queues where rows are sparse across tiles, and the autotuner may pick either")
    ap.add_argument("--no-cpu-parallel", action="store_true", help="skip the P-process oracle timing")
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
    scaling = args.workload == "scaling"
    if args.steps is None:
        args.steps = 20 if scaling else 5
    if args.cpu_steps is None:
        args.cpu_steps = 5 if scaling else 40
    if scaling:
        # the FP64 plain comparison would rebuild the 1.28e9-synapse network in
        # double; the scaling runs compare static and plastic synapses instead
        args.no_fp64 = True
    def progress(msg):
        print(f"[bench] {msg} ({time.perf_counter() - t_start:.0f} s)", file=sys.stderr, flush=True)

    t_start = time.perf_counter()
    print(f"[bench] generating workload {args.workload}", file=sys.stderr, flush=True)
    wl = W.WORKLOADS[args.workload](**({"batch_size": args.batch} if args.batch else {}))
    net_w = wl.network
    if args.online:
        return bench_online(args, wl, progress)
    T = max(int(wl.make_batch(0, 0, 1).n_steps.max()), 1)
    if args.workload == "c2_evidence":
        T = 1800
    print(f"[bench] workload {wl.name}: J={net_w.n_rec} I={net_w.n_in} K={net_w.n_out} "
          f"synapses={net_w.in_rec.nnz + net_w.rec_rec.nnz} batch={wl.batch_size} T={T}", file=sys.stderr, flush=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        net = E.Network(net_w, "fp32", max_trials=wl.batch_size, max_steps=T, delivery=args.delivery,
                        stream=E.C.c_void_p(stream.cuda_stream), autotune=not args.no_autotune,
                        scatter_form=args.scatter_form if args.delivery == "scatter" else "auto")
        progress("network built")
        staged = stage_batches(wl, args.warmup + args.steps, 0)
        torch.cuda.synchronize()
        progress("batches staged")
        warm_losses = []
        for i in range(args.warmup):
            _, wloss = run_staged(net, staged[i], time_driven=args.time_driven)
            net.apply()
            warm_losses.append(float(wloss.mean()))
        torch.cuda.synchronize()
        progress("warm-up done")
        tot = {"events": 0, "updates": 0, "rec_spikes": 0, "in_spikes": 0}
        phases = {k: 0.0 for k in E.PHASES}
        losses = []
        t0 = time.perf_counter()
        for i in range(args.steps):
            res, loss = run_staged(net, staged[args.warmup + i], profile=True, time_driven=args.time_driven)
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
        progress(f"timed steps done, {elapsed / args.steps * 1000.0:.2f} ms per step")
        static = None
        if scaling:
            # the same samples with static synapses: forward pass and readout only
            t1 = time.perf_counter()
            for i in range(args.steps):
                run_staged(net, staged[args.warmup + i], train=False)
            torch.cuda.synchronize()
            el_s = time.perf_counter() - t1
            progress(f"static run done, {el_s / args.steps * 1000.0:.2f} ms per sample")
            bio_s = args.steps * T * net_w.params.dt / 1000.0
            static = {"ms_per_sample": el_s / args.steps * 1000.0, "real_time_factor": bio_s / el_s,
                      "eprop_real_time_factor": bio_s / elapsed, "biological_seconds": bio_s,
                      "note": "real-time factor = simulated biological time / wall-clock time; static: "
                              "the same samples without plasticity (no gradient, no update)"}
    steps = args.steps
    n_tr = wl.batch_size
    rate_hz = tot["rec_spikes"] / (steps * n_tr * net_w.n_rec * T * net_w.params.dt / 1000.0)
    lay = net.layout()
    gather = args.delivery == "gather"
    # the forward kernel runs once per block of steps (scatter) or once per step (gather)
    launches = T if gather else -(-T // lay["steps_per_launch"])
    per_step = {k: v / steps for k, v in tot.items()}
    per_step["neuron_steps"] = float(np.mean([int(staged[args.warmup + i][0].n_steps.sum()) for i in range(steps)])
                                     * net_w.n_rec)
    fwd_ms = phases["forward"] / steps
    fwd_b = forward_bytes(per_step, net_w)
    achieved = fwd_b / launches / (fwd_ms / launches / 1000.0) / 1e9
    roof = {"kernel": "k_neuron_gather" if gather else "k_forward_tiled", "bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "avg_launch_ms": round(fwd_ms / launches, 4), "algorithmic_bytes_per_launch": int(fwd_b / launches)}
    step_s = elapsed / steps
    pb = path_bytes(per_step, net_w, n_tr, net_w.params.optimizer == 1)
    db = design_bytes(per_step, net_w, n_tr, net_w.params.optimizer == 1, bool(lay["blocked_update"]), net_w.n_out)
    dsum = sum(db.values())
    path_roof = {
        "design": {"bytes_per_step": int(dsum), "achieved": round(dsum / step_s / 1e9, 1), "unit": "GB/s",
                   "frac": round(dsum / step_s / 1e9 / HBM_PEAK_GBS, 4),
                   "bytes_by_kernel": {k: int(v) for k, v in db.items()},
                   "note": "the bytes this design's kernels need (their own algorithms)"},
        "survey_model": {"bytes_per_step": int(pb), "achieved": round(pb / step_s / 1e9, 1), "unit": "GB/s",
                         "frac": round(pb / step_s / 1e9 / HBM_PEAK_GBS, 4),
                         "note": "the survey's per-unit model: 24-32 B of per-synapse trace and gradient traffic "
                                 "per event, which the archive design never moves; a model, not a measurement"},
        "measured": None}
    tr = measured_traffic(wl.name, roof["kernel"])
    if tr is not None:
        roof["traffic"] = round(tr / 1e9, 3)
        roof["traffic_unit"] = "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    tstep = measured_traffic(wl.name, "step")
    if tstep is not None:
        path_roof["measured"] = {"bytes_per_step": int(tstep), "achieved": round(tstep / step_s / 1e9, 1),
                                 "unit": "GB/s", "frac": round(tstep / step_s / 1e9 / HBM_PEAK_GBS, 4),
                                 "note": "rocprofv3 FETCH_SIZE + WRITE_SIZE of every kernel of one step, "
                                         "copy-calibrated"}

    fp64 = None
    if not args.no_fp64 and (args.seeds > 1 or args.seed_start > 0):
        fp64 = equal_loss(args, W, E, T, max(1, args.fp64_iters), stream, progress)
    elif not args.no_fp64:
        # the FP64 plain path (same kernels in double, one trial at a time,
        # deterministic gather delivery), trained on the same batches from
        # the same initial weights as the FP32 run's first iterations
        m = max(1, min(args.fp64_iters, args.warmup + steps))
        all32 = warm_losses + losses
        with torch.cuda.stream(stream):
            net64 = E.Network(net_w, "fp64", max_trials=1, max_steps=T, delivery="gather",
                              stream=E.C.c_void_p(stream.cuda_stream))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ev64, loss64 = 0, []
            for it in range(m):
                bb = staged[it][0]
                lt = []
                for i in range(bb.n_trials):
                    r = net64.simulate(bb.trial(i), train=True)
                    ev64 += r.n_syn_events
                    lt.append(float(r.loss[0]))
                net64.apply()
                loss64.append(float(np.mean(lt)))
            torch.cuda.synchronize()
            el64 = time.perf_counter() - t1
            net64.close()
        # final loss: the mean over the last 10% of the compared iterations (at least one)
        nl = max(1, m // 10)
        l64, l32 = float(np.mean(loss64[-nl:])), float(np.mean(all32[m - nl:m]))
        fp64 = {"value": ev64 / el64, "unit": "synaptic events/s", "seconds_per_iteration": el64 / m,
                "iterations": m, "speedup_fp32_batched": (el64 / m) / (elapsed / steps),
                "loss_fp64": loss64, "loss_fp32": all32[:m], "final_loss_fp64": l64, "final_loss_fp32": l32,
                "final_loss_rel_diff": abs(l32 - l64) / abs(l64),
                "comparison": ("trained: final loss = mean over the last %d of %d training iterations" % (nl, m))
                if m >= 100 else ("first %d batch(es) from the same initial weights: a forward and gradient "
                                  "comparison, not a trained run" % m),
                "note": "same batches and initial weights; speedup = FP64 plain seconds per iteration / "
                        "FP32 batched"}
    net.close()

    cpu = None
    if not args.no_cpu_baseline:
        progress("CPU oracle baseline")
        cpu = cpu_baseline(wl, min(args.cpu_steps, T))
        progress("CPU oracle baseline done")
        if not args.no_cpu_parallel:
            cpu["parallel"] = cpu_parallel(wl, min(args.cpu_steps, T))
            progress("parallel CPU oracle baseline done")

    out = {"metric": "synaptic events/s (event-driven e-prop training, FP32 batched)",
           "value": tot["events"] / elapsed, "unit": "synaptic events/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": elapsed / steps * 1000.0, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": f"{wl.name}: {wl.description}", "n_rec": net_w.n_rec, "n_in": net_w.n_in,
                      "n_out": net_w.n_out, "synapses": int(net_w.in_rec.nnz + net_w.rec_rec.nnz),
                      "trials_per_batch": n_tr, "steps_per_trial": T,
                      "delivery": "gather (target side)" if gather else "scatter (LDS tiles)",
                      "gradient": "time-driven baseline" if args.time_driven else "event-driven"},
           "eprop_updates_per_s": tot["updates"] / elapsed,
           "recurrent_rate_hz": rate_hz,
           "phase_ms_per_step": {k: round(v / steps, 3) for k, v in phases.items()},
           "mean_loss": losses,
           "layout": lay, "roofline": roof, "path_roofline": path_roof, "cpu_baseline": cpu, "fp64_plain": fp64}
    if static is not None:
        out["scaling_run"] = static
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
