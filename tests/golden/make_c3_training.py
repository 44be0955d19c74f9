"""Writes c3_training_oracle.json: the FP64 oracle's free-running training of
the event-camera classification task (2312 inputs, 180 LIF neurons with
sparse recurrence, 10 softmax readouts, cross-entropy over the last 30
steps; gradient descent with eta 1e-3 as in the task's configuration) for
100 iterations of 32 trials, from eight network seeds.  Per iteration it
records the mean loss over the batch's trials and the fraction of trials
whose predicted class equals the label.

Calls only the oracle and the seeded input generators.  Run from the
repository root: python tests/golden/make_c3_training.py  (about 35 minutes
on 8 cores: one process per seed).
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

ITERATIONS, BATCH, ETA, SEEDS = 100, 32, 1e-3, 8
SEED_STEP = 7919


def seeds():
    from paper_2511_21674_amd import workloads as W
    return [W.SEED_BASE + 3 + SEED_STEP * s for s in range(SEEDS)]


def run(seed):
    import numpy as np
    import oracle as O
    from paper_2511_21674_amd import workloads as W
    wl = W.c3_events(seed=seed, batch_size=BATCH)
    wl.network.params.eta = ETA
    h = O.train(wl, iterations=ITERATIONS, grad_mode=2, batch_size=BATCH)
    acc = []
    for it in range(ITERATIONS):
        lab = wl.make_batch(it, 0, BATCH).label
        acc.append(float(np.mean(h["pred"][it] == lab)))
    return {"seed": seed, "mean_loss": [float(x.mean()) for x in h["loss"]], "accuracy": acc}


def main():
    import oracle as O
    O.build(force=False)
    with ProcessPoolExecutor(min(SEEDS, os.cpu_count() or 1)) as ex:
        runs = list(ex.map(run, seeds()))
    out = {"workload": "c3_events", "batch": BATCH, "iterations": ITERATIONS, "optimizer": "gd", "eta": ETA,
           "gradient": "event-driven (oracle)", "runs": runs}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_training_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
