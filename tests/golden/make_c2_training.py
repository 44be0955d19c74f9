"""Writes c2_training_oracle.json: the FP64 oracle's free-running training of
the evidence-accumulation task (softmax cross-entropy in the recall window,
50 LIF + 50 ALIF neurons, Adam with eta 5e-3 as in the task's configuration;
Results, "Evidence accumulation") for 100 iterations of 32 trials, from three
network seeds.  Per iteration it records the mean loss over the batch's
trials and the fraction of trials whose predicted class equals the label.

Calls only the oracle and the seeded input generators.  Run from the
repository root: python tests/golden/make_c2_training.py  (about 7 minutes
on 3 cores).
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

ITERATIONS, BATCH = 100, 32
SEED_STEP = 7919


def seeds():
    from paper_2511_21674_amd import workloads as W
    return [W.SEED_BASE + 2 + SEED_STEP * s for s in range(3)]


def run(seed):
    import numpy as np
    import oracle as O
    from paper_2511_21674_amd import workloads as W
    wl = W.c2_evidence(seed=seed, batch_size=BATCH)
    h = O.train(wl, iterations=ITERATIONS, grad_mode=2, batch_size=BATCH)
    acc = []
    for it in range(ITERATIONS):
        lab = wl.make_batch(it, 0, BATCH).label
        acc.append(float(np.mean(h["pred"][it] == lab)))
    return {"seed": seed, "mean_loss": [float(x.mean()) for x in h["loss"]], "accuracy": acc}


def main():
    import oracle as O
    O.build(force=False)
    with ProcessPoolExecutor(3) as ex:
        runs = list(ex.map(run, seeds()))
    out = {"workload": "c2_evidence", "batch": BATCH, "iterations": ITERATIONS, "optimizer": "adam", "eta": 5e-3,
           "gradient": "event-driven (oracle)", "runs": runs}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_training_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
