"""Train the learned preconditioner on Newton systems of the weak Landau
(64^4, from t = 4) and two-stream (128^4, from t = 15) workloads and save
its parameters.

    python -m paper_2606_29027_amd.train_precond [--iters N] [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=1500)
    ap.add_argument("--steps", type=int, default=150)
    ap.add_argument("--capacity", type=int, default=200)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    from paper_2606_29027_amd import cnn as CNN
    t0 = time.perf_counter()
    data = CNN.collect(CNN.training_problems(), steps=args.steps, capacity=args.capacity,
                       skip=CNN.TRAINING_SKIP)
    t1 = time.perf_counter()
    net = CNN.make()
    hist = CNN.train(net, data, iters=args.iters, lr=args.lr)
    t2 = time.perf_counter()
    out = args.out or CNN.WEIGHTS
    CNN.save(net, out, meta={"pairs": [int(d[0].shape[0]) for d in data],
                             "loss_first": float(np.mean(hist[:10])),
                             "loss_last": float(np.mean(hist[-10:]))})
    print(json.dumps({"pairs": [int(d[0].shape[0]) for d in data], "collect_s": t1 - t0,
                      "train_s": t2 - t1, "loss_first10": float(np.mean(hist[:10])),
                      "loss_last10": float(np.mean(hist[-10:])), "saved": out}))


if __name__ == "__main__":
    main()
