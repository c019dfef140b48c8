"""Writes learned_params.json: a network for the learned criterion's parity
tests, trained by the oracle alone (FP64 Adam on the oracle's own training
pairs of a 16384-body Plummer sphere).  The parity tests need a smooth,
trained network: a random one moves its output so much at a bf16 rounding
step that most decisions would be near a threshold.

    python tests/golden/make_learned_params.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import mlp  # noqa: E402
from paper_2203_08966_amd import workloads as W  # noqa: E402


def main():
    b = W.plummer(16384, 41)
    bb = oracle.build_all(b.pos, b.mass, 16)
    feat, lab, _, cnt = oracle.group_samples(bb, 0.005, 0.2, 1.5, 0.5, 7, cap=4096)
    X = np.concatenate([feat[q, :cnt[q]] for q in range(len(cnt))])
    y = np.concatenate([lab[q, :cnt[q]] for q in range(len(cnt))])
    th = mlp.init(7)
    th[-1] = y.mean()
    opt = mlp.Adam(mlp.NPARAM, lr=1e-3)
    rng = np.random.default_rng(0)
    for ep in range(6):
        perm = rng.permutation(len(y))
        for b0 in range(0, len(y), 1024):
            idx = perm[b0:b0 + 1024]
            th = opt.step(th, mlp.grad(th, X[idx], y[idx]))
        print(f"epoch {ep}: loss {mlp.loss(th, X, y):.4f} on {len(y)} pairs")
    with open(os.path.join(HERE, "learned_params.json"), "w") as fh:
        json.dump({"source": "tests/golden/make_learned_params.py (oracle only)",
                   "pairs": int(len(y)), "loss": float(mlp.loss(th, X, y)),
                   "params": [float(v) for v in th]}, fh)


if __name__ == "__main__":
    main()
