"""Training pipeline of the learned acceptance criterion.

Host orchestration only: every step is a call into libbh.so (simulation
snapshots, training pairs, training kernels); torch tensors carry the device
buffers.  Training systems are small Plummer spheres evolved with the
library's own FP64 leapfrog; a pair (body, cell) is labelled with the error
of the cell's quadrupole term against the direct sum over its bodies,
normalised by M l^3 / d^5, so that the network learns the per-cell
coefficient k_C of the error model k_C (l/d)^3 M/d^2.
"""
from __future__ import annotations

import numpy as np

from . import binding as B
from . import workloads as W

NF, NH = 10, 32


def init_params(seed: int, label_mean: float = 0.0) -> np.ndarray:
    """He-uniform hidden layers, small output layer, output bias at the
    label mean; flat layout W1 b1 W2 b2 w3 b3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.uniform(-1, 1, (NH, NF)) * np.sqrt(6.0 / NF)
    W2 = rng.uniform(-1, 1, (NH, NH)) * np.sqrt(6.0 / NH)
    w3 = rng.uniform(-1, 1, NH) * np.sqrt(6.0 / NH) * 0.1
    return np.concatenate([W1.ravel(), np.zeros(NH), W2.ravel(), np.zeros(NH), w3,
                           [label_mean]])


def training_set(ctx, seeds=range(41, 51), n=4096, snapshots=(0, 4, 8), dt=1e-3, eps=0.01,
                 leaf=8, theta_lo=0.3, theta_max=1.0, keep=0.1, pair_seed=7):
    """Pairs (feat, label) as GPU tensors from Plummer spheres of n bodies
    (one per seed), sampled at the given leapfrog step counts."""
    import torch
    feats, labels = [], []
    dev = torch.device("cuda")
    for s in seeds:
        b = W.plummer(n, int(s))
        P = torch.from_numpy(b.pos).to(dev)
        V = torch.from_numpy(b.vel).to(dev)
        M = torch.from_numpy(b.mass).to(dev)
        B.bh_sim_init(ctx, P, V, M, leaf, 0.5, eps)
        step = 0
        for snap in sorted(snapshots):
            while step < snap:
                B.bh_leapfrog_step(ctx, dt)
                step += 1
            tree = B.bh_sim_tree(ctx)
            f, lab, _, _ = B.bh_mlp_samples(tree, eps, theta_lo, theta_max, keep,
                                            pair_seed ^ (int(s) << 8) ^ snap)
            feats.append(f.clone())
            labels.append(lab.clone())
    return torch.cat(feats), torch.cat(labels)


def train(ctx, feat, label, epochs=8, batch=4096, lr=1e-3, seed=7, quantile=0.9):
    """Initialise, train on the GPU, leave the packed network in ctx.

    With quantile q in (0, 1) the network is fitted to the q-quantile of the
    label (pinball loss) instead of its mean: a cell is accepted for every
    body direction at once, so its coefficient should bound the error of most
    directions rather than describe the average one.  Returns the per-epoch
    mean loss."""
    import torch
    if quantile > 0:
        start = float(torch.quantile(label[: 1 << 24].double(), quantile).item())
    else:
        start = float(label.double().mean().item())
    B.bh_mlp_set(ctx, init_params(seed, start))
    return B.bh_mlp_train(ctx, feat, label, epochs=epochs, batch=batch, lr=lr, seed=seed,
                          quantile=quantile)
