"""Training pipeline of the learned acceptance criterion.

Host orchestration only: every step is a call into libbh.so (simulation
snapshots, training pairs, training kernels); torch tensors carry the device
buffers.  Training systems are Plummer spheres evolved with the library's
own FP64 leapfrog; a pair (group, cell) is labelled with the largest error
the cell's quadrupole term makes on the group's 64 bodies against the direct
sum over the cell's bodies, in units of the error budget's model
M l^3 / d_g^5, so that the network learns a coefficient k_C of that model per
group and cell from their geometry.
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


def training_set(ctx, seeds=range(41, 47), n=16384, snapshots=(0, 4, 8), dt=1e-3, eps=0.005,
                 leaf=16, theta_lo=0.2, theta_max=1.5, keep=0.5, pair_seed=7):
    """Pairs (feat, label) as GPU tensors from Plummer spheres of n bodies
    (one per seed), sampled at the given leapfrog step counts: for every
    group of 64 consecutive bodies, the cells with theta_lo <= l/d_g <
    theta_max whose cube misses the group's box, kept with probability
    keep."""
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


def train(ctx, feat, label, epochs=8, batch=4096, lr=1e-3, seed=7, quantile=0.99):
    """Initialise, train on the GPU, leave the packed network in ctx.

    quantile 0 fits the label's mean (mean-squared error); q in (0, 1) its
    q-quantile (pinball loss).  The rms force error is set by the cells
    whose error the network underestimates, so a high quantile (0.99) makes
    the predicted coefficient an upper bound for nearly every pair with the
    same features; measured with the oracle on 2^16-body Plummer spheres,
    the mean (MSE) could not reach rms 1e-3 at any tau.  Returns the
    per-epoch mean loss."""
    import torch
    if quantile > 0:
        start = float(torch.quantile(label[: 1 << 24].double(), quantile).item())
    else:
        start = float(label.double().mean().item())
    B.bh_mlp_set(ctx, init_params(seed, start))
    return B.bh_mlp_train(ctx, feat, label, epochs=epochs, batch=batch, lr=lr, seed=seed,
                          quantile=quantile)
