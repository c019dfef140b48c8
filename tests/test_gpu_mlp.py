"""GPU learned acceptance criterion against the oracle: bf16 MFMA inference,
training gradients, training pairs (features and labels), and the walk with
the learned decision."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp
from paper_2203_08966_amd import binding as B
from tests.conftest import case_bodies, say

pytestmark = pytest.mark.gpu


def _params(seed, noise=0.2):
    rng = np.random.default_rng(seed)
    return mlp.init(seed) + rng.normal(size=mlp.NPARAM) * noise


def _features(n, seed):
    """Feature rows in the ranges the walk produces."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.2, 1.2, n)
    f = np.stack([r, r * r, rng.uniform(0, 0.5, n), rng.uniform(-0.5, 0.5, n),
                  rng.uniform(0, 0.8, n), rng.normal(0, 0.3, n), rng.uniform(0, 1.5, n),
                  rng.integers(1, 12, n) / 21.0, rng.uniform(0, 0.05, n),
                  rng.integers(0, 2, n).astype(float)], axis=1)
    return f.astype(np.float32)


def test_inference_matches_bf16_oracle(ctx):
    th = _params(11)
    B.bh_mlp_set(ctx, th)
    th32 = B.bh_mlp_get(ctx)  # FP32 rounding of the parameters
    X = _features(5000, 3)    # 5000: a ragged last wave
    say("bf16 MFMA inference vs oracle bf16 view, 5000 rows")
    pred = B.bh_mlp_infer(ctx, torch.from_numpy(X).cuda()).cpu().numpy()
    ref = mlp.forward_bf16(th32, X.astype(np.float64))
    err = np.abs(pred - ref)
    say(f"  max |d| {err.max():.2e}  rms {np.sqrt(np.mean(err ** 2)):.2e}")
    assert np.sqrt(np.mean(err ** 2)) < 1e-3
    assert err.max() < 2e-2
    # and close to the full-precision network (bf16 quantisation only)
    full, _ = mlp.forward(th32, X.astype(np.float64))
    assert np.sqrt(np.mean((pred - full) ** 2)) < 0.05 * np.std(full) + 1e-3


def test_gradient_matches_oracle(ctx):
    th = _params(12, 0.1)
    B.bh_mlp_set(ctx, th)
    th32 = B.bh_mlp_get(ctx)
    X = _features(3000, 4)
    rng = np.random.default_rng(5)
    y = (rng.normal(size=3000) - 3.0).astype(np.float32)
    say("training gradient (one batch of 3000) vs oracle FP64 backprop")
    g, lv = B.bh_mlp_grad(ctx, torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda())
    g = g.cpu().numpy().astype(np.float64)
    ref = mlp.grad(th32, X.astype(np.float64), y.astype(np.float64))
    assert abs(lv - mlp.loss(th32, X.astype(np.float64), y.astype(np.float64))) < 1e-5 * abs(lv) + 1e-7
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    say(f"  relative gradient error {rel:.2e}")
    assert rel < 1e-4
    np.testing.assert_allclose(g, ref, rtol=1e-3, atol=1e-5 * np.abs(ref).max())


def test_training_reduces_loss_like_oracle(ctx):
    rng = np.random.default_rng(6)
    X = _features(8192, 7)
    y = (np.sin(3 * X[:, 0]) - 2 * X[:, 2] + X[:, 5]).astype(np.float32)
    th = mlp.init(8)
    B.bh_mlp_set(ctx, th)
    say("GPU training, 30 epochs of 8192 pairs, batch 512")
    Xt, yt = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    loss = B.bh_mlp_train(ctx, Xt, yt, epochs=30, batch=512, lr=3e-3, seed=1)
    assert np.all(np.isfinite(loss))
    assert loss[-1] < 0.1 * loss[0]
    th_gpu = B.bh_mlp_get(ctx)
    final = mlp.loss(th_gpu, X.astype(np.float64), y.astype(np.float64))
    assert abs(final - loss[-1]) < 0.5 * loss[-1] + 1e-4
    # the oracle trained the same way reaches a comparable loss
    opt = mlp.Adam(mlp.NPARAM, lr=3e-3)
    tho = th.copy()
    for ep in range(30):
        perm = rng.permutation(8192)
        for b0 in range(0, 8192, 512):
            idx = perm[b0:b0 + 512]
            tho = opt.step(tho, mlp.grad(tho, X[idx].astype(np.float64), y[idx].astype(np.float64)))
    lo = mlp.loss(tho, X.astype(np.float64), y.astype(np.float64))
    say(f"  final loss GPU {final:.3e}  oracle {lo:.3e}  (start {loss[0]:.3e})")
    assert final < 3 * lo + 1e-3


def test_training_pairs_match_oracle(ctx):
    pos, _, mass = case_bodies("plummer", 2048, 41, np.float64)
    theta_lo, theta_hi, keep, seed, eps = 0.3, 1.0, 0.25, 7, 0.01
    say("training pairs: FP64 tree of 2048 bodies vs oracle")
    P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda()
    t = B.bh_build(ctx, P, M, 8)
    feat, label, node, body = B.bh_mlp_samples(t, eps, theta_lo, theta_hi, keep, seed)
    feat, label = feat.cpu().numpy(), label.cpu().numpy()
    node, body = node.cpu().numpy(), body.cpu().numpy()
    B.bh_tree_free(t)
    ref = oracle.build_all(pos, mass, 8)
    f, lab, nd, cnt = oracle.mac_samples(ref, eps, theta_lo, theta_hi, keep, seed, cap=1024)
    assert len(label) == cnt.sum()
    starts = np.concatenate([[0], np.cumsum(cnt)])
    same = 0
    for i in range(len(cnt)):
        g = slice(starts[i], starts[i + 1])
        if np.array_equal(node[g], nd[i, :cnt[i]]):
            same += 1
            assert np.all(body[g] == i)
            np.testing.assert_allclose(feat[g], f[i, :cnt[i]], rtol=1e-5, atol=1e-6)
            np.testing.assert_allclose(label[g], lab[i, :cnt[i]], rtol=0, atol=1e-4)
    say(f"  bodies with identical pair lists: {same} of {len(cnt)}")
    assert same >= 0.999 * len(cnt)


def test_learned_walk_matches_oracle(ctx):
    """The walk with the learned decision, against the oracle's walk with the
    bf16 view of the same network: identical interaction counts for every
    body with no near-threshold decision, forces within the FP32 bound."""
    pos, _, mass = case_bodies("plummer", 20000, 3, np.float32)
    th = _params(21, 0.3)
    th[-1] = 0.0
    B.bh_mlp_set(ctx, th)
    th32 = B.bh_mlp_get(ctx)
    pred = mlp.forward_bf16(th32, _features(20000, 1).astype(np.float64))
    tau = float(np.median(pred))  # a threshold that splits the decisions
    lo, hi, eps = 0.35, 0.9, 0.005
    say(f"learned walk: 20000 bodies, band [{lo}, {hi}], log10 tau {tau:.3f}")
    P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda()
    t = B.bh_build(ctx, P, M, 16)
    n = len(mass)
    acc = torch.empty_like(P)
    npp = torch.zeros(n, dtype=torch.int32, device="cuda")
    npc = torch.zeros(n, dtype=torch.int32, device="cuda")
    o = B.force_opts(mac=B.BH_MAC_MLP, n_pp=npp, n_pc=npc, mlp_theta_lo=lo, mlp_theta_hi=hi,
                     mlp_log10_tau=tau)
    B.bh_forces(t, 0.5, eps, acc, o)
    torch.cuda.synchronize()
    B.bh_tree_free(t)
    ref = oracle.build_all(pos.astype(np.float64), mass.astype(np.float64), 16)
    r = oracle.walk_mlp(ref, eps, lo, hi, tau, th32)
    rank = np.empty(n, dtype=np.int64)
    rank[ref["perm"]] = np.arange(n)
    a = acc.cpu().numpy().astype(np.float64)[ref["perm"]]
    cp, cc = npp.cpu().numpy()[ref["perm"]], npc.cpu().numpy()[ref["perm"]]
    ok = r.flag == 0
    match = (cp == r.npp) & (cc == r.npc)
    say(f"  unflagged {ok.sum()}, of those with identical counts {match[ok].sum()}")
    assert ok.sum() > 0.5 * n
    assert match[ok].mean() >= 0.99
    e = np.linalg.norm(a - r.acc, axis=1) / np.linalg.norm(r.acc, axis=1)
    assert np.sqrt(np.mean(e[ok & match] ** 2)) < 1e-5
    assert np.sqrt(np.mean(e ** 2)) < 1e-3


def test_learned_walk_state_and_band_errors(ctx):
    pos, _, mass = case_bodies("plummer", 1000, 3, np.float64)
    t = B.bh_build(ctx, torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda(), 8)
    acc = torch.empty((1000, 3), dtype=torch.float64, device="cuda")
    B.bh_mlp_set(ctx, _params(1))
    with pytest.raises(B.BHError) as e:  # FP64 tree: the learned walk is FP32 only
        B.bh_forces(t, 0.5, 0.01, acc, B.force_opts(mac=B.BH_MAC_MLP))
    assert e.value.code == B.BH_E_INVALID
    B.bh_tree_free(t)
