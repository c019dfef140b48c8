"""The larger workloads at their full sizes: the two-sphere collision of
2^24 bodies and the Plummer sphere of 2^22 bodies against the oracle on
sampled bodies and groups (tree arrays bit for bit), and the clumpy field of
2^26 bodies through properties that hold at any size."""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_08966_amd import binding as B
from paper_2203_08966_amd import workloads as W
from tests.conftest import say

pytestmark = pytest.mark.gpu

TOL32_RMS, TOL32_MAX = 1e-5, 1e-4


def _perm(tree, n):
    """Only the permutation of a tree (sorted rank -> caller index)."""
    import ctypes as C
    perm = np.zeros(n, dtype=np.uint32)
    rc = B.load().bh_tree_export(tree, None, C.c_void_p(perm.ctypes.data), *([None] * 10))
    assert rc == B.BH_OK
    return perm.astype(np.int64)


def _ranks(perm):
    r = np.empty(len(perm), dtype=np.int64)
    r[perm] = np.arange(len(perm))
    return r


@pytest.mark.parametrize("name", ["c4", "c3"])
def test_full_size_sampled_against_oracle(ctx, name):
    b, cfg = W.config(name)
    n, leaf, eps, theta = b.n, cfg["leaf"], cfg["eps"], cfg["theta"]
    say(f"{name}: {cfg['workload']} n={n} theta {theta} eps {eps}")
    P, M = torch.from_numpy(b.pos).cuda(), torch.from_numpy(b.mass).cuda()
    t = B.bh_build(ctx, P, M, leaf)
    acc = torch.empty_like(P)
    B.bh_forces(t, theta, eps, acc)
    gacc = torch.empty_like(P)
    B.bh_forces(t, 0.7, eps, gacc, B.force_opts(walk=B.BH_WALK_GROUP))
    torch.cuda.synchronize()
    ex = B.bh_tree_export(t)
    B.bh_tree_free(t)
    ref = oracle.build_all(b.pos.astype(np.float64), b.mass.astype(np.float64), leaf)
    assert np.array_equal(ex["keys"], ref["keys"])
    assert np.array_equal(ex["perm"].astype(np.int64), ref["perm"])
    assert np.array_equal(ex["next"], ref["tree"]["next"])
    sample = W.subsample(n, 4096, cfg["sub_seed"])
    rs = _ranks(ref["perm"])[sample]
    r = oracle.walk(ref["tree"], ref["mom"], ref["spos"], ref["smass"], ref["L"], theta, eps,
                    targets=rs)
    ok = r.flag == 0
    a = acc.cpu().numpy().astype(np.float64)[sample]
    e = np.linalg.norm(a - r.acc, axis=1) / np.linalg.norm(r.acc, axis=1)
    say(f"  per body: unflagged {ok.mean():.4f}, rms {np.sqrt(np.mean(e[ok] ** 2)):.2e}")
    assert ok.mean() > 0.98
    assert np.sqrt(np.mean(e[ok] ** 2)) <= TOL32_RMS and e[ok].max() <= TOL32_MAX
    # sampled groups of the group walk
    ga = gacc.cpu().numpy().astype(np.float64)[ref["perm"]]
    rng = np.random.default_rng(7)
    checked = 0
    G = B.BH_GROUP_BODIES
    for g in rng.choice(n // G, 16, replace=False):
        rg = oracle.walk_group(ref, eps, group=G, theta=0.7, target_range=(G * g, G * g + G))
        if rg.flag.any():
            continue
        checked += 1
        eg = np.linalg.norm(ga[G * g:G * g + G] - rg.acc, axis=1) / np.linalg.norm(rg.acc, axis=1)
        assert eg.max() <= TOL32_MAX
    say(f"  group walk: unflagged sampled groups {checked} of 16")
    assert checked >= 8


def test_clumpy_full_size_properties(ctx):
    """2^26 clumpy bodies: a sub-range of sorted ranks walked alone gives the
    full walk's forces bit for bit (per body, and per group on group
    boundaries), and the error against FP64 direct summation on sampled
    bodies stays within the opening angle's error."""
    b, cfg = W.config("c5")
    n, leaf, eps, theta = b.n, cfg["leaf"], cfg["eps"], cfg["theta"]
    say(f"c5: clumpy n={n} theta {theta} eps {eps}")
    P, M = torch.from_numpy(b.pos).cuda(), torch.from_numpy(b.mass).cuda()
    del b
    t = B.bh_build(ctx, P, M, leaf)
    perm = torch.from_numpy(_perm(t, n)).cuda()
    for walk in (B.BH_WALK_BODY, B.BH_WALK_GROUP):
        th = theta if walk == B.BH_WALK_BODY else 0.8
        full = torch.empty_like(P)
        B.bh_forces(t, th, eps, full, B.force_opts(walk=walk))
        lo, hi = 64 * 123457, 64 * 123457 + 64 * 1000
        part = torch.zeros_like(P)
        B.bh_forces(t, th, eps, part, B.force_opts(walk=walk, target_range=(lo, hi)))
        torch.cuda.synchronize()
        sel = perm[lo:hi]
        assert torch.equal(part.index_select(0, sel), full.index_select(0, sel))
        # error against FP64 direct summation on 512 sampled bodies
        sample = torch.from_numpy(W.subsample(n, 512, cfg["sub_seed"])).cuda()
        ref = torch.empty((512, 3), dtype=torch.float64, device="cuda")
        B.bh_direct(ctx, P, M, sample, eps, ref)
        a = full.index_select(0, sample.long()).double()
        e = ((a - ref).norm(dim=1) / ref.norm(dim=1)).cpu().numpy()
        rms = float(np.sqrt(np.mean(e * e)))
        say(f"  walk {walk}: rms rel err vs FP64 direct {rms:.2e}")
        assert rms < 5e-3
    B.bh_tree_free(t)
