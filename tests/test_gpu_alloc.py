"""Device memory from the caller's allocator (bh_ctx_set_allocator): torch's
caching allocator serves every buffer of a context, its trees and its
simulation, with results identical to hipMalloc'd buffers."""
import numpy as np
import pytest
import torch

from paper_2203_08966_amd import binding as B
from tests.conftest import case_bodies, say

pytestmark = pytest.mark.gpu


def _run(ctx, P, V, M):
    t = B.bh_build(ctx, P, M, 16)
    acc = torch.empty_like(P)
    B.bh_forces(t, 0.6, 0.01, acc, B.force_opts(walk=B.BH_WALK_GROUP))
    acc2 = torch.empty_like(P)
    B.bh_forces(t, 0.6, 0.01, acc2, B.force_opts(mac=B.BH_MAC_BUDGET, mlp_log10_tau=-2.0,
                                                  mlp_theta_max=1.5))
    B.bh_sim_init(ctx, P, V, M, 16, 0.6, 0.01)
    for _ in range(3):
        B.bh_leapfrog_step(ctx, 1e-3)
    x = torch.empty_like(P)
    B.bh_sim_get(ctx, x)
    e = B.bh_energy(ctx)
    torch.cuda.synchronize()
    return t, acc.cpu(), acc2.cpu(), x.cpu(), e


def test_torch_allocator_same_results():
    pos, vel, mass = case_bodies("plummer", 50000, 3, np.float32)
    P, V, M = (torch.from_numpy(a).cuda() for a in (pos, vel, mass))
    say("allocator: 50000 bodies, hipMalloc vs torch caching allocator")
    c1 = B.bh_ctx_create(0)
    t1, *ref = _run(c1, P, V, M)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    c2 = B.bh_ctx_create(0)
    B.use_torch_allocator(c2)
    t2, *got = _run(c2, P, V, M)
    held = torch.cuda.memory_allocated() - before
    say(f"  torch allocator holds {held / 2**20:.1f} MiB for the context")
    assert held > 50000 * 64  # tree, simulation state and scratch at least
    for a, b in zip(ref[:3], got[:3]):
        assert torch.equal(a, b)
    assert ref[3] == got[3]
    B.bh_tree_free(t2)
    B.bh_ctx_destroy(c2)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    B.bh_tree_free(t1)
    B.bh_ctx_destroy(c1)


def test_allocator_refusal_is_nomem():
    """An allocator that returns NULL makes the call fail with BH_E_NOMEM;
    after switching back to hipMalloc the context works."""
    pos, _, mass = case_bodies("plummer", 4096, 4, np.float32)
    P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda()
    c = B.bh_ctx_create(0)
    B.bh_ctx_set_allocator(c, lambda n, d, s: 0, lambda p, n, d, s: None)
    with pytest.raises(B.BHError) as e:
        B.bh_build(c, P, M, 16)
    assert e.value.code == B.BH_E_NOMEM
    with pytest.raises(ValueError):
        B.bh_ctx_set_allocator(c, lambda n, d, s: 0)
    B.bh_ctx_set_allocator(c)
    t = B.bh_build(c, P, M, 16)
    B.bh_tree_free(t)
    B.bh_ctx_destroy(c)
