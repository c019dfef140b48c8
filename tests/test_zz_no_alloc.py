"""bh_direct_static, the direct sum for callers that cannot allocate, called
through the C ABI: bitwise the results of bh_direct on two calls in a row
(the second smaller, so it reads only what it wrote itself), and a target
count beyond its fixed scratch refused before any launch."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2203_08966_amd import binding as B
from tests.conftest import case_bodies, say

pytestmark = pytest.mark.gpu


def _raw(fn, ctx, P, M, tg, eps, acc, phi):
    """Direct ctypes call of one of the two entry points."""
    lib = B.load()
    return getattr(lib, fn)(ctx, C.c_void_p(P.data_ptr()), C.c_void_p(M.data_ptr()),
                            B.BH_F32 if P.dtype == torch.float32 else B.BH_F64,
                            int(M.shape[0]), C.c_void_p(tg.data_ptr()), int(tg.shape[0]),
                            float(eps), C.c_void_p(acc.data_ptr()),
                            C.c_void_p(phi.data_ptr()) if phi is not None else None)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_static_scratch_matches_bh_direct(dtype):
    ctx = B.bh_ctx_create(0)
    try:
        for k, (n, nt) in enumerate(((70000, 30000), (9000, 777))):
            pos, _, mass = case_bodies("plummer", n, 40 + k, dtype)
            P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda()
            rng = np.random.default_rng(k)
            tg = torch.from_numpy(rng.choice(n, nt, replace=False).astype(np.int64)).cuda()
            say(f"no-alloc direct: call {k + 1}, n={n}, {nt} targets, {np.dtype(dtype).name}")
            a0 = torch.full((nt, 3), np.nan, dtype=torch.float64, device="cuda")
            p0 = torch.full((nt,), np.nan, dtype=torch.float64, device="cuda")
            a1, p1 = a0.clone(), p0.clone()
            assert _raw("bh_direct", ctx, P, M, tg, 0.01, a0, p0) == B.BH_OK
            assert _raw("bh_direct_static", ctx, P, M, tg, 0.01, a1, p1) == B.BH_OK
            torch.cuda.synchronize()
            assert torch.isfinite(a1).all() and torch.isfinite(p1).all()
            assert torch.equal(a0, a1) and torch.equal(p0, p1)
        # a target count the fixed scratch cannot hold is refused on the host
        n = 4096
        pos, _, mass = case_bodies("plummer", n, 45, np.float32)
        P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda()
        big = 524289
        tg = torch.zeros(big, dtype=torch.int64, device="cuda")
        a = torch.zeros((big, 3), dtype=torch.float64, device="cuda")
        assert _raw("bh_direct_static", ctx, P, M, tg, 0.01, a, None) == B.BH_E_INVALID
        assert "nt" in B.bh_last_error()
        torch.cuda.synchronize()
        assert torch.count_nonzero(a).item() == 0
    finally:
        B.bh_ctx_destroy(ctx)
