import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    oracle.build(force=False)
    yield


@pytest.fixture(scope="session")
def ctx():
    """One library context on cuda:0 for the GPU tests (the default stream)."""
    import torch
    from paper_2203_08966_amd import binding as B
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load()
    c = B.bh_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    B.bh_ctx_destroy(c)


def case_bodies(kind, n, seed, dtype):
    """Seeded bodies as numpy arrays of `dtype` (the same values feed both the
    GPU and, promoted exactly to float64, the oracle)."""
    import numpy as np
    from paper_2203_08966_amd import workloads as W
    if kind == "plummer":
        b = W.plummer(n, seed)
    elif kind == "two_spheres":
        b = W.two_spheres(n, seed)
    elif kind == "clumpy":
        b = W.clumpy(n, seed, n_clumps=max(1, n // 1000))
    elif kind == "coincident":
        rng = np.random.default_rng(seed)
        base = rng.normal(size=(-(-n // 7), 3))
        pos = np.repeat(base, 7, axis=0)[:n]
        b = W.Bodies(pos, np.zeros_like(pos), rng.random(n) + 0.1)
    elif kind == "tiny_cluster":
        rng = np.random.default_rng(seed)
        pos = rng.normal(size=(n, 3)) * 1e-5 + np.array([3.0, -1.0, 0.5])
        b = W.Bodies(pos, np.zeros_like(pos), np.full(n, 1.0 / n))
    else:
        raise ValueError(kind)
    return (np.ascontiguousarray(b.pos, dtype=dtype), np.ascontiguousarray(b.vel, dtype=dtype),
            np.ascontiguousarray(b.mass, dtype=dtype))


def say(*a):
    print(*a, flush=True)


def check_flagged(ref, orc_acc, gpu_acc, flag, eps, max_frac):
    """Bodies with a decision near its threshold (``flag``, sorted order):
    their share is at most ``max_frac``, and each one's GPU force is within
    the method's own error: its relative error against FP64 direct
    summation is at most the largest the oracle's walk (same criterion and
    parameters) makes on any body.  A decision taken the other way swaps one
    particle-cell term for the exact sum over the cell or back, so it can
    move a force by no more than the approximation the method accepts."""
    import numpy as np

    import oracle
    flag = np.asarray(flag) != 0
    frac = float(flag.mean())
    say(f"  flagged {flag.sum()} of {flag.size} ({frac:.4%}), bound {max_frac:.2%}")
    assert frac <= max_frac
    if not flag.any():
        return
    d, _ = oracle.direct(ref["spos"], ref["smass"], eps)
    nd = np.linalg.norm(d, axis=1)
    e_orc = np.linalg.norm(orc_acc - d, axis=1) / nd
    e_gpu = np.linalg.norm(gpu_acc[flag] - d[flag], axis=1) / nd[flag]
    say(f"  flagged: max error vs direct {e_gpu.max():.3e}, method's max {e_orc.max():.3e}")
    assert np.all(e_gpu <= e_orc.max())
