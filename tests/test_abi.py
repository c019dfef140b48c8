"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/bh.h declares, and rejects bad arguments with the
documented status before touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2203_08966_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bh.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bh_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = B.load()
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTED)


def test_version_and_defaults():
    assert B.bh_version().startswith("bh-gfx950")
    o = B.bh_force_opts_default()
    assert o.order == 2 and o.mac == B.BH_MAC_THETA
    assert o.target_begin == 0 and o.target_end == 0
    assert o.mlp_theta_max == 1.0 and o.mlp_log10_tau == -3.0 and o.mlp_theta_est == 0.8
    assert o.mlp_acc_norm is None and o.mlp_acc_floor == 0.0
    assert o.mlp_precision == B.BH_MLP_BF16
    assert o.n_pq is None


def test_null_handles_rejected():
    lib = B.load()
    assert lib.bh_ctx_create(0, None, None) == B.BH_E_INVALID
    h = C.c_void_p()
    assert lib.bh_ctx_create(-1, None, C.byref(h)) == B.BH_E_INVALID
    assert lib.bh_build(None, None, None, 0, 10, 8, C.byref(h)) == B.BH_E_INVALID
    assert "ctx" in B.bh_last_error()
    assert lib.bh_forces(None, 0.5, 0.0, None, None) == B.BH_E_INVALID
    assert lib.bh_leapfrog_step(None, 1e-3) == B.BH_E_INVALID
    assert lib.bh_sim_init(None, None, None, None, 0, 10, 8, 0.5, 0.0, None) == B.BH_E_INVALID
    assert lib.bh_sim_get(None, None, None, None) == B.BH_E_INVALID
    assert lib.bh_direct(None, None, None, 0, 1, None, 1, 0.0, None, None) == B.BH_E_INVALID
    assert lib.bh_standard_units(None, None, None, None, 0, 10, None) == B.BH_E_INVALID
    assert lib.bh_ctx_set_allocator(None, B.ALLOC_FN(), B.FREE_FN(), None) == B.BH_E_INVALID
    assert lib.bh_ctx_set_curve(None, B.BH_CURVE_HILBERT) == B.BH_E_INVALID
    assert lib.bh_ctx_set_sort(None, B.BH_SORT_FULL) == B.BH_E_INVALID
    assert lib.bh_tree_free(None) == B.BH_E_INVALID
    assert lib.bh_ctx_destroy(None) == B.BH_E_INVALID
    assert lib.bh_sync(None) == B.BH_E_INVALID
    assert lib.bh_tree_info_get(None, None) == B.BH_E_INVALID
    assert lib.bh_tree_export(None, *([None] * 12)) == B.BH_E_INVALID
    ek, ep = C.c_double(), C.c_double()
    assert lib.bh_energy(None, C.byref(ek), C.byref(ep)) == B.BH_E_INVALID
    assert lib.bh_sim_timing(None, 1) == B.BH_E_INVALID
    assert lib.bh_mlp_set(None, None) == B.BH_E_INVALID
    assert lib.bh_mlp_get(None, None) == B.BH_E_INVALID
    tot = C.c_int64()
    assert lib.bh_mlp_samples(None, 0.0, 0.3, 1.0, 1.0, 1, 0, None, None, None, None, C.byref(tot)) == B.BH_E_INVALID
    assert lib.bh_mlp_train(None, None, None, 1, None, None) == B.BH_E_INVALID
    assert lib.bh_mlp_grad(None, None, None, 1, 0.0, None, None) == B.BH_E_INVALID
    assert lib.bh_mlp_infer(None, None, 1, B.BH_MLP_BF16, None) == B.BH_E_INVALID
    assert lib.bh_sim_timing_get(None, None, None) == B.BH_E_INVALID
    assert lib.bh_sim_counts_get(None, None, None) == B.BH_E_INVALID
    assert lib.bh_sim_counts_pq_get(None, None) == B.BH_E_INVALID


def test_build_argument_checks_precede_device_use():
    """A stand-in context pointer is never dereferenced when the arguments
    are invalid, so these run without a GPU."""
    lib = B.load()
    dummy = C.create_string_buffer(256)
    ctx = C.c_void_p(C.addressof(dummy))
    buf = C.create_string_buffer(64)
    p = C.c_void_p(C.addressof(buf))
    tree = C.c_void_p()
    cases = [
        (None, p, B.BH_F32, 10, 8),   # null pos
        (p, None, B.BH_F32, 10, 8),   # null mass
        (p, p, 7, 10, 8),             # bad dtype
        (p, p, B.BH_F32, 0, 8),       # n < 1
        (p, p, B.BH_F32, 1 << 31, 8), # n too large
        (p, p, B.BH_F32, 10, 0),      # leaf < 1
        (p, p, B.BH_F32, 10, 257),    # leaf > 256
    ]
    for pos, mass, dt, n, leaf in cases:
        assert lib.bh_build(ctx, pos, mass, dt, n, leaf, C.byref(tree)) == B.BH_E_INVALID
        assert B.bh_last_error()
    assert lib.bh_build(ctx, p, p, B.BH_F32, 10, 8, None) == B.BH_E_INVALID


def test_force_parameter_checks_precede_device_use():
    lib = B.load()
    dummy = C.create_string_buffer(1024)
    t = C.c_void_p(C.addressof(dummy))
    buf = C.create_string_buffer(64)
    acc = C.c_void_p(C.addressof(buf))
    for theta, eps in [(-0.1, 0.0), (float("nan"), 0.0), (float("inf"), 0.0), (0.5, -1.0),
                       (0.5, float("nan"))]:
        assert lib.bh_forces(t, theta, eps, acc, None) == B.BH_E_INVALID
    assert lib.bh_forces(t, 0.5, 0.0, None, None) == B.BH_E_INVALID
    for f in (-0.5, float("nan"), float("inf")):
        o = B.force_opts(mac=B.BH_MAC_BUDGET, mlp_acc_floor=f)
        assert lib.bh_forces(t, 0.5, 0.0, acc, C.byref(o)) == B.BH_E_INVALID
        assert "learned-criterion" in B.bh_last_error()
    o = B.force_opts(mac=B.BH_MAC_MLP, mlp_precision=2)
    assert lib.bh_forces(t, 0.5, 0.0, acc, C.byref(o)) == B.BH_E_INVALID
    # the mixed order runs with the error budget only; order 4 does not exist
    for mac, order in ((B.BH_MAC_THETA, B.BH_ORDER_MIXED), (B.BH_MAC_MLP, B.BH_ORDER_MIXED),
                       (B.BH_MAC_BUDGET, 4)):
        o = B.force_opts(mac=mac, order=order)
        assert lib.bh_forces(t, 0.5, 0.0, acc, C.byref(o)) == B.BH_E_INVALID
        assert "order" in B.bh_last_error()
    ctx = C.c_void_p(C.addressof(dummy))
    assert lib.bh_mlp_infer(ctx, acc, 1, 2, acc) == B.BH_E_INVALID
    assert "precision" in B.bh_last_error()


def test_sim_argument_checks():
    lib = B.load()
    dummy = C.create_string_buffer(256)
    ctx = C.c_void_p(C.addressof(dummy))
    buf = C.create_string_buffer(64)
    p = C.c_void_p(C.addressof(buf))
    assert lib.bh_sim_init(ctx, p, None, p, 0, 10, 8, 0.5, 0.0, None) == B.BH_E_INVALID
    assert lib.bh_sim_init(ctx, p, p, p, 0, 10, 8, -0.5, 0.0, None) == B.BH_E_INVALID
    assert lib.bh_sim_init(ctx, p, p, p, 0, 0, 8, 0.5, 0.0, None) == B.BH_E_INVALID
    assert lib.bh_direct(ctx, p, p, 0, 10, p, 0, 0.0, p, None) == B.BH_E_INVALID
    assert lib.bh_direct(ctx, p, p, 3, 10, p, 5, 0.0, p, None) == B.BH_E_INVALID
    assert lib.bh_direct(ctx, p, p, 0, 10, p, 5, -1.0, p, None) == B.BH_E_INVALID


def test_no_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert B.load().bh_ctx_create(0, None, C.byref(h)) == B.BH_E_DEVICE
    assert "device" in B.bh_last_error().lower()


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus 2 exits with status 2 and a JSON
    line that says so, before touching a device."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]
