"""ctypes binding of libbh.so: argument marshalling only.

Every function carries the name of the C entry point it calls (see
include/bh.h) and takes torch tensors on the GPU; all work runs in the HIP
library on the current torch stream.  There is no fallback: if the library
is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbh.so")

BH_OK, BH_E_INVALID, BH_E_NOMEM, BH_E_DEVICE, BH_E_STATE, BH_E_NONFINITE = 0, -1, -2, -3, -4, -5
BH_F32, BH_F64 = 0, 1
BH_MAC_THETA, BH_MAC_MLP, BH_MAC_BUDGET, BH_MAC_THETA_GUARD = 0, 1, 2, 3
BH_MLP_BF16, BH_MLP_FP16 = 0, 1
BH_WALK_BODY, BH_WALK_GROUP, BH_WALK_DIRECT = 0, 1, 2
BH_GROUP_BODIES = 64  # bodies per group of BH_WALK_GROUP
BH_CURVE_MORTON, BH_CURVE_HILBERT = 0, 1
BH_SORT_ADAPTIVE, BH_SORT_FULL = 0, 1
BH_ORDER_MIXED = 1  # opts.order of the error budget: monopole or quadrupole per cell

EXPORTED = [
    "bh_version", "bh_last_error", "bh_force_opts_default", "bh_ctx_create", "bh_ctx_set_stream",
    "bh_ctx_destroy", "bh_sync", "bh_build", "bh_tree_free", "bh_forces", "bh_tree_info_get",
    "bh_tree_export", "bh_sim_init", "bh_leapfrog_step", "bh_sim_get", "bh_energy",
    "bh_sim_tree", "bh_direct", "bh_direct_static", "bh_sim_timing", "bh_sim_timing_get", "bh_sim_counts_get",
    "bh_sim_counts_pq_get",
    "bh_mlp_set",
    "bh_mlp_get", "bh_mlp_samples", "bh_mlp_train", "bh_mlp_grad", "bh_mlp_infer",
    "bh_standard_units", "bh_ctx_set_allocator", "bh_ctx_set_curve", "bh_ctx_set_sort",
]
BH_MLP_PARAMS = 1441


__all__ = EXPORTED + [
    "BHError", "ForceOpts", "TreeInfo", "force_opts", "load", "BH_OK", "BH_E_INVALID",
    "BH_E_NOMEM", "BH_E_DEVICE", "BH_E_STATE", "BH_E_NONFINITE", "BH_F32", "BH_F64",
    "use_torch_allocator", "BH_MAC_THETA", "BH_MAC_MLP", "BH_MAC_BUDGET", "BH_MAC_THETA_GUARD", "BH_WALK_BODY", "BH_WALK_GROUP", "BH_WALK_DIRECT",
    "BH_GROUP_BODIES",
]


class BHError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class ForceOpts(C.Structure):
    _fields_ = [
        ("order", C.c_int), ("mac", C.c_int), ("phi", C.c_void_p), ("n_pp", C.c_void_p),
        ("n_pc", C.c_void_p), ("target_begin", C.c_int64), ("target_end", C.c_int64),
        ("mlp_theta_max", C.c_double), ("mlp_log10_tau", C.c_double),
        ("mlp_acc_norm", C.c_void_p), ("mlp_theta_est", C.c_double),
        ("walk", C.c_int), ("walk_stack", C.c_int), ("walk_cap", C.c_int),
        ("mlp_acc_floor", C.c_double), ("mlp_precision", C.c_int), ("n_pq", C.c_void_p),
    ]


class MlpTrainCfg(C.Structure):
    _fields_ = [("epochs", C.c_int), ("batch", C.c_int), ("lr", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("seed", C.c_uint64), ("quantile", C.c_double)]


class TreeInfo(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("m", C.c_int64), ("depth", C.c_int32), ("dtype", C.c_int32),
        ("leaf_size", C.c_int32), ("last_mac", C.c_int32), ("curve", C.c_int32),
        ("reserved", C.c_int32), ("lo", C.c_double * 3), ("side", C.c_double),
        ("movers", C.c_int64),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Load libbh.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not built: run __graft_entry__.build() or "
                          "python paper_2203_08966_amd/build_lib.py")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
    pp = C.POINTER(C.c_void_p)
    sig = {
        "bh_version": ([], C.c_char_p),
        "bh_last_error": ([], C.c_char_p),
        "bh_force_opts_default": ([C.POINTER(ForceOpts)], None),
        "bh_ctx_create": ([i32, vp, pp], i32),
        "bh_ctx_set_stream": ([vp, vp], i32),
        "bh_ctx_set_curve": ([vp, i32], i32),
        "bh_ctx_set_sort": ([vp, i32], i32),
        "bh_ctx_destroy": ([vp], i32),
        "bh_sync": ([vp], i32),
        "bh_build": ([vp, vp, vp, i32, i64, i32, pp], i32),
        "bh_tree_free": ([vp], i32),
        "bh_forces": ([vp, dbl, dbl, vp, C.POINTER(ForceOpts)], i32),
        "bh_tree_info_get": ([vp, C.POINTER(TreeInfo)], i32),
        "bh_tree_export": ([vp] + [vp] * 12, i32),
        "bh_sim_init": ([vp, vp, vp, vp, i32, i64, i32, dbl, dbl, C.POINTER(ForceOpts)], i32),
        "bh_leapfrog_step": ([vp, dbl], i32),
        "bh_sim_get": ([vp, vp, vp, vp], i32),
        "bh_energy": ([vp, C.POINTER(dbl), C.POINTER(dbl)], i32),
        "bh_sim_tree": ([vp, pp], i32),
        "bh_direct": ([vp, vp, vp, i32, i64, vp, i64, dbl, vp, vp], i32),
        "bh_direct_static": ([vp, vp, vp, i32, i64, vp, i64, dbl, vp, vp], i32),
        "bh_standard_units": ([vp, vp, vp, vp, i32, i64, vp], i32),
        "bh_ctx_set_allocator": ([vp, ALLOC_FN, FREE_FN, vp], i32),
        "bh_sim_timing": ([vp, i32], i32),
        "bh_sim_timing_get": ([vp, C.POINTER(dbl), C.POINTER(i64)], i32),
        "bh_sim_counts_get": ([vp, C.POINTER(i64), C.POINTER(i64)], i32),
        "bh_sim_counts_pq_get": ([vp, C.POINTER(i64)], i32),
        "bh_mlp_set": ([vp, vp], i32),
        "bh_mlp_get": ([vp, vp], i32),
        "bh_mlp_samples": ([vp, dbl, dbl, dbl, dbl, C.c_uint64, i64, vp, vp, vp, vp,
                            C.POINTER(i64)], i32),
        "bh_mlp_train": ([vp, vp, vp, i64, C.POINTER(MlpTrainCfg), vp], i32),
        "bh_mlp_grad": ([vp, vp, vp, i64, dbl, vp, C.POINTER(dbl)], i32),
        "bh_mlp_infer": ([vp, vp, i64, i32, vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != BH_OK:
        raise BHError(rc, load().bh_last_error().decode())


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return BH_F32
    if t.dtype == torch.float64:
        return BH_F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev(t, name):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _bodies(pos, mass, vel=None):
    """Shape/dtype checks shared by the entry points that take bodies."""
    n = int(mass.shape[0])
    if mass.dim() != 1 or tuple(pos.shape) != (n, 3):
        raise ValueError(f"pos must be (n, 3) and mass (n,); got {tuple(pos.shape)}, {tuple(mass.shape)}")
    if vel is not None and tuple(vel.shape) != (n, 3):
        raise ValueError("vel must be (n, 3)")
    for t in (mass, vel):
        if t is not None and t.dtype != pos.dtype:
            raise TypeError("pos, vel and mass must share a dtype")
    return n


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def force_opts(order=2, mac=BH_MAC_THETA, phi=None, n_pp=None, n_pc=None, target_range=None,
               mlp_theta_max=None, mlp_log10_tau=None, mlp_acc_norm=None,
               mlp_theta_est=None, walk=BH_WALK_BODY, walk_stack=0, walk_cap=0,
               mlp_acc_floor=None, mlp_precision=None, n_pq=None) -> ForceOpts:
    """Walk options.  mlp_acc_norm: device tensor of |a_i| in caller order
    and the tree's dtype (kept alive by the caller until the walk ran);
    mlp_acc_floor: f in max(|a_i|, f <|a|>)."""
    o = ForceOpts()
    load().bh_force_opts_default(C.byref(o))
    o.order = order
    o.mac = mac
    o.phi = _dev(phi, "phi")
    o.n_pp = _dev(n_pp, "n_pp")
    o.n_pc = _dev(n_pc, "n_pc")
    if target_range is not None:
        o.target_begin, o.target_end = int(target_range[0]), int(target_range[1])
    if mlp_theta_max is not None:
        o.mlp_theta_max = mlp_theta_max
    if mlp_log10_tau is not None:
        o.mlp_log10_tau = mlp_log10_tau
    o.mlp_acc_norm = _dev(mlp_acc_norm, "mlp_acc_norm")
    if mlp_theta_est is not None:
        o.mlp_theta_est = mlp_theta_est
    o.walk = walk
    o.walk_stack = walk_stack
    o.walk_cap = walk_cap
    if mlp_acc_floor is not None:
        o.mlp_acc_floor = mlp_acc_floor
    if mlp_precision is not None:
        o.mlp_precision = mlp_precision
    o.n_pq = _dev(n_pq, "n_pq")
    return o


# ----------------------------------------------------------------- entry points
def bh_version() -> str:
    return load().bh_version().decode()


def bh_last_error() -> str:
    return load().bh_last_error().decode()


def bh_force_opts_default() -> ForceOpts:
    o = ForceOpts()
    load().bh_force_opts_default(C.byref(o))
    return o


def bh_ctx_create(device: int = 0, stream=None) -> C.c_void_p:
    h = C.c_void_p()
    s = _stream() if stream is None else C.c_void_p(stream)
    _check(load().bh_ctx_create(device, s, C.byref(h)))
    return h


def bh_ctx_set_stream(ctx, stream=None):
    _check(load().bh_ctx_set_stream(ctx, _stream() if stream is None else C.c_void_p(stream)))


def bh_ctx_set_curve(ctx, curve: int):
    _check(load().bh_ctx_set_curve(ctx, int(curve)))


def bh_ctx_set_sort(ctx, mode: int):
    _check(load().bh_ctx_set_sort(ctx, int(mode)))


def bh_ctx_destroy(ctx):
    _check(load().bh_ctx_destroy(ctx))
    _ALLOCATORS.pop(ctx.value, None)


# bh_alloc_fn / bh_free_fn
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_int, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p, C.c_void_p)
_ALLOCATORS = {}  # ctx -> callbacks, kept alive while the context lives


def bh_ctx_set_allocator(ctx, alloc=None, free=None):
    """Route the context's device memory through alloc(bytes, device,
    stream) -> int and free(ptr, bytes, device, stream) (Python callables;
    None, None: hipMalloc)."""
    if (alloc is None) != (free is None):
        raise ValueError("give both allocator functions or neither")
    if alloc is None:
        _check(load().bh_ctx_set_allocator(ctx, ALLOC_FN(), FREE_FN(), None))
        return

    def _a(nbytes, dev, stream, user):
        try:
            return alloc(int(nbytes), int(dev), stream or 0) or None
        except Exception:  # the library reports BH_E_NOMEM
            return None

    def _f(ptr, nbytes, dev, stream, user):
        try:
            free(int(ptr), int(nbytes), int(dev), stream or 0)
        except Exception:
            pass
    cbs = (ALLOC_FN(_a), FREE_FN(_f))
    _check(load().bh_ctx_set_allocator(ctx, cbs[0], cbs[1], None))
    _ALLOCATORS.setdefault(ctx.value, []).append(cbs)


def use_torch_allocator(ctx):
    """Take the context's device memory from torch's caching allocator."""
    import torch
    bh_ctx_set_allocator(
        ctx, lambda n, dev, stream: torch.cuda.caching_allocator_alloc(n, dev, stream),
        lambda p, n, dev, stream: torch.cuda.caching_allocator_delete(p))


def bh_sync(ctx):
    _check(load().bh_sync(ctx))


def bh_build(ctx, pos, mass, leaf_size: int, tree=None) -> C.c_void_p:
    n = _bodies(pos, mass)
    h = C.c_void_p(tree.value if tree is not None else None)
    _check(load().bh_build(ctx, _dev(pos, "pos"), _dev(mass, "mass"), _dtype_code(pos),
                           n, int(leaf_size), C.byref(h)))
    return h


def bh_tree_free(tree):
    _check(load().bh_tree_free(tree))


def bh_forces(tree, theta: float, eps: float, acc, opts: ForceOpts | None = None):
    info = TreeInfo()
    _check(load().bh_tree_info_get(tree, C.byref(info)))
    if tuple(acc.shape) != (info.n, 3) or _dtype_code(acc) != info.dtype:
        raise ValueError("acc must be (n, 3) in the tree's dtype")
    _check(load().bh_forces(tree, float(theta), float(eps), _dev(acc, "acc"),
                            C.byref(opts) if opts is not None else None))


def bh_tree_info_get(tree) -> dict:
    info = TreeInfo()
    _check(load().bh_tree_info_get(tree, C.byref(info)))
    return dict(n=info.n, m=info.m, depth=info.depth, dtype=info.dtype,
                leaf_size=info.leaf_size, last_mac=info.last_mac, curve=info.curve,
                lo=np.array(info.lo[:]), side=info.side, movers=info.movers)


def bh_tree_export(tree) -> dict:
    info = bh_tree_info_get(tree)
    n, m = info["n"], info["m"]
    out = dict(
        keys=np.zeros(n, np.uint64), perm=np.zeros(n, np.uint32), hkey=np.zeros(m, np.uint64),
        level=np.zeros(m, np.int32), begin=np.zeros(m, np.int32), count=np.zeros(m, np.int32),
        next=np.zeros(m, np.int32), parent=np.zeros(m, np.int32), cmask=np.zeros(m, np.int32),
        mass=np.zeros(m), com=np.zeros((m, 3)), quad=np.zeros((m, 6)),
    )
    order = ["keys", "perm", "hkey", "level", "begin", "count", "next", "parent", "cmask",
             "mass", "com", "quad"]
    _check(load().bh_tree_export(tree, *[C.c_void_p(out[k].ctypes.data) for k in order]))
    out.update(info)
    return out


def bh_sim_init(ctx, pos, vel, mass, leaf_size: int, theta: float, eps: float,
                opts: ForceOpts | None = None):
    n = _bodies(pos, mass, vel)
    _check(load().bh_sim_init(ctx, _dev(pos, "pos"), _dev(vel, "vel"), _dev(mass, "mass"),
                              _dtype_code(pos), n, int(leaf_size),
                              float(theta), float(eps), C.byref(opts) if opts else None))


def bh_leapfrog_step(ctx, dt: float):
    _check(load().bh_leapfrog_step(ctx, float(dt)))


def bh_sim_get(ctx, pos=None, vel=None, acc=None):
    info = bh_tree_info_get(bh_sim_tree(ctx))
    for t, name in ((pos, "pos"), (vel, "vel"), (acc, "acc")):
        if t is not None and (tuple(t.shape) != (info["n"], 3) or _dtype_code(t) != info["dtype"]):
            raise ValueError(f"{name} must be (n, 3) in the simulation's dtype")
    _check(load().bh_sim_get(ctx, _dev(pos, "pos"), _dev(vel, "vel"), _dev(acc, "acc")))


def bh_energy(ctx) -> tuple[float, float]:
    ek, ep = C.c_double(), C.c_double()
    _check(load().bh_energy(ctx, C.byref(ek), C.byref(ep)))
    return ek.value, ep.value


def bh_sim_tree(ctx) -> C.c_void_p:
    h = C.c_void_p()
    _check(load().bh_sim_tree(ctx, C.byref(h)))
    return h


def _direct_args(pos, mass, targets, acc, phi):
    import torch
    if targets.dtype != torch.int64:
        raise TypeError("targets must be int64")
    _bodies(pos, mass)
    nt = int(targets.shape[0])
    if tuple(acc.shape) != (nt, 3) or acc.dtype != torch.float64:
        raise ValueError("acc must be (len(targets), 3) float64")
    if phi is not None and (tuple(phi.shape) != (nt,) or phi.dtype != torch.float64):
        raise ValueError("phi must be (len(targets),) float64")
    return (_dev(pos, "pos"), _dev(mass, "mass"), _dtype_code(pos), int(mass.shape[0]),
            _dev(targets, "targets"), nt)


def bh_direct(ctx, pos, mass, targets, eps: float, acc, phi=None):
    _check(load().bh_direct(ctx, *_direct_args(pos, mass, targets, acc, phi), float(eps),
                            _dev(acc, "acc"), _dev(phi, "phi")))


def bh_direct_static(ctx, pos, mass, targets, eps: float, acc, phi=None):
    """bh_direct without any device allocation (fixed per-GPU scratch)."""
    _check(load().bh_direct_static(ctx, *_direct_args(pos, mass, targets, acc, phi), float(eps),
                                   _dev(acc, "acc"), _dev(phi, "phi")))


def bh_standard_units(ctx, pos, vel, mass) -> tuple[float, float, float]:
    """Scale (pos, vel, mass) in place to standard units; returns E_kin,
    E_pot and the total mass before the scaling."""
    _bodies(pos, mass)
    if tuple(vel.shape) != tuple(pos.shape) or vel.dtype != pos.dtype:
        raise ValueError("vel must match pos in shape and dtype")
    st = (C.c_double * 3)()
    _check(load().bh_standard_units(ctx, _dev(pos, "pos"), _dev(vel, "vel"), _dev(mass, "mass"),
                                    _dtype_code(pos), int(mass.shape[0]), st))
    return st[0], st[1], st[2]


def bh_sim_timing(ctx, enable: bool = True):
    _check(load().bh_sim_timing(ctx, 1 if enable else 0))


def bh_sim_timing_get(ctx) -> tuple[list, int]:
    ms = (C.c_double * 5)()
    steps = C.c_int64()
    _check(load().bh_sim_timing_get(ctx, ms, C.byref(steps)))
    return list(ms), steps.value


def bh_sim_counts_get(ctx) -> tuple[int, int]:
    """(sum n_pp, sum n_pc) over the walks of the recorded steps."""
    pp, pc = C.c_int64(), C.c_int64()
    _check(load().bh_sim_counts_get(ctx, C.byref(pp), C.byref(pc)))
    return pp.value, pc.value


def bh_sim_counts_pq_get(ctx) -> int:
    """Of the recorded steps' particle-cell terms, those with the quadrupole."""
    pq = C.c_int64()
    _check(load().bh_sim_counts_pq_get(ctx, C.byref(pq)))
    return pq.value


# ----------------------------------------------------------------- learned criterion
def bh_mlp_set(ctx, params):
    p = np.ascontiguousarray(params, dtype=np.float64)
    if p.shape != (BH_MLP_PARAMS,):
        raise ValueError(f"params must have {BH_MLP_PARAMS} values")
    _check(load().bh_mlp_set(ctx, C.c_void_p(p.ctypes.data)))


def bh_mlp_get(ctx) -> np.ndarray:
    p = np.zeros(BH_MLP_PARAMS)
    _check(load().bh_mlp_get(ctx, C.c_void_p(p.ctypes.data)))
    return p


def bh_mlp_samples(tree, eps, theta_lo, theta_max, keep, seed):
    """Training pairs of an FP64 tree: (feat, label, node, group's first
    sorted rank) GPU tensors."""
    import torch
    tot = C.c_int64()
    lib = load()
    _check(lib.bh_mlp_samples(tree, float(eps), float(theta_lo), float(theta_max), float(keep),
                              int(seed), 0, None, None, None, None, C.byref(tot)))
    n = tot.value
    dev = torch.device("cuda")
    feat = torch.empty((max(n, 1), 10), dtype=torch.float32, device=dev)
    label = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
    node = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    group = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    _check(lib.bh_mlp_samples(tree, float(eps), float(theta_lo), float(theta_max), float(keep),
                              int(seed), n, _dev(feat, "feat"), _dev(label, "label"),
                              _dev(node, "node"), _dev(group, "group"), C.byref(tot)))
    return feat[:n], label[:n], node[:n], group[:n]


def _pairs(feat, label):
    import torch
    if feat.dtype != torch.float32 or label.dtype != torch.float32:
        raise TypeError("feat and label must be float32")
    n = int(label.shape[0])
    if tuple(feat.shape) != (n, 10):
        raise ValueError("feat must be (n, 10)")
    return n


def bh_mlp_train(ctx, feat, label, epochs=10, batch=4096, lr=1e-3, beta1=0.9, beta2=0.999,
                 eps=1e-8, seed=7, quantile=0.0) -> np.ndarray:
    n = _pairs(feat, label)
    cfg = MlpTrainCfg(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps),
                      int(seed), float(quantile))
    loss = np.zeros(max(int(epochs), 1))
    _check(load().bh_mlp_train(ctx, _dev(feat, "feat"), _dev(label, "label"), n, C.byref(cfg),
                               C.c_void_p(loss.ctypes.data)))
    return loss[:int(epochs)]


def bh_mlp_grad(ctx, feat, label, quantile=0.0):
    import torch
    n = _pairs(feat, label)
    g = torch.empty(BH_MLP_PARAMS, dtype=torch.float32, device="cuda")
    lv = C.c_double()
    _check(load().bh_mlp_grad(ctx, _dev(feat, "feat"), _dev(label, "label"), n, float(quantile),
                              _dev(g, "grad"), C.byref(lv)))
    return g, lv.value


def bh_mlp_infer(ctx, feat, precision=None):
    import torch
    if feat.dtype != torch.float32 or feat.dim() != 2 or feat.shape[1] != 10:
        raise ValueError("feat must be (n, 10) float32")
    n = int(feat.shape[0])
    pred = torch.empty(n, dtype=torch.float32, device="cuda")
    prec = BH_MLP_BF16 if precision is None else precision
    _check(load().bh_mlp_infer(ctx, _dev(feat, "feat"), n, prec, _dev(pred, "pred")))
    return pred
