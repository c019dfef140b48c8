"""FP64 CPU oracle for the Barnes-Hut hot path (arXiv:2203.08966).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU library; the heavy loops live in ``oracle.c`` (plain C, FP64,
built with ``build()``), the glue here is plain numpy.

Pins (see ``tests/test_oracle_*.py``) tie every function to something other
than itself: the paper's worked Morton example and its 21-point quadtree
figure, closed forms (two-body force, two-mass quadrupole field, Plummer
energies, circular orbits), brute force on tiny inputs, invariants
(momentum conservation, coverage, time reversal) and theta = 0 equal to
direct summation.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None

_P = np.ctypeslib.ndpointer
_f64 = _P(np.float64, flags="C_CONTIGUOUS")
_i64 = _P(np.int64, flags="C_CONTIGUOUS")
_i32 = _P(np.int32, flags="C_CONTIGUOUS")
_u64 = _P(np.uint64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = C.CDLL(_LIB)
    lib.orc_num_threads.restype = C.c_int
    lib.orc_direct.argtypes = [C.c_int64, _f64, _f64, C.c_double, C.c_int64, _i64, _f64, _f64]
    lib.orc_root_cube.argtypes = [C.c_int64, _f64, _f64, C.POINTER(C.c_double)]
    lib.orc_interleave.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32]
    lib.orc_interleave.restype = C.c_uint64
    lib.orc_keys.argtypes = [C.c_int64, _f64, _f64, C.c_double, _u64]
    lib.orc_sort.argtypes = [C.c_int64, _u64, _i64]
    opt_u64 = C.c_void_p
    lib.orc_build.argtypes = [C.c_int64, _u64, C.c_int] + [opt_u64] * 7
    lib.orc_build.restype = C.c_int64
    lib.orc_build_curve.argtypes = [C.c_int64, _u64, _u64, C.c_int] + [opt_u64] * 7
    lib.orc_build_curve.restype = C.c_int64
    lib.orc_hilbert.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_uint32)]
    lib.orc_hilbert.restype = C.c_uint64
    lib.orc_keys_hilbert.argtypes = [C.c_int64, _f64, _f64, C.c_double, _u64]
    lib.orc_moments.argtypes = [C.c_int64, _i32, _u64, _i32, _i32, _f64, _f64, _f64,
                                C.c_double, _f64, _f64, _f64, C.c_void_p]
    lib.orc_walk.argtypes = [C.c_int64, _i32, _i32, _i32, _i32, _f64, _f64, _f64, _f64, _f64,
                             C.c_double, C.c_double, C.c_double, C.c_int, C.c_int64, _i64,
                             _f64, _f64, _i64, _i64, _i64, _i32, C.c_void_p, C.c_void_p,
                             C.c_int, C.c_double, C.c_void_p]
    lib.orc_octopole.argtypes = [C.c_int64, _i32, _i32, _f64, _f64, _f64, _f64]
    _lib = lib
    return lib


def num_threads() -> int:
    return int(_load().orc_num_threads())


def _pos64(pos):
    return np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(-1, 3))


def direct(pos, mass, eps: float, targets=None):
    """FP64 direct sum: (acc[t], phi[t]) for each body index in ``targets``
    (all bodies by default), original order."""
    lib = _load()
    p = _pos64(pos)
    m = np.ascontiguousarray(mass, dtype=np.float64)
    n = m.shape[0]
    t = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    acc = np.zeros((t.shape[0], 3))
    phi = np.zeros(t.shape[0])
    lib.orc_direct(n, p.ravel(), m, float(eps), t.shape[0], t, acc.ravel(), phi)
    return acc, phi


def root_cube(pos):
    lib = _load()
    p = _pos64(pos)
    lo = np.zeros(3)
    L = C.c_double()
    lib.orc_root_cube(p.shape[0], p.ravel(), lo, C.byref(L))
    return lo, L.value


def interleave(qx: int, qy: int, qz: int) -> int:
    return int(_load().orc_interleave(qx, qy, qz))


def keys(pos, lo, L, curve: str = "morton"):
    """Space-filling-curve keys of bodies in the root cube (lo, L): the
    Morton key (default) or the Peano-Hilbert index, 21 bits per axis."""
    lib = _load()
    p = _pos64(pos)
    k = np.zeros(p.shape[0], dtype=np.uint64)
    f = {"morton": lib.orc_keys, "hilbert": lib.orc_keys_hilbert}[curve]
    f(p.shape[0], p.ravel(), np.ascontiguousarray(lo, dtype=np.float64), float(L), k)
    return k


def hilbert(q, bits: int) -> int:
    """Peano-Hilbert index of the integer point q (any dimension, axis 0
    first) on a grid of 2^bits per axis."""
    a = (C.c_uint32 * len(q))(*[int(v) for v in q])
    return int(_load().orc_hilbert(len(q), int(bits), a))


def sort(k):
    lib = _load()
    k = np.ascontiguousarray(k, dtype=np.uint64)
    perm = np.zeros(k.shape[0], dtype=np.int64)
    lib.orc_sort(k.shape[0], k, perm)
    return perm


def build_tree(sorted_keys, leaf_size: int, cell_keys=None) -> dict:
    """Pre-order node arrays of the canonical octree over key-sorted bodies.
    With ``cell_keys`` (the Morton keys of the same sorted bodies, when they
    were sorted by another curve) cells are ordered by the curve and named
    by their Morton hashed keys."""
    lib = _load()
    k = np.ascontiguousarray(sorted_keys, dtype=np.uint64)
    n = k.shape[0]
    if cell_keys is not None:
        ck = np.ascontiguousarray(cell_keys, dtype=np.uint64)
        build = lambda *a: lib.orc_build_curve(n, k, ck, int(leaf_size), *a)  # noqa: E731
    else:
        build = lambda *a: lib.orc_build(n, k, int(leaf_size), *a)  # noqa: E731
    m = build(None, None, None, None, None, None, None)
    t = {
        "hkey": np.zeros(m, dtype=np.uint64),
        "level": np.zeros(m, dtype=np.int32),
        "begin": np.zeros(m, dtype=np.int32),
        "count": np.zeros(m, dtype=np.int32),
        "next": np.zeros(m, dtype=np.int32),
        "parent": np.zeros(m, dtype=np.int32),
        "cmask": np.zeros(m, dtype=np.int32),
    }
    m2 = build(*(t[f].ctypes.data for f in
                 ("hkey", "level", "begin", "count", "next", "parent", "cmask")))
    assert m2 == m
    return t


def moments(tree: dict, spos, smass, lo, L):
    lib = _load()
    m = tree["hkey"].shape[0]
    p = _pos64(spos)
    ms = np.ascontiguousarray(smass, dtype=np.float64)
    M = np.zeros(m)
    com = np.zeros((m, 3))
    Q = np.zeros((m, 6))
    trT = np.zeros(m)
    lib.orc_moments(m, tree["level"], tree["hkey"], tree["begin"], tree["count"], p.ravel(), ms,
                    np.ascontiguousarray(lo, dtype=np.float64), float(L), M, com.ravel(), Q.ravel(),
                    trT.ctypes.data)
    moments.trT = trT  # the last call's trace of the second moment
    return M, com, Q


class WalkResult(tuple):
    """(acc, phi, npp, npc, ncov, flag) of a tree walk; fields by name too.
    The budget walks add npq: of the npc particle-cell terms, those that
    carry the quadrupole."""
    _fields = ("acc", "phi", "npp", "npc", "ncov", "flag", "npq")

    def __new__(cls, *vals):
        return super().__new__(cls, vals)

    def __getattr__(self, name):
        try:
            return self[self._fields.index(name)]
        except ValueError:
            raise AttributeError(name) from None


def octopole(b):
    """Octopole moments per cell (n_cells x 10: xxx xxy xxz xyy xyz xzz yyy
    yyz yzz zzz), symmetric and traceless, about the COM; cached in b."""
    if "oct" not in b:
        t = b["tree"]
        com = b["mom"][1]
        m = com.shape[0]
        O = np.zeros((m, 10))
        _load().orc_octopole(m, t["begin"], t["count"], _pos64(b["spos"]).ravel(),
                             np.ascontiguousarray(b["smass"], dtype=np.float64), com.ravel(),
                             O.ravel())
        b["oct"] = O
    return b["oct"]


def walk(tree, mom, spos, smass, L, theta, eps, order=2, targets=None, guard_lo=None,
         tol=1e-5, oct=None):
    """Per-body tree walk over sorted bodies; ``targets`` are sorted ranks.
    ``guard_lo``: the root cube's corner, to open every cell whose cube holds
    the body (the containment guard, a variant); None: the paper's test.
    ``tol``: a body is flagged when an opening-angle test it takes lies
    within this relative margin of its threshold.  ``order`` 0 (monopole), 2
    (with the quadrupole) or 3 (and the octopole: ``oct`` from
    ``octopole``)."""
    if order >= 3 and oct is None:
        raise ValueError("order 3 needs the octopole moments (oct=octopole(b))")
    lib = _load()
    M, com, Q = mom
    p = _pos64(spos)
    ms = np.ascontiguousarray(smass, dtype=np.float64)
    n = ms.shape[0]
    t = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = t.shape[0]
    acc = np.zeros((nt, 3))
    phi = np.zeros(nt)
    npp = np.zeros(nt, dtype=np.int64)
    npc = np.zeros(nt, dtype=np.int64)
    ncov = np.zeros(nt, dtype=np.int64)
    flag = np.zeros(nt, dtype=np.int32)
    hk = np.ascontiguousarray(tree["hkey"], dtype=np.uint64)
    lo = None if guard_lo is None else np.ascontiguousarray(guard_lo, dtype=np.float64)
    lib.orc_walk(M.shape[0], tree["level"], tree["begin"], tree["count"], tree["next"],
                 M, com.ravel(), Q.ravel(), p.ravel(), ms, float(L), float(theta), float(eps),
                 int(order), nt, t, acc.ravel(), phi, npp, npc, ncov, flag,
                 hk.ctypes.data, None if lo is None else lo.ctypes.data,
                 0 if lo is None else 1, float(tol),
                 None if oct is None else np.ascontiguousarray(oct).ctypes.data)
    return WalkResult(acc, phi, npp, npc, ncov, flag)


def build_all(pos, mass, leaf_size: int, curve: str = "morton"):
    """Root cube, keys, stable sort, tree and moments for bodies in any order
    (bodies ordered along the Morton or the Peano-Hilbert curve)."""
    p = _pos64(pos)
    m = np.ascontiguousarray(mass, dtype=np.float64)
    lo, L = root_cube(p)
    k = keys(p, lo, L, curve)
    perm = sort(k)
    sk = k[perm]
    tree = build_tree(sk, leaf_size, None if curve == "morton" else keys(p, lo, L)[perm])
    spos = p[perm]
    smass = m[perm]
    mom = moments(tree, spos, smass, lo, L)
    return dict(lo=lo, L=L, keys=sk, perm=perm, tree=tree, mom=mom, trT=moments.trT, spos=spos,
                smass=smass)


def barnes_hut(pos, mass, theta, eps, leaf_size, order=2, targets=None, built=None):
    """Barnes-Hut forces on bodies ``targets`` (original indices; all by default).
    Returns a WalkResult (acc, phi, npp, npc, ncov, flag) in the order of
    ``targets``."""
    b = built if built is not None else build_all(pos, mass, leaf_size)
    n = b["perm"].shape[0]
    rank = np.empty(n, dtype=np.int64)
    rank[b["perm"]] = np.arange(n, dtype=np.int64)
    t = np.arange(n, dtype=np.int64) if targets is None else np.asarray(targets, dtype=np.int64)
    return walk(b["tree"], b["mom"], b["spos"], b["smass"], b["L"], theta, eps, order, rank[t],
                oct=octopole(b) if order >= 3 else None)


def energy(pos, vel, mass, eps):
    """(E_kin, E_pot) with E_pot = 1/2 sum_i m_i phi_i from the direct sum:
    each pair counted once (the double sum over i != j in the energy formula
    of Sec. 2.4 counts every pair twice), softened like the force."""
    m = np.asarray(mass, dtype=np.float64)
    v = np.asarray(vel, dtype=np.float64)
    ekin = 0.5 * float(np.sum(m * np.sum(v * v, axis=1)))
    _, phi = direct(pos, m, eps)
    epot = 0.5 * float(np.sum(m * phi))
    return ekin, epot


def standard_units(pos, vel, mass):
    """Scale a system to the standard units of Sec. 2.4, in the paper's
    order: total mass 1; shift to the centre-of-mass frame; one velocity
    factor so that E_kin = -E_pot / 2 (virial equilibrium); then lengths by
    b and velocities by 1 / sqrt(b), which divides the total energy by b,
    with b chosen so that it becomes -1/4.  E_pot is the unsoftened direct
    sum.  Returns (pos, vel, mass, (E_kin, E_pot, M)) with E_kin and E_pot
    of the shifted system before the two scalings and M the input's total
    mass."""
    m = np.asarray(mass, dtype=np.float64)
    M = float(m.sum())
    m = m / M
    x = _pos64(pos)
    v = _pos64(vel)
    x = x - np.sum(m[:, None] * x, axis=0)
    v = v - np.sum(m[:, None] * v, axis=0)
    ek, ep = energy(x, v, m, 0.0)
    v = v * np.sqrt(-ep / (2.0 * ek))  # now E = E_pot / 2
    b = -2.0 * ep                     # E / b = -1/4
    return x * b, v / np.sqrt(b), m, (ek, ep, M)


def kdk(pos, vel, mass, dt, steps, force):
    """Kick-drift-kick leapfrog (Sec. 2.3) with a fixed step: the acceleration
    at the start is computed once, then each step is half kick, drift, new
    acceleration, half kick.  ``force(pos) -> acc``.  Returns (pos, vel, acc)."""
    x = np.array(pos, dtype=np.float64)
    v = np.array(vel, dtype=np.float64)
    a = force(x)
    for _ in range(int(steps)):
        v = v + a * (0.5 * dt)
        x = x + v * dt
        a = force(x)
        v = v + a * (0.5 * dt)
    return x, v, a


def rms_rel(acc, ref):
    """sqrt(mean_i |a_i - a_i^ref|^2 / |a_i^ref|^2) with the median, p99, max."""
    e = np.linalg.norm(np.asarray(acc) - ref, axis=1) / np.linalg.norm(ref, axis=1)
    return dict(rms=float(np.sqrt(np.mean(e * e))), median=float(np.median(e)),
                p99=float(np.quantile(e, 0.99)), max=float(e.max()))


# ------------------------------------------------------------------ learned criterion
def _mac_sigs(lib):
    lib.orc_splitmix64.argtypes = [C.c_uint64]
    lib.orc_splitmix64.restype = C.c_uint64
    lib.orc_mlp_bf16.argtypes = [_f64, _f64]
    lib.orc_mlp_bf16.restype = C.c_double
    lib.orc_mlp_f16.argtypes = [_f64, _f64]
    lib.orc_mlp_f16.restype = C.c_double
    lib.orc_f16r.argtypes = [C.c_double]
    lib.orc_f16r.restype = C.c_double
    lib.orc_cell_kc.argtypes = [C.c_int64, _i32, _f64, C.c_double, _f64]
    lib.orc_walk_kc.argtypes = [_i32, _u64, _i32, _i32, _i32, _f64, _f64, _f64, _f64, _f64, _f64,
                                C.c_double, C.c_double, C.c_double, C.c_double, _f64, _f64,
                                C.c_int64, _i64, _f64, _f64, _i64, _i64, _i64, _i32, C.c_int, _i64]
    lib.orc_walk_group.argtypes = [_i32, _u64, _i32, _i32, _i32, _f64, _f64, _f64, _f64, _f64,
                                   _f64, C.c_double, C.c_double, C.c_int, C.c_int, C.c_double,
                                   C.c_double, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_int, C.c_int64, C.c_int64, C.c_int64, C.c_int64,
                                   C.c_double, _u64,
                                   _i32, C.c_int, _f64, _f64, _i64, _i64, _i64, _i32, C.c_void_p,
                                   _i64]
    lib.orc_gfeatures.argtypes = [_f64, _f64, _f64, C.c_double, _f64, C.c_double, _f64, C.c_int,
                                  C.c_int, C.c_double, _f64]
    lib.orc_gnet_bound.argtypes = [_f64, _f64, C.POINTER(C.c_double), C.c_int]
    lib.orc_gnet_bound.restype = C.c_double
    lib.orc_group_samples.argtypes = [_i32, _u64, _i32, _i32, _i32, _f64, _f64, _f64, _f64,
                                      _f64, _f64, C.c_double, C.c_int64, C.c_int64, C.c_double,
                                      C.c_double, C.c_double, C.c_double, C.c_uint64, C.c_int64,
                                      C.c_int64, _f64, _f64, _i32, _i64]
    return lib


def _mlib():
    lib = _load()
    if not getattr(lib, "_mac_ready", False):
        _mac_sigs(lib)
        lib._mac_ready = True
    return lib


def splitmix64(x: int) -> int:
    return int(_mlib().orc_splitmix64(x))


def mlp_bf16(params, f) -> float:
    return float(_mlib().orc_mlp_bf16(np.ascontiguousarray(params, dtype=np.float64),
                                      np.ascontiguousarray(f, dtype=np.float64)))


def mlp_f16(params, f) -> float:
    """The network with fp16 operands (IEEE binary16, nearest even)."""
    return float(_mlib().orc_mlp_f16(np.ascontiguousarray(params, dtype=np.float64),
                                     np.ascontiguousarray(f, dtype=np.float64)))


def f16r(x: float) -> float:
    """The C oracle's rounding of an FP32 value to binary16."""
    return float(_mlib().orc_f16r(float(x)))


def cell_kc(b):
    """Per cell M l^3: the error budget's coefficient k_C M l^3 with
    k_C = 1."""
    lib = _mlib()
    t = b["tree"]
    M = b["mom"][0]
    kc = np.zeros(M.shape[0])
    lib.orc_cell_kc(M.shape[0], t["level"], M, float(b["L"]), kc)
    return kc


def floored_norms(anorm, floor):
    """|a_i| as the error-budget test uses it: max(|a_i|, floor <|a|>), the
    mean taken over every given norm (the library's reading of the budget:
    error relative to the larger of the body's acceleration and a fraction
    of the mean one; floor = 0 leaves the norms as they are)."""
    a = np.asarray(anorm, dtype=np.float64)
    if floor <= 0:
        return a
    return np.maximum(a, floor * a.mean())


# mixed expansion order of the budget walks: per cell the monopole where the
# budget charged with the dropped quadrupole's bound holds, else the
# quadrupole where the plain budget holds, else the cell is opened
ORDER_MIXED = 1


def walk_kc(b, eps, theta_max, tau, kc, anorm, targets=None, floor=0.0, order=2):
    """Walk with the error budget (kc from ``cell_kc``); anorm is |a_i| per
    sorted rank, floored by ``floored_norms``.  order 0: monopole terms, the
    budget charging each cell the bound on its dropped quadrupole term too;
    ORDER_MIXED: the cheaper of the two orders that meets the budget."""
    anorm = floored_norms(anorm, floor)
    lib = _mlib()
    t = b["tree"]
    M, com, Q = b["mom"]
    n = b["smass"].shape[0]
    tg = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = tg.shape[0]
    acc = np.zeros((nt, 3))
    phi = np.zeros(nt)
    npp = np.zeros(nt, dtype=np.int64)
    npc = np.zeros(nt, dtype=np.int64)
    ncov = np.zeros(nt, dtype=np.int64)
    flag = np.zeros(nt, dtype=np.int32)
    npq = np.zeros(nt, dtype=np.int64)
    lib.orc_walk_kc(t["level"], t["hkey"], t["begin"], t["count"], t["next"], M, com.ravel(),
                    Q.ravel(), b["spos"].ravel(), b["smass"], np.ascontiguousarray(b["lo"]),
                    float(b["L"]), float(eps), float(theta_max),
                    float(tau), np.ascontiguousarray(kc, dtype=np.float64),
                    np.ascontiguousarray(anorm, dtype=np.float64), nt, tg, acc.ravel(), phi, npp,
                    npc, ncov, flag, int(order), npq)
    return WalkResult(acc, phi, npp, npc, ncov, flag, npq)


# ------------------------------------------------------------------ group walk
def leaf_levels(b):
    """Level of the leaf holding each sorted rank (cached in ``b``).  The
    leaves, in pre-order, cover the sorted bodies left to right."""
    if "_leaf_levels" in b:
        return b["_leaf_levels"]
    t = b["tree"]
    leaves = np.nonzero(t["next"] == np.arange(len(t["next"])) + 1)[0]
    cnt = t["count"][leaves].astype(np.int64)
    start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    assert np.array_equal(t["begin"][leaves], start) and cnt.sum() == len(b["smass"])
    out = np.repeat(t["level"][leaves], cnt).astype(np.int32)
    b["_leaf_levels"] = out
    return out


def walk_group(b, eps, *, cap, split, group=64, mode=0, theta=0.5, theta_max=1.0, tau=1e-3,
               kc=None, anorm=None, params=None, f16=False, order=2, target_range=None,
               tol=1e-5, floor=0.0):
    """Walk with one acceptance decision per group of ``group`` consecutive
    sorted ranks in ``target_range`` (all bodies by default): mode 0 opening
    angle, mode 1 error budget (kc per cell, anorm per sorted rank), mode 2
    the learned criterion (network ``params``, anorm per sorted rank; a run
    over the cap takes the learned decision with each body as its own
    group).  With
    ``split`` a group straddling a jump of the space-filling curve is cut
    into runs walked as groups of their own.  A run whose work (particle-cell
    terms plus particle-particle bodies) exceeds ``cap`` is walked per body.
    Both are part of the walk's definition and have no default: every caller
    states them.  Results are indexed by rank - t0."""
    lib = _mlib()
    t = b["tree"]
    M, com, Q = b["mom"]
    n = b["smass"].shape[0]
    t0, t1 = (0, n) if target_range is None else (int(target_range[0]), int(target_range[1]))
    nt = max(t1 - t0, 0)
    acc = np.zeros((nt, 3))
    phi = np.zeros(nt)
    npp = np.zeros(nt, dtype=np.int64)
    npc = np.zeros(nt, dtype=np.int64)
    ncov = np.zeros(nt, dtype=np.int64)
    flag = np.zeros(nt, dtype=np.int32)
    npq = np.zeros(nt, dtype=np.int64)
    kcv = None if kc is None else np.ascontiguousarray(kc, dtype=np.float64)
    anv = None if anorm is None else np.ascontiguousarray(floored_norms(anorm, floor))
    if mode == 1 and (kcv is None or anv is None):
        raise ValueError("the error-budget mode needs kc and anorm")
    pv = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
    if mode == 2 and (pv is None or anv is None):
        raise ValueError("the learned mode needs params and anorm")
    if nt:
        lib.orc_walk_group(t["level"], t["hkey"], t["begin"], t["count"], t["next"], M,
                           com.ravel(), Q.ravel(), b["spos"].ravel(), b["smass"],
                           np.ascontiguousarray(b["lo"]), float(b["L"]), float(eps), int(order),
                           int(mode), float(theta), float(theta_max), float(tau),
                           None if kcv is None else kcv.ctypes.data,
                           None if anv is None else anv.ctypes.data,
                           None if pv is None else pv.ctypes.data, 1 if f16 else 0, int(group),
                           t0, t1,
                           int(cap), float(tol), np.ascontiguousarray(b["keys"], dtype=np.uint64),
                           leaf_levels(b), 1 if split else 0, acc.ravel(), phi, npp, npc, ncov,
                           flag, octopole(b).ctypes.data if order >= 3 else None, npq)
    return WalkResult(acc, phi, npp, npc, ncov, flag, npq)


# ------------------------------------------------------------------ learned group criterion
def gfeatures(box_lo, box_hi, centre, side, com, M, Q, count, is_leaf, eps):
    """The 10 features of a (group box, cell) pair."""
    f = np.zeros(10)
    _mlib().orc_gfeatures(np.ascontiguousarray(box_lo, dtype=np.float64),
                          np.ascontiguousarray(box_hi, dtype=np.float64),
                          np.ascontiguousarray(centre, dtype=np.float64), float(side),
                          np.ascontiguousarray(com, dtype=np.float64), float(M),
                          np.ascontiguousarray(Q, dtype=np.float64), int(count), int(is_leaf),
                          float(eps), f)
    return f


def gnet_bound(params, f, f16=False):
    """(prediction, bound on the move of a reduced-precision evaluation) of
    the network with bf16 (or fp16) operands."""
    d = C.c_double()
    out = _mlib().orc_gnet_bound(np.ascontiguousarray(params, dtype=np.float64),
                                 np.ascontiguousarray(f, dtype=np.float64), C.byref(d),
                                 1 if f16 else 0)
    return float(out), d.value


def group_samples(b, eps, theta_lo, theta_max, keep, seed, group=64, cap=4096,
                  target_range=None):
    """Training pairs of the learned criterion from a tree of build_all:
    groups of ``group`` consecutive sorted ranks of ``target_range`` (all
    bodies by default), per group up to ``cap`` kept candidates in
    pre-order.  Returns (feat (ng, cap, 10), label (ng, cap), node (ng, cap),
    count (ng,))."""
    lib = _mlib()
    t = b["tree"]
    M, com, Q = b["mom"]
    n = b["smass"].shape[0]
    t0, t1 = (0, n) if target_range is None else (int(target_range[0]), int(target_range[1]))
    ng = (t1 - t0 + group - 1) // group
    feat = np.zeros((ng, cap, 10))
    label = np.zeros((ng, cap))
    node = np.full((ng, cap), -1, dtype=np.int32)
    cnt = np.zeros(ng, dtype=np.int64)
    lib.orc_group_samples(t["level"], t["hkey"], t["begin"], t["count"], t["next"], M,
                          com.ravel(), Q.ravel(), b["spos"].ravel(), b["smass"],
                          np.ascontiguousarray(b["lo"]), float(b["L"]), t0, t1, float(eps),
                          float(theta_lo), float(theta_max), float(keep), int(seed), int(group),
                          int(cap), feat.ravel(), label.ravel(), node.ravel(), cnt)
    return feat, label, node, cnt
