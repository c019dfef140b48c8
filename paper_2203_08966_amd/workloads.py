"""Seeded synthetic N-body initial conditions.

This module only draws random numbers and lays out initial conditions; it holds
none of the Barnes-Hut arithmetic (no keys, trees, moments or forces), so both
the GPU path and the FP64 oracle can be fed the identical arrays it returns.

Workloads (the paper's test problem is two colliding Plummer clusters in
standard units, Sec. 5; the sizes below are the measured configurations):

* ``plummer``   -- one Plummer sphere, equal masses.
* ``two_spheres`` -- two Plummer spheres on a collision course, lognormal masses.
* ``two_clusters`` -- the paper's test problem: two equal-mass Plummer
  clusters of n/2 bodies each, offset in every dimension, at rest relative
  to each other (to be scaled to standard units before use).
* ``clumpy``    -- many small Plummer clumps in a unit cube plus a uniform
  background at rest.

Plummer sampling follows the method of Aarseth, Henon and Wielen (1974):
invert the cumulative mass profile for r, draw the speed ratio q from
g(q) ~ q^2 (1-q^2)^(7/2) by rejection, isotropic directions, then shift to the
centre-of-mass frame.  Units: G = 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Bodies",
    "plummer",
    "two_spheres",
    "two_clusters",
    "clumpy",
    "subsample",
    "config",
    "CONFIGS",
]


@dataclass
class Bodies:
    pos: np.ndarray   # (N, 3) float64 or float32
    vel: np.ndarray   # (N, 3)
    mass: np.ndarray  # (N,)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.mass.shape[0])

    def astype(self, dtype) -> "Bodies":
        return Bodies(self.pos.astype(dtype), self.vel.astype(dtype),
                      self.mass.astype(dtype), dict(self.meta))


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    """Unit vectors uniform on the sphere."""
    cz = 1.0 - 2.0 * rng.random(n)
    ph = 2.0 * np.pi * rng.random(n)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return np.stack([sz * np.cos(ph), sz * np.sin(ph), cz], axis=1)


def _plummer_unit(rng: np.random.Generator, n: int):
    """Positions/velocities of an n-body Plummer sphere with G = M = a = 1
    (before the centre-of-mass shift)."""
    # radius: mass fraction X in (0, 0.999) -> r = (X^(-2/3) - 1)^(-1/2)
    x = rng.random(n) * 0.999
    x = np.where(x <= 0.0, 1e-300, x)
    r = 1.0 / np.sqrt(x ** (-2.0 / 3.0) - 1.0)
    pos = r[:, None] * _isotropic(rng, n)
    # speed ratio q in [0,1) with density ~ q^2 (1 - q^2)^(7/2); max < 0.1
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        q4 = rng.random(todo.size)
        q5 = rng.random(todo.size)
        ok = 0.1 * q5 < q4 * q4 * (1.0 - q4 * q4) ** 3.5
        q[todo[ok]] = q4[ok]
        todo = todo[~ok]
    vesc = np.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
    vel = (q * vesc)[:, None] * _isotropic(rng, n)
    return pos, vel


def _com_shift(pos, vel, mass):
    m = mass[:, None]
    mt = mass.sum()
    pos = pos - (m * pos).sum(0) / mt
    vel = vel - (m * vel).sum(0) / mt
    return pos, vel


def plummer(n: int, seed: int, a: float = 1.0, total_mass: float = 1.0) -> Bodies:
    """Equal-mass Plummer sphere of scale radius ``a`` and mass ``total_mass``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, vel = _plummer_unit(rng, n)
    mass = np.full(n, total_mass / n)
    pos, vel = _com_shift(pos, vel, mass)
    pos *= a
    vel *= np.sqrt(total_mass / a)
    return Bodies(pos, vel, mass, {"kind": "plummer", "n": n, "seed": seed, "a": a})


def two_spheres(n: int, seed: int, a1: float = 1.0, a2: float = 0.3,
                separation: float = 10.0, approach_speed: float = 0.5,
                sigma_ln_mass: float = 0.5) -> Bodies:
    """Two Plummer spheres of n/2 bodies each (scale radii a1, a2), each of
    total mass 1/2 with lognormal body masses, centres ``separation`` apart
    along (1,1,1)/sqrt(3) and approaching each other at ``approach_speed``
    with zero total momentum.  Velocities are drawn independently of mass."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n1 = n // 2
    n2 = n - n1
    u = np.ones(3) / np.sqrt(3.0)
    parts = []
    for nk, ak, sgn in ((n1, a1, -1.0), (n2, a2, 1.0)):
        p, v = _plummer_unit(rng, nk)
        m = np.exp(sigma_ln_mass * rng.standard_normal(nk))
        m *= 0.5 / m.sum()
        p, v = _com_shift(p, v, m)
        p = p * ak
        v = v * np.sqrt(0.5 / ak)
        p = p + sgn * 0.5 * separation * u
        v = v - sgn * 0.5 * approach_speed * u
        parts.append((p, v, m))
    pos = np.concatenate([parts[0][0], parts[1][0]])
    vel = np.concatenate([parts[0][1], parts[1][1]])
    mass = np.concatenate([parts[0][2], parts[1][2]])
    return Bodies(pos, vel, mass, {"kind": "two_spheres", "n": n, "seed": seed})


def two_clusters(n: int, seed: int, offset: float = 2.0) -> Bodies:
    """Two Plummer clusters (scale radius 1, mass 1/2 each, equal-mass
    bodies) centred at -offset (1, 1, 1) and +offset (1, 1, 1), each in its
    own equilibrium and at rest relative to the other, so that mutual
    gravity brings them together (Sec. 5's collision of two globular
    clusters).  The paper runs it in standard units, which needs the
    system's potential energy: apply that scaling (with the library or the
    oracle) before integrating."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n1 = n // 2
    parts = []
    for nk, sgn in ((n1, -1.0), (n - n1, 1.0)):
        p, v = _plummer_unit(rng, nk)
        m = np.full(nk, 1.0 / n)
        p, v = _com_shift(p, v, m)
        v = v * np.sqrt(0.5)  # virialised with the cluster's own mass 1/2
        parts.append((p + sgn * offset, v, m))
    pos = np.concatenate([parts[0][0], parts[1][0]])
    vel = np.concatenate([parts[0][1], parts[1][1]])
    mass = np.concatenate([parts[0][2], parts[1][2]])
    return Bodies(pos, vel, mass, {"kind": "two_clusters", "n": n, "seed": seed,
                                   "offset": offset})


def clumpy(n: int, seed: int, n_clumps: int = 4096, mean_radius: float = 0.05,
           sigma_ln_radius: float = 0.5, background_fraction: float = 0.1) -> Bodies:
    """Clumpy field: ``n_clumps`` Plummer clumps with lognormal scale radii
    (arithmetic mean ``mean_radius``) at uniform random centres in [0,1]^3,
    each virialised with its own mass, holding (1 - background_fraction) of
    the bodies split as evenly as possible; the rest uniform in [0,1]^3 at
    rest.  Equal masses 1/n."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_bg = int(round(background_fraction * n))
    n_cl = n - n_bg
    mu = np.log(mean_radius) - 0.5 * sigma_ln_radius ** 2
    radii = np.exp(mu + sigma_ln_radius * rng.standard_normal(n_clumps))
    centres = rng.random((n_clumps, 3))
    counts = np.full(n_clumps, n_cl // n_clumps)
    counts[: n_cl - counts.sum()] += 1
    mb = 1.0 / n
    pos = np.empty((n, 3))
    vel = np.zeros((n, 3))
    p_unit, v_unit = _plummer_unit(rng, n_cl)
    off = 0
    for c in range(n_clumps):
        k = int(counts[c])
        p = p_unit[off:off + k]
        v = v_unit[off:off + k]
        p = p - p.mean(0)
        v = v - v.mean(0)
        mc = k * mb
        pos[off:off + k] = centres[c] + radii[c] * p
        vel[off:off + k] = v * np.sqrt(mc / radii[c])
        off += k
    pos[n_cl:] = rng.random((n_bg, 3))
    mass = np.full(n, mb)
    return Bodies(pos, vel, mass, {"kind": "clumpy", "n": n, "seed": seed})


def subsample(n: int, k: int, seed: int) -> np.ndarray:
    """Seeded uniform sample of min(k, n) distinct body indices, sorted."""
    if k >= n:
        return np.arange(n, dtype=np.int64)
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


# The measured configurations.  theta/eps/leaf/dt/steps are the method's
# parameters; "dtype" is the walk's arithmetic type.
CONFIGS = {
    "c1": dict(workload="plummer", n=4096, seed=1, theta=0.5, eps=0.01, leaf=8,
               dtype="f64", dt=1e-3, steps=10),
    "c2": dict(workload="plummer", n=1 << 20, seed=2, theta=0.5, eps=0.005, leaf=16,
               dtype="f32", dt=5e-4, steps=100, sub_seed=102),
    "c3": dict(workload="two_spheres", n=1 << 24, seed=3, theta=0.6, eps=0.002, leaf=16,
               dtype="f32", dt=5e-4, steps=10, sub_seed=103),
    "c4": dict(workload="plummer", n=1 << 22, seed=4, theta=0.5, eps=0.005, leaf=16,
               dtype="f32", dt=5e-4, steps=10, sub_seed=104, mlp="bf16"),
    "c5": dict(workload="clumpy", n=1 << 26, seed=5, theta=0.7, eps=1e-4, leaf=16,
               dtype="f32", dt=1e-3, steps=10, sub_seed=105, mlp="fp16"),
}


def config(name: str, n: int | None = None) -> tuple[Bodies, dict]:
    """Bodies and parameters of a named configuration (optionally resized)."""
    cfg = dict(CONFIGS[name])
    if n is not None:
        cfg["n"] = int(n)
    gen = {"plummer": plummer, "two_spheres": two_spheres, "clumpy": clumpy}[cfg["workload"]]
    kw = {}
    if cfg["workload"] == "clumpy" and cfg["n"] < (1 << 20):
        kw["n_clumps"] = max(1, min(4096, cfg["n"] // 1024))
    b = gen(cfg["n"], cfg["seed"], **kw)
    if cfg["dtype"] == "f32":
        b = b.astype(np.float32)
    return b, cfg
