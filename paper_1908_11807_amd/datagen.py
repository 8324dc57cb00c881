"""Seeded synthetic inputs shaped like the ArborX paper's workloads.

This module holds no part of the search method: it only draws coordinates,
radii and request streams.  Both the HIP path and the CPU oracle consume its
arrays, so the two sides always see identical fp32 bytes.

Every generator draws with numpy's PCG64 (``numpy.random.default_rng(seed)``)
in float64 and rounds once to float32.

Workload recipes (paper section 3, "Experimental data sets"):

* uniform unit cube ``U[0,1)^3`` (the filled cube used by the benchmark
  configurations), and the paper's own four shapes with ``a = p**(1/3)`` and
  ``Omega = [-a, a]^3``: filled cube, hollow cube (faces taken cyclically),
  filled sphere (rejection from Omega) and hollow sphere (a cube point
  projected onto the sphere of radius ``a``);
* a thin spherical shell (radius uniform by volume in ``[R0, R1]``, direction
  a normalised Gaussian draw);
* Gaussian clusters (uniform centres plus isotropic normal offsets).

The radius rule follows the paper's choice of ``r`` such that a filled cube
gives ``k`` neighbours on average (section 3, data sets; ``k = 10``).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "uniform_cube", "shell", "clusters", "boxes_around",
    "paper_filled_cube", "paper_hollow_cube", "paper_filled_sphere",
    "paper_hollow_sphere", "radius_for_density", "radius_for_shell",
    "box_side_for_density", "forest_sizes", "request_stream", "CONFIGS",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def uniform_cube(n: int, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """``n`` points uniform in ``[lo, hi)^3``, float32 ``[n, 3]``."""
    r = _rng(seed)
    x = r.random((n, 3))
    return (lo + (hi - lo) * x).astype(np.float32)


def shell(n: int, seed: int, r0: float = 1.0 - 5e-4, r1: float = 1.0 + 5e-4) -> np.ndarray:
    """``n`` points uniform (by volume) in the shell ``r0 <= |x| <= r1``.

    Draw order: ``n x 3`` standard normals (direction), then ``n`` uniforms
    (radius, inverted through the ``R^2`` density).
    """
    r = _rng(seed)
    d = r.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    u = r.random(n)
    rad = np.cbrt(u * (r1 ** 3 - r0 ** 3) + r0 ** 3)
    return (d * rad[:, None]).astype(np.float32)


def clusters(n: int, seed: int, n_centres: int = 50, sigma: float = 0.02) -> np.ndarray:
    """Gaussian clusters: centres ``U[0,1)^3``, labels uniform, offsets ``N(0, sigma^2 I)``."""
    r = _rng(seed)
    c = r.random((n_centres, 3))
    lab = r.integers(0, n_centres, size=n)
    off = r.standard_normal((n, 3)) * sigma
    return (c[lab] + off).astype(np.float32)


def boxes_around(points: np.ndarray, seed: int, max_half: float) -> np.ndarray:
    """Axis-aligned boxes ``[p - h, p + h]`` with per-axis ``h ~ U[0, max_half)``.

    Returns float32 ``[n, 6]`` laid out ``lo x, lo y, lo z, hi x, hi y, hi z``.
    Corners are rounded from float64 once, so ``lo <= hi`` holds exactly.
    """
    r = _rng(seed)
    p = points.astype(np.float64)
    h = r.random(p.shape) * max_half
    lo = (p - h).astype(np.float32)
    hi = (p + h).astype(np.float32)
    return np.ascontiguousarray(np.concatenate([lo, hi], axis=1))


# -- the paper's four shapes (section 3, data sets) -------------------------

def paper_filled_cube(p: int, seed: int) -> np.ndarray:
    a = p ** (1.0 / 3.0)
    return (_rng(seed).random((p, 3)) * 2 * a - a).astype(np.float32)


def paper_hollow_cube(p: int, seed: int) -> np.ndarray:
    """Point ``i`` lies on face ``i mod 6`` of ``Omega``, uniform on that face."""
    a = p ** (1.0 / 3.0)
    r = _rng(seed)
    x = r.random((p, 3)) * 2 * a - a
    face = np.arange(p) % 6
    axis = face // 2
    sign = np.where(face % 2 == 0, -a, a)
    x[np.arange(p), axis] = sign
    return x.astype(np.float32)


def paper_filled_sphere(p: int, seed: int) -> np.ndarray:
    """Rejection sampling of ``Omega`` against the ball of radius ``a``."""
    a = p ** (1.0 / 3.0)
    r = _rng(seed)
    out = np.empty((0, 3))
    while out.shape[0] < p:
        x = r.random((2 * p, 3)) * 2 * a - a
        x = x[np.einsum("ij,ij->i", x, x) <= a * a]
        out = np.concatenate([out, x])
    return out[:p].astype(np.float32)


def paper_hollow_sphere(p: int, seed: int) -> np.ndarray:
    """``U[-1,1]^3`` points projected radially onto the sphere of radius ``a``."""
    a = p ** (1.0 / 3.0)
    x = _rng(seed).random((p, 3)) * 2 - 1
    nrm = np.linalg.norm(x, axis=1, keepdims=True)
    nrm[nrm == 0] = 1.0
    return (a * x / nrm).astype(np.float32)


# -- radius rules -------------------------------------------------------------

def radius_for_density(n: int, k: int = 10, volume: float = 1.0) -> float:
    """``r`` with ``k`` expected neighbours among ``n`` uniform points in ``volume``.

    Solves ``(n / volume) * (4/3) pi r^3 = k``.  Unit cube, n = 1e4 gives
    0.06203505; the paper's Omega (density 1/8) gives ``(6k/pi)^(1/3)``.
    """
    return (3.0 * k * volume / (4.0 * math.pi * n)) ** (1.0 / 3.0)


def radius_for_shell(n: int, thickness: float, k: int = 10) -> float:
    """``r`` with ``k`` expected neighbours for a query on a unit shell's mid-surface.

    A ball of radius ``r >= t/2`` centred in a slab of thickness ``t`` cuts
    volume ``pi (r^2 t - t^3/12)``; with density ``n / (4 pi t)`` that holds
    ``(n/4)(r^2 - t^2/12)`` points.
    """
    return math.sqrt(4.0 * k / n + thickness ** 2 / 12.0)


def box_side_for_density(n: int, k: int = 10, volume: float = 1.0) -> float:
    """Side ``s`` of a cube holding ``k`` expected points: ``(n/volume) s^3 = k``."""
    return (k * volume / n) ** (1.0 / 3.0)


# -- batched forest and serving streams ---------------------------------------

def forest_sizes(n_trees: int, seed: int, lo_exp: float = 3.0, hi_exp: float = 6.0) -> np.ndarray:
    """Tree sizes ``round(10**U(lo_exp, hi_exp))`` (log-uniform), int64."""
    e = _rng(seed).uniform(lo_exp, hi_exp, size=n_trees)
    return np.rint(10.0 ** e).astype(np.int64)


def forest_tree(t: int, size: int, base_seed: int = 401) -> tuple[np.ndarray, np.ndarray]:
    """Primitives and queries of tree ``t``: even ids uniform cube, odd ids clusters.

    Queries follow the tree's own distribution with the same count.  Seeds:
    primitives ``base_seed + t``, queries ``base_seed + t + 100000``.
    """
    gen = uniform_cube if t % 2 == 0 else clusters
    return gen(size, base_seed + t), gen(size, base_seed + t + 100000)


def forest_inputs(n_trees: int, seed: int = 401):
    """The forest workload: ``n_trees`` trees with sizes log-uniform in
    [1e3, 1e6]; even ids uniform cube, odd ids Gaussian clusters; each tree
    has as many queries as points, from its own distribution.  Returns
    (points, offsets, queries, query offsets), offsets int64 of length T+1."""
    sizes = forest_sizes(n_trees, seed)
    pts, qs = [], []
    for t, n in enumerate(sizes):
        p, q = forest_tree(t, int(n), seed)
        pts.append(p)
        qs.append(q)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return np.concatenate(pts), off, np.concatenate(qs), off.copy()


def request_stream(n_req: int, seed: int, rate_hz: float, n_trees: int,
                   lo_exp: float = 0.0, hi_exp: float = 5.0,
                   kinds=("radius", 1, 8, 32)):
    """Poisson request stream.

    Returns a list of dicts ``{t_arrival, tree, kind, m, seed}``: exponential
    inter-arrival gaps at ``rate_hz``, query counts ``floor(10**U(lo,hi))``,
    kind uniform over ``kinds`` (``"radius"`` or an int ``k``), tree uniform.
    """
    r = _rng(seed)
    gaps = r.exponential(1.0 / rate_hz, size=n_req)
    t = np.cumsum(gaps)
    m = np.maximum(1, np.floor(10.0 ** r.uniform(lo_exp, hi_exp, size=n_req))).astype(np.int64)
    kind = r.integers(0, len(kinds), size=n_req)
    tree = r.integers(0, n_trees, size=n_req)
    qseed = r.integers(0, 2 ** 31 - 1, size=n_req)
    return [dict(t_arrival=float(t[i]), tree=int(tree[i]), kind=kinds[kind[i]],
                 m=int(m[i]), seed=int(qseed[i])) for i in range(n_req)]


# -- the five benchmark configurations ----------------------------------------

CONFIGS = {
    "C1": dict(desc="1e4 uniform-cube points, 1e4 uniform-cube queries", n=10_000, m=10_000,
               prim_seed=101, query_seed=102, k=10,
               radius=float(np.float32(radius_for_density(10_000)))),
    "C2": dict(desc="1e6 uniform-cube points, 1e6 uniform-cube queries", n=1_000_000, m=1_000_000,
               prim_seed=201, query_seed=202, k=10,
               radius=float(np.float32(radius_for_density(1_000_000)))),
    "C3": dict(desc="1e7 points on a unit shell of thickness 1e-3, 1e7 queries uniform in [-1,1]^3",
               n=10_000_000, m=10_000_000, prim_seed=301, query_seed=302, k=10,
               radius=float(np.float32(radius_for_shell(10_000_000, 1e-3)))),
}


def config_inputs(name: str, n: int | None = None, m: int | None = None):
    """Primitives and queries of configuration ``name`` (C1-C3), optionally truncated sizes."""
    c = CONFIGS[name]
    n = c["n"] if n is None else n
    m = c["m"] if m is None else m
    if name == "C3":
        return shell(n, c["prim_seed"]), uniform_cube(m, c["query_seed"], -1.0, 1.0)
    return uniform_cube(n, c["prim_seed"]), uniform_cube(m, c["query_seed"])
