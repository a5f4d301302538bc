"""Poisson request trace for the serving benchmark (inputs only).

512 requests drawn from ``numpy.random.default_rng(seed)`` (PCG64) in a fixed
draw order per request: inter-arrival gap ~ Exp(mean 1/rate); icosphere level
uniform in 1..6; mesh-vs-mesh with probability 0.3 (else against S^2); large
frequency rule with probability ``p_large``; per-vertex radial noise
N(0, (1e-3*h)^2) with h the mean edge length of the unperturbed mesh; a
uniformly random rotation.  A mesh-vs-mesh request draws its second mesh with
the same level/noise/rotation steps.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .meshes import icosphere, mean_edge_length, perturb_radial, random_rotation, rotate


@dataclass
class Request:
    index: int
    arrival: float
    level: int
    rule: str                     # "small" or "large"
    verts: np.ndarray
    tris: np.ndarray
    verts2: np.ndarray | None = None   # second mesh (mesh-vs-mesh) or None (vs S^2)
    tris2: np.ndarray | None = None
    level2: int | None = None
    meta: dict = field(default_factory=dict)


def _draw_mesh(rng: np.random.Generator, level: int):
    v, f = icosphere(level)
    h = mean_edge_length(v, f)
    v = perturb_radial(v, 1e-3 * h, rng)
    v = rotate(v, random_rotation(rng))
    return v, f


def serving_trace(n: int = 512, rate: float = 20.0, seed: int = 0,
                  p_large: float = 0.01, max_level: int = 6,
                  materialize: bool = True) -> list[Request]:
    rng = np.random.default_rng(seed)
    t = 0.0
    out: list[Request] = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        level = int(rng.integers(1, max_level + 1))
        mesh_vs_mesh = rng.random() < 0.3
        rule = "large" if rng.random() < p_large else "small"
        v, f = _draw_mesh(rng, level)
        req = Request(index=i, arrival=t, level=level, rule=rule, verts=v, tris=f)
        if mesh_vs_mesh:
            level2 = int(rng.integers(1, max_level + 1))
            v2, f2 = _draw_mesh(rng, level2)
            req.verts2, req.tris2, req.level2 = v2, f2, level2
        out.append(req)
    return out
