"""Triangulated test surfaces (inputs only; no transform arithmetic here).

The icosahedral discretisation follows the recursive construction of
Section 4.2 (icosahedral discretization): start from the regular icosahedron
inscribed in the unit sphere, split every face into four through its edge
midpoints, and push the new vertices radially onto the sphere.  Level ``N``
has ``10*4**N + 2`` vertices and ``20*4**N`` triangles.
"""
from __future__ import annotations

import numpy as np

GOLDEN = (1.0 + 5.0 ** 0.5) / 2.0


def icosphere_counts(level: int) -> tuple[int, int]:
    """(vertices, triangles) of the level-``level`` icosphere (Section 4.2)."""
    return 10 * 4 ** level + 2, 20 * 4 ** level


def icosahedron() -> tuple[np.ndarray, np.ndarray]:
    """Regular icosahedron on the unit sphere.

    Vertices are the cyclic permutations of (0, +-1, +-phi), normalised.
    Faces are the 20 vertex triples that are pairwise at the minimal edge
    distance, oriented so that the normal (v1-v0)x(v2-v0) points outward.
    """
    base = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            base.append((0.0, s1, s2 * GOLDEN))
    verts = []
    for shift in range(3):
        for p in base:
            verts.append(tuple(p[(i - shift) % 3] for i in range(3)))
    v = np.array(verts, dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    emin = d[d > 1e-12].min()
    adj = np.abs(d - emin) < 1e-9
    faces = []
    n = len(v)
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if adj[i, k] and adj[j, k]:
                    f = [i, j, k]
                    nrm = np.cross(v[j] - v[i], v[k] - v[i])
                    if np.dot(nrm, v[i] + v[j] + v[k]) < 0.0:
                        f = [i, k, j]
                    faces.append(f)
    f = np.array(faces, dtype=np.int32)
    assert f.shape == (20, 3)
    return v, f


def _subdivide(v: np.ndarray, f: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """One midpoint refinement; new vertices are projected onto the sphere."""
    verts = [tuple(x) for x in v]
    edge_mid: dict[tuple[int, int], int] = {}

    def mid(i: int, j: int) -> int:
        key = (i, j) if i < j else (j, i)
        idx = edge_mid.get(key)
        if idx is None:
            m = (v[i] + v[j]) * 0.5
            m = m / np.linalg.norm(m)
            idx = len(verts)
            verts.append(tuple(m))
            edge_mid[key] = idx
        return idx

    out = np.empty((4 * len(f), 3), dtype=np.int32)
    for t, (a, b, c) in enumerate(f):
        ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
        out[4 * t + 0] = (a, ab, ca)
        out[4 * t + 1] = (b, bc, ab)
        out[4 * t + 2] = (c, ca, bc)
        out[4 * t + 3] = (ab, bc, ca)
    return np.array(verts, dtype=np.float64), out


_CACHE: dict[int, tuple[np.ndarray, np.ndarray]] = {}


def icosphere(level: int) -> tuple[np.ndarray, np.ndarray]:
    """Level-``level`` icosahedral discretisation of S^2 (Section 4.2).

    Returns ``(verts[nv,3] float64, tris[nt,3] int32)``; copies, so callers
    may modify them.
    """
    if level < 0:
        raise ValueError("level must be >= 0")
    if level not in _CACHE:
        v, f = icosahedron() if level == 0 else icosphere(level - 1)
        if level > 0:
            v, f = _subdivide(v, f)
        _CACHE[level] = (v, f)
    v, f = _CACHE[level]
    return v.copy(), f.copy()


def mean_edge_length(verts: np.ndarray, tris: np.ndarray) -> float:
    """Mean length of the unique edges of a triangle mesh."""
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e = np.sort(e, axis=1)
    e = np.unique(e, axis=0)
    return float(np.linalg.norm(verts[e[:, 0]] - verts[e[:, 1]], axis=1).mean())


def perturb_radial(verts: np.ndarray, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """v <- v_hat * (1 + eta), eta ~ N(0, sigma^2) drawn per vertex."""
    eta = rng.normal(0.0, sigma, size=len(verts))
    vh = verts / np.linalg.norm(verts, axis=1, keepdims=True)
    return vh * (1.0 + eta)[:, None]


def perturb_harmonic(verts: np.ndarray, amp: float = 0.05) -> np.ndarray:
    """v <- v_hat * (1 + amp*sin(3*theta)*cos(2*phi)).

    theta is the polar angle from +z, phi = atan2(y, x).
    """
    vh = verts / np.linalg.norm(verts, axis=1, keepdims=True)
    theta = np.arccos(np.clip(vh[:, 2], -1.0, 1.0))
    phi = np.arctan2(vh[:, 1], vh[:, 0])
    return vh * (1.0 + amp * np.sin(3.0 * theta) * np.cos(2.0 * phi))[:, None]


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform rotation matrix from a normalised 4-D Gaussian quaternion."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def rotate(verts: np.ndarray, rot: np.ndarray) -> np.ndarray:
    return verts @ rot.T


def random_triangles(n: int, rng: np.random.Generator, scale: float = 1.0,
                     spread: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    """``n`` independent triangles: centre in a ball of radius ``spread``,
    vertex offsets of size ~``scale``.  Returns (verts[3n,3], tris[n,3])."""
    c = rng.uniform(-spread, spread, size=(n, 1, 3))
    off = rng.normal(0.0, scale, size=(n, 3, 3))
    v = (c + off).reshape(-1, 3)
    t = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    return v, t


def random_points(n: int, rng: np.random.Generator, rmax: float) -> np.ndarray:
    """``n`` points uniform in direction, radius uniform in [0, rmax]."""
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rng.uniform(0.0, rmax, size=(n, 1))
    return d * r


def ellipsoid_mesh(level: int, a: float, b: float, c: float) -> tuple[np.ndarray, np.ndarray]:
    """Level-N icosphere stretched to the ellipsoid x^2/a^2 + y^2/b^2 +
    z^2/c^2 = 1 (vertices on the surface; the inscribed polyhedron)."""
    v, f = icosphere(level)
    return v * np.array([a, b, c]), f


def torus_mesh(n_u: int, n_v: int, R: float, r: float) -> tuple[np.ndarray, np.ndarray]:
    """Triangulated torus ((R + r cos v) cos u, (R + r cos v) sin u, r sin v)
    on an n_u x n_v grid of the parameter square (vertices on the surface),
    two triangles per cell, consistently oriented."""
    u = 2.0 * np.pi * np.arange(n_u) / n_u
    w = 2.0 * np.pi * np.arange(n_v) / n_v
    U, W = np.meshgrid(u, w, indexing="ij")
    rho = R + r * np.cos(W)
    v = np.stack([rho * np.cos(U), rho * np.sin(U), r * np.sin(W)], axis=-1).reshape(-1, 3)
    i, j = np.meshgrid(np.arange(n_u), np.arange(n_v), indexing="ij")
    a = i * n_v + j
    b = ((i + 1) % n_u) * n_v + j
    c = ((i + 1) % n_u) * n_v + (j + 1) % n_v
    d = i * n_v + (j + 1) % n_v
    f = np.concatenate([np.stack([a, b, c], -1).reshape(-1, 3), np.stack([a, c, d], -1).reshape(-1, 3)])
    return v, f.astype(np.int32)
