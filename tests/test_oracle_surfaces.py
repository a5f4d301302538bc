"""Pins of the oracle's smooth-surface measures (the extension closing
Section 5: a smooth surface known by an exact parametrisation, sampled on its
parameter domain) and of the library's own quadrature of the same surfaces
(independent code, compared on the CPU through a host test hook)."""
import ctypes as C
import math
import os

import numpy as np
import pytest
from scipy import special

from hsd_inputs import icosphere, random_rotation, rotate, ellipsoid_mesh, torus_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2304_06340_amd", "libhsd_testhooks.so")


def test_sphere_quadrature_matches_closed_form(orc):
    """Unit sphere as an ellipsoid a = b = c = 1: the sampled measure's
    transform against 4 pi sin r / r (eq. ft_nsphere_sinc) at random
    directions up to r = 60; spectral convergence makes 96 x 192 nodes exact
    to rounding."""
    pts, w = orc.surface_points("ellipsoid", 96, 192)
    assert math.fsum(w) == pytest.approx(4 * math.pi, rel=1e-14)
    rng = np.random.default_rng(0)
    n = rng.normal(size=(40, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    r = np.repeat([0.5, 5.0, 20.0, 60.0], 10)
    xi = n * r[:, None]
    got = orc.point_sum(pts, w, xi)
    ref = orc.nu_hat_sphere(r)
    assert np.max(np.abs(got - ref)) <= 5e-13 * 4 * math.pi


@pytest.mark.parametrize("a,c", [(1.0, 1.7), (1.3, 0.6), (2.0, 2.0)])
def test_spheroid_area(orc, a, c):
    _, w = orc.surface_points("ellipsoid", 48, 96, a, a, c)
    assert math.fsum(w) == pytest.approx(orc.spheroid_area(a, c), rel=1e-13)


def test_torus_area_and_axial_transform(orc):
    """Torus (R, r): area 4 pi^2 R r, and along the axis the transform is
    int e^{-ik r sin v} r (R + r cos v) du dv = 4 pi^2 R r J0(k r) (the cos v
    part integrates to zero)."""
    R, r = 2.0, 0.5
    pts, w = orc.surface_points("torus", 128, 64, R, r)
    assert math.fsum(w) == pytest.approx(4 * math.pi ** 2 * R * r, rel=1e-14)
    k = np.array([0.0, 1.0, 7.0, 25.0])
    got = orc.point_sum(pts, w, np.stack([0 * k, 0 * k, k], axis=1))
    ref = 4 * math.pi ** 2 * R * r * special.j0(k * r)
    assert np.max(np.abs(got - ref)) <= 1e-12 * 4 * math.pi ** 2 * R * r


def test_point_measure_target_reproduces_sphere_distance(orc):
    """The distance to the sampled sphere equals the distance to the
    closed-form sphere target (same mesh, same rule)."""
    spec = dict(r_max=24.0, n_panels=3, n_per_panel=8, n_cos=8, n_phi=16)
    rule = orc.spherical_product_rule(**spec)
    v, f = icosphere(2)
    pts = orc.surface_points("ellipsoid", 48, 96)
    d_closed = orc.distance(v, f, rule)
    d_points = orc.distance(v, f, rule, nu_points=pts)
    assert d_points == pytest.approx(d_closed, rel=1e-11)


def test_inputs_lie_on_their_surfaces():
    v, f = ellipsoid_mesh(2, 1.2, 0.8, 0.6)
    assert np.allclose((v[:, 0] / 1.2) ** 2 + (v[:, 1] / 0.8) ** 2 + (v[:, 2] / 0.6) ** 2, 1.0)
    v, f = torus_mesh(24, 12, 2.0, 0.5)
    rho = np.hypot(v[:, 0], v[:, 1])
    assert np.allclose((rho - 2.0) ** 2 + v[:, 2] ** 2, 0.25)
    assert len(f) == 2 * 24 * 12 and f.max() == len(v) - 1
    # closed surface: every edge is shared by exactly two triangles
    e = np.sort(np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]]), axis=1)
    _, counts = np.unique(e, axis=0, return_counts=True)
    assert np.all(counts == 2)


class _SurfaceDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_u", C.c_int32), ("n_v", C.c_int32), ("a", C.c_double),
                ("b", C.c_double), ("c", C.c_double), ("center", C.c_double * 3), ("reserved", C.c_int32 * 4)]


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhsd_testhooks.so not built")
@pytest.mark.parametrize("kind,args", [(0, (1.2, 0.8, 0.6)), (1, (2.0, 0.5, 0.0))])
def test_library_surface_quadrature_matches_oracle(orc, kind, args):
    """The library's C++ quadrature of its built-in surfaces (host test hook)
    against the oracle's independent construction (area element from the
    cross product of the partial derivatives)."""
    L = C.CDLL(LIB)
    f = L.hsd__host_surface_points
    f.argtypes = [C.POINTER(_SurfaceDesc), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    d = _SurfaceDesc()
    d.kind, d.n_u, d.n_v = kind, 24, 40
    d.a, d.b, d.c = args
    d.center[:] = [0.3, -0.2, 0.1]
    n = d.n_u * d.n_v
    pts = np.zeros((n, 3))
    w = np.zeros(n)
    assert f(C.byref(d), pts.ctypes.data_as(C.POINTER(C.c_double)), w.ctypes.data_as(C.POINTER(C.c_double))) == 0
    name = "ellipsoid" if kind == 0 else "torus"
    op, ow = orc.surface_points(name, 24, 40, *args, center=(0.3, -0.2, 0.1))
    assert np.max(np.abs(pts - op)) <= 1e-14 * 4
    assert np.max(np.abs(w - ow)) <= 1e-14 * np.max(ow) * 4


def test_ellipsoid_meshes_converge_quadratically(orc):
    """Section 5's programme on a surface other than S^2: inscribed
    icosahedral meshes of an ellipsoid against its exact measure; the
    distance falls by about 4 per subdivision as for the sphere (Section 4.2)."""
    rule = orc.spherical_product_rule(24.0, 3, 8, 8, 16)
    pts = orc.surface_points("ellipsoid", 48, 96, 1.2, 0.8, 0.6)
    d = [math.sqrt(orc.distance(*ellipsoid_mesh(L, 1.2, 0.8, 0.6), rule, nu_points=pts)) for L in (2, 3, 4)]
    ratios = [d[0] / d[1], d[1] / d[2]]
    assert 3.8 < ratios[0] < ratios[1] < 4.1
