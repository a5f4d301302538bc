"""Pins of the oracle's target, weights, rule and distance.

Closed forms of Sections 2.2 and 4.1, the icosahedral counts of Section 4.2,
exact symmetries of the product rule and the quadratic convergence the paper
observes for icosahedral meshes (Section 4.2, Fig. 3(b)).
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

from hsd_inputs import icosphere, icosphere_counts, random_rotation, rotate


def test_nu_hat_matches_bessel_form(orc):
    """4 pi sin r / r equals the Bessel form of eq. ft_nsphere,
    2 pi |eta|^-1/2 J_{1/2}(2 pi |eta|), at eta = xi / (2 pi)."""
    r = np.concatenate([np.linspace(1e-6, 1e-3, 7), np.linspace(0.01, 300.0, 501)])
    eta = r / (2.0 * math.pi)
    bessel = 2.0 * math.pi * eta ** -0.5 * special.jv(0.5, 2.0 * math.pi * eta)
    got = orc.nu_hat_sphere(r)
    assert np.max(np.abs(got - bessel)) <= 1e-13 * 4 * math.pi
    # spherical Bessel j0 form and the r -> 0 limit (surface area 4 pi)
    assert np.allclose(got, 4 * math.pi * special.spherical_jn(0, r), rtol=0, atol=1e-14)
    assert orc.nu_hat_sphere(np.array([0.0]))[0] == 4 * math.pi


@pytest.mark.parametrize("s", [-1.0, -1.5, -5.0, -10.0])
def test_paper_closed_form_sphere_norm(orc, s):
    """eq. sphere_sobolev_exact against the radial integral of
    g_s = (1+|eta|^2)^s |sigma^|^2 with sigma^ = 2 sin(2 pi|eta|)/|eta|
    (eq. ft_nsphere_sinc):  16 pi int_0^inf (1+r^2)^s sin^2(2 pi r) dr."""
    f = lambda r: 16.0 * math.pi * (1.0 + r * r) ** s * math.sin(2.0 * math.pi * r) ** 2
    val = 0.0
    edges = np.arange(0.0, 400.5, 0.5)
    for a, b in zip(edges[:-1], edges[1:]):
        val += integrate.quad(f, a, b, epsabs=1e-15, epsrel=1e-13)[0]
    tail_bound = 16.0 * math.pi * 400.0 ** (2 * s + 1) / (-2 * s - 1)
    exact = orc.sphere_norm_paper(s)
    assert abs(val - exact) <= 1e-10 * exact + tail_bound
    if s == -1.0:
        assert exact == pytest.approx(4 * math.pi ** 2 * (1 - math.exp(-4 * math.pi)), rel=1e-14)


def test_rule_weights_and_exactness(orc):
    for R, P, n, nc, nphi in [(64.0, 8, 16, 32, 64), (256.0, 16, 16, 8, 16), (10.0, 3, 5, 7, 9)]:
        rule = orc.spherical_product_rule(R, P, n, nc, nphi)
        assert len(rule) == P * n * nc * nphi
        assert math.fsum(rule.weights) == pytest.approx(4 * math.pi * R ** 3 / 3, rel=1e-13)
        # radial Gauss-Legendre panels integrate r^k exactly up to degree 2n-1-2
        for k in (0, 3, 2 * n - 3):
            got = math.fsum(rule.weights * rule.radii ** k)
            assert got == pytest.approx(4 * math.pi * R ** (k + 3) / (k + 3), rel=1e-12)
        # the angular part integrates z^2 exactly: int_S2 z^2 = 4 pi / 3
        z2 = math.fsum(rule.weights * rule.nodes[:, 2] ** 2 / np.maximum(rule.radii, 1e-300) ** 2)
        assert z2 == pytest.approx(4 * math.pi / 3 * R ** 3 / 3, rel=1e-12)


def test_cube_trapezoid_rule(orc):
    rule = orc.cube_trapezoid_rule(5.0, 8)
    assert len(rule) == 9 ** 3
    assert math.fsum(rule.weights) == pytest.approx(1000.0, rel=1e-14)
    # trapezoid is exact for functions linear in each coordinate
    f = (1 + rule.nodes[:, 0]) * (2 - rule.nodes[:, 1]) * (3 + 0.5 * rule.nodes[:, 2])
    assert math.fsum(rule.weights * f) == pytest.approx(1000.0 * 1 * 2 * 3, rel=1e-13)


def test_empty_mesh_distance_closed_form(orc):
    """With no triangles, d^2 = (2pi)^-3 sum W |nu^|^2 and the angular sum is
    exact: 8 sum_r w_r sin^2 r/(1+r^2); R -> inf gives 2 pi (1 - e^-2)."""
    rule = orc.spherical_product_rule(64.0, 8, 16, 32, 64)
    v = np.zeros((0, 3))
    t = np.zeros((0, 3), np.int32)
    d2 = orc.distance(v, t, rule, s=1.0)
    xg, wg = np.polynomial.legendre.leggauss(16)
    r = np.concatenate([8 * p + 4 * (xg + 1) for p in range(8)])
    wr = np.concatenate([4 * wg for _ in range(8)])
    closed = orc.empty_mesh_distance_radial(r, wr, 1.0)
    assert d2 == pytest.approx(closed, rel=1e-13)
    trunc = 8.0 * integrate.quad(lambda x: math.sin(x) ** 2 / (1 + x * x), 0, 64, limit=500,
                                 epsabs=1e-14, epsrel=1e-14)[0]
    assert d2 == pytest.approx(trunc, rel=1e-6)
    full = 2 * math.pi * (1 - math.exp(-2))
    assert abs(d2 - full) < 8.0 / 64.0  # the neglected tail is below 8/R


def test_icosphere_counts_and_geometry():
    """10*4^N+2 vertices, 20*4^N triangles (Section 4.2); vertices on S^2;
    closed surface (Euler characteristic 2, every edge shared by two faces)."""
    for level in range(5):
        v, f = icosphere(level)
        nv, nt = icosphere_counts(level)
        assert v.shape == (nv, 3) and f.shape == (nt, 3)
        assert np.allclose(np.linalg.norm(v, axis=1), 1.0, atol=1e-15)
        e = np.sort(np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]]), axis=1)
        ue, cnt = np.unique(e, axis=0, return_counts=True)
        assert np.all(cnt == 2)
        assert nv - len(ue) + nt == 2


def test_mesh_against_itself_and_symmetry(orc):
    rule = orc.spherical_product_rule(16.0, 2, 6, 8, 12)
    v, f = icosphere(1)
    assert orc.distance(v, f, rule, verts2=v, tris2=f) == 0.0
    rng = np.random.default_rng(3)
    v2 = rotate(v, random_rotation(rng)) * 1.01
    a = orc.distance(v, f, rule, verts2=v2, tris2=f)
    b = orc.distance(v2, f, rule, verts2=v, tris2=f)
    assert a > 0 and a == pytest.approx(b, rel=1e-13)


def test_rule_symmetries_leave_distance_unchanged(orc):
    """Rotation about z by 2 pi m / n_phi and the reflections z -> -z,
    y -> -y map the product rule onto itself, so d^2 is unchanged up to
    rounding."""
    rule = orc.spherical_product_rule(24.0, 3, 8, 12, 16)
    rng = np.random.default_rng(5)
    v, f = icosphere(2)
    v = rotate(v, random_rotation(rng)) * (1 + 0.01 * rng.normal(size=(len(v), 1)))
    base = orc.distance(v, f, rule)
    ang = 2 * math.pi * 3 / 16
    Rz = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0], [0, 0, 1]])
    for M in (Rz, np.diag([1.0, 1.0, -1.0]), np.diag([1.0, -1.0, 1.0])):
        assert orc.distance(v @ M.T, f, rule) == pytest.approx(base, rel=1e-11)


def test_quadratic_convergence_of_icosahedral_meshes(orc):
    """Section 4.2 / Fig. 3(b): the distance between T_N and S^2 falls like
    4^-N; ratios of d = sqrt(d^2) between consecutive levels approach 4."""
    rule = orc.spherical_product_rule(32.0, 4, 8, 16, 32)
    d = []
    for level in range(1, 5):
        v, f = icosphere(level)
        d.append(math.sqrt(orc.distance(v, f, rule)))
    ratios = [d[i] / d[i + 1] for i in range(len(d) - 1)]
    assert 3.0 < ratios[0] < 4.5
    assert 3.7 < ratios[1] < 4.3 and 3.85 < ratios[2] < 4.15, ratios


def test_paper_convention_trapezoid_reaches_closed_form(orc):
    """Paper convention (section 2.1: exp(-2 pi i eta.x), order -10): the
    empty-mesh distance is the sphere's own H_-10 norm, which the trapezoid
    rule on [-5, 5]^3 (eq. trap_rule_R3) approximates to about 1e-13 at
    M = 128 (section 4.1, Fig. 1(b)); eq. sphere_sobolev_exact gives it in
    closed form.  Nodes are xi = 2 pi eta and freq_unit = 2 pi."""
    exact = orc.sphere_norm_paper(-10.0)
    rule = orc.cube_trapezoid_rule(2 * math.pi * 5.0, 128)
    W = orc.sobolev_weights(rule, 10.0, 2 * math.pi)
    nu = orc.nu_hat_sphere(rule.radii)
    got = math.fsum((W * nu * nu).tolist())
    assert abs(got - exact) <= 1e-12 * exact
    # the same norm from a radial product rule on |eta| <= 5 (tail below 1e-14)
    sp = orc.spherical_product_rule(2 * math.pi * 5.0, 8, 16, 4, 4)
    W = orc.sobolev_weights(sp, 10.0, 2 * math.pi)
    nu = orc.nu_hat_sphere(sp.radii)
    assert abs(math.fsum((W * nu * nu).tolist()) - exact) <= 1e-12 * exact


def test_paper_convention_quadratic_convergence(orc):
    """Section 4.2, Fig. 3(b): relative H_-10 errors ||T_N - S^2|| / ||S^2||
    fall by about 4 per subdivision and reach the level of 1e-5 at N = 7
    (trapezoid rule, xi_max = 5).  Levels 0-2 on an M = 64 grid (whose own
    error is 1.4e-7 relative, far below these) must show the ratio rising
    towards 4, and extrapolating by 4^-5 from N = 2 must land at that level."""
    from hsd_inputs import icosphere
    exact = orc.sphere_norm_paper(-10.0)
    rule = orc.cube_trapezoid_rule(2 * math.pi * 5.0, 64)
    rel = []
    for level in (0, 1, 2):
        v, f = icosphere(level)
        rel.append(math.sqrt(orc.distance(v, f, rule, 10.0, freq_unit=2 * math.pi) / exact))
    r01, r12 = rel[0] / rel[1], rel[1] / rel[2]
    assert 3.0 < r01 < r12 < 4.2
    assert 5e-6 < rel[2] / 4 ** 5 < 5e-5
