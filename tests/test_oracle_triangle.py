"""Pins of the oracle's exact triangle transform (eq. simplex32_ft).

Each check is independent of the oracle's own arithmetic: the triangle's
area at xi = 0, a 30-digit brute-force quadrature of the defining integral,
the paper's closed form evaluated at 50 digits, the normal-direction
invariance of eq. simplex32_ft_orth, and exact symmetries of the integral.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from hsd_inputs import random_triangles


def _area(v0, v1, v2):
    return 0.5 * np.linalg.norm(np.cross(v1 - v0, v2 - v0))


def brute_force(v0, v1, v2, xi, dps=30):
    """Definition: int_T exp(-i xi.x) dS = J int_{Q0} exp(-i xi.L(u)) du with
    L(u) = v0 + u1 e1 + u2 e2, J = |e1 x e2| (eq. change_variable), by an
    iterated Gauss-Legendre quadrature (mpmath.quad) at ``dps`` digits."""
    with mp.workdps(dps):
        V0 = [mp.mpf(float(x)) for x in v0]
        E1 = [mp.mpf(float(a)) - mp.mpf(float(b)) for a, b in zip(v1, v0)]
        E2 = [mp.mpf(float(a)) - mp.mpf(float(b)) for a, b in zip(v2, v0)]
        X = [mp.mpf(float(x)) for x in xi]
        cr = [E1[1] * E2[2] - E1[2] * E2[1], E1[2] * E2[0] - E1[0] * E2[2],
              E1[0] * E2[1] - E1[1] * E2[0]]
        J = mp.sqrt(sum(c * c for c in cr))
        t0 = sum(a * b for a, b in zip(X, V0))
        d1 = sum(a * b for a, b in zip(X, E1))
        d2 = sum(a * b for a, b in zip(X, E2))

        def inner(u1):
            return mp.quad(lambda u2: mp.expj(-(t0 + u1 * d1 + u2 * d2)), [0, 1 - u1])

        val = J * mp.quad(inner, [0, 1])
        return complex(val)


def paper_closed_form(v0, v1, v2, xi, dps=60):
    """Eq. simplex32_ft in the exp(-i xi.x) convention:
    -J sum_i exp(-i theta_i) / prod_{j != i} (theta_i - theta_j),
    theta_i = xi.p_i, evaluated at ``dps`` digits (exact for distinct
    theta when the working precision swamps the cancellation)."""
    with mp.workdps(dps):
        P = [[mp.mpf(float(x)) for x in v] for v in (v0, v1, v2)]
        X = [mp.mpf(float(x)) for x in xi]
        e1 = [P[1][c] - P[0][c] for c in range(3)]
        e2 = [P[2][c] - P[0][c] for c in range(3)]
        cr = [e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
              e1[0] * e2[1] - e1[1] * e2[0]]
        J = mp.sqrt(sum(c * c for c in cr))
        th = [sum(X[c] * P[i][c] for c in range(3)) for i in range(3)]
        tot = mp.mpc(0)
        for i in range(3):
            den = mp.mpf(1)
            for j in range(3):
                if j != i:
                    den *= th[i] - th[j]
            tot += mp.expj(-th[i]) / den
        return complex(-J * tot)


def test_transform_at_zero_is_area(orc):
    rng = np.random.default_rng(1)
    v, t = random_triangles(50, rng, scale=0.7)
    for tri in t:
        p = v[tri]
        val = orc.tri_ft(p[0], p[1], p[2], [0.0, 0.0, 0.0])
        assert abs(val.imag) == 0.0
        assert val.real == pytest.approx(_area(*p), rel=1e-15, abs=0)


@pytest.mark.parametrize("seed", range(6))
def test_against_brute_force_quadrature(orc, seed):
    rng = np.random.default_rng(100 + seed)
    v, _ = random_triangles(1, rng, scale=0.5)
    xi = rng.normal(size=3) * [0.5, 3.0, 8.0][seed % 3]
    ref = brute_force(v[0], v[1], v[2], xi)
    got = orc.tri_ft(v[0], v[1], v[2], xi)
    scale = _area(v[0], v[1], v[2])
    assert abs(got - ref) <= 1e-14 * scale


@pytest.mark.parametrize("case", ["generic", "small_gap_a", "small_gap_b", "both_small",
                                  "near_normal", "large_freq", "thin_triangle"])
def test_against_paper_closed_form(orc, case):
    rng = np.random.default_rng(hash(case) % 2 ** 32)
    v0 = rng.normal(size=3) * 0.3
    e1 = rng.normal(size=3) * 0.2
    e2 = rng.normal(size=3) * 0.2
    xi = rng.normal(size=3) * 20.0
    n = np.cross(e1, e2)
    n /= np.linalg.norm(n)
    if case == "small_gap_a":          # xi almost orthogonal to e1
        xi = xi - (xi @ e1) / (e1 @ e1) * e1 + 1e-9 * e1
    elif case == "small_gap_b":        # xi almost orthogonal to e2 - e1
        d = e2 - e1
        xi = xi - (xi @ d) / (d @ d) * d + 3e-7 * d
    elif case == "both_small":         # xi almost along the normal
        xi = 40.0 * n + 1e-5 * e1 + 2e-5 * e2
    elif case == "near_normal":
        xi = 7.0 * n + 0.3 * e1
    elif case == "large_freq":
        xi = xi * 12.0
    elif case == "thin_triangle":      # nearly degenerate triangle
        e2 = 0.5 * e1 + 1e-6 * rng.normal(size=3)
    v1, v2 = v0 + e1, v0 + e2
    ref = paper_closed_form(v0, v1, v2, xi, dps=80)
    got = orc.tri_ft(v0, v1, v2, xi)
    # J = |e1 x e2| is rounded relative to |e1||e2| (a thin triangle's area is
    # ill-conditioned in its vertices); the phases theta = xi.v are rounded
    # relative to |xi| -- those are the only FP64 errors left.
    scale = 0.5 * np.linalg.norm(e1) * np.linalg.norm(e2)
    tol = 4e-15 * max(1.0, np.linalg.norm(xi) * 1.5) * scale + 1e-300
    assert abs(got - ref) <= tol, (got, ref, abs(got - ref) / scale)


def test_normal_invariance_eq_simplex32_ft_orth(orc):
    """|mu_T(a n + xi_perp)| does not depend on a, and the phase is
    exp(-i a n.p0) (eq. simplex32_ft_orth)."""
    rng = np.random.default_rng(7)
    v, _ = random_triangles(5, rng, scale=0.4)
    for k in range(5):
        p = v[3 * k:3 * k + 3]
        n = np.cross(p[1] - p[0], p[2] - p[0])
        n /= np.linalg.norm(n)
        xp = rng.normal(size=3) * 6.0
        xp -= (xp @ n) * n
        base = orc.tri_ft(p[0], p[1], p[2], xp)
        for a in (-30.0, -1.0, 0.37, 5.0, 60.0):
            val = orc.tri_ft(p[0], p[1], p[2], xp + a * n)
            pred = np.exp(-1j * a * (n @ p[0])) * base
            assert abs(val - pred) <= 1e-13 * _area(*p)


def test_symmetries(orc):
    rng = np.random.default_rng(11)
    v, _ = random_triangles(8, rng, scale=0.5)
    for k in range(8):
        p = v[3 * k:3 * k + 3]
        xi = rng.normal(size=3) * 5.0
        A = _area(*p)
        val = orc.tri_ft(p[0], p[1], p[2], xi)
        # Hermitian symmetry of the transform of a real measure
        assert abs(orc.tri_ft(p[0], p[1], p[2], -xi) - np.conj(val)) <= 1e-14 * A
        # vertex order is irrelevant (Section 2.2)
        for perm in ((1, 2, 0), (2, 1, 0), (0, 2, 1)):
            q = p[list(perm)]
            assert abs(orc.tri_ft(q[0], q[1], q[2], xi) - val) <= 1e-14 * A
        # translation by b multiplies by exp(-i xi.b)
        b = rng.normal(size=3)
        q = p + b
        assert abs(orc.tri_ft(q[0], q[1], q[2], xi) - np.exp(-1j * xi @ b) * val) <= 1e-13 * A
        # dilation: mu_{lam T}(xi) = lam^2 mu_T(lam xi)
        lam = 1.7
        q = p * lam
        assert abs(orc.tri_ft(q[0], q[1], q[2], xi) - lam ** 2 * orc.tri_ft(p[0], p[1], p[2], lam * xi)) \
            <= 1e-13 * A * lam ** 2


def test_midpoint_subdivision_additivity(orc):
    """Linearity (Section 3.1): a flat triangle equals the sum of its four
    midpoint children."""
    rng = np.random.default_rng(12)
    for _ in range(10):
        p = rng.normal(size=(3, 3)) * 0.6
        xi = rng.normal(size=3) * 9.0
        a, b, c = p
        ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
        kids = [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        tot = sum(orc.tri_ft(*k, xi) for k in kids)
        assert abs(tot - orc.tri_ft(a, b, c, xi)) <= 1e-14 * max(1.0, _area(a, b, c))


def test_continuity_across_tau(orc):
    """The series branch and the closed branch agree where both are valid:
    the closed branch carries an absolute error of about eps/G, so it is
    compared only for G >= 1e-2 (the series is exact there to 1e-20)."""
    rng = np.random.default_rng(13)
    p = rng.normal(size=(3, 3)) * 0.2
    n = np.cross(p[1] - p[0], p[2] - p[0])
    n /= np.linalg.norm(n)
    A = _area(*p)
    for eps in (1e-4, 1e-3, 3e-3, 8e-3, 1.2e-2, 3e-2):
        xi = 50.0 * n + eps * rng.normal(size=3)
        vals = [orc.tri_ft(p[0], p[1], p[2], xi, tau=t) for t in (1e-2, 5e-2)]
        assert abs(vals[1] - vals[0]) <= 5e-14 * A


def test_transform_sums_triangles(orc):
    rng = np.random.default_rng(14)
    v, t = random_triangles(20, rng, scale=0.3)
    nodes = rng.normal(size=(7, 3)) * 4.0
    got = orc.transform(v, t, nodes)
    for k, xi in enumerate(nodes):
        ref = math.fsum(orc.tri_ft(*v[tri], xi).real for tri in t) + \
            1j * math.fsum(orc.tri_ft(*v[tri], xi).imag for tri in t)
        assert abs(got[k] - ref) <= 1e-15 * 20
