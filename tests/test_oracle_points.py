"""Pins of the point-cloud model (Section 3.1) and its direct exponential sum."""
import math

import numpy as np
import pytest

from hsd_inputs import icosphere, random_triangles


def _monomial_exact(a, b):
    # int over the standard triangle of u^a v^b = a! b! / (a+b+2)!
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


@pytest.mark.parametrize("rule,deg_ok,deg_bad", [("dunavant7", 5, 6), ("gl8x8", 14, None)])
def test_triangle_rule_exactness(orc, rule, deg_ok, deg_bad):
    bary, w = orc.dunavant7() if rule == "dunavant7" else orc.gl_collapsed_rule(8)
    assert math.fsum(w) == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(bary.sum(axis=1), 1.0, atol=1e-15)
    u, v = bary[:, 1], bary[:, 2]
    for a in range(deg_ok + 1):
        for b in range(deg_ok + 1 - a):
            got = 0.5 * math.fsum(w * u ** a * v ** b)     # area of Q0 is 1/2
            assert got == pytest.approx(_monomial_exact(a, b), rel=2e-14, abs=1e-17)
    if deg_bad is not None:
        errs = [abs(0.5 * math.fsum(w * u ** a * v ** (deg_bad - a)) - _monomial_exact(a, deg_bad - a))
                for a in range(deg_bad + 1)]
        assert max(errs) > 1e-6


def test_point_sum_direct(orc):
    rng = np.random.default_rng(21)
    x = rng.normal(size=(40, 3))
    c = rng.normal(size=40)
    nodes = rng.normal(size=(9, 3)) * 6
    got = orc.point_sum(x, c, nodes)
    ref = np.array([np.sum(c * np.exp(-1j * (x @ k))) for k in nodes])
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.sum(np.abs(c))


def test_point_cloud_converges_to_exact_transform(orc):
    """The Dirac cloud of a triangle rule reproduces the exact transform when
    the phase span per triangle is small (eq. change_variable_approx)."""
    v, f = icosphere(3)
    rng = np.random.default_rng(22)
    nodes = rng.normal(size=(16, 3))
    nodes *= (4.0 / np.linalg.norm(nodes, axis=1))[:, None]
    exact = orc.transform(v, f, nodes)
    for rule, tol in (("dunavant7", 1e-8), ("gl8x8", 1e-13)):
        p, c = orc.point_cloud(v, f, rule)
        assert len(p) == len(f) * (7 if rule == "dunavant7" else 64)
        approx = orc.point_sum(p, c, nodes)
        assert np.max(np.abs(approx - exact)) <= tol * 4 * math.pi, rule
