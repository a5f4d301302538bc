"""Pins of the oracle's gradient (dual numbers through the exact transform).

Independent checks: high-precision finite differences of the paper's closed
form (eq. simplex32_ft at 80 digits), the translation identity
sum_j d mu_T / d v_j = -i xi mu_T, and central differences of the oracle's
own distance.
"""
import mpmath as mp
import numpy as np
import pytest

from hsd_inputs import icosphere, perturb_harmonic
from test_oracle_triangle import paper_closed_form


@pytest.mark.parametrize("case", ["generic", "near_edge_orth", "near_normal"])
def test_triangle_gradient_vs_high_precision_fd(orc, case):
    rng = np.random.default_rng(len(case))
    p = rng.normal(size=(3, 3)) * 0.3
    xi = rng.normal(size=3) * 6.0
    if case == "near_edge_orth":
        e1 = p[1] - p[0]
        xi = xi - (xi @ e1) / (e1 @ e1) * e1 + 1e-7 * e1
    elif case == "near_normal":
        n = np.cross(p[1] - p[0], p[2] - p[0])
        xi = 30.0 * n / np.linalg.norm(n) + 1e-4 * (p[1] - p[0])
    val, g = orc.tri_ft_grad(p[0], p[1], p[2], xi)
    h = 1e-20
    with mp.workdps(80):
        for j in range(3):
            for c in range(3):
                pp, pm = p.copy(), p.copy()
                # FD on the exact closed form at 80 digits: perturbations are
                # exact in mpmath (passed as mpf through float offsets of 0)
                def f(sgn):
                    P = [[mp.mpf(float(x)) for x in row] for row in p]
                    P[j][c] += sgn * mp.mpf(h)
                    X = [mp.mpf(float(x)) for x in xi]
                    e1 = [P[1][k] - P[0][k] for k in range(3)]
                    e2 = [P[2][k] - P[0][k] for k in range(3)]
                    cr = [e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                          e1[0] * e2[1] - e1[1] * e2[0]]
                    J = mp.sqrt(sum(x * x for x in cr))
                    th = [sum(X[k] * P[i][k] for k in range(3)) for i in range(3)]
                    tot = mp.mpc(0)
                    for i in range(3):
                        den = mp.mpf(1)
                        for jj in range(3):
                            if jj != i:
                                den *= th[i] - th[jj]
                        tot += mp.expj(-th[i]) / den
                    return -J * tot
                d = complex((f(1) - f(-1)) / (2 * mp.mpf(h)))
                scale = np.linalg.norm(xi) * 0.3 + 1.0
                assert abs(g[j, c] - d) <= 1e-12 * scale, (j, c, g[j, c], d)


def test_translation_identity(orc):
    rng = np.random.default_rng(31)
    for _ in range(20):
        p = rng.normal(size=(3, 3)) * 0.5
        xi = rng.normal(size=3) * rng.choice([0.01, 1.0, 30.0])
        val, g = orc.tri_ft_grad(p[0], p[1], p[2], xi)
        lhs = g.sum(axis=0)
        rhs = -1j * xi * val
        assert np.max(np.abs(lhs - rhs)) <= 1e-12 * (1 + np.linalg.norm(xi))


def test_distance_gradient_vs_central_differences(orc):
    rule = orc.spherical_product_rule(12.0, 2, 6, 8, 10)
    v, f = icosphere(1)
    v = perturb_harmonic(v, 0.05)
    d2, g = orc.gradient(v, f, rule)
    rng = np.random.default_rng(33)
    h = 1e-6
    for _ in range(8):
        i, c = int(rng.integers(len(v))), int(rng.integers(3))
        vp, vm = v.copy(), v.copy()
        vp[i, c] += h
        vm[i, c] -= h
        fd = (orc.distance(vp, f, rule) - orc.distance(vm, f, rule)) / (2 * h)
        assert g[i, c] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(g).max())
    # d^2 of a closed mesh vs S^2 is not translation invariant, but mesh vs a
    # rigidly moved copy of itself is: the two gradient sums cancel.
    w = v + np.array([0.01, -0.02, 0.005])
    _, g1 = orc.gradient(v, f, rule, verts2=w, tris2=f)
    _, g2 = orc.gradient(w, f, rule, verts2=v, tris2=f)
    tot = g1.sum(axis=0) + g2.sum(axis=0)
    assert np.max(np.abs(tot)) <= 1e-10 * np.abs(g1).max()
