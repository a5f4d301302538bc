"""CPU run of the adjoint kernel's per-pair derivative math against the
oracle's dual-number derivative of the exact triangle transform."""
import ctypes as C
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2304_06340_amd", "libhsd_testhooks.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhsd_testhooks.so not built")
dp = C.POINTER(C.c_double)


def pair_grad_host(theta_mid, a, b, tau):
    L = C.CDLL(LIB)
    L.hsd__host_pair_grad.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp]
    out = np.zeros(8)
    L.hsd__host_pair_grad(theta_mid, a, b, tau, out.ctypes.data_as(dp))
    c = out[0::2] + 1j * out[1::2]
    return c[0], c[1], c[2], c[3]   # E, D_lo, D_mid, D_hi


def library_tri_grad(p, xi, tau=1e-2):
    """d mu_T / d v_j assembled from the kernel's pair math:
    a_j E J-part + J D_j xi (a_j = n x (v_{j+2} - v_{j+1}))."""
    e1, e2 = p[1] - p[0], p[2] - p[0]
    cr = np.cross(e1, e2)
    J = np.linalg.norm(cr)
    n = cr / J
    th = np.array([xi @ p[0], xi @ p[1], xi @ p[2]])
    s = np.array([0.0, xi @ e1, xi @ e2])
    order = np.argsort(s, kind="stable")
    lo, mid, hi = s[order]
    E, Dlo, Dmid, Dhi = pair_grad_host(xi @ p[0] + mid, mid - lo, hi - mid, tau)
    D = np.zeros(3, complex)
    D[order[0]], D[order[1]], D[order[2]] = Dlo, Dmid, Dhi
    g = np.zeros((3, 3), complex)
    for j in range(3):
        opp = p[(j + 2) % 3] - p[(j + 1) % 3]
        g[j] = np.cross(n, opp) * E + J * D[j] * xi
    return J * E, g


@pytest.mark.parametrize("case", ["generic", "small_gap", "near_normal", "tiny_xi", "large_xi"])
def test_pair_derivatives_match_oracle(orc, case):
    rng = np.random.default_rng(abs(hash(case)) % 2 ** 31)
    for _ in range(20):
        p = rng.normal(size=(3, 3)) * 0.3
        xi = rng.normal(size=3) * 5.0
        nrm = np.cross(p[1] - p[0], p[2] - p[0])
        nrm /= np.linalg.norm(nrm)
        if case == "small_gap":
            e1 = p[1] - p[0]
            xi = xi - (xi @ e1) / (e1 @ e1) * e1 + rng.uniform(0, 1e-3) * e1
        elif case == "near_normal":
            xi = 20 * nrm + rng.normal(size=3) * 1e-3
        elif case == "tiny_xi":
            xi = xi * 1e-4
        elif case == "large_xi":
            xi = xi * 40
        val, g = library_tri_grad(p, xi)
        ref_val, ref_g = orc.tri_ft_grad(p[0], p[1], p[2], xi)
        scale = 0.5 * np.linalg.norm(np.cross(p[1] - p[0], p[2] - p[0])) * (1 + np.linalg.norm(xi))
        assert abs(val - ref_val) <= 1e-12 * scale
        assert np.max(np.abs(g - ref_g)) <= 2e-11 * scale, (case, np.max(np.abs(g - ref_g)) / scale)


def test_series_branch_agrees_with_closed_branch():
    for a, b in [(0.004, 0.003), (0.02, 0.025), (0.0, 0.03), (0.03, 0.0)]:
        for tau_lo, tau_hi in [(1e-4, 0.05)]:
            x = pair_grad_host(0.7, a, b, tau_lo)     # closed branch
            y = pair_grad_host(0.7, a, b, tau_hi)     # series branch
            G = a + b
            for u, v in zip(x, y):
                assert abs(u - v) <= 1e-15 / G ** 2 + 1e-15


@pytest.mark.parametrize("P,n", [(3, 8), (4, 16), (2, 6)])
def test_sp_lane_matches_per_node_lane(P, n):
    """The adjoint's spherical-product lane body (phases by radial products,
    direct at panel 0's small radii, reciprocals by multiplication) against
    the per-node lane body on the same rule, residuals and weights, for
    generic and nearly flat (series-branch) triangles."""
    L = C.CDLL(LIB)
    f = L.hsd__host_adjoint_lane_sp
    f.argtypes = [dp, dp, dp, C.c_double, dp, C.c_int64, dp, C.c_int, C.c_int, C.c_double, dp, dp, dp, dp,
                  C.c_double, dp, dp]
    rng = np.random.default_rng(P * 100 + n)
    r_max = 20.0
    x, wx = np.polynomial.legendre.leggauss(n)
    h = r_max / P / 2
    radii = np.concatenate([(2 * p + 1) * h + h * x for p in range(P)])
    hx = np.ascontiguousarray(h * x[n // 2:])
    n_dir = 7
    dirs = rng.normal(size=(n_dir, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    resid = rng.normal(size=(n_dir * P * n, 2))
    wdir = rng.uniform(0.5, 1.5, n_dir)
    wtab = rng.uniform(0.1, 1.0, P * n)
    for scale in (0.3, 3e-4):
        p = rng.normal(size=(3, 3)) * scale
        e1, e2 = p[1] - p[0], p[2] - p[0]
        J = np.linalg.norm(np.cross(e1, e2))
        a_sp, a_ref = np.zeros(10), np.zeros(10)
        args = [np.ascontiguousarray(v) for v in (p[0], e1, e2)]
        f(*[a.ctypes.data_as(dp) for a in args], J, dirs.ctypes.data_as(dp), n_dir, radii.ctypes.data_as(dp),
          P, n, h, hx.ctypes.data_as(dp), resid.ctypes.data_as(dp), wdir.ctypes.data_as(dp),
          wtab.ctypes.data_as(dp), 0.05, a_sp.ctypes.data_as(dp), a_ref.ctypes.data_as(dp))
        scale_ref = np.max(np.abs(a_ref))
        # the library runs the adjoint with series threshold 0.05, where the
        # closed-branch derivatives lose ~eps / G^3 ~ 1e-12
        assert np.max(np.abs(a_sp - a_ref)) <= 1e-11 * scale_ref, (scale, a_sp, a_ref)
