"""CPU run of the HIP kernels' lane bodies against the oracle.

The direct-sum kernels are thin wrappers around __host__ __device__ lane
functions; libhsd exports a host-side driver of those functions (not part of
the public ABI) so their arithmetic is checked here, on the CPU, before any
GPU run.  The host pass differs from the device only in 1/x (IEEE division
instead of the hardware estimate plus Newton steps) and, for the mixed form,
in sin/cos of FP32 revolutions (libm instead of the transcendental unit).
"""
import ctypes as C
import os

import numpy as np
import pytest

from hsd_inputs import icosphere, perturb_radial, random_rotation, rotate, random_triangles

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2304_06340_amd", "libhsd_testhooks.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhsd_testhooks.so not built")

dp = C.POINTER(C.c_double)


def _lib():
    L = C.CDLL(LIB)
    L.hsd__host_transform_sp.argtypes = [dp, C.c_void_p, C.c_int64, dp, C.c_int64, dp, C.c_int, C.c_int,
                                         C.c_double, C.c_double, C.c_int, dp]
    L.hsd__host_transform_gen.argtypes = [dp, C.c_void_p, C.c_int64, dp, C.c_int64, C.c_double, C.c_int, dp]
    L.hsd__host_sincos64.argtypes = [dp, C.c_int64, dp, dp]
    L.hsd__host_sincos64_tab.argtypes = [dp, C.c_int64, dp, dp]
    fp = C.POINTER(C.c_float)
    L.hsd__host_sincos32.argtypes = [dp, C.c_int64, fp, fp]
    return L


def _p(a):
    return a.ctypes.data_as(dp)


def host_sp(v, f, spec, form=0, tau=1e-2):
    L = _lib()
    P, n, nc, nphi, R = spec["n_panels"], spec["n_per_panel"], spec["n_cos"], spec["n_phi"], spec["r_max"]
    x, _ = np.polynomial.legendre.leggauss(n)
    mu, _ = np.polynomial.legendre.leggauss(nc)
    phi = 2 * np.pi * np.arange(nphi) / nphi
    st = np.sqrt(1 - mu * mu)
    dirs = np.ascontiguousarray(np.stack([(st[:, None] * np.cos(phi)).ravel(),
                                          (st[:, None] * np.sin(phi)).ravel(),
                                          np.repeat(mu, nphi)], axis=1))
    h = R / P / 2
    hx = np.ascontiguousarray(h * x[n // 2:])
    v = np.ascontiguousarray(v, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.int32)
    out = np.zeros(2 * len(dirs) * P * n)
    L.hsd__host_transform_sp(_p(v), f.ctypes.data, len(f), _p(dirs), len(dirs), _p(hx), n, P, h, tau,
                             form, _p(out))
    return out[0::2] + 1j * out[1::2]


def host_gen(v, f, nodes, form=0, tau=1e-2):
    L = _lib()
    v = np.ascontiguousarray(v, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.int32)
    x = np.ascontiguousarray(nodes, dtype=np.float64)
    out = np.zeros(2 * len(x))
    L.hsd__host_transform_gen(_p(v), f.ctypes.data, len(f), _p(x), len(x), tau, form, _p(out))
    return out[0::2] + 1j * out[1::2]


def _area(v, f):
    return 0.5 * np.linalg.norm(np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]]), axis=1).sum()


def mu_tol(v, f, nodes, k=20.0, tau=1e-2, h=None):
    """Per-node bound for two FP64 evaluations of mu_h^: phase rounding
    (eps |xi| per vertex phase) plus the closed branch's eps/G error with
    G >= tau, each times the triangle's J = 2 area.

    h: half panel width of a spherical-product rule evaluated by the
    wave-per-direction kernel.  It forms the phase of node r = m -+ h x
    (panel centre m) as the product of exp(-i m c) and exp(-+i h x c): a
    half-gap sine then carries an absolute rounding proportional to the
    larger angle (m + h |x|) c rather than r c, so the closed branch's
    eps/(r G) term grows by rho = (m + h |x|) / r (1 above the panel centre,
    up to 188 at the smallest node of the first panel)."""
    eps = 1.1e-16
    A = _area(v, f)
    r = np.linalg.norm(nodes, axis=1)
    rho = 1.0
    if h is not None:
        m = (2.0 * np.floor(r / (2.0 * h)) + 1.0) * h
        rho = (m + np.abs(r - m)) / np.maximum(r, 1e-300)
    return k * eps * (1.0 + r) * A + 8.0 * eps * rho / tau * A


def test_sincos64_against_libm():
    L = _lib()
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-1, 1, 20000) * 10.0 ** rng.uniform(-8, 4, 20000),
                        np.arange(-50, 51) * np.pi / 4, [0.0, -0.0, 1e-300]])
    c = np.zeros_like(x)
    s = np.zeros_like(x)
    L.hsd__host_sincos64(_p(x), len(x), _p(c), _p(s))
    tol = 2.5e-16 + 1.2e-16 * np.abs(x) * 1e-16 * 16
    assert np.max(np.abs(c - np.cos(x)) - tol) <= 0
    assert np.max(np.abs(s - np.sin(x)) - tol) <= 0


def test_sincos64_tab_against_libm():
    """The pi/16-reduced FP64 sin/cos of the wave kernel's producer: ~1 ulp
    against libm over a wide range, and full relative accuracy for small
    angles (no table rotation there)."""
    L = _lib()
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-1, 1, 20000) * 10.0 ** rng.uniform(-8, 3.5, 20000),
                        np.arange(-64, 65) * np.pi / 16, [0.0, -0.0, 1e-300]])
    c = np.zeros_like(x)
    s = np.zeros_like(x)
    L.hsd__host_sincos64_tab(_p(x), len(x), _p(c), _p(s))
    tol = 3.5e-16 + 2.3e-16 * np.abs(x) * 1e-16 * 16
    assert np.max(np.abs(c - np.cos(x)) - tol) <= 0
    assert np.max(np.abs(s - np.sin(x)) - tol) <= 0
    small = np.abs(x) < np.pi / 32
    assert np.all(np.abs(s[small] - np.sin(x[small])) <= 3e-16 * np.abs(np.sin(x[small])))


def test_sincos32_unbiased():
    """The mixed form's FP32 sin/cos: within a few FP32 ulps, and without a
    systematic error along the exact phase (mean of the projection of
    computed - exact on e^{ix} below 2e-11 over 4e6 spread angles; a biased
    polynomial shows about -2e-10)."""
    L = _lib()
    rng = np.random.default_rng(2)
    x = rng.uniform(-60.0, 60.0, 4_000_000)
    c = np.zeros(len(x), np.float32)
    s = np.zeros(len(x), np.float32)
    fp = C.POINTER(C.c_float)
    L.hsd__host_sincos32(_p(x), len(x), c.ctypes.data_as(fp), s.ctypes.data_as(fp))
    ce, se = np.cos(x), np.sin(x)
    dc, ds = c.astype(np.float64) - ce, s.astype(np.float64) - se
    assert np.max(np.abs(dc) + np.abs(ds)) < 2.5e-7
    par = dc * ce + ds * se
    assert abs(par.mean()) < 2e-11 + 4 * par.std() / np.sqrt(len(x))


@pytest.mark.parametrize("spec", [
    dict(r_max=64.0, n_panels=8, n_per_panel=16, n_cos=4, n_phi=6),
    dict(r_max=20.0, n_panels=6, n_per_panel=6, n_cos=5, n_phi=7),
    dict(r_max=9.0, n_panels=3, n_per_panel=2, n_cos=3, n_phi=5),
])
@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("perturb", [True, False])
def test_sp_lane_matches_oracle(orc, spec, form, perturb):
    """perturb=False keeps the symmetric icosphere, whose edges are exactly
    orthogonal to some rule directions (zero phase gaps)."""
    rng = np.random.default_rng(5)
    v, f = icosphere(1)
    if perturb:
        v = rotate(perturb_radial(v, 0.01, rng), random_rotation(rng))
    got = host_sp(v, f, spec, form)
    o = orc.spherical_product_rule(**spec)
    ref = orc.transform(v, f, o.nodes)
    err = np.abs(got - ref)
    if form == 0:
        assert np.all(err <= mu_tol(v, f, o.nodes)), err.max()
    else:
        assert np.all(np.isfinite(got))
        assert err.max() <= 2e-5 * _area(v, f)


@pytest.mark.parametrize("form", [0, 1])
def test_gen_lane_matches_oracle(orc, form):
    rng = np.random.default_rng(8)
    v, f = random_triangles(30, rng, scale=0.3)
    v = np.concatenate([v, [[0.1, 0.2, 0.3], [0.1, 0.2, 0.3], [0.5, 0.0, 0.0]]])
    f = np.concatenate([f, [[90, 91, 92]]]).astype(np.int32)
    p = v[f[0]]
    nrm = np.cross(p[1] - p[0], p[2] - p[0])
    nrm /= np.linalg.norm(nrm)
    perp = np.cross(p[1] - p[0], nrm)
    nodes = np.array([nrm * 17.0, perp * 23.0, [1e-9, 2e-9, -1e-9], [0.0, 0.0, 0.0]]
                     + list(rng.normal(size=(200, 3)) * rng.choice([0.01, 1.0, 30.0, 200.0], size=(200, 1))))
    got = host_gen(v, f, nodes, form)
    ref = orc.transform(v, f, nodes)
    err = np.abs(got - ref)
    if form == 0:
        assert np.all(err <= mu_tol(v, f, nodes, 40.0)), err.max()
    else:
        assert err.max() <= 3e-6 * _area(v, f)


def host_wave(v, f, spec, form=0, tau=1e-2):
    L = _lib()
    L.hsd__host_transform_wave.argtypes = [dp, C.c_void_p, C.c_int64, dp, C.c_int64, dp, C.c_int,
                                           C.c_double, C.c_double, C.c_int, dp]
    P, n, nc, nphi, R = spec["n_panels"], spec["n_per_panel"], spec["n_cos"], spec["n_phi"], spec["r_max"]
    assert n == 16 and P % 8 == 0
    x, _ = np.polynomial.legendre.leggauss(n)
    mu, _ = np.polynomial.legendre.leggauss(nc)
    phi = 2 * np.pi * np.arange(nphi) / nphi
    st = np.sqrt(1 - mu * mu)
    dirs = np.ascontiguousarray(np.stack([(st[:, None] * np.cos(phi)).ravel(),
                                          (st[:, None] * np.sin(phi)).ravel(),
                                          np.repeat(mu, nphi)], axis=1))
    h = R / P / 2
    hx = np.ascontiguousarray(h * x[n // 2:])
    v = np.ascontiguousarray(v, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.int32)
    out = np.zeros(2 * len(dirs) * P * n)
    assert L.hsd__host_transform_wave(_p(v), f.ctypes.data, len(f), _p(dirs), len(dirs), _p(hx), P, h, tau,
                                      form, _p(out)) == 0
    return out[0::2] + 1j * out[1::2]


@pytest.mark.parametrize("spec", [
    dict(r_max=64.0, n_panels=8, n_per_panel=16, n_cos=3, n_phi=4),     # one panel per lane
    dict(r_max=96.0, n_panels=16, n_per_panel=16, n_cos=2, n_phi=3),    # two panels per lane
    dict(r_max=64.0, n_panels=32, n_per_panel=16, n_cos=2, n_phi=2),    # two waves per direction
])
@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("perturb", [True, False])
def test_wave_kernel_bodies_match_oracle(orc, spec, form, perturb):
    """Producer/consumer bodies of the wave-per-direction kernel, run on the
    CPU lane by lane, against the oracle at every rule node.  75 triangles:
    two full FP64 record blocks of 32 and a ragged one of 11 (batches of
    4, 4, 3); for the mixed form 9 batches of 8 and a ragged one of 3."""
    rng = np.random.default_rng(9)
    v, f = icosphere(1)
    if perturb:
        v = rotate(perturb_radial(v, 0.01, rng), random_rotation(rng))
    f = f[:75]       # ragged block and batch
    got = host_wave(v, f, spec, form)
    o = orc.spherical_product_rule(**spec)
    ref = orc.transform(v, f, o.nodes)
    err = np.abs(got - ref)
    if form == 0:
        h = spec["r_max"] / spec["n_panels"] / 2
        assert np.all(err <= mu_tol(v, f, o.nodes, h=h)), err.max()
    else:
        assert np.all(np.isfinite(got))
        assert err.max() <= 2e-5 * _area(v, f)


@pytest.mark.parametrize("tau", [0.005, 0.015, 0.05])
@pytest.mark.parametrize("n_panels", [8, 16])
def test_wave_fp64_series_slot_and_general_path(orc, tau, n_panels):
    """FP64 wave bodies where the series branch is taken: level-3 triangles
    (G about 0.1-0.2) against a rule whose first panel reaches down to
    r = 0.0106 h, so that the smallest-radius slot of the first panel
    group takes the series value its producer lane stored, and directions
    near a face normal (small G) send whole triangles through the path that
    compares every slot.  Elementwise against the oracle; thresholds on
    both sides of the r^5 / r^7 switch."""
    rng = np.random.default_rng(21)
    v, f = icosphere(3)
    v = rotate(v, random_rotation(rng))
    f = f[rng.choice(len(f), 70, replace=False)]
    spec = dict(r_max=2.0 * n_panels, n_panels=n_panels, n_per_panel=16, n_cos=4, n_phi=5)
    got = host_wave(v, f, spec, 0, tau=tau)
    o = orc.spherical_product_rule(**spec)
    ref = orc.transform(v, f, o.nodes, tau=tau)
    err = np.abs(got - ref)
    assert np.all(err <= mu_tol(v, f, o.nodes, tau=tau, h=1.0)), err.max()


@pytest.mark.parametrize("level", [0, 1, 2])
@pytest.mark.parametrize("spec", [
    dict(r_max=16.0, n_panels=8, n_per_panel=16, n_cos=3, n_phi=4),
    dict(r_max=64.0, n_panels=8, n_per_panel=16, n_cos=3, n_phi=5),
    dict(r_max=256.0, n_panels=16, n_per_panel=16, n_cos=2, n_phi=3),
])
def test_wave_kernel_small_radius_nodes(orc, level, spec):
    """FP64 wave-kernel bodies on coarse meshes (edges up to 1.05), where the
    nodes below the first panel centre take the closed branch near its
    threshold r G = tau: every node within the per-node bound, and the
    nodes at r >= h (rho <= 2 there) within the bound for directly
    evaluated phases (rho = 1)."""
    rng = np.random.default_rng(level)
    v, f = icosphere(level)
    v = rotate(perturb_radial(v, 0.05, rng), random_rotation(rng))
    got = host_wave(v, f, spec, 0)
    o = orc.spherical_product_rule(**spec)
    ref = orc.transform(v, f, o.nodes)
    err = np.abs(got - ref)
    h = spec["r_max"] / spec["n_panels"] / 2
    r = np.linalg.norm(o.nodes, axis=1)
    assert np.all(err <= mu_tol(v, f, o.nodes, h=h)), err.max()
    assert np.all(err[r >= h] <= mu_tol(v, f, o.nodes[r >= h])), err[r >= h].max()
