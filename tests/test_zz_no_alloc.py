"""hsd_distance_noalloc (the entry point that allocates no device memory)
against hsd_distance, through the C ABI: FP64 parity bar 1e-10 relative in
d^2 (the two differ only in the device-built weight tables and, where the
fixed scratch array is too small for hsd_distance's split count, in the
split order).  Two calls in a row, the second on a smaller input, then the
first again; the empty surface; a rule too large for the array is refused
before anything is launched."""
import numpy as np
import pytest

import paper_2304_06340_amd as hsd
from hsd_inputs import icosphere, perturb_radial, random_rotation, rotate

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return abs(a - b) / abs(b)


def test_noalloc_matches_distance_on_two_calls(hsd_ctx):
    rng = np.random.default_rng(21)
    v3, f3 = icosphere(3)
    v3 = rotate(perturb_radial(v3, 1e-3, rng), random_rotation(rng))
    v2, f2 = icosphere(2)
    v1, f1 = icosphere(1)
    big_mesh = hsd.Mesh(hsd_ctx, v3, f3)
    small_mesh = hsd.Mesh(hsd_ctx, v2, f2)
    other = hsd.Mesh(hsd_ctx, v1, f1)
    big_rule = hsd.Rule.spherical_product(hsd_ctx, 64.0, 8, 16, 32, 64)        # 262,144 nodes
    nodes = rng.normal(size=(3000, 3)) * rng.choice([0.5, 4.0, 20.0], size=(3000, 1))
    small_rule = hsd.Rule.explicit(hsd_ctx, nodes, rng.uniform(0.1, 1.0, 3000))
    cases = [
        ("level 3 vs S^2, 262,144-node rule, FP64", big_mesh, None, big_rule, hsd.Params(s=1.0)),
        ("level 2 vs level 1, 3,000 explicit nodes, FP64", small_mesh, other, small_rule, hsd.Params(s=1.5)),
        ("level 3 vs S^2, 262,144-node rule, FP64 again", big_mesh, None, big_rule, hsd.Params(s=1.0)),
        ("level 2 vs S^2, 262,144-node rule, mixed", small_mesh, None, big_rule, hsd.Params(form="mixed")),
    ]
    for name, mu, nu, rule, p in cases:
        ref = hsd.distance(hsd_ctx, mu, nu, rule, p)
        got = hsd.distance_noalloc(hsd_ctx, mu, nu, rule, p)
        print(f"{name}: d2 {got.d2!r} vs {ref.d2!r}, rel {_rel(got.d2, ref.d2):.2e}", flush=True)
        assert got.pairs == ref.pairs
        assert _rel(got.d2, ref.d2) <= 1e-10
    for m in (big_mesh, small_mesh, other):
        m.close()
    big_rule.close()
    small_rule.close()


def test_noalloc_empty_surface_and_oversized_rule(hsd_ctx):
    empty = hsd.Mesh(hsd_ctx, np.zeros((0, 3)), np.zeros((0, 3), np.int32))
    rule = hsd.Rule.spherical_product(hsd_ctx, 64.0, 8, 16, 32, 64)
    ref = hsd.distance(hsd_ctx, empty, None, rule, hsd.Params())
    got = hsd.distance_noalloc(hsd_ctx, empty, None, rule, hsd.Params())
    print(f"empty surface: {got.d2!r} vs {ref.d2!r}", flush=True)
    assert _rel(got.d2, ref.d2) <= 1e-12
    # 128 panels x 16 x 128 x 256 = 67,108,864 nodes: 1 GiB of partials
    huge = hsd.Rule.spherical_product(hsd_ctx, 256.0, 128, 16, 128, 256)
    with pytest.raises(hsd.HsdError, match="no-allocation"):
        hsd.distance_noalloc(hsd_ctx, empty, None, huge, hsd.Params())
    with pytest.raises(hsd.HsdError, match="direct method"):
        hsd.distance_noalloc(hsd_ctx, empty, None, rule, hsd.Params(method="nufft3"))
    huge.close()
    rule.close()
    empty.close()
