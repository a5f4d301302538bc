"""GPU tests of the serving loop: every result of a mixed batch is bitwise
equal to the same request run alone through hsd_distance; cancellation and
a tight memory budget behave."""
import numpy as np
import pytest

import paper_2304_06340_amd as hsd
from hsd_inputs import serving_trace

pytestmark = pytest.mark.gpu

SMALL = dict(r_max=64.0, n_panels=8, n_per_panel=16, n_cos=32, n_phi=64)
TINY = dict(r_max=16.0, n_panels=2, n_per_panel=8, n_cos=8, n_phi=16)


def test_results_alone_equal_results_in_the_mix(hsd_ctx):
    rules = {"small": hsd.Rule.spherical_product(hsd_ctx, **SMALL),
             "large": hsd.Rule.spherical_product(hsd_ctx, **TINY)}
    trace = serving_trace(n=24, rate=200.0, seed=3, p_large=0.3, max_level=4)
    for form in ("fp64", "mixed"):
        p = hsd.Params(form=form)
        with hsd.Server(hsd_ctx, slots=4, chunk_pairs=50_000_000) as srv:
            tks = [(r, srv.submit(r.verts, r.tris, rules[r.rule], p, r.verts2, r.tris2)) for r in trace]
            res = [(r, srv.wait(t, 120.0)) for r, t in tks]
        for r, t in res:
            assert t.status == 0
            m1 = hsd.Mesh(hsd_ctx, r.verts, r.tris)
            m2 = hsd.Mesh(hsd_ctx, r.verts2, r.tris2) if r.verts2 is not None else None
            alone = hsd.distance(hsd_ctx, m1, m2, rules[r.rule], p)
            assert t.result.d2 == alone.d2, (r.index, form, t.result.d2, alone.d2)


def test_cancel_and_tight_budget(hsd_ctx):
    rule = hsd.Rule.spherical_product(hsd_ctx, **SMALL)
    trace = serving_trace(n=6, rate=1000.0, seed=5, p_large=0.0, max_level=5)
    with hsd.Server(hsd_ctx, slots=2, chunk_pairs=10_000_000) as srv:
        tks = [srv.submit(r.verts, r.tris, rule) for r in trace]
        srv.cancel(tks[0])
        res = [srv.wait(t, 120.0) for t in tks]
        assert res[0].status in (0, -5)
        assert all(r.status == 0 for r in res[1:])
    # a budget that admits one request at a time: results unchanged
    fp = max(r.footprint for r in res[1:])
    with hsd.Server(hsd_ctx, slots=4, budget_bytes=int(fp * 1.2), chunk_pairs=10_000_000) as srv:
        tks = [srv.submit(r.verts, r.tris, rule) for r in trace[1:]]
        res2 = [srv.wait(t, 120.0) for t in tks]
    assert [a.result.d2 for a in res2] == [b.result.d2 for b in res[1:]]
    for a, b in zip(res2[:-1], res2[1:]):
        assert b.admitted_s >= a.finished_s - 1e-3 or b.footprint + a.footprint <= fp * 1.2
