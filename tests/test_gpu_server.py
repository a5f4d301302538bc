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
    """Every result of a mixed batch is bitwise the result of the same
    request served alone (one slot, nothing else submitted), and agrees with
    hsd_distance within the form's stated error (the server may split the
    triangles differently, to fill the device per chunk)."""
    rules = {"small": hsd.Rule.spherical_product(hsd_ctx, **SMALL),
             "large": hsd.Rule.spherical_product(hsd_ctx, **TINY)}
    trace = serving_trace(n=24, rate=200.0, seed=3, p_large=0.3, max_level=4)
    for form in ("fp64", "mixed"):
        p = hsd.Params(form=form)
        with hsd.Server(hsd_ctx, slots=4, chunk_pairs=50_000_000) as srv:
            tks = [(r, srv.submit(r.verts, r.tris, rules[r.rule], p, r.verts2, r.tris2)) for r in trace]
            res = [(r, srv.wait(t, 120.0)) for r, t in tks]
        with hsd.Server(hsd_ctx, slots=1, chunk_pairs=50_000_000) as srv:
            solo = [srv.wait(srv.submit(r.verts, r.tris, rules[r.rule], p, r.verts2, r.tris2), 120.0)
                    for r in trace]
        for (r, t), s in zip(res, solo):
            assert t.status == 0 and s.status == 0
            assert t.result.d2 == s.result.d2, (r.index, form, t.result.d2, s.result.d2)
            m1 = hsd.Mesh(hsd_ctx, r.verts, r.tris)
            m2 = hsd.Mesh(hsd_ctx, r.verts2, r.tris2) if r.verts2 is not None else None
            alone = hsd.distance(hsd_ctx, m1, m2, rules[r.rule], p)
            assert abs(t.result.d2 - alone.d2) <= alone.rel_err_stated * abs(alone.d2), (r.index, form)


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


def test_nufft_requests_under_a_tight_budget(hsd_ctx):
    """NUFFT3 requests through the serving loop: their footprint covers the
    whole transform plan (points, sort, spread tiles, spread and FFT grids),
    so a budget of 1.2 times the largest footprint runs them one at a time
    with the device bytes they leave behind within it, and every result
    equals the same request run alone."""
    rule = hsd.Rule.spherical_product(hsd_ctx, **SMALL)
    p = hsd.Params(method="nufft3", nufft_tol=1e-9)
    trace = serving_trace(n=5, rate=1000.0, seed=11, p_large=0.0, max_level=4)
    base = hsd_ctx.bytes_in_use()
    with hsd.Server(hsd_ctx, slots=1, chunk_pairs=10_000_000) as srv:
        probe = srv.wait(srv.submit(trace[0].verts, trace[0].tris, rule, p), 120.0)
        assert probe.status == 0
        kept = hsd_ctx.bytes_in_use() - base
        assert kept <= probe.footprint, (kept, probe.footprint)
    budget = None
    alone = []
    for r in trace:
        m1 = hsd.Mesh(hsd_ctx, r.verts, r.tris)
        m2 = hsd.Mesh(hsd_ctx, r.verts2, r.tris2) if r.verts2 is not None else None
        alone.append(hsd.distance(hsd_ctx, m1, m2, rule, p).d2)
    with hsd.Server(hsd_ctx, slots=4, chunk_pairs=10_000_000) as srv:
        fps = [srv.wait(srv.submit(r.verts, r.tris, rule, p, r.verts2, r.tris2), 120.0).footprint for r in trace]
    budget = int(max(fps) * 1.2)
    with hsd.Server(hsd_ctx, slots=4, budget_bytes=budget, chunk_pairs=10_000_000) as srv:
        tks = [srv.submit(r.verts, r.tris, rule, p, r.verts2, r.tris2) for r in trace]
        res = [srv.wait(t, 120.0) for t in tks]
    assert all(t.status == 0 for t in res), [t.error for t in res]
    assert [t.result.d2 for t in res] == alone
    order = sorted(res, key=lambda t: t.admitted_s)
    for a, b in zip(order[:-1], order[1:]):
        assert b.admitted_s >= a.finished_s - 1e-3 or a.footprint + b.footprint <= budget
    rule.close()
