"""Replay a request trace against the serving loop and summarise it.

Requests are submitted at their arrival times (a Poisson process in the
traces of hsd_inputs.serving_trace; time_scale 0 submits them all at once,
which saturates the server); latency is measured on the server's clock from
submit to result.  Reported: p50/p99 latency, completed distances per second
over the span from the first arrival to the last result, the fraction of
that span during which the device had at least one request admitted, the
offered load (the trace's work per second of arrivals over the server's
measured capacity, when that capacity is given) and a per-rule breakdown.
"""
from __future__ import annotations

import time

import numpy as np

from .api import Params, Rule, Server


def _busy_fraction(intervals, t0: float, t1: float) -> float:
    """Length of the union of [a, b) intervals within [t0, t1), over t1 - t0."""
    busy, end = 0.0, t0
    for a, b in sorted(intervals):
        a, b = max(a, end), min(b, t1)
        if b > a:
            busy += b - a
            end = b
    return busy / max(t1 - t0, 1e-12)


def replay(server: Server, trace, rules: dict[str, Rule], params: Params,
           time_scale: float = 1.0, capacity_pairs_per_s: float | None = None) -> dict:
    t_start = time.perf_counter()
    tickets = []
    for req in trace:
        due = t_start + req.arrival * time_scale
        now = time.perf_counter()
        if due > now:
            time.sleep(due - now)
        tk = server.submit(req.verts, req.tris, rules[req.rule], params, req.verts2, req.tris2,
                           tag=req.index)
        tickets.append((req, tk))
    out = []
    for req, tk in tickets:
        t = server.wait(tk, 600.0)
        out.append((req, t))
        server.release(tk)
    wall = time.perf_counter() - t_start
    lat = np.array([t.latency_s for _, t in out])
    ok = np.array([t.status == 0 for _, t in out])
    first = min(t.arrival_s for _, t in out)
    last_arrival = max(t.arrival_s for _, t in out)
    last = max(t.finished_s for _, t in out)
    pairs = float(sum(t.result.pairs for _, t in out))
    per_rule = {}
    for name in sorted(set(r.rule for r, _ in out)):
        ls = np.array([t.latency_s for r, t in out if r.rule == name])
        per_rule[name] = {"requests": int(len(ls)), "p50_ms": float(np.percentile(ls, 50) * 1e3),
                          "p99_ms": float(np.percentile(ls, 99) * 1e3)}
    res = {
        "requests": len(out),
        "failed": int((~ok).sum()),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "distances_per_s": float(ok.sum()) / (last - first),
        "pairs_per_s": pairs / (last - first),
        "span_s": last - first,
        "wall_s": wall,
        "pairs": pairs,
        "device_busy_frac": _busy_fraction([(t.admitted_s, t.finished_s) for _, t in out], first, last),
        "per_rule": per_rule,
        "results": {r.index: t.result.d2 for r, t in out},
    }
    if capacity_pairs_per_s and last_arrival > first:
        res["offered_load"] = pairs / (last_arrival - first) / capacity_pairs_per_s
    return res
