"""Benchmark: tri*freq pair evaluations per second of the direct-sum H^-s
distance on one MI355X, FP64 form (value) and mixed form, with the error of
each against the FP64 reference, the roofline of the dominant kernel and the
CPU oracle timed on a bounded sample.

Default workload (the large configuration, stated factors): level-7
icosphere (327,680 triangles) against the unit sphere S^2, spherical product
rule with 16 radial Gauss-Legendre panels x 16 nodes on [0, 256], 128
Gauss-Legendre nodes in cos(theta), 256 trapezoid nodes in phi (8,388,608
nodes), s = 1.  One step = one complete hsd_distance call (direct sum over all
2.75e12 triangle-node pairs, residual against 4 pi sin r / r, Sobolev
weights, two-level reduction, 8-byte readback), with the mesh and the rule
already resident in HBM.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (level, rule spec, description)
    "level7-large-rule": (7, dict(r_max=256.0, n_panels=16, n_per_panel=16, n_cos=128, n_phi=256),
                          "level-7 icosphere (327,680 tri) vs S^2; rule r<=256: 16 GL panels x 16 "
                          "radial x 128 GL cos(theta) x 256 phi = 8,388,608 nodes; s=1"),
    "level7-large-rule-128panels": (7, dict(r_max=256.0, n_panels=128, n_per_panel=16, n_cos=128, n_phi=256),
                                    "level-7 icosphere vs S^2; rule r<=256: 128 GL panels x 16 radial "
                                    "x 128 x 256 = 67,108,864 nodes; s=1"),
    "level2-small-rule": (2, dict(r_max=64.0, n_panels=8, n_per_panel=16, n_cos=32, n_phi=64),
                          "level-2 icosphere (320 tri) vs S^2; rule r<=64: 8 GL panels x 16 radial "
                          "x 32 x 64 = 262,144 nodes; s=1"),
    "level7-small-rule": (7, dict(r_max=64.0, n_panels=8, n_per_panel=16, n_cos=32, n_phi=64),
                          "level-7 icosphere vs S^2; rule r<=64: 262,144 nodes; s=1"),
}

FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector (256 CU x 2.4 GHz x 128 FLOP/clk)
FP32_PEAK_TFLOPS = 157.3    # MI355X FP32 vector (256 CU x 2.4 GHz x 256 FLOP/clk)

# Sources whose compiled code is the FP64 direct-sum kernel (with the triangle
# record's layout from the internal header); their hash stamps the HBM
# traffic measured for it below.
KERNEL_SOURCES = ("paper_2304_06340_amd/csrc/hsd_direct_wave.hip", "paper_2304_06340_amd/csrc/hsd_math.hpp")
TRIREC_HEADER = "paper_2304_06340_amd/csrc/hsd_internal.hpp"

# HBM bytes per launch of k_direct_wave<2, true> (FP64) from rocprofv3:
# FETCH_SIZE x 2.00 + WRITE_SIZE x 1.00, the factors read off a 1 GiB device
# copy in the same runs (profiles/k_direct_wave_fp64_level7_large_rule.md),
# with the hash of KERNEL_SOURCES when they were taken.  A kernel whose
# sources hash differently reports traffic null: the counters no longer
# describe it.
MEASURED_TRAFFIC = {"level7-large-rule": (7.0089e9, "983bd74a62007f99")}


def kernel_revision() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, TRIREC_HEADER)) as fh:
        text = fh.read()
    i = text.index("struct TriRec {")
    h.update(text[i:text.index("};", i)].encode())
    return h.hexdigest()[:16]


def flops_per_pair(spec, form="fp64") -> float:
    """Algorithmic FLOPs (FMA = 2) per triangle-node pair of the
    wave-per-direction direct-sum kernel (16-node panels), counted from its
    source along the closed branch (the series branch replaces it for the
    pairs with a small phase spread).  A wave covers 8 PG panels, 128 PG
    nodes of one direction.

    FP64 form, consumer per node: 3 phase products (6 each) + the closed
    branch's two numerators from the sqrt(K)-scaled half-gap phases (2 MUL +
    2 FMA = 6) + complex multiply-accumulate (8)                          = 32
    one FP64 sin/cos with its argument (turn-table reduction, degree-9/8
        polynomials, rotation)                                             = 30
    per (triangle, wave), once:
        record: dot products, gaps and phase constants (20), sqrt(K_a),
        sqrt(K_b) (reciprocal, products, two square roots: 10), series
        coefficients through r^7 and threshold (46)                        = 76
        8 half-node lanes: 3 sin/cos, the two sqrt(K) scalings (4) and the
        series value of the wave's smallest radius (through r^5: 12)       = 106 each
        8 panel-centre lanes: 3 PG sin/cos, or with one wave per direction
        (PG = 2) 3 sin/cos and the second panel's phase as a product with
        the square of the first panel's phase: 3 (30 + 12)                 = 126 each
    running-sum merges: 2 * 2 PG adds per lane every 32 triangles.
    Per pair: 32 + (8 * 106 + 8 * panel lane + 76) / (128 PG) + 1 / 16.

    Mixed form (FP32 node arithmetic): consumer 34 per node (the K factors
    applied to the phase sines: 2 more MUL); per (triangle, wave) a record of
    20 (dot products, gaps, constants) + 60 (K_a, K_b, threshold and series
    coefficients through r^11) and 8 producer lanes of 3 (1 + PG) FP32
    sin/cos of 36 each (FP64 reduction 5, polynomials with two-float leading
    coefficients 31); batch flush: 2 adds per slot and batch of 8.
    """
    P = spec["n_panels"]
    PG = 2 if P % 16 == 0 else 1
    if form == "mixed":
        return 34.0 + (8 * 3 * (1 + PG) * 36.0 + 80.0) / (128 * PG) + 2.0 / 8
    one_wave = P == 8 * PG
    panel_lane = 3 * (30.0 + 12.0) if (one_wave and PG == 2) else 3 * PG * 30.0
    return 32.0 + (8 * 106.0 + 8 * panel_lane + 76.0) / (128 * PG) + 1.0 / 16


HBM_PEAK_GBS = 8000.0       # MI355X HBM3E


def _nufft_roofline(ctx, mesh, rule, params) -> dict:
    """Per-stage device times of one NUFFT distance (HIP events at the stage
    boundaries, on the library's stream) with each stage's algorithmic bytes
    (the library's count of what the stage must read and write), and the
    HBM roofline of the FFT passes (the stage whose design is HBM-bound) and
    of the whole pipeline."""
    import paper_2304_06340_amd as hsd
    ctx.set_stage_timing(True)
    hsd.distance(ctx, mesh, None, rule, params)
    st = ctx.nufft_stage_stats()
    ctx.set_stage_timing(False)
    stages = {k: {"ms": ms, "bytes": b, "GB_per_s": b / (ms * 1e-3) / 1e9 if ms > 0 else None}
              for k, (ms, b) in st.items()}
    fft_ms, fft_b = st["fft"]
    tot_ms = sum(ms for ms, _ in st.values())
    tot_b = sum(b for _, b in st.values())
    ach = fft_b / (fft_ms * 1e-3) / 1e9
    return {"roofline": {"bound": "hbm", "kernel": "k_fft_axis (three pruned passes)", "achieved": ach,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                         "traffic": None, "kernel_ms": fft_ms, "algorithmic_bytes": fft_b,
                         "pipeline_GB_per_s": tot_b / (tot_ms * 1e-3) / 1e9,
                         "pipeline_frac": tot_b / (tot_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "stages": stages}


def _cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_full_runs() -> list:
    """Complete oracle d2 evaluations stored with the parity fixtures (wall
    seconds on the machine that wrote them, named in each entry): level 2
    and level 7 on the 262,144-node rule, levels 3-5 on the 8,388,608-node
    rule."""
    import json
    runs = []
    for name, nodes in (("small_rule_levels.json", 262144), ("large_rule_levels.json", 8388608)):
        path = os.path.join(ROOT, "tests", "golden", name)
        if not os.path.exists(path):
            continue
        g = json.load(open(path))
        host = g.get("host", {})
        for L, sec in sorted(g.get("seconds", {}).items(), key=lambda kv: int(kv[0])):
            pairs = 20.0 * 4 ** int(L) * nodes
            runs.append({"level": int(L), "nodes": nodes, "pairs": pairs, "seconds": sec,
                         "pairs_per_s": pairs / sec, "host": host.get("cpu", "unknown"),
                         "threads": host.get("threads")})
    return runs


def _progress(msg: str) -> None:
    """One line per finished section on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="level7-large-rule", choices=sorted(WORKLOADS))
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-nodes", type=int, default=10240)
    ap.add_argument("--no-nufft", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-paper", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (reference kernel for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (the sharded path is design only); --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2304_06340_amd as hsd
    from hsd_inputs import icosphere

    level, spec, desc = WORKLOADS[args.workload]
    v, f = icosphere(level)
    torch.cuda.init()
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    ctx = hsd.Context(0)
    mesh = hsd.Mesh(ctx, v, f)
    rule = hsd.Rule.spherical_product(ctx, **spec)
    pairs = float(len(f)) * len(rule)

    def run(params, steps, warmup):
        for _ in range(warmup):
            hsd.distance(ctx, mesh, None, rule, params)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        results = [hsd.distance(ctx, mesh, None, rule, params) for _ in range(steps)]
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        return wall, results

    fp64 = hsd.Params(s=1.0, form="fp64")
    wall64, res64 = run(fp64, args.steps, args.warmup)
    _progress(f"fp64 {wall64 * 1e3:.1f} ms per distance")
    d2_64 = res64[-1].d2
    assert all(r.d2 == d2_64 for r in res64), "non-deterministic FP64 result"
    kern_ms = float(np.mean([r.transform_ms for r in res64]))
    out = {
        "metric": "tri*freq evals/s (FP64 direct-sum H^-s distance, reduction included)",
        "value": pairs / wall64,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (icosahedral mesh built in-process)",
        "config": {"workload": args.workload, "description": desc, "triangles": len(f),
                   "nodes": len(rule), "pairs_per_step": pairs, "s": 1.0},
        "distances_per_s": 1.0 / wall64,
        "d2": d2_64,
    }
    flop_pair = flops_per_pair(spec)
    achieved = flop_pair * pairs / (kern_ms * 1e-3) / 1e12
    rev = kernel_revision()
    traffic, traffic_rev = MEASURED_TRAFFIC.get(args.workload, (None, ""))
    out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                       "traffic": traffic if traffic_rev == rev else None,
                       "traffic_note": "HBM bytes per launch from rocprofv3 FETCH_SIZE/WRITE_SIZE, "
                                       "scaled by a plain copy's counters, for kernel revision "
                                       f"{traffic_rev or 'none'} (this build: {rev}; null when they differ)",
                       "kernel": "k_direct_wave (FP64)", "kernel_ms": kern_ms,
                       "kernel_revision": rev, "flops_per_pair": flop_pair}
    if not args.no_mixed:
        mixed = hsd.Params(s=1.0, form="mixed")
        wallm, resm = run(mixed, args.steps, args.warmup)
        _progress(f"mixed {wallm * 1e3:.1f} ms per distance")
        rel = abs(resm[-1].d2 - d2_64) / d2_64
        kern_m = float(np.mean([r.transform_ms for r in resm]))
        flop_m = flops_per_pair(spec, "mixed")
        ach_m = flop_m * pairs / (kern_m * 1e-3) / 1e12
        out["mixed"] = {"pairs_per_s": pairs / wallm, "ms_per_step": wallm * 1e3,
                        "distances_per_s": 1.0 / wallm, "rel_err_vs_fp64": rel,
                        "rel_err_stated": resm[-1].rel_err_stated,
                        "speedup_vs_fp64": wall64 / wallm, "kernel_ms": kern_m,
                        "roofline": {"bound": "alu", "achieved": ach_m, "peak": FP32_PEAK_TFLOPS,
                                     "unit": "TFLOP/s", "frac": ach_m / FP32_PEAK_TFLOPS,
                                     "kernel": "k_direct_wave_mixed", "flops_per_pair": flop_m,
                                     "note": "FP32 peak; the kernel's FP64 phase reduction, "
                                             "series-branch accumulation and batch flushes run at "
                                             "the FP64 rate"}}
    if not args.no_nufft:
        # type-3 NUFFT fast path (Dunavant-7 points, tol 1e-9) on the same mesh and rule
        pn = hsd.Params(s=1.0, method="nufft3", nufft_tol=1e-9)
        walln, resn = run(pn, max(1, args.steps), 1)
        _progress(f"nufft {walln * 1e3:.1f} ms per distance")
        out["nufft"] = {"ms_per_step": walln * 1e3, "distances_per_s": 1.0 / walln,
                        "points": resn[-1].pairs, "rel_err_vs_fp64_direct": abs(resn[-1].d2 - d2_64) / d2_64,
                        "note": "error vs the exact-triangle d2 includes the 7-point rule's model error",
                        **_nufft_roofline(ctx, mesh, rule, pn)}
    if not args.no_paper:
        # The paper's own configuration (section 4, Figs. 3(b) and 4): level 7,
        # exp(-2 pi i eta.x) convention with order -10, trapezoid rule on
        # [-5, 5]^3 with M = 128 (nodes xi = 2 pi eta), 64-point GL triangle
        # rule, NUFFT tolerance 1e-7 as in its timings; relative H_-10 error
        # against the empty surface's norm on the same rule.
        cube = hsd.Rule.cube_trapezoid(ctx, 2.0 * math.pi * 5.0, 128)
        pp = hsd.Params(s=10.0, freq_unit=2.0 * math.pi, method="nufft3", tri_rule="gl8x8", nufft_tol=1e-7)
        hsd.distance(ctx, mesh, None, cube, pp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        resp = [hsd.distance(ctx, mesh, None, cube, pp) for _ in range(3)]
        torch.cuda.synchronize()
        wp = (time.perf_counter() - t0) / 3
        _progress(f"paper configuration {wp * 1e3:.1f} ms per distance")
        empty = hsd.Mesh(ctx, np.zeros((0, 3)), np.zeros((0, 3), np.int32))
        norm2 = hsd.distance(ctx, empty, None, cube, pp).d2
        out["paper_config"] = {
            "workload": "level-7 icosphere, paper convention, s=-10, xi_max=5, M=128 (129^3 lattice), "
                        "GL 8x8 points (20,971,520), NUFFT tol 1e-7 (type 1 on the lattice)",
            "ms_per_distance": wp * 1e3, "transform_ms": resp[-1].transform_ms,
            "relative_H-10_error": math.sqrt(resp[-1].d2 / norm2),
            **_nufft_roofline(ctx, mesh, cube, pp),
            "paper_reference": "0.94 s on an RTX A6000 for the same N, M, xi_max and point rule "
                               "(context: other hardware, allocation and reductions excluded there)"}
        cube.close()
        # the paper's second timed configuration: level 5, M = 416 (417^3 lattice)
        m5 = hsd.Mesh(ctx, *icosphere(5))
        cube = hsd.Rule.cube_trapezoid(ctx, 2.0 * math.pi * 5.0, 416)
        hsd.distance(ctx, m5, None, cube, pp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        resp = [hsd.distance(ctx, m5, None, cube, pp) for _ in range(3)]
        torch.cuda.synchronize()
        wp = (time.perf_counter() - t0) / 3
        _progress(f"paper configuration M=416 {wp * 1e3:.1f} ms per distance")
        norm2 = hsd.distance(ctx, empty, None, cube, pp).d2
        out["paper_config_m416"] = {
            "workload": "level-5 icosphere, paper convention, s=-10, xi_max=5, M=416 (417^3 lattice), "
                        "GL 8x8 points (1,310,720), NUFFT tol 1e-7 (type 1 on the lattice)",
            "ms_per_distance": wp * 1e3, "transform_ms": resp[-1].transform_ms,
            "relative_H-10_error": math.sqrt(resp[-1].d2 / norm2),
            "paper_reference": "1.44 s on an RTX A6000 for the same N, M, xi_max and point rule "
                               "(context: other hardware, allocation and reductions excluded there)"}
        empty.close()
        m5.close()
        cube.close()
    if not args.no_adjoint:
        from hsd_inputs import perturb_harmonic
        va, fa = icosphere(4)
        va = perturb_harmonic(va, 0.05)
        ma = hsd.Mesh(ctx, va, fa)
        ra = hsd.Rule.spherical_product(ctx, r_max=64.0, n_panels=8, n_per_panel=16, n_cos=32, n_phi=64)
        hsd.distance_grad(ctx, ma, None, ra)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            ga = hsd.distance_grad(ctx, ma, None, ra)[0]
        torch.cuda.synchronize()
        wa = (time.perf_counter() - t0) / 3
        _progress(f"adjoint {wa * 1e3:.1f} ms per gradient")
        gm = hsd.distance_grad(ctx, ma, None, ra, hsd.Params(s=1.0, form="mixed"))[1]
        g64 = hsd.distance_grad(ctx, ma, None, ra)[1]
        out["adjoint"] = {"workload": "level-4 icosphere, v(1+0.05 sin3t cos2p), 262,144-node rule",
                          "ms_per_gradient": wa * 1e3, "pairs": ga.pairs,
                          "mixed_grad_rel_err": float(np.max(np.abs(gm - g64)) / np.max(np.abs(g64))),
                          "note": "mixed: residuals from the mixed forward, FP64 adjoint"}
        ma.close()
        ra.close()
    if not args.no_serve:
        from hsd_inputs import serving_trace
        from paper_2304_06340_amd.serving import replay
        trace = serving_trace(n=args.serve_requests, rate=20.0, seed=0, p_large=0.01)
        rules = {"small": hsd.Rule.spherical_product(ctx, r_max=64.0, n_panels=8, n_per_panel=16,
                                                     n_cos=32, n_phi=64),
                 "large": rule}
        out["serving"] = {"trace": f"{len(trace)} requests, Poisson 20/s, seed 0, levels 1-6, 30% "
                                   "mesh-vs-mesh, 1% on the large rule", "slots": 4,
                          "note": "saturated: the same requests all submitted at t = 0 (capacity); "
                                  "offered_load = the trace's pairs per second of arrivals / the "
                                  "saturated pairs per second; device_busy_frac = share of the span "
                                  "with at least one request admitted"}
        for form in ("fp64", "mixed"):
            prm = hsd.Params(s=1.0, form=form)
            with hsd.Server(ctx, slots=4, chunk_pairs=20_000_000_000) as srv:
                sat = replay(srv, trace, rules, prm, time_scale=0.0)
            with hsd.Server(ctx, slots=4, chunk_pairs=20_000_000_000) as srv:
                st = replay(srv, trace, rules, prm, capacity_pairs_per_s=sat["pairs_per_s"])
            for x in (sat, st):
                x.pop("results")
            st["saturated"] = {k: sat[k] for k in ("distances_per_s", "pairs_per_s", "span_s", "p50_ms",
                                                   "p99_ms", "failed", "device_busy_frac")}
            out["serving"][form] = st
            _progress(f"serving {form}: p50 {st['p50_ms']:.1f} ms, p99 {st['p99_ms']:.1f} ms, load "
                      f"{st.get('offered_load', float('nan')):.2f}; saturated {sat['distances_per_s']:.1f}/s")
    if not args.no_sweep:
        # per-request device time of the direct sum by mesh level, rule and
        # form: the service times behind the serving trace's latencies
        rules_sw = {"small": hsd.Rule.spherical_product(ctx, r_max=64.0, n_panels=8, n_per_panel=16,
                                                        n_cos=32, n_phi=64), "large": rule}
        sweep = {}
        for rname, rl in rules_sw.items():
            for level in range(1, 7):
                vs, fs = icosphere(level)
                ms = hsd.Mesh(ctx, vs, fs)
                row = {}
                for form in ("fp64", "mixed"):
                    prm = hsd.Params(s=1.0, form=form)
                    hsd.distance(ctx, ms, None, rl, prm)
                    row[form + "_ms"] = float(np.median([hsd.distance(ctx, ms, None, rl, prm).transform_ms
                                                         for _ in range(3)]))
                row["mixed_speedup"] = row["fp64_ms"] / row["mixed_ms"]
                sweep[f"{rname}-L{level}"] = row
                ms.close()
        rules_sw["small"].close()
        out["kernel_ms_by_level"] = sweep
        _progress("sweep " + ", ".join(f"{k} {v['mixed_speedup']:.2f}x" for k, v in sweep.items()))
    if not args.no_cpu:
        import oracle
        orule = oracle.spherical_product_rule(**spec)
        rng = np.random.default_rng(0)
        idx = rng.choice(len(orule), size=min(args.cpu_nodes, len(orule)), replace=False)
        t0 = time.perf_counter()
        oracle.transform(v, f, orule.nodes[idx])
        dt = time.perf_counter() - t0
        _progress(f"cpu oracle {dt:.1f} s")
        cores = oracle.num_threads()
        rate = len(idx) * len(f) / dt
        out["cpu_baseline"] = {"value": rate, "unit": "pairs/s", "cores": cores, "kind": "oracle",
                               "per_core": rate / cores, "cpu": _cpu_model(),
                               "sample": f"oracle.transform of the same mesh at {len(idx)} seeded "
                                         f"rule nodes ({len(idx) * len(f):.3e} pairs, {dt:.1f} s)",
                               "full_runs": _oracle_full_runs()}
    print(json.dumps(out), flush=True)
    mesh.close()
    rule.close()
    ctx.close()


if __name__ == "__main__":
    main()
