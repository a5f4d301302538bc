"""Write the stored expected values used by the GPU parity tests.

Calls only the CPU oracle (``oracle``) and the seeded input generators
(``hsd_inputs``).  Usage:  python tests/golden/make_golden.py [name ...]
Each fixture is an .npz/.json file next to this script; its header fields say
what it is and how it was made.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from hsd_inputs import icosphere, perturb_harmonic  # noqa: E402

# the configurations (rule parameters) the fixtures refer to
RULE_SMALL = dict(r_max=64.0, n_panels=8, n_per_panel=16, n_cos=32, n_phi=64)      # 262,144 nodes
RULE_LARGE = dict(r_max=256.0, n_panels=16, n_per_panel=16, n_cos=128, n_phi=256)  # 8,388,608 nodes


def _rule(spec):
    return oracle.spherical_product_rule(spec["r_max"], spec["n_panels"], spec["n_per_panel"],
                                         spec["n_cos"], spec["n_phi"])


def sampled(name, level, spec, n_samples=4096, seed=7):
    """mu_h^ of the level-``level`` icosphere at ``n_samples`` seeded nodes of a rule."""
    rule = _rule(spec)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(len(rule), size=n_samples, replace=False))
    v, f = icosphere(level)
    t = time.time()
    mu = oracle.transform(v, f, rule.nodes[idx])
    dt = time.time() - t
    np.savez(os.path.join(HERE, name + ".npz"), idx=idx, nodes=rule.nodes[idx], mu_re=mu.real,
             mu_im=mu.imag, level=level, rule=json.dumps(spec),
             note="oracle.transform at sampled rule nodes; written by make_golden.py")
    print(f"{name}: {n_samples} nodes x {len(f)} triangles in {dt:.1f}s", flush=True)


def _host():
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu": model, "threads": oracle.num_threads(),
            "note": "the machine make_golden.py ran on (its oracle timings)"}


def d2_levels(name, levels, spec, s=1.0):
    rule = _rule(spec)
    out = {"rule": spec, "s": s, "d2": {}, "seconds": {},
           "note": "oracle.distance vs the unit sphere; written by make_golden.py", "host": _host()}
    path = os.path.join(HERE, name + ".json")
    if os.path.exists(path):
        old = json.load(open(path))
        if old.get("rule") == spec:
            out["d2"].update(old.get("d2", {}))
            out["seconds"].update(old.get("seconds", {}))
    for L in levels:
        if str(L) in out["d2"]:
            continue
        v, f = icosphere(L)
        t = time.time()
        out["d2"][str(L)] = oracle.distance(v, f, rule, s=s)
        out["seconds"][str(L)] = time.time() - t
        print(f"{name}: level {L} d2={out['d2'][str(L)]!r} ({out['seconds'][str(L)]:.1f}s)", flush=True)
        json.dump(out, open(path, "w"), indent=1)


def adjoint_case(name, level=4, spec=RULE_SMALL, amp=0.05, s=1.0):
    """d^2 and its vertex gradient for the radially perturbed icosphere
    v <- v_hat (1 + amp sin(3 theta) cos(2 phi)) against S^2."""
    v, f = icosphere(level)
    v = perturb_harmonic(v, amp)
    rule = _rule(spec)
    t = time.time()
    d2, g = oracle.gradient(v, f, rule, s=s)
    dt = time.time() - t
    np.savez(os.path.join(HERE, name + ".npz"), d2=d2, grad=g, level=level, amp=amp, s=s,
             rule=json.dumps(spec), note="oracle.gradient (dual numbers); written by make_golden.py")
    print(f"{name}: d2={d2!r} |grad|max={np.abs(g).max():.3e} ({dt:.1f}s)", flush=True)


def nufft_sampled(name, level, tri_rule, rule, n_samples=512, seed=13):
    """The direct point sum of a level-``level`` icosphere's point cloud
    (``tri_rule``: the 7-point or the 8x8 Gauss-Legendre triangle rule) at
    ``n_samples`` seeded nodes of ``rule`` (the full-size NUFFT parity case);
    sum |c| is stored for the tolerance tol * sum |c|."""
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(len(rule), size=n_samples, replace=False))
    v, f = icosphere(level)
    pts, c = oracle.point_cloud(v, f, tri_rule)
    t = time.time()
    mu = oracle.point_sum(pts, c, rule.nodes[idx])
    dt = time.time() - t
    np.savez(os.path.join(HERE, name + ".npz"), idx=idx, nodes=rule.nodes[idx], mu_re=mu.real,
             mu_im=mu.imag, level=level, tri_rule=tri_rule, sum_abs_c=np.sum(np.abs(c)),
             n_points=len(c), note="oracle.point_sum of oracle.point_cloud at sampled rule nodes; "
                                   "written by make_golden.py")
    print(f"{name}: {n_samples} nodes x {len(c)} points in {dt:.1f}s", flush=True)


JOBS = {
    "adjoint_level4_small_rule": lambda: adjoint_case("adjoint_level4_small_rule"),
    "small_rule_levels": lambda: d2_levels("small_rule_levels", range(0, 6), RULE_SMALL),
    "level7_small_rule_sampled": lambda: sampled("level7_small_rule_sampled", 7, RULE_SMALL),
    "level7_large_rule_sampled": lambda: sampled("level7_large_rule_sampled", 7, RULE_LARGE),
    "large_rule_level3": lambda: d2_levels("large_rule_levels", [3], RULE_LARGE),
    "large_rule_level4": lambda: d2_levels("large_rule_levels", [3, 4], RULE_LARGE),
    "large_rule_level5": lambda: d2_levels("large_rule_levels", [3, 4, 5], RULE_LARGE),
    # level 7, 7-point rule (2,293,760 points) on the 8,388,608-node ball rule
    "nufft_level7_large_rule_sampled": lambda: nufft_sampled(
        "nufft_level7_large_rule_sampled", 7, "dunavant7", _rule(RULE_LARGE)),
    # the paper's configuration: level 7, 8x8 GL rule (20,971,520 points) on
    # the M = 128 lattice of [-xi_max, xi_max]^3 with xi_max = 2 pi 5
    "nufft_level7_paper_lattice_sampled": lambda: nufft_sampled(
        "nufft_level7_paper_lattice_sampled", 7, "gl8x8", oracle.cube_trapezoid_rule(2.0 * np.pi * 5.0, 128)),
    "small_rule_level7": lambda: d2_levels("small_rule_levels", [6, 7], RULE_SMALL),
}

if __name__ == "__main__":
    names = sys.argv[1:] or ["small_rule_levels", "level7_small_rule_sampled", "level7_large_rule_sampled"]
    for n in names:
        JOBS[n]()
