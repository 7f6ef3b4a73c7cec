"""Full-run parity: the GPU solver over many consecutive steps against the
oracle's stored runs (tests/golden/*_fp64.json, written by
tests/golden/make_golden.py from oracle/ alone).

- homogeneous32: a homogeneous plate with a notch run to the fracture point.
  FP64: every step's E, Sigma, D, T and G_eff (Eq. 32-33) within 1e-8
  relative, and the same fracture step.  Mixed precision (FP32 fields and
  transforms, FP64 reductions, constraint and curve): G_eff within 1e-3.
- composite64: the first 60 steps of the 64 x 64 two-phase composite, FP64,
  every step within 1e-8.

The curve integral T accumulates the iterative tolerances (stagger 1e-10,
Krylov and constraint 1e-12) of every step, so a run is held to a looser
bound than one step (1e-9) or one operator (1e-12).
"""
import json
import math
import os

import pytest

from paper_2508_07424_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
CURVE_TOL = 1e-8


def _golden(name):
    with open(os.path.join(HERE, "golden", name + "_fp64.json")) as fh:
        return json.load(fh)


def _compare(infos, gold):
    worst = {}
    for info, ref in zip(infos, gold["steps"]):
        for key in ("E", "Sigma", "D", "T"):
            d = abs(info[key] - ref[key]) / max(abs(ref[key]), 1e-300)
            worst[key] = max(worst.get(key, 0.0), d)
        # instantaneous energy release rate (Eq. 34): None / NaN where the
        # crack surface did not grow
        g, gr = info["G_inst"], ref["G_inst"]
        if gr is None:
            assert math.isnan(g), (info["step"], g)
        else:
            d = abs(g - gr) / max(abs(gr), 1e-300)
            worst["G_inst"] = max(worst.get("G_inst", 0.0), d)
    print("worst relative deviation per quantity", worst, flush=True)
    for key, d in worst.items():
        assert d < CURVE_TOL, (key, d)


def _fp64_tol(gold):
    return dict(gold["tolerances"], tol_pcg=1e-13)


def test_homogeneous_full_run_fp64():
    from paper_2508_07424_amd import mirve
    gold = _golden("homogeneous32")
    w = W.homogeneous_2d(nx=32, ny=32, crack=8)
    r = mirve.from_workload(w, **_fp64_tol(gold))
    infos = []
    for _ in range(len(gold["steps"]) + 5):
        infos.append(r.rve_step_dissipation(w.dtau))
        if infos[-1]["fractured"]:
            break
    print("steps gpu", len(infos), "oracle", len(gold["steps"]), flush=True)
    assert len(infos) == len(gold["steps"]) and infos[-1]["fractured"]
    _compare(infos, gold)
    G = r.rve_effective_toughness()
    print("G_eff gpu", G, "oracle", gold["G_eff"], flush=True)
    assert abs(G - gold["G_eff"]) <= CURVE_TOL * abs(gold["G_eff"])


def test_homogeneous_full_run_mixed_toughness():
    from paper_2508_07424_amd import mirve
    gold = _golden("homogeneous32")
    w = W.homogeneous_2d(nx=32, ny=32, crack=8)
    r = mirve.from_workload(w, precision=mirve.RVE_PREC_MIXED)
    n = 0
    for n in range(1, len(gold["steps"]) + 40):
        if r.rve_step_dissipation(w.dtau)["fractured"]:
            break
    G = r.rve_effective_toughness()
    print("steps mixed", n, "oracle", len(gold["steps"]), "G_eff mixed", G, "oracle",
          gold["G_eff"], flush=True)
    assert abs(G - gold["G_eff"]) <= 1e-3 * abs(gold["G_eff"])


def test_composite_60_steps_fp64():
    from paper_2508_07424_amd import mirve
    gold = _golden("composite64")
    w = W.composite_2d_small()
    r = mirve.from_workload(w, **_fp64_tol(gold))
    infos = [r.rve_step_dissipation(w.dtau) for _ in gold["steps"]]
    _compare(infos, gold)


def test_crack_position_sampling_fp64():
    """Toughness as the minimum over initial-crack positions (Sec. 3): four
    positions of the 24 x 24 plate with one inclusion run as the slots of
    one batched handle, each at its own pace, against the oracle's runs of
    the same positions (tests/golden/sampling24_fp64.json)."""
    from paper_2508_07424_amd import sampling
    with open(os.path.join(HERE, "golden", "sampling24_fp64.json")) as fh:
        gold = json.load(fh)
    w = W.inclusion_2d()
    res = sampling.min_toughness_over_crack_positions(w, 4, **_fp64_tol(gold))
    print("G_eff per shift", list(zip(res["shifts"], res["G_eff"])), flush=True)
    for ref, G, n in zip(gold["runs"], res["G_eff"], res["steps"]):
        assert n == ref["steps"]
        assert abs(G - ref["G_eff"]) <= CURVE_TOL * abs(ref["G_eff"]), (ref["shift"], G, ref["G_eff"])
    assert res["shift_min"] == gold["shift_min"]
    assert abs(res["G_min"] - gold["G_min"]) <= CURVE_TOL * gold["G_min"]
