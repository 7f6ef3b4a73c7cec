"""Effective toughness as the minimum over initial-crack positions.

The estimate of Eq. 32-33 depends on where the initial crack sits: the
crack starts there and may be biased away from the weakest path.  Sec. 3
proposes sampling several crack positions in the same RVE and taking the
minimum toughness.  The positions are independent RVE problems of one grid,
so they run as the slots of one batched handle, each at its own pace, until
each reaches its fracture point.  All solver work runs in libmirve; this
module only builds the samples and collects the results.
"""
from . import mirve
from . import workloads as W


def min_toughness_over_crack_positions(w, count, precision=mirve.RVE_PREC_FP64, max_steps=400,
                                       stream=None, **cfg):
    """Run `count` crack positions of workload w (workloads.crack_position_samples)
    to fracture in one batched handle.

    Returns a dict: shifts (voxels along the load axis), G_eff per shift
    (None where the run failed or did not fracture within max_steps),
    status and steps per shift, G_min and the shift that gives it."""
    samples = W.crack_position_samples(w, count)
    ws = [s for _, s in samples]
    r = mirve.from_workloads(ws, precision=precision, stream=stream, **cfg)
    try:
        infos, status = r.rve_run_slots([s.dtau for s in ws], [max_steps] * len(ws),
                                        stop_at_fracture=True)
        G = []
        for b, (info, st) in enumerate(zip(infos, status)):
            G.append(r.rve_effective_toughness(b) if st == 0 and info["fractured"] else None)
    finally:
        r.close()
    valid = [(g, sh) for g, (sh, _) in zip(G, samples) if g is not None]
    g_min, sh_min = min(valid) if valid else (None, None)
    return {"shifts": [sh for sh, _ in samples], "G_eff": G, "status": list(status),
            "steps": [i["step"] for i in infos], "G_min": g_min, "shift_min": sh_min}
