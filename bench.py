#!/usr/bin/env python
"""Benchmark of the FFT Green-operator solve of the phase-field-fracture
toughness solver on one MI355X.

Default workload: a batch of 64 synthetic 2D elastic polycrystals of
512 x 512 voxels (200 Voronoi grains, rotated cubic stiffness, orientation-
dependent cleavage toughness, l = 2, a notch of 0.1 L_x), FP32 bulk with
FP64 reductions and constraint, in one batched handle.  A step is one
dissipation-controlled step (Eq. 16 of the paper: mechanics CG with the
fused Green operator, damage PCG, arc-length constraint, commit and
fracture test) of every RVE of the batch.  W warm-up steps, then K timed
steps, inputs resident in HBM: the batch of B RVEs commits W x B, then
K x B RVE-steps in one call each, every RVE at its own pace (a fast RVE
takes more steps than a slow one, so the launches keep covering the whole
batch).  An RVE caught in the middle of a step when the total is reached
returns to the start of that step, and the work of that step is not
counted.  With --schedule fixed every RVE takes exactly W, then K steps,
and a call ends with its slowest RVE.

value = sum over RVEs of (voxels x Green-operator applications of their
committed steps) / seconds.

The JSON line also carries the roofline of the dominant kernel (HIP events
on its stream) on the algorithmic bytes of a Green-operator application,
the in-solve rate and a plain-operator microbenchmark against the same
bytes, and the CPU oracle's rate on a bounded sample of the workload.
"""
import argparse
import json
import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
os.environ.setdefault("MKL_NUM_THREADS", "1")

HBM_PEAK_GBS = 8000.0
T_START = time.perf_counter()


def progress(msg):
    """Progress on stderr (the JSON result is the only line on stdout)."""
    print("[bench %6.1fs] %s" % (time.perf_counter() - T_START, msg), file=sys.stderr, flush=True)
PASS_NAMES = {3: "x-forward + constitutive + CG direction (k_xfwd)",
              1: "axis pass: last-axis FFT, projection, inverse FFT (k_axis)",
              4: "x-inverse + CG update (k_xinv)"}
PASS_SYMBOLS = {3: "k_xfwd", 1: "k_axis", 4: "k_xinv"}


def _workloads(size, batch, seed0=1):
    from paper_2508_07424_amd import workloads as W
    combos = [(e, g) for e in (2.0, 5.0, 10.0) for g in (1.0, 2.0, 4.0)]
    out = []
    for i in range(batch):
        e, g = combos[i % len(combos)]
        out.append(W.composite_2d(n=size, seed=seed0 + i, E_ratio=e, Gc_ratio=g, vf=0.3, ell=2.0,
                                  crack=int(round(40 * size / 256))))
    return out


def _polycrystals(size, batch):
    """Elastic polycrystals: 200 periodic Voronoi grains per realization
    (seed 1000 + r), in-plane orientations U[0, 2 pi), cubic C11 = 1,
    C12 = 0.5, C44 = z / 4 with the Zener ratio z ~ U[1, 4] and cleavage
    toughness Gc = 1 + a cos^2(4 theta), a ~ U[0, 3], per realization;
    l = 2, a notch of 0.1 L_x (Sec. 5.3)."""
    import numpy as np
    from paper_2508_07424_amd import workloads as W
    rng = np.random.default_rng(77)
    return [W.polycrystal_2d(n=size, grains=200, seed=1000 + r, zener=float(rng.uniform(1, 4)),
                             a_cleave=float(rng.uniform(0, 3)), ell=2.0) for r in range(batch)]


def _spheres(size, batch):
    """3D composites: 40 spheres by RSA at volume fraction 0.2, E contrast 5,
    Gc contrast 3, nu = 0.3, l = 2, a square notch L/2 x L/2 in the z
    mid-plane, load e_z (x) e_z."""
    from paper_2508_07424_amd import workloads as W
    return [W.composite_3d(n=size, seed=1 + r, spheres=40, vf=0.2, E_ratio=5.0, Gc_ratio=3.0)
            for r in range(batch)]


WORKLOADS = {
    # name: (builder, default size, default batch, default precision, description)
    "composite256": (_workloads, 256, 63, "fp64",
                     "2D fibre composite {n}x{n}, vf 0.3, r~U[5,9], E ratio {{2,5,10}} x Gc ratio "
                     "{{1,2,4}} x {r} realizations, l=2, 40-voxel notch"),
    "polycrystal512": (_polycrystals, 512, 64, "mixed",
                       "2D cubic polycrystal {n}x{n}, 200 Voronoi grains, Zener U[1,4], "
                       "Gc = 1 + a cos^2(4 theta) with a U[0,3], l=2, notch 0.1 L, {b} realizations"),
    "spheres128": (_spheres, 128, 1, "mixed",
                   "3D sphere composite {n}^3, 40 spheres vf 0.2, E ratio 5, Gc ratio 3, l=2, "
                   "square notch L/2 x L/2, load zz, {b} realization(s)"),
}


def alg_bytes(dim, w, m=2):
    """Algorithmic bytes per voxel of one Green-operator application on the
    minimal-pass schedule (the compulsory traffic of the hot path): in 2D
    three passes, [x-R2C + constitutive: read s+1 fields and the material id,
    write s] + [y forward, projection, y inverse: 2s] + [x-C2R: 2s], i.e.
    (6s + 1) w + m; in 3D five passes, (10s + 1) w + m.  Returns the total
    and each pass's share."""
    s = 3 if dim == 2 else 6
    share = {"x-forward": (s + 1) * w + m + s * w, "axis": 2 * s * w, "x-inverse": 2 * s * w}
    total = (6 * s + 1) * w + m if dim == 2 else (10 * s + 1) * w + m
    return total, share


def roofline(r, torch, dim, w, repeat=50):
    """Average duration of each pass of a mechanics CG iteration (one launch
    covers every RVE of the batch), by HIP events on the handle's stream.
    The dominant pass (the x-forward pass, which carries the constitutive
    law and the CG direction update) is priced at its share of the
    algorithmic bytes of a Green-operator application; the bytes it moves
    for the Krylov vectors (r, p, x) are reported beside it."""
    stream = torch.cuda.current_stream() if r.stream is None else r.stream
    B_alg, share = alg_bytes(dim, w)
    shares = {3: share["x-forward"], 1: share["axis"], 4: share["x-inverse"]}
    res = {}
    for p in (3, 1, 4):
        r.rve_profile_pass(p, 3)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        nbytes = r.rve_profile_pass(p, repeat)
        b.record(stream)
        torch.cuda.synchronize()
        res[p] = (a.elapsed_time(b) / repeat, nbytes)
    dom = max(res, key=lambda k: res[k][0])
    ms, krylov_bytes = res[dom]
    vox = r.N * r.B
    alg = shares[dom] * vox
    gbs = alg / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": PASS_NAMES[dom], "kernel_symbol": PASS_SYMBOLS[dom],
            "avg_us": round(ms * 1e3, 2),
            "algorithmic_bytes_per_launch": alg,
            "algorithmic_bytes_per_voxel": shares[dom],
            "krylov_inclusive_bytes_per_launch": krylov_bytes,
            "krylov_inclusive_gbs": round(krylov_bytes / (ms * 1e-3) / 1e9, 1),
            "passes_us": {PASS_NAMES[k]: round(v[0] * 1e3, 2) for k, v in res.items()}}


def operator_bench(r, torch, dim, w, repeat=1000):
    """The plain Green operator out = F^-1{P : F[g C : eps]} applied `repeat`
    times to a fixed strain on the batch's current (mid-run) damage, every
    RVE of the batch per application: voxel-iter/s and its fraction of the
    HBM roofline on the algorithmic bytes."""
    stream = torch.cuda.current_stream() if r.stream is None else r.stream
    dt = torch.float64 if w == 8 else torch.float32
    n = r.B * r.s * r.N
    with torch.cuda.stream(stream):
        g = torch.Generator(device="cuda")
        g.manual_seed(3)
        eps = torch.randn(n, dtype=dt, device="cuda", generator=g)
        out = torch.empty_like(eps)
    torch.cuda.synchronize()
    r.rve_apply_green_op_device(eps, out, 5)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    r.rve_apply_green_op_device(eps, out, repeat)
    b.record(stream)
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) * 1e-3
    B_alg, _ = alg_bytes(dim, w)
    rate = repeat * r.N * r.B / sec
    return {"applications": repeat, "voxel_iter_per_s": round(rate, 1),
            "us_per_application": round(1e6 * sec / repeat, 2),
            "algorithmic_bytes_per_voxel": B_alg,
            "achieved_gbs": round(rate * B_alg / 1e9, 1),
            "frac": round(rate * B_alg / 1e9 / HBM_PEAK_GBS, 4)}


def copy_bandwidth(torch, mib=1024, repeat=10):
    """Plain device-to-device copy of `mib` MiB (beyond the 256 MB last-level
    cache): the measured HBM bandwidth the roofline is also quoted against."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(repeat):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / repeat
    del src, dst
    return round(2 * n * 8 / (ms * 1e-3) / 1e9, 1)


# the files the Green-operator passes are compiled from
GREENOP_SOURCES = ("common.h", "fft2l.h", "fft_device.h", "greenop.hip", "kernels.h", "reduce.h")


def stored_traffic(kernel_file):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, if it was taken on the current
    sources of that kernel (else None)."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", kernel_file)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    h = hashlib.sha256()
    for name in GREENOP_SOURCES:
        with open(os.path.join(here, "paper_2508_07424_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    if vals.get("kernel_sources_sha256") != h.hexdigest():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


SERVE_SIZES = {
    # name: (2D sides, 3D sides), drawn log-uniform and rounded to the nearest listed side
    "small": ((32, 48, 64), (16, 24)),
    "full": ((64, 128, 256, 512), (64, 128)),
}


def serving(n_requests, seed, rate, sizes="small", max_steps=300, forms="both"):
    """The serving form against the plain form on one seeded request stream
    (2D fibre composites and polycrystals, 3D sphere composites, elastic
    contrast U[1, 10], toughness contrast U[1, 4], Poisson arrivals; sizes
    "small": 32^2-64^2 and 16^3-24^3, "full": 64^2-512^2 and 64^3-128^3):
    continuous batching in mixed precision versus one RVE at a time in
    FP64, same arrivals.  Reports solves/s, p50/p99 latency and the largest
    relative G_eff difference between the two."""
    import torch
    from paper_2508_07424_amd import mirve, serve
    from paper_2508_07424_amd import workloads as W
    s2, s3 = SERVE_SIZES[sizes]
    stream = W.serving_stream(n_requests, seed=seed, sizes_2d=s2, sizes_3d=s3,
                              frac_3d=0.25, rate=rate, dtau_frac=0.02)
    reqs = [serve.Request(i, w, arrival=a, max_steps=max_steps) for i, (a, w) in enumerate(stream)]
    progress("stream: " + ", ".join("%d:%s" % (i, "x".join(map(str, w.n)))
                                    for i, (a, w) in enumerate(stream)))
    torch.cuda.synchronize()
    res_s = res_p = None
    if forms in ("both", "batched"):
        progress("serving %d requests, mixed precision, continuous batching" % n_requests)
        t0 = time.perf_counter()
        srv = serve.Server(precision=mirve.RVE_PREC_MIXED, slots_per_pool=16)
        try:
            res_s = srv.run(reqs, realtime=True,
                            on_result=lambda r: progress("  served %d: G_eff %s after %d steps"
                                                         % (r.rid, r.G_eff, r.steps)))
        finally:
            srv.close()
        wall_s = time.perf_counter() - t0
    if forms in ("both", "plain"):
        progress("same requests, plain FP64, one at a time")
        t0 = time.perf_counter()
        res_p = serve.serve_sequential(
            reqs, precision=mirve.RVE_PREC_FP64,
            on_result=lambda r: progress("  solved %d: G_eff %s after %d steps" % (r.rid, r.G_eff, r.steps)),
            on_chunk=lambda rid, n: progress("    request %d: %d steps" % (rid, n)))
        wall_p = time.perf_counter() - t0
    if res_s is None or res_p is None:
        one, wall, name = (res_s, wall_s, "served_mixed_batched") if res_p is None else \
            (res_p, wall_p, "plain_fp64_one_at_a_time")
        return {"requests": n_requests, "arrival_rate_per_s": rate, "sizes": sizes,
                "grids": ["x".join(map(str, r.workload.n)) for r in reqs],
                name: serve.summarize(one, wall),
                "per_request": [{"rid": a.rid, "G_eff": a.G_eff, "steps": a.steps, "status": a.status,
                                 "latency_s": round(a.latency, 2)} for a in one]}
    both = [(a, b) for a, b in zip(res_s, res_p) if a.G_eff is not None and b.G_eff is not None]
    dev = max((abs(a.G_eff - b.G_eff) / abs(b.G_eff) for a, b in both), default=None)
    out = {"requests": n_requests, "arrival_rate_per_s": rate, "sizes": sizes,
           "grids": ["x".join(map(str, r.workload.n)) for r in reqs],
           "per_request": [{"rid": a.rid, "G_eff_mixed_batched": a.G_eff, "G_eff_plain_fp64": b.G_eff,
                            "steps": [a.steps, b.steps], "latency_s": [round(a.latency, 2),
                                                                       round(b.latency, 2)]}
                           for a, b in zip(res_s, res_p)],
           "served_mixed_batched": serve.summarize(res_s, wall_s),
           "plain_fp64_one_at_a_time": serve.summarize(res_p, wall_p),
           "max_rel_G_eff_diff": None if dev is None else float("%.3g" % dev),
           "compared": len(both), "admission_stalls": srv.stalls,
           "peak_workspace_bytes": srv.peak_bytes}
    ps = out["plain_fp64_one_at_a_time"]["solves_per_s"]
    if ps:
        out["solves_speedup"] = round(out["served_mixed_batched"]["solves_per_s"] / ps, 2)
    return out


def host_cpu():
    """Cores this process may use and the CPU model of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": usable, "cpu_count": os.cpu_count(), "model": model}


def newton_compare(torch, size=32, steps=3, oracle=True):
    """The monolithic Newton-Raphson step (Sec. 4.1) against the staggered
    step on one FP64 RVE (homogeneous size x size plate, notch size / 4):
    after one untimed step each, `steps` steps timed per solver on the GPU,
    and one Newton step of the oracle on the host from the same state."""
    from paper_2508_07424_amd import mirve
    from paper_2508_07424_amd import workloads as W
    w = W.homogeneous_2d(nx=size, ny=size, crack=size // 4)
    tight = dict(tol=1e-10, tol_cg=1e-12, tol_pcg=1e-14, tol_al=1e-12)
    stream = torch.cuda.Stream()
    a = mirve.from_workload(w, stream=stream, **tight)
    b = mirve.from_workload(w, stream=stream, **tight)
    a.rve_step_dissipation(w.dtau)
    b.rve_step_newton(w.dtau, tol=1e-10)
    out = {"workload": "homogeneous %dx%d plate, notch %d, FP64, %d steps after the first"
           % (size, size, size // 4, steps)}
    for name, r, fn in (("staggered", a, lambda: a.rve_step_dissipation(w.dtau)),
                        ("newton", b, lambda: b.rve_step_newton(w.dtau, tol=1e-10))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tot = {"n_greenop": 0, "n_stagger": 0, "n_cg": 0, "n_pcg": 0}
        for _ in range(steps):
            info = fn()
            for key in tot:
                tot[key] += info[key]
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out[name] = {"ms_per_step": round(1e3 * sec / steps, 2),
                     "greenops_per_step": round(tot["n_greenop"] / steps, 1),
                     "voxel_iter_per_s": round(tot["n_greenop"] * r.N / sec, 1),
                     "E": info["E"]}
        if name == "newton":
            out[name]["newton_iterations_per_step"] = round(tot["n_stagger"] / steps, 2)
            out[name]["gmres_iterations_per_step"] = round(tot["n_cg"] / steps, 1)
        else:
            out[name]["stagger_iterations_per_step"] = round(tot["n_stagger"] / steps, 2)
        progress("newton comparison: %s %.1f ms per step" % (name, out[name]["ms_per_step"]))
    out["rel_E_diff"] = abs(out["newton"]["E"] - out["staggered"]["E"]) / abs(out["staggered"]["E"])
    out["newton_over_staggered_time"] = round(out["newton"]["ms_per_step"] / out["staggered"]["ms_per_step"], 2)
    if oracle:
        from oracle import newton, solver
        prob = solver.Problem(w.n, w.h, w.ell, w.phases, w.phase_id, w.f, theta=w.theta, void=w.void,
                              phi_disc=w.phi_disc, phi_M=w.phi_M, k=w.k, tol=1e-10, tol_cg=1e-12,
                              tol_al=1e-12)
        st = solver.State(prob)
        newton.step(prob, st, w.dtau, tol=1e-10)
        t0 = time.perf_counter()
        rec = newton.step(prob, st, w.dtau, tol=1e-10)
        sec = time.perf_counter() - t0
        out["oracle_newton"] = {"ms_per_step": round(1e3 * sec, 1), "kind": "oracle", "cores": 1,
                                "newton_iterations": rec["n_newton"], "krylov_iterations": rec["n_krylov"],
                                "sample": "the second step, after an untimed first"}
        progress("newton comparison: oracle %.1f ms per step" % out["oracle_newton"]["ms_per_step"])
    return out


def cpu_baseline(w, seconds):
    """The oracle's conjugate-gradient Green-operator solve on the host,
    bounded to about `seconds` of work: voxel-iterations per second."""
    import numpy as np
    from oracle import solver
    prob = solver.Problem(w.n, w.h, w.ell, w.phases, w.phase_id, w.f, theta=w.theta, void=w.void,
                          phi_disc=w.phi_disc, phi_M=w.phi_M, k=w.k, tol_cg=1e-300, max_cg=5)
    st = solver.State(prob)
    t0 = time.perf_counter()
    x, it = solver.mechanics(prob, st.phi, st.x)
    t1 = time.perf_counter()
    per = (t1 - t0) / max(it + 2, 1)                 # CG iterations + the two set-up applications
    n_it = max(5, int(seconds / max(per, 1e-6)))
    prob.max_cg = n_it
    t0 = time.perf_counter()
    x, it = solver.mechanics(prob, st.phi, st.x)
    t1 = time.perf_counter()
    N = int(np.prod(w.n))
    host = host_cpu()
    return {"value": round(N * (it + 2) / (t1 - t0), 1), "unit": "voxel-iter/s", "cores": 1,
            "kind": "oracle", "host_nproc": host["nproc"], "host_cpu": host["model"],
            "sample": "%d CG iterations (+2 set-up Green operators) of the oracle's mechanics solve on "
                      "one %s RVE at its enriched initial state, numpy FFT, 1 thread, %.1f s"
                      % (it, "x".join(map(str, w.n)), t1 - t0)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="polycrystal512")
    ap.add_argument("--batch", type=int, default=None,
                    help="RVEs (default: 64 polycrystals; 63 = 9 contrast cases x 7 realizations "
                         "for composite256)")
    ap.add_argument("--size", type=int, default=None)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--operator-repeat", type=int, default=1000)
    ap.add_argument("--serve-requests", type=int, default=0,
                    help="requests of the serving comparison (0: skip it)")
    ap.add_argument("--serve-rate", type=float, default=2.0, help="Poisson arrivals per second")
    ap.add_argument("--serve-sizes", choices=sorted(SERVE_SIZES), default="small")
    ap.add_argument("--serve-seed", type=int, default=5)
    ap.add_argument("--serve-only", action="store_true",
                    help="only the serving comparison (one JSON line with its field)")
    ap.add_argument("--serve-form", choices=["both", "batched", "plain"], default="both",
                    help="run one form only (the stream and arrivals are the same)")
    ap.add_argument("--schedule", choices=["budget", "fixed"], default="budget",
                    help="budget: the batch commits steps x B RVE-steps, each RVE at its own pace; "
                         "fixed: every RVE takes exactly the steps (a call ends with its slowest RVE)")
    ap.add_argument("--newton-size", type=int, default=32,
                    help="grid side of the Newton-against-staggered comparison (0: skip it)")
    ap.add_argument("--newton-steps", type=int, default=3)
    ap.add_argument("--newton-only", action="store_true",
                    help="only the Newton-against-staggered comparison (one JSON line)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="set up the batch and time the Green-operator passes only (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: there is no multi-GPU path here "
              "(independent RVEs would shard across GPUs with no collective)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2508_07424_amd import mirve
    if args.serve_only:
        out = {"serving": serving(max(1, args.serve_requests), seed=args.serve_seed,
                                  rate=args.serve_rate, sizes=args.serve_sizes, forms=args.serve_form)}
        print(json.dumps(out), flush=True)
        return
    if args.newton_only:
        out = {"newton": newton_compare(torch, args.newton_size, args.newton_steps,
                                        oracle=not args.no_cpu_baseline)}
        print(json.dumps(out), flush=True)
        return
    build, size0, batch0, prec0, desc = WORKLOADS[args.workload]
    args.size = args.size or size0
    args.batch = args.batch or batch0
    args.precision = args.precision or prec0
    prec = mirve.RVE_PREC_FP64 if args.precision == "fp64" else mirve.RVE_PREC_MIXED
    w_bytes = 8 if prec == mirve.RVE_PREC_FP64 else 4
    progress("generating %d %s inputs" % (args.batch, args.workload))
    wls = build(args.size, args.batch)
    dim = len(wls[0].n)
    # one batched handle; each RVE advances at its own pace within a call
    progress("setting up %d RVEs" % len(wls))
    rve = mirve.from_workloads(wls, precision=prec, stream=torch.cuda.Stream())
    dtaus = [w.dtau for w in wls]
    torch.cuda.synchronize()
    progress("set up")
    shape = rve.rve_autotune(10)
    progress("autotuned launch shape (x rows, y lines, z columns, non-temporal) = %s" % (shape,))
    if args.roofline_only:
        roof = roofline(rve, torch, dim, w_bytes)
        roof["copy_gbs"] = copy_bandwidth(torch)
        print(json.dumps({"roofline": roof}), flush=True)
        return

    failed = {}
    occupancy = {}

    def run(nsteps, label):
        t0 = time.perf_counter()
        live = [d if b not in failed else 0.0 for b, d in enumerate(dtaus)]
        if args.schedule == "budget":
            infos, st = rve.rve_run_budget(live, nsteps * sum(1 for d in live if d > 0.0))
        else:
            infos, st = rve.rve_run_slots(live, [nsteps] * len(live))
        for b, (i, s) in enumerate(zip(infos, st)):
            if s != 0 and b not in failed:
                failed[b] = {"slot": b, "status": s, "reason": mirve.WHY.get(i["reason"], "?"),
                             "phase": label, "steps_done": i["n_steps"]}
        done = sum(i["n_steps"] for i in infos)
        rounds, occ = rve.rve_run_stats()
        progress("%s: %d RVE-steps in %.2f s, %d failed slots, %d rounds at %.3f mean slot occupancy"
                 % (label, done, time.perf_counter() - t0, len(failed), rounds, occ))
        per = [i["n_steps"] for i in infos]
        occupancy[label] = {"rounds": rounds, "mean_active_slot_fraction": round(occ, 4),
                            "rve_steps": done, "steps_per_rve_min": min(per),
                            "steps_per_rve_max": max(per)}
        return infos

    per = " on average" if args.schedule == "budget" else ""
    if args.warmup > 0:
        run(args.warmup, "warm-up (%d steps per RVE%s)" % (args.warmup, per))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = run(args.steps, "timed (%d steps per RVE%s)" % (args.steps, per))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = t1 - t0
    greenops = sum(rve.N * i["n_greenop"] for i in infos)
    rve_steps = sum(i["n_steps"] for i in infos)
    value = greenops / sec

    B_alg, _ = alg_bytes(dim, w_bytes)
    roof = roofline(rve, torch, dim, w_bytes)
    roof["copy_gbs"] = copy_bandwidth(torch)
    roof["frac_of_copy"] = round(roof["achieved"] / roof["copy_gbs"], 4)
    tag = "f64" if prec == mirve.RVE_PREC_FP64 else "mixed"
    roof["traffic"] = stored_traffic("traffic_%s_%s_b%d_%s.txt" % (
        roof["kernel_symbol"], "x".join([str(args.size)] * dim), args.batch, tag))
    roof["in_solve"] = {"voxel_iter_per_s": round(value, 1), "algorithmic_bytes_per_voxel": B_alg,
                        "achieved_gbs": round(value * B_alg / 1e9, 1),
                        "frac": round(value * B_alg / 1e9 / HBM_PEAK_GBS, 4)}
    progress("operator microbenchmark (%d applications)" % args.operator_repeat)
    roof["operator"] = operator_bench(rve, torch, dim, w_bytes, args.operator_repeat)
    out = {
        "metric": "voxel-iter/s FFT Green-op solve",
        "value": round(value, 1),
        "unit": "voxel-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * sec / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == mirve.RVE_PREC_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": desc.format(n=args.size, r=(args.batch + 8) // 9, b=args.batch),
                   "batch": args.batch, "precision": args.precision, "schedule": args.schedule,
                   "rve_steps": rve_steps,
                   "rve_steps_per_s": round(rve_steps / sec, 3),
                   "greenops_per_rve_step": round(greenops / max(rve_steps, 1) / rve.N, 1),
                   "failed_slots": sorted(failed.values(), key=lambda d: d["slot"]),
                   "slot_occupancy": occupancy,
                   "launch_shape": {"x_rows_per_block": shape[0], "y_lines_per_block": shape[1],
                                    "y_pass": "one wave per line" if shape[1] == 0 else "block",
                                    "z_columns_per_tile": shape[2],
                                    "krylov_vectors_nontemporal": shape[3]}},
        "roofline": roof,
    }
    if args.serve_requests > 0:
        rve = None
        torch.cuda.empty_cache()
        out["serving"] = serving(args.serve_requests, seed=args.serve_seed, rate=args.serve_rate,
                                 sizes=args.serve_sizes)
    if args.newton_size > 0:
        rve = None
        torch.cuda.empty_cache()
        out["newton"] = newton_compare(torch, args.newton_size, args.newton_steps,
                                       oracle=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        progress("oracle on the host")
        out["cpu_baseline"] = cpu_baseline(wls[0], args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
