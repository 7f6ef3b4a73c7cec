"""Batched form: RVEs advanced together by the same launches give the same
results as each RVE alone (per-RVE reductions have the same shape, so the
results are bitwise equal)."""
import numpy as np
import pytest

from paper_2508_07424_amd import workloads as W

pytestmark = pytest.mark.gpu


def _three():
    return [W.homogeneous_2d(nx=48, ny=40, crack=8),
            W.laminate_2d(nx=48, ny=40, widths=(0.5, 0.5), Gcs=(1.0, 2.0), ell=1.5),
            W.homogeneous_2d(nx=48, ny=40, crack=12, E=2.0, Gc=1.5)]


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_equals_alone(prec):
    from paper_2508_07424_amd import mirve
    ws = _three()
    for w in ws:
        w.f = W.load_yy(2)
    batch = mirve.from_workloads(ws, precision=prec)
    alone = [mirve.from_workload(w, precision=prec, max_materials=4096) for w in ws]
    for k in range(2):
        info_b, st = batch.rve_step_dissipation_slots([w.dtau for w in ws])
        assert all(v == 0 for v in st), st
        for i, (w, r) in enumerate(zip(ws, alone)):
            info = r.rve_step_dissipation(w.dtau)
            print("step", k + 1, "rve", i, info_b[i]["E"], info["E"], flush=True)
            for key in ("E", "Sigma", "D", "T", "n_cg", "n_stagger"):
                assert info_b[i][key] == info[key], (k, i, key, info_b[i][key], info[key])
    for i, r in enumerate(alone):
        assert np.array_equal(batch.rve_get_field("phi", slot=i), r.rve_get_field("phi"))


def test_idle_slot_and_release():
    from paper_2508_07424_amd import mirve
    ws = _three()
    batch = mirve.from_workloads(ws)
    before = batch.rve_get_field("phi", slot=1)
    info, st = batch.rve_step_dissipation_slots([ws[0].dtau, 0.0, ws[2].dtau])
    assert st == [0, 0, 0]
    assert np.array_equal(batch.rve_get_field("phi", slot=1), before)
    assert batch.rve_get_scalars(slot=1)["step"] == 0
    assert batch.rve_get_scalars(slot=0)["step"] == 1
    batch.rve_release_slot(1)
    info, st = batch.rve_step_dissipation_slots([ws[0].dtau, 1.0, 0.0])
    assert st[0] == 0 and st[1] == mirve.RVE_ESTATE


def test_autotune_keeps_results():
    """The tuner only changes launch shapes: a tuned handle gives the same
    steps as an untuned one up to the summation order of the partials."""
    from paper_2508_07424_amd import mirve
    w = W.composite_2d_small()
    tight = dict(tol=1e-12, tol_cg=1e-13, tol_pcg=1e-14, tol_al=1e-13)
    a = mirve.from_workload(w, **tight)
    b = mirve.from_workload(w, **tight)
    shape = b.rve_autotune(5)
    print("tuned shape", shape, flush=True)
    assert shape[0] >= 2 and shape[0] % 2 == 0 and shape[1] >= 1
    assert b.rve_autotune(5) == shape            # cached
    for _ in range(2):
        ia = a.rve_step_dissipation(w.dtau)
        ib = b.rve_step_dissipation(w.dtau)
        for key in ("E", "Sigma", "D", "T"):
            assert abs(ia[key] - ib[key]) <= 1e-9 * abs(ia[key]), (key, ia[key], ib[key])


def test_streaming_policies_match():
    """The non-temporal and the cached policy of the Krylov x passes run the
    same arithmetic: a batch stepped under each gives bitwise-equal steps
    and fields, in both precisions."""
    from paper_2508_07424_amd import mirve
    for prec in (mirve.RVE_PREC_FP64, mirve.RVE_PREC_MIXED):
        ws = _three()
        for w in ws:
            w.f = W.load_yy(2)
        a = mirve.from_workloads(ws, precision=prec, streaming=0)
        b = mirve.from_workloads(ws, precision=prec, streaming=1)
        print("precision", prec, flush=True)
        for _ in range(2):
            ia, sa = a.rve_step_dissipation_slots([w.dtau for w in ws])
            ib, sb = b.rve_step_dissipation_slots([w.dtau for w in ws])
            assert list(sa) == list(sb) and all(v == 0 for v in sa), (sa, sb)
            for x, y in zip(ia, ib):
                for key in ("E", "Sigma", "D", "T"):
                    assert x[key] == y[key], (prec, key, x[key], y[key])
        for slot in range(len(ws)):
            assert np.array_equal(a.rve_get_field("phi", slot=slot), b.rve_get_field("phi", slot=slot))


def test_graph_replays_match_launches():
    """Krylov chunks replayed from captured HIP graphs (several replays of
    each graph, with eager work in between) give the same steps as direct
    launches, bitwise."""
    from paper_2508_07424_amd import mirve
    ws = _three()
    for w in ws:
        w.f = W.load_yy(2)
    import torch
    a = mirve.from_workloads(ws)
    b = mirve.from_workloads(ws, graphs=1, stream=torch.cuda.Stream())   # capture needs a stream
    for k in range(3):
        ia, sa = a.rve_step_dissipation_slots([w.dtau for w in ws])
        ib, sb = b.rve_step_dissipation_slots([w.dtau for w in ws])
        assert sa == sb == [0, 0, 0]
        for i in range(len(ws)):
            for key in ("E", "Sigma", "D", "T", "n_cg", "n_pcg"):
                assert ia[i][key] == ib[i][key], (k, i, key, ia[i][key], ib[i][key])
    for i in range(len(ws)):
        assert np.array_equal(a.rve_get_field("phi", slot=i), b.rve_get_field("phi", slot=i))


def test_run_slots_each_at_its_own_pace():
    """rve_run_slots: slots asked for different numbers of steps advance at
    their own pace in one call (a slot that commits starts its next step
    while others still iterate) and end bitwise where the same RVE stepped
    alone ends, with the same work counters."""
    from paper_2508_07424_amd import mirve
    ws = _three()
    for w in ws:
        w.f = W.load_yy(2)
    batch = mirve.from_workloads(ws)
    todo = [3, 1, 2]
    infos, st = batch.rve_run_slots([w.dtau for w in ws], todo)
    assert st == [0, 0, 0]
    for i, w in enumerate(ws):
        r = mirve.from_workload(w, max_materials=4096)
        tot = {"n_cg": 0, "n_pcg": 0, "n_stagger": 0, "n_greenop": 0}
        for _ in range(todo[i]):
            one = r.rve_step_dissipation(w.dtau)
            for key in tot:
                tot[key] += one[key]
        b = infos[i]
        print("rve", i, "steps", b["n_steps"], "E", b["E"], one["E"], flush=True)
        assert b["n_steps"] == todo[i] and b["step"] == todo[i]
        for key in ("E", "Sigma", "D", "T", "tau"):
            assert b[key] == one[key], (i, key)
        for key, v in tot.items():
            assert b[key] == v, (i, key, b[key], v)
        assert np.array_equal(batch.rve_get_field("phi", slot=i), r.rve_get_field("phi"))
        assert np.array_equal(batch.rve_get_field("hist", slot=i), r.rve_get_field("hist"))


def test_run_stats_report_slot_occupancy():
    """rve_run_stats: the rounds of the last rve_run_slots call and the mean
    fraction of the batch they covered.  With one of three slots idle every
    round covers at most two thirds of the batch; a slot that finishes its
    steps early lowers it further."""
    from paper_2508_07424_amd import mirve as m
    ws = [W.composite_2d_small(seed=s) for s in (1, 2, 3)]
    r = m.from_workloads(ws)
    infos, st = r.rve_run_slots([ws[0].dtau, ws[1].dtau, 0.0], [2, 1, 0])
    assert st == [0, 0, 0]
    rounds, occ = r.rve_run_stats()
    print("rounds", rounds, "occupancy", occ, flush=True)
    assert rounds > 0 and 0.0 < occ < 2.0 / 3.0
    infos, st = r.rve_run_slots([w.dtau for w in ws], [1, 1, 1])
    rounds1, occ1 = r.rve_run_stats()
    assert rounds1 > 0 and occ < occ1 <= 1.0


@pytest.mark.parametrize("case", ["plain", "halving"])
def test_run_budget_ends_on_committed_states(case):
    """rve_run_budget: slots step at their own pace until the batch has
    committed the budget; every round covers the whole batch, and each slot
    ends bitwise where the same RVE stepped alone for the slot's committed
    steps ends (a slot caught in the middle of a step, also after sub-steps
    of it had committed, returns to the step's start and drops its work).
    The slots then go on from there as the lone RVEs do.  "halving" takes
    doubled steps under a small stagger limit so that steps split."""
    from paper_2508_07424_amd import mirve
    ws = _three()
    kw = {}
    for w in ws:
        w.f = W.load_yy(2)
        if case == "halving":
            w.dtau = 2.0 * w.dtau
    if case == "halving":
        kw = dict(max_stagger=6)
    batch = mirve.from_workloads(ws, **kw)
    alone = [mirve.from_workload(w, max_materials=4096, **kw) for w in ws]
    dt = [w.dtau for w in ws]
    split = 0
    for call, budget in enumerate((4, 1, 2)):
        infos, st = batch.rve_run_budget(dt, budget)
        assert st == [0, 0, 0], st
        done = [i["n_steps"] for i in infos]
        rounds, occ = batch.rve_run_stats()
        print("call", call, "budget", budget, "steps", done, "substeps",
              [i["n_substeps"] for i in infos], "rounds", rounds, "occupancy", occ, flush=True)
        assert budget <= sum(done) < budget + len(ws)
        assert rounds > 0 and occ == 1.0
        for i, r in enumerate(alone):
            tot = {"n_cg": 0, "n_pcg": 0, "n_stagger": 0, "n_greenop": 0, "n_substeps": 0}
            one = None
            for _ in range(done[i]):
                one = r.rve_step_dissipation(dt[i])
                for key in tot:
                    tot[key] += one[key]
            split += tot["n_substeps"] - done[i]
            b = infos[i]
            for key, v in tot.items():
                assert b[key] == v, (call, i, key, b[key], v)
            sb, sa = batch.rve_get_scalars(slot=i), r.rve_get_scalars()
            for key in ("E", "Sigma", "T", "tau", "step"):
                assert sb[key] == sa[key], (call, i, key, sb[key], sa[key])
            if one is not None:
                for key in ("E", "Sigma", "D", "T", "Gamma"):
                    assert b[key] == one[key], (call, i, key)
            assert np.array_equal(batch.rve_get_field("phi", slot=i), r.rve_get_field("phi"))
            assert np.array_equal(batch.rve_get_field("hist", slot=i), r.rve_get_field("hist"))
    if case == "halving":
        assert split > 0, "no step split: the case does not reach the sub-step path"
    with pytest.raises(RuntimeError):
        batch._chk(mirve.lib.rve_run_budget(batch.h, mirve._dptr(np.array(dt)), None, -1, 0, None, None))


@pytest.mark.parametrize("case", ["plain", "halving"])
def test_run_budget_keep_resumes_steps_in_flight(case):
    """RVE_RUN_KEEP: budget calls of one step each leave the slots' steps in
    flight on the handle, and the next keep call resumes them.  A last keep
    call with max_steps = 1 lets every slot finish the step it is in.  Each
    slot then holds bitwise the state of the same RVE stepped alone as many
    times, and the work counters summed over the calls equal the lone RVE's
    (nothing counted twice, nothing dropped).  A read of the scalars in
    between returns the slots to their steps' starts; the next keep call
    begins those steps again."""
    from paper_2508_07424_amd import mirve
    ws = _three()
    kw = {}
    for w in ws:
        w.f = W.load_yy(2)
        if case == "halving":
            w.dtau = 2.0 * w.dtau
    if case == "halving":
        kw = dict(max_stagger=6)
    dt = [w.dtau for w in ws]
    keys = ("n_cg", "n_pcg", "n_stagger", "n_greenop", "n_substeps", "n_steps")
    batch = mirve.from_workloads(ws, **kw)
    tot = [dict.fromkeys(keys, 0) for _ in ws]

    def add(infos):
        for i, info in enumerate(infos):
            for key in keys:
                tot[i][key] += info[key]

    for call in range(6 if case == "plain" else 3):
        infos, st = batch.rve_run_budget(dt, 1, keep=True)
        assert st == [0, 0, 0], st
        add(infos)
        print("keep call", call, "steps", [i["n_steps"] for i in infos], flush=True)
    infos, last = batch.rve_run_budget(dt, 100, keep=True, max_steps=[1, 1, 1])
    add(infos)
    for i, w in enumerate(ws):
        # the lone RVE takes the same steps; a step that fails for good (the
        # halving case can exhaust its halvings) fails there too, with the
        # same work and the same state left behind
        r = mirve.from_workload(w, max_materials=4096, **kw)
        ref = dict.fromkeys(keys, 0)
        for k in range(tot[i]["n_steps"] + (0 if last[i] == 0 else 1)):
            one, s1 = r.rve_run_slots([w.dtau], [1])
            for key in keys:
                ref[key] += one[0][key]
        assert s1[0] == last[i], (i, s1, last)
        print("rve", i, "status", last[i], "batch", tot[i], "alone", ref, flush=True)
        assert tot[i] == ref, (i, tot[i], ref)
        sb, sa = batch.rve_get_scalars(slot=i), r.rve_get_scalars()
        for key in ("E", "Sigma", "T", "tau", "step"):
            assert sb[key] == sa[key], (i, key)
        assert np.array_equal(batch.rve_get_field("phi", slot=i), r.rve_get_field("phi"))
        assert np.array_equal(batch.rve_get_field("hist", slot=i), r.rve_get_field("hist"))
    if case != "plain":
        return
    # a read between keep calls drops the steps in flight: the slots restart
    # them, and stay on the lone RVEs' path
    nsteps = [t["n_steps"] for t in tot]
    for _ in range(3):
        batch.rve_get_scalars(slot=_)
    infos, _st = batch.rve_run_budget(dt, 1, keep=True)
    nsteps = [n + i["n_steps"] for n, i in zip(nsteps, infos)]
    for i in range(3):
        batch.rve_get_scalars(slot=i)
    infos, st = batch.rve_run_budget(dt, 100, keep=True, max_steps=[1, 1, 1])
    nsteps = [n + i["n_steps"] for n, i in zip(nsteps, infos)]
    for i, w in enumerate(ws):
        r = mirve.from_workload(w, max_materials=4096, **kw)
        for _ in range(nsteps[i]):
            r.rve_step_dissipation(w.dtau)
        assert batch.rve_get_scalars(slot=i)["step"] == r.rve_get_scalars()["step"]
        assert np.array_equal(batch.rve_get_field("phi", slot=i), r.rve_get_field("phi"))
