"""Serving: continuous batching of independent scenes through hot_batch_*.

A scene's result must not depend on what else is resident, nor on how it is
served: each request's particles after its steps, run inside a stream of
overlapping requests (scenes created by the batch's slot threads from its
device pool, V-cycles launched as captured HIP graphs, or scenes created by
the loop and stepped eagerly), are bit-identical to the same scene stepped
alone and eagerly (every kernel of the step is deterministic: fixed-order
reductions, no floating-point atomics across waves).  A captured V-cycle
graph is replayed at every quasi-Newton iteration of a step, with the
iteration's eager kernels and host synchronisations between replays, and the
step must equal the eager step bit for bit.  Admission must respect the HBM
budget, and a request larger than the budget is refused.
"""
import numpy as np
import pytest

import hot_scenes as hs

pytestmark = pytest.mark.gpu

N_REQ = 10
STEPS = 3


def _mods():
    from paper_1911_07913_amd import hot, serving
    hot.lib()
    return hot, serving


def small_requests():
    return [hs.serving_scene(i, seed_base=4500, n_min=2000, n_max=24000) for i in range(N_REQ)]


def alone(hot, sc, precision, smoother=0):
    g = hot.Scene.from_scene(sc, precision=precision, smoother=smoother)
    try:
        for _ in range(STEPS):
            g.step()
        return g.read()
    finally:
        g.close()


@pytest.mark.parametrize("submit,graph", [(True, True), (False, False)],
                         ids=["submitted-graph", "loop-created-eager"])
@pytest.mark.parametrize("precision,smoother", [(0, 0), (1, 0), (1, 1)],
                         ids=["fp64", "mixed", "mixed-gauss-seidel"])
def test_results_identical_alone_and_in_the_mix(precision, smoother, submit, graph):
    hot, serving = _mods()
    reqs = small_requests()
    ref = [alone(hot, sc, precision, smoother) for sc in reqs]
    got = {}

    def collect(k, scene):
        got[k] = scene.read()

    arrivals = serving.poisson_arrivals(N_REQ, rate=200.0, seed=7)
    records, summary, trace = serving.serve(reqs, arrivals, budget_bytes=8 << 30, max_slots=4,
                                            precision=precision, n_steps=STEPS, collect=collect,
                                            smoother=smoother, submit=submit, graph=graph)
    print(summary, trace)
    assert len(records) == N_REQ and summary["failed"] == 0
    assert trace["peak_resident"] > 1, "requests never overlapped"
    for r in records:
        assert r["steps"] == STEPS and r["status"] >= 0
    for k in range(N_REQ):
        for f in ("x", "v", "F", "C"):
            assert np.array_equal(got[k][f], ref[k][f]), f"request {k} field {f}"


def test_admission_respects_budget():
    hot, serving = _mods()
    reqs = small_requests()[:6]
    need = [hot.footprint(hot.params_of(sc, hot.HOT_MIXED), sc.x) for sc in reqs]
    budget = int(max(need) * 1.5)
    records, summary, trace = serving.serve(reqs, np.zeros(len(reqs)), budget_bytes=budget,
                                            max_slots=8, precision=hot.HOT_MIXED, n_steps=1)
    assert len(records) == len(reqs) and summary["failed"] == 0
    assert trace["peak_reserved_bytes"] <= budget
    # a scene's working set stays within its admission estimate
    for sc in reqs[:2]:
        g = hot.Scene.from_scene(sc, precision=hot.HOT_MIXED)
        g.step()
        live, est = g.memory()
        g.close()
        assert live <= est, (live, est)


def test_oversized_request_is_refused():
    hot, serving = _mods()
    sc = small_requests()[0]
    b = hot.Batch(1 << 20, 2)
    g = hot.Scene.from_scene(sc)
    try:
        assert b.add(g, 1, 0) is False
        done, resident = b.poll()
        assert done == [] and resident == 0
    finally:
        b.close()
        g.close()


@pytest.mark.parametrize("precision,smoother", [(0, 0), (1, 0), (0, 1), (1, 1)],
                         ids=["fp64", "mixed", "fp64-gauss-seidel", "mixed-gauss-seidel"])
def test_graph_vcycle_steps_equal_eager_steps(precision, smoother):
    """Three steps of a three-level scene with the V-cycle captured as a HIP
    graph (recaptured at every step, replayed at every iteration) against the
    same steps run eagerly: identical decisions and bit-identical particles."""
    hot, _ = _mods()
    sc = hs.twisting_bars(side=4, length=24, n_steps=3)
    sc.mg_levels = 3
    out = []
    for graph in (0, 1):
        g = hot.Scene.from_scene(sc, precision=precision, smoother=smoother, graph=graph)
        try:
            its = []
            for _ in range(3):
                g.step()
                its.append((g.stats["iters"], g.stats["cg_iters_total"]))
            out.append((its, g.read()))
        finally:
            g.close()
    (ie, re_), (ig, rg) = out
    print("eager", ie, "graph", ig)
    assert ie == ig
    for f in ("x", "v", "F", "C"):
        assert np.array_equal(re_[f], rg[f]), f


def test_more_slots_than_grid_tickets():
    """Twenty slots of scenes whose coarsest levels use the grid-barrier
    solve: at most 16 such solves run at once (the rest wait for a ticket),
    and every result is still bit-identical to the scene stepped alone."""
    hot, serving = _mods()
    reqs = [hs.serving_scene(i, seed_base=4600, n_min=20000, n_max=40000) for i in range(24)]
    for sc in reqs:
        sc.mg_levels = 2  # coarsest levels of several hundred rows: grid solves
    ref = [alone(hot, sc, 0) for sc in reqs]
    got = {}

    def collect(k, scene):
        got[k] = scene.read()

    records, summary, trace = serving.serve(reqs, np.zeros(len(reqs)), budget_bytes=32 << 30,
                                            max_slots=20, precision=0, n_steps=STEPS,
                                            collect=collect)
    print(summary, trace)
    assert summary["failed"] == 0 and trace["peak_resident"] > 16
    for k in range(len(reqs)):
        for f in ("x", "v"):
            assert np.array_equal(got[k][f], ref[k][f]), f"request {k} field {f}"


def test_submitted_request_with_invalid_scene_comes_back_with_its_error():
    """A scene description that fails validation is refused on the slot
    thread: its result carries the status and message and no scene, and the
    batch serves the next request normally."""
    hot, serving = _mods()
    good = small_requests()[0]
    bad = small_requests()[1]
    bad.v = bad.v.copy()
    bad.v[3, 1] = np.nan
    b = hot.Batch(8 << 30, 2)
    try:
        args = [hot.SceneArgs(hot.params_of(sc), sc.x, sc.v, sc.F, sc.C, sc.vol0, sc.mat_id,
                              sc.materials, sc.bcs) for sc in (bad, good)]
        assert b.submit(args[0], 1, 0) and b.submit(args[1], 1, 1)
        got = {}
        for _ in range(200):
            done, resident = b.poll(wait_ms=50)
            for r in done:
                got[r["tag"]] = r
            if len(got) == 2:
                break
        assert got[0]["status"] == hot.HOT_E_INVALID and not got[0]["scene"]
        assert "finite" in got[0]["message"]
        assert got[1]["status"] == 0 and got[1]["steps"] == 1 and got[1]["scene"]
        hot.Scene.adopt(got[1]["scene"], args[1].n, args[1].params).close()
    finally:
        b.close()
