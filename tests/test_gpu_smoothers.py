"""The V-cycle smoothers on the HIP path, through the C ABI, against the
oracle.  The other GPU tests run the default l1 block-Jacobi smoother; this
file covers the paper's coloured symmetric block Gauss-Seidel
(HOT_SMOOTH_SGS):

* rows ordered by colour (grid coordinate mod 3 per axis, ascending row
  index within a colour), bit-exact at every smoothed level;
* one V-cycle element by element (FP64 sums in another order);
* full FP64 steps with every discrete decision of the solve (halvings,
  fallbacks, skipped pairs, coarse-PCG counts, iteration count) identical and
  x, v, F within 1e-10;
* mixed precision with either smoother: the V-cycle differs from the FP64
  oracle by the BF16 block rounding only, and a step converged to a tight
  tolerance lands on the FP64 oracle's step.
"""
import numpy as np
import pytest

import oracle as O
from test_gpu_parity import SCENES, _grip_scene, _hot, oracle_prepare, rel

pytestmark = pytest.mark.gpu

SMOOTHERS = {"l1jacobi": 0, "sgs": 1}


def _scene(name):
    return _grip_scene() if name == "bars_small_grips" else SCENES[name]()


@pytest.fixture(scope="module", params=list(SCENES))
def prepared_sgs(request):
    hot = _hot()
    sc = _scene(request.param)
    dt = O.time_step(sc)
    st, hz = oracle_prepare(sc, dt)
    g = hot.Scene.from_scene(sc, smoother=hot.HOT_SMOOTH_SGS)
    g.debug_prepare(dt)
    yield request.param, sc, dt, st, hz, g
    g.close()


def test_color_rows_bit_exact(prepared_sgs):
    hot = _hot()
    name, sc, dt, st, hz, g = prepared_sgs
    for m in range(len(hz.levels) - 1):
        lev = hz.levels[m]
        want = np.lexsort((np.arange(lev.n), O.node_colors(lev)))
        got = g.debug_read(hot.DBG_LEVEL_COLOR_ROWS, m, dtype=np.int32)
        assert np.array_equal(got, want), f"level {m}"


def test_vcycle_sgs(prepared_sgs):
    name, sc, dt, st, hz, g = prepared_sgs
    n = st.lev0.n
    rng = np.random.Generator(np.random.PCG64(15))
    for k in range(2):
        b = rng.normal(size=3 * n) * hz.free[0]
        uo = O.vcycle(hz, b, sweeps=sc.smoother_sweeps, smoother="sgs")
        ug = g.debug_apply(0, b)
        assert rel(ug, uo) < 1e-11, f"cycle {k}"
        assert np.all(ug[hz.free[0] == 0] == 0.0)


@pytest.mark.parametrize("name", list(SCENES))
def test_full_step_sgs_fp64(name):
    hot = _hot()
    sc = _scene(name)
    dt = O.time_step(sc)
    out, info = O.step(sc, dt=dt, smoother="sgs")
    g = hot.Scene.from_scene(sc, smoother=hot.HOT_SMOOTH_SGS)
    try:
        g.step(dt)
        res = g.read()
        logi = g.debug_read(hot.DBG_LOG_INT, dtype=np.int32).reshape(-1, 4)
        stats = dict(g.stats)
    finally:
        g.close()
    log = info["log"]
    print(f"{name}: Gauss-Seidel iterations {stats['iters']}")
    assert stats["iters"] == info["iters"]
    assert list(logi[:, 0]) == log["alpha_halvings"]
    assert list(logi[:, 2]) == log["fallback"]
    assert list(logi[: len(log["skipped"]), 1]) == log["skipped"]
    assert list(logi[:, 3]) == [sum(c) for c in log["cg"]]
    assert rel(res["x"], out.x) < 1e-10
    assert rel(res["v"], out.v) < 1e-10
    assert rel(res["F"], out.F) < 1e-10


@pytest.mark.parametrize("smoother", list(SMOOTHERS))
def test_mixed_vcycle_and_tight_step(smoother):
    hot = _hot()
    sc = _scene("box_walls_fcr")
    dt = O.time_step(sc)
    st, hz = oracle_prepare(sc, dt)
    g = hot.Scene.from_scene(sc, precision=hot.HOT_MIXED, smoother=SMOOTHERS[smoother])
    try:
        g.debug_prepare(dt)
        rng = np.random.Generator(np.random.PCG64(16))
        b = rng.normal(size=3 * st.lev0.n) * hz.free[0]
        err = rel(g.debug_apply(0, b), O.vcycle(hz, b, sweeps=sc.smoother_sweeps, smoother=smoother))
        print(f"mixed {smoother} V-cycle relative error {err:.2e}")
        assert err < 2e-2
    finally:
        g.close()
    sc.tol = 1e-10
    out, info = O.step(sc, dt=dt, smoother=smoother)
    g = hot.Scene.from_scene(sc, precision=hot.HOT_MIXED, smoother=SMOOTHERS[smoother])
    try:
        status = g.step(dt)
        res = g.read()
        stats = dict(g.stats)
    finally:
        g.close()
    assert status == 0 and stats["converged"] and info["converged"]
    assert rel(res["x"], out.x) < 1e-9
    assert rel(res["v"], out.v) < 1e-8
