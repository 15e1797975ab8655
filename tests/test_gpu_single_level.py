"""The single-level configuration (mg_levels = 1: the V-cycle reduces to the
Jacobi-preconditioned CG on level 0, stopped at relative 1/2, i.e. L-BFGS
with an inexact Hessian solve as initial inverse Hessian) next to HOT with
three levels, on a stretched box (initial singular values drawn from
[0.7, 1.3], the convergence set-up of Sec. 8), through the C ABI against
the oracle: every discrete decision of the solve identical and x, v, F
within 1e-10.
"""
import numpy as np
import pytest

import hot_scenes as hs
import oracle as O
from test_gpu_parity import _hot, assert_dt_matches, rel

pytestmark = pytest.mark.gpu


def _stretched_box(levels):
    return hs.small_box(seed=131, cells=(12, 12, 12), box_lo=(3, 3, 3), box_hi=(9, 9, 9), walls=2,
                        levels=levels, F_spread=0.3, E=1e5, tol=1e-6, history=5)


@pytest.mark.parametrize("levels", [1, 3])
def test_stretched_box_step(levels):
    hot = _hot()
    sc = _stretched_box(levels)
    dt = O.time_step(sc)
    out, info = O.step(sc, dt=dt)
    g = hot.Scene.from_scene(sc)
    try:
        status = g.step(dt)
        res = g.read()
        logi = g.debug_read(hot.DBG_LOG_INT, dtype=np.int32).reshape(-1, 4)
        stats = dict(g.stats)
    finally:
        g.close()
    log = info["log"]
    print(f"levels {levels}: {stats['iters']} iterations, "
          f"{sum(sum(c) for c in log['cg'])} coarse CG iterations")
    assert status == 0 and info["converged"]
    assert stats["iters"] == info["iters"]
    assert list(logi[:, 0]) == log["alpha_halvings"]
    assert list(logi[:, 2]) == log["fallback"]
    assert list(logi[: len(log["skipped"]), 1]) == log["skipped"]
    assert list(logi[:, 3]) == [sum(c) for c in log["cg"]]
    assert rel(res["x"], out.x) < 1e-10
    assert rel(res["v"], out.v) < 1e-10
    assert rel(res["F"], out.F) < 1e-10


# The bench's stretched-box workload at reduced size (6^3 cells of particles,
# one diagonal F in [0.7, 1.3] for the box, no gravity, no walls, CN
# tolerance 1e-7) under the three solver configurations the bench compares.
STRETCHED = {
    "lbfgs_h": (dict(levels=1, sweeps=1), "l1jacobi", 0),
    "hot_sgs": (dict(levels=3, sweeps=1), "sgs", 1),
    "hot_l1jacobi": (dict(levels=3, sweeps=5), "l1jacobi", 0),
}


@pytest.mark.parametrize("case", list(STRETCHED))
def test_stretched_box_diagonal_F(case):
    hot = _hot()
    kw, smoother, hs_smoother = STRETCHED[case]
    sc = hs.stretched_box(side=6, margin=3, levels=kw["levels"])
    sc.smoother_sweeps = kw["sweeps"]
    out, info = O.step(sc, smoother=smoother)
    g = hot.Scene.from_scene(sc, smoother=hs_smoother)
    try:
        status = g.step(0.0)  # the library's own CFL time step
        res = g.read()
        logi = g.debug_read(hot.DBG_LOG_INT, dtype=np.int32).reshape(-1, 4)
        stats = dict(g.stats)
    finally:
        g.close()
    log = info["log"]
    print(f"{case}: {stats['iters']} iterations (oracle {info['iters']})")
    assert status == 0 and info["converged"]
    assert_dt_matches(stats["dt"], sc)
    assert stats["iters"] == info["iters"]
    assert list(logi[:, 0]) == log["alpha_halvings"]
    assert list(logi[:, 2]) == log["fallback"]
    assert list(logi[:, 3]) == [sum(c) for c in log["cg"]]
    assert rel(res["x"], out.x) < 1e-10
    assert rel(res["v"], out.v) < 1e-10
    assert rel(res["F"], out.F) < 1e-10
