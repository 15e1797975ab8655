"""The paper's Newton-Krylov baselines (Alg. 1) on the library's kernels,
against the oracle through the C ABI: PN-PCG (CG with the scalar diagonal as
preconditioner) and PN-MGPCG (CG preconditioned by one V-cycle of the
hierarchy rebuilt from each Newton iteration's Hessian), both with the
adaptive inexact tolerance of Sec. 5.3 and HOT's line search.

Bar as for HOT: every discrete decision (Newton iterations, step-length
halvings, CG iterations of every linear solve) identical, x, v, F within
1e-10 relative.  Scenes: two boxes (single- and three-material) and the
three-material twisted bar of the varying-stiffness experiment at a soft and
a stiff middle (E = 1e5 and 1e8 Pa).
"""
import numpy as np
import pytest

import hot_scenes as hs
import oracle as O
from test_gpu_parity import SCENES, _hot, assert_dt_matches, rel

pytestmark = pytest.mark.gpu

CASES = {
    "box_walls_fcr": SCENES["box_walls_fcr"],
    "box_nh_3mat": SCENES["box_nh_3mat"],
    "stiffness_bar_1e5": lambda: hs.stiffness_bar(E_mid=1e5, side=4, length=48),
    "stiffness_bar_1e8": lambda: hs.stiffness_bar(E_mid=1e8, side=4, length=48),
}
SOLVERS = {"pn-pcg": 1, "pn-mgpcg": 2}


@pytest.mark.parametrize("solver", list(SOLVERS))
@pytest.mark.parametrize("name", list(CASES))
def test_newton_krylov_step_matches_oracle(name, solver):
    hot = _hot()
    sc = CASES[name]()
    dt = O.time_step(sc)
    out, info = O.step(sc, dt=dt, solver=solver)
    g = hot.Scene.from_scene(sc, solver=SOLVERS[solver])
    try:
        status = g.step(0.0)
        assert_dt_matches(g.stats["dt"], sc)
        res = g.read()
        logi = g.debug_read(hot.DBG_LOG_INT, dtype=np.int32).reshape(-1, 4)
        stats = dict(g.stats)
    finally:
        g.close()
    log = info["log"]
    print(f"{name} {solver}: {stats['iters']} Newton iterations, CG {list(logi[:, 3])} "
          f"(oracle {log['cg']})")
    assert status == 0 and info["converged"] and stats["converged"]
    assert stats["iters"] == info["iters"]
    assert list(logi[:, 0]) == log["alpha_halvings"]
    assert list(logi[:, 3]) == log["cg"]
    assert stats["cg_iters_total"] == sum(log["cg"])
    assert rel(res["x"], out.x) < 1e-10
    assert rel(res["v"], out.v) < 1e-10
    assert rel(res["F"], out.F) < 1e-10
