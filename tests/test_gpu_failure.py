"""Failure handling and resume, through the C ABI (conditions forced from the
host; every kernel runs to completion).

* An iteration cap that stops the solve early returns HOT_W_NOT_CONVERGED,
  and the step is still taken: it matches the oracle's step with the same
  cap.
* A non-finite incremental potential (one particle with the finite but huge
  deformation gradient 1e200 I, whose determinant overflows) returns
  HOT_E_NONFINITE and leaves the particles as they were.
* Resume: reading the particles after one step and starting a new scene from
  them gives the same second step as stepping on (positions, velocities, F
  and C within 1e-12; the new scene bins particles from the caller's order,
  so sums may run in another order).
"""
import numpy as np
import pytest

import hot_scenes as hs
import oracle as O
from test_gpu_parity import _hot, rel

pytestmark = pytest.mark.gpu


def _box(**kw):
    base = dict(seed=121, cells=(12, 12, 12), box_lo=(3, 3, 3), box_hi=(8, 9, 7), walls=2,
                levels=2, F_spread=0.1)
    base.update(kw)
    return hs.small_box(**base)


def test_iteration_cap_returns_warning_and_takes_the_step():
    hot = _hot()
    sc = _box()
    sc.max_iters = 1
    dt = O.time_step(sc)
    out, info = O.step(sc, dt=dt, max_iters=1)
    assert not info["converged"] and info["iters"] == 1
    g = hot.Scene.from_scene(sc)
    try:
        status = g.step(dt)
        res = g.read()
        st = dict(g.stats)
    finally:
        g.close()
    assert status == hot.HOT_W_NOT_CONVERGED
    assert st["iters"] == 1 and not st["converged"]
    assert st["E"] < st["E0"]
    assert rel(res["x"], out.x) < 1e-10
    assert rel(res["v"], out.v) < 1e-10


def test_nonfinite_energy_is_reported_and_state_kept():
    hot = _hot()
    sc = _box()
    sc.F[0] = np.eye(3) * 1e200
    g = hot.Scene.from_scene(sc)
    try:
        before = g.read()
        with pytest.raises(hot.HotError) as e:
            g.step()
        assert e.value.status == hot.HOT_E_NONFINITE
        after = g.read()
    finally:
        g.close()
    for f in ("x", "v", "F", "C"):
        assert np.array_equal(after[f], before[f]), f


def test_resume_from_read_particles():
    hot = _hot()
    sc = _box(seed=122)
    g = hot.Scene.from_scene(sc)
    try:
        g.step()
        mid = g.read()
        g.step()
        two = g.read()
    finally:
        g.close()
    r = sc.copy()
    r.x, r.v, r.F, r.C = mid["x"], mid["v"], mid["F"], mid["C"]
    h = hot.Scene.from_scene(r)
    try:
        h.step()
        res = h.read()
    finally:
        h.close()
    for f in ("x", "v", "F", "C"):
        d = rel(res[f], two[f])
        print(f"resume {f}: {d:.2e}")
        assert d < 1e-12, f
