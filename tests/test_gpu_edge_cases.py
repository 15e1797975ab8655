"""Degenerate and ragged inputs through the C ABI against the oracle, each
stepped once in FP64 with every discrete decision of the solve identical
and x, v, F within 1e-10:

* one stretched particle alone in the grid (27 active nodes);
* a box in which one cell holds 29 particles, so that one cell column spans
  four 8-particle assembly chunks (the last partial), plus one isolated
  particle away from the box (a second, disconnected node island);
* a box with a third of its particles on the planes where the base cell
  changes (near-tie binning decisions, and nodes left without mass);
* fixed-corotated and Neo-Hookean particles in one box, with particles at
  both ends of the valid region on every axis.
"""
import numpy as np
import pytest

import hot_scenes as hs
import oracle as O
from test_gpu_parity import _hot, rel

pytestmark = pytest.mark.gpu


def _take(sc, idx):
    for f in ("x", "v", "F", "C", "vol0", "mat_id"):
        setattr(sc, f, np.ascontiguousarray(getattr(sc, f)[idx]))
    return sc


def _append(sc, x, v):
    k = x.shape[0]
    sc.x = np.concatenate([sc.x, x])
    sc.v = np.concatenate([sc.v, v])
    sc.F = np.concatenate([sc.F, np.repeat(np.eye(3)[None], k, 0)])
    sc.C = np.concatenate([sc.C, np.zeros((k, 3, 3))])
    sc.vol0 = np.concatenate([sc.vol0, np.full(k, sc.vol0[0])])
    sc.mat_id = np.concatenate([sc.mat_id, np.zeros(k, np.int32)])
    return sc


def single_particle():
    sc = hs.small_box(seed=141, cells=(10, 10, 10), box_lo=(4, 4, 4), box_hi=(5, 5, 5), levels=2)
    sc = _take(sc, [0])
    sc.F[0] = np.diag([1.2, 0.9, 1.1])  # stressed, so the solve has work to do
    return sc


def crowded_cell_and_island():
    sc = hs.small_box(seed=142, cells=(14, 14, 14), box_lo=(3, 3, 3), box_hi=(7, 7, 7), walls=2,
                      levels=2, F_spread=0.1)
    rng = np.random.Generator(np.random.PCG64(143))
    dx = sc.dx
    # 21 more particles whose base cell is (5, 5, 5): x / dx in [5.55, 6.45)
    crowd = (5.55 + 0.9 * rng.random((21, 3))) * dx
    island = np.array([[10.2, 10.3, 4.6]]) * dx
    xs = np.concatenate([crowd, island])
    vs = 0.1 * rng.normal(size=xs.shape)
    return _append(sc, xs, vs)


def on_cell_faces():
    """A box with a third of its particles moved onto the planes where the
    base cell changes (x / dx - 1/2 an integer, up to rounding of the
    products): the binning decision there is a near tie, taken with the same
    IEEE operations on both sides."""
    sc = hs.small_box(seed=144, cells=(12, 12, 12), box_lo=(3, 3, 3), box_hi=(8, 8, 8), walls=2,
                      levels=2, F_spread=0.05)
    k = np.arange(0, sc.n, 3)
    a = k % 3
    t = sc.x[k, a] / sc.dx
    sc.x[k, a] = (np.round(t - 0.5) + 0.5) * sc.dx
    return sc


def mixed_models_at_region_edges():
    """Fixed-corotated and Neo-Hookean particles side by side (the material
    branch diverges inside a wave), plus particles at both ends of the valid
    region on each axis (x / dx exactly 2 and exactly cells - 3)."""
    sc = hs.small_box(seed=145, cells=(12, 12, 12), box_lo=(3, 3, 3), box_hi=(8, 8, 8), walls=None,
                      levels=2, n_mats=2, E=2e4, F_spread=0.05)
    sc.materials[1]["model"] = hs.NEOHOOKEAN
    lo, hi = 2.0 * sc.dx, (sc.grid_cells[0] - 3) * sc.dx
    edge = np.array([[lo, 5.5 * sc.dx, 5.5 * sc.dx], [hi, 5.5 * sc.dx, 5.5 * sc.dx],
                     [5.5 * sc.dx, lo, 5.5 * sc.dx], [5.5 * sc.dx, hi, 5.5 * sc.dx],
                     [5.5 * sc.dx, 5.5 * sc.dx, lo], [5.5 * sc.dx, 5.5 * sc.dx, hi]])
    return _append(sc, edge, np.zeros_like(edge))


CASES = {"single_particle": single_particle, "crowded_cell_and_island": crowded_cell_and_island,
         "on_cell_faces": on_cell_faces, "mixed_models_at_region_edges": mixed_models_at_region_edges}


SMOOTHERS = {"l1jacobi": 0, "sgs": 1}


@pytest.mark.parametrize("smoother", list(SMOOTHERS))
@pytest.mark.parametrize("name", list(CASES))
def test_degenerate_step_fp64(name, smoother):
    """FP64 step with either smoother (tiny levels leave Gauss-Seidel colours
    without rows)."""
    hot = _hot()
    sc = CASES[name]()
    dt = O.time_step(sc)
    out, info = O.step(sc, dt=dt, smoother=smoother)
    g = hot.Scene.from_scene(sc, smoother=SMOOTHERS[smoother])
    try:
        status = g.step(dt)
        res = g.read()
        logi = g.debug_read(hot.DBG_LOG_INT, dtype=np.int32).reshape(-1, 4)
        stats = dict(g.stats)
    finally:
        g.close()
    log = info["log"]
    print(f"{name} ({smoother}): n = {sc.n}, {stats['iters']} iterations")
    assert status == 0 and info["converged"]
    assert stats["iters"] == info["iters"]
    assert list(logi[:, 0]) == log["alpha_halvings"]
    assert list(logi[:, 2]) == log["fallback"]
    assert list(logi[: len(log["skipped"]), 1]) == log["skipped"]
    assert list(logi[:, 3]) == [sum(c) for c in log["cg"]]
    assert rel(res["x"], out.x) < 1e-10
    assert rel(res["v"], out.v) < 1e-10
    assert rel(res["F"], out.F) < 1e-10


@pytest.mark.parametrize("name", list(CASES))
def test_degenerate_step_mixed(name):
    """Mixed precision (BF16 blocks, FP32 V-cycle) on the same inputs against
    the FP64 oracle at the same CN tolerance, eps = 1e-10, where every case
    converges with the default smoother: x and v within 1e-6 relative."""
    hot = _hot()
    sc = CASES[name]()
    sc.tol = 1e-10
    dt = O.time_step(sc)
    ref, rinfo = O.step(sc, dt=dt)
    g = hot.Scene.from_scene(sc, precision=hot.HOT_MIXED)
    try:
        status = g.step(dt)
        res = g.read()
        stats = dict(g.stats)
    finally:
        g.close()
    mx, mv, mF = rel(res["x"], ref.x), rel(res["v"], ref.v), rel(res["F"], ref.F)
    print(f"{name} eps=1e-10: iterations mixed {stats['iters']}, fp64 {rinfo['iters']}; "
          f"mixed vs fp64 oracle: x {mx:.2e} v {mv:.2e} F {mF:.2e}")
    assert status == 0 and stats["converged"] and rinfo["converged"]
    assert mx <= 1e-6 and mv <= 1e-6 and mF <= 1e-6
