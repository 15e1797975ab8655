"""Elastoplastic steps (von Mises return on the Hencky strain after the solve)
and the moving-sphere boundary, FP64 through the C ABI against the oracle.

Parity bar as for the elastic steps: every discrete decision of the solve
identical, positions, velocities and F within 1e-10 relative.  On top of it,
the GPU output must satisfy the return mapping's own invariant: every
particle's deviatoric Hencky strain on or inside the yield surface.
"""
import math

import numpy as np
import pytest

import hot_scenes as hs
import oracle as O
from test_gpu_parity import _hot, assert_dt_matches, rel

pytestmark = pytest.mark.gpu


def box_plastic():
    # F drawn with singular values in [0.9, 1.1]: the deviatoric Hencky
    # strain of most particles lies beyond a 100 Pa yield stress at E = 1e4
    sc = hs.small_box(seed=103, cells=(12, 12, 12), box_lo=(3, 3, 3), box_hi=(9, 8, 8),
                      walls=2, levels=2, F_spread=0.1)
    sc.materials[0]["yield_stress"] = 100.0
    return sc


def sphere_slab_small():
    # the sphere-impact scene at 24^3 cells: slab 12x5x12 cells, sphere of
    # radius 0.15 m one cell above it moving down at 3 m/s
    return hs.sphere_slab(n=24, slab=(12, 5, 12), y0=6, radius=0.15, levels=3, n_steps=2)


SCENES = {"box_plastic": box_plastic, "sphere_slab_small": sphere_slab_small}


def hencky_dev_norm(F):
    s = np.linalg.svd(F, compute_uv=False)
    eps = np.log(s)
    dev = eps - eps.mean(axis=1, keepdims=True)
    return np.linalg.norm(dev, axis=1)


@pytest.mark.parametrize("name", list(SCENES))
def test_plastic_steps_fp64(name):
    hot = _hot()
    sc = SCENES[name]()
    g = hot.Scene.from_scene(sc)
    mu, lam = O.lame(sc.materials[0]["E"], sc.materials[0]["nu"])
    ys = sc.materials[0]["yield_stress"]
    lim = math.sqrt(2.0 / 3.0) * ys / (2.0 * mu)
    cur = sc
    t = 0.0
    try:
        for k in range(sc.n_steps):
            dt = O.time_step(cur)
            out, info = O.step(cur, dt=dt, t=t)
            t += dt
            # the library takes its own time step (CFL rule over particle and
            # prescribed boundary speeds); after the first step the two sides
            # start from states that agree to the parity bar
            status = g.step(0.0)
            if k == 0:
                assert_dt_matches(g.stats["dt"], cur)
            else:
                assert abs(g.stats["dt"] - dt) <= 1e-10 * dt
            res = g.read()
            logi = g.debug_read(hot.DBG_LOG_INT, dtype=np.int32).reshape(-1, 4)
            log = info["log"]
            assert status in (0, 1)
            assert g.stats["iters"] == info["iters"], f"step {k}"
            assert list(logi[:, 0]) == log["alpha_halvings"]
            assert list(logi[:, 3]) == [sum(c) for c in log["cg"]]
            assert rel(res["x"], out.x) < 1e-10, f"step {k}"
            assert rel(res["v"], out.v) < 1e-10, f"step {k}"
            assert rel(res["F"], out.F) < 1e-10, f"step {k}"
            # return-mapping invariants on the GPU's own output
            nd = hencky_dev_norm(res["F"])
            assert np.all(nd <= lim * (1.0 + 1e-9))
            on_surface = np.count_nonzero(nd > lim * (1.0 - 1e-9))
            print(f"{name} step {k}: {on_surface} of {sc.n} particles on the yield surface, "
                  f"iters {info['iters']}")
            if name == "box_plastic":
                assert on_surface > sc.n // 2
            # each side continues from its own output
            cur = out
    finally:
        g.close()


def test_snow_clamp_steps_fp64():
    """Snow-type plastic flow (singular values of F clamped into
    [0.99, 1.001] after each step): two steps against the oracle, every
    decision identical, x, v, F within 1e-10; the GPU's output F has its
    singular values inside the interval and many particles sit on a bound."""
    hot = _hot()
    sc = hs.small_box(seed=104, cells=(12, 12, 12), box_lo=(3, 3, 3), box_hi=(9, 8, 8),
                      walls=2, levels=2, F_spread=0.05)
    sc.materials[0]["snow_clamp"] = (0.99, 1.001)
    sc.n_steps = 2
    g = hot.Scene.from_scene(sc)
    cur, t = sc, 0.0
    try:
        for k in range(sc.n_steps):
            dt = O.time_step(cur)
            out, info = O.step(cur, dt=dt, t=t)
            t += dt
            # the library takes its own time step (CFL rule over particle and
            # prescribed boundary speeds); after the first step the two sides
            # start from states that agree to the parity bar
            status = g.step(0.0)
            if k == 0:
                assert_dt_matches(g.stats["dt"], cur)
            else:
                assert abs(g.stats["dt"] - dt) <= 1e-10 * dt
            res = g.read()
            logi = g.debug_read(hot.DBG_LOG_INT, dtype=np.int32).reshape(-1, 4)
            log = info["log"]
            assert status in (0, 1)
            assert g.stats["iters"] == info["iters"], f"step {k}"
            assert list(logi[:, 0]) == log["alpha_halvings"]
            assert list(logi[:, 3]) == [sum(c) for c in log["cg"]]
            assert rel(res["x"], out.x) < 1e-10, f"step {k}"
            assert rel(res["v"], out.v) < 1e-10, f"step {k}"
            assert rel(res["F"], out.F) < 1e-10, f"step {k}"
            s = np.linalg.svd(res["F"], compute_uv=False)
            assert s.min() >= 0.99 - 1e-12 and s.max() <= 1.001 + 1e-12
            on_bound = np.count_nonzero(np.any((np.abs(s - 0.99) < 1e-12) |
                                               (np.abs(s - 1.001) < 1e-12), axis=1))
            print(f"snow step {k}: {on_bound} of {sc.n} particles on a clamp bound, "
                  f"iters {info['iters']}")
            assert on_bound > sc.n // 2
            cur = out
    finally:
        g.close()


def test_snow_clamp_step_mixed():
    """The snow clamp after a mixed-precision solve: the clamp runs on the
    FP64 particle state, so the GPU's F keeps its singular values inside
    [0.99, 1.001]; at the same CN tolerance as the FP64 oracle, eps = 1e-10,
    x and v agree within 1e-6 relative."""
    hot = _hot()
    sc = hs.small_box(seed=104, cells=(12, 12, 12), box_lo=(3, 3, 3), box_hi=(9, 8, 8),
                      walls=2, levels=2, F_spread=0.05)
    sc.materials[0]["snow_clamp"] = (0.99, 1.001)
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
    assert status == 0 and stats["converged"] and rinfo["converged"]
    s = np.linalg.svd(res["F"], compute_uv=False)
    assert s.min() >= 0.99 - 1e-12 and s.max() <= 1.001 + 1e-12
    mx, mv = rel(res["x"], ref.x), rel(res["v"], ref.v)
    print(f"snow mixed eps=1e-10: iterations mixed {stats['iters']}, fp64 {rinfo['iters']}; "
          f"mixed vs fp64 oracle x {mx:.2e} v {mv:.2e}")
    assert mx <= 1e-6 and mv <= 1e-6
