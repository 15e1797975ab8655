"""A large level against the oracle.

Levels of at least 16,384 rows run the smoothing and residual sweeps as
work-groups over runs of 16 consecutive rows with the iterate window staged
in LDS (the form the 1.5M-particle bars spend most of their V-cycle time
in); smaller levels one row per wave.  This scene is a one-cell-thick slab of
128 x 128 cells with two particles per cell (the lattice sub-positions
(1/4, 1/4, 1/4) and (3/4, 3/4, 3/4), volume dx^3/2 each), so that its fine
level holds 68,118 rows while the oracle still builds it in seconds.  The
V-cycle, the level-0 product and a full FP64 step (the library choosing its
own time step) are compared with the oracle at the usual bars: V-cycle
1e-11, every discrete decision identical, x, v, F within 1e-10.
"""
import numpy as np
import pytest

import hot_scenes as hs
import oracle as O
from test_gpu_parity import _hot, assert_dt_matches, oracle_prepare, rel

pytestmark = pytest.mark.gpu

RUN_MIN = 16384


def slab_two_per_cell():
    sc = hs.small_box(seed=205, cells=(136, 136, 8), box_lo=(3, 3, 3), box_hi=(131, 131, 4),
                      dx=0.01, walls=2, levels=3)
    keep = np.zeros(sc.n, dtype=bool)
    keep[0::8] = True
    keep[7::8] = True
    for f in ("x", "v", "F", "C", "vol0", "mat_id"):
        setattr(sc, f, getattr(sc, f)[keep].copy())
    sc.vol0 *= 4.0
    return sc


def test_large_level_vcycle_and_product():
    hot = _hot()
    sc = slab_two_per_cell()
    dt = O.time_step(sc)
    st, hz = oracle_prepare(sc, dt)
    n = st.lev0.n
    print(f"slab: {sc.n} particles, level sizes {[l.n for l in hz.levels]}")
    assert n >= RUN_MIN
    g = hot.Scene.from_scene(sc)
    try:
        g.debug_prepare(0.0)
        nodes = g.debug_read(hot.DBG_LEVEL_NODES, 0, dtype=np.int32)
        assert np.array_equal(nodes.astype(np.int64), hz.levels[0].lin)
        rng = np.random.Generator(np.random.PCG64(9))
        x = rng.normal(size=3 * n) * hz.free[0]
        assert rel(g.debug_apply(3, x), hz.A[0] @ x) < 1e-12
        u = g.debug_apply(0, x)
        assert rel(u, O.vcycle(hz, x, sweeps=sc.smoother_sweeps)) < 1e-11
        # the same cycle with one row per wave on every level, bit for bit
        try:
            hot.debug_set(hot.SET_MULTIROW_MIN, 1 << 30)
            u1 = g.debug_apply(0, x)
        finally:
            hot.debug_set(hot.SET_MULTIROW_MIN, -1)
        assert np.array_equal(u, u1)
    finally:
        g.close()


def test_large_level_full_step_fp64():
    hot = _hot()
    sc = slab_two_per_cell()
    dt = O.time_step(sc)
    out, info = O.step(sc, dt=dt)
    g = hot.Scene.from_scene(sc)
    try:
        status = g.step(0.0)
        assert_dt_matches(g.stats["dt"], sc)
        res = g.read()
        logi = g.debug_read(hot.DBG_LOG_INT, dtype=np.int32).reshape(-1, 4)
        stats = dict(g.stats)
    finally:
        g.close()
    log = info["log"]
    print(f"slab step: {stats['iters']} iterations, level 0 {stats['n_nodes']} rows")
    assert stats["n_nodes"] >= RUN_MIN
    assert status == 0 and info["converged"]
    assert stats["iters"] == info["iters"]
    assert list(logi[:, 0]) == log["alpha_halvings"]
    assert list(logi[:, 2]) == log["fallback"]
    assert list(logi[: len(log["skipped"]), 1]) == log["skipped"]
    assert list(logi[:, 3]) == [sum(c) for c in log["cg"]]
    assert rel(res["x"], out.x) < 1e-10
    assert rel(res["v"], out.v) < 1e-10
    assert rel(res["F"], out.F) < 1e-10
