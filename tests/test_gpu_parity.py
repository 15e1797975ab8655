"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Integer work (binning permutation, active nodes per level, block patterns,
constrained DOFs) must match bit for bit.  Floating-point fields are compared
element by element: intermediate kernels to 1e-12 relative (FP64 sums in a
different order), and the full step to the 1e-10 relative bound on positions
and velocities, with every discrete decision of the solve (step-length
halvings, descent fallbacks, skipped secant pairs, coarse-PCG iteration
counts, iteration count) identical.
"""
import math

import numpy as np
import pytest

import hot_scenes as hs
import oracle as O

pytestmark = pytest.mark.gpu


def _hot():
    from paper_1911_07913_amd import hot
    hot.lib()
    return hot


def unpack_pattern(words, n):
    bits = np.unpackbits(words.view(np.uint8).reshape(n, 16), axis=1, bitorder="little")
    return bits[:, :125].astype(bool)


def rel(a, b):
    d = np.abs(np.asarray(a) - np.asarray(b)).max() if np.size(a) else 0.0
    s = np.abs(np.asarray(b)).max() if np.size(b) else 1.0
    return d / (s if s > 0 else 1.0)


SCENES = {
    "box_walls_fcr": lambda: hs.small_box(seed=101, cells=(12, 12, 12), box_lo=(3, 3, 3),
                                          box_hi=(8, 9, 7), walls=2, levels=2, F_spread=0.1),
    "box_nh_3mat": lambda: hs.small_box(seed=102, cells=(14, 12, 12), box_lo=(3, 3, 3),
                                        box_hi=(11, 8, 8), walls=2, levels=3, model=1,
                                        n_mats=3, E=3e4, nu=0.4),
    "bars_small_grips": lambda: hs.twisting_bars(side=4, length=24, n_steps=1),
}


def _grip_scene():
    sc = SCENES["bars_small_grips"]()
    sc.mg_levels = 3
    return sc


def oracle_prepare(sc, dt):
    st = O.prepare(sc, dt)
    H0, nbr0 = O.hessian_slots(st)
    hz = O.build_hierarchy(st, H0, nbr0, sc.mg_levels)
    return st, hz


@pytest.fixture(scope="module", params=list(SCENES))
def prepared(request):
    hot = _hot()
    sc = _grip_scene() if request.param == "bars_small_grips" else SCENES[request.param]()
    dt = O.time_step(sc)
    st, hz = oracle_prepare(sc, dt)
    g = hot.Scene.from_scene(sc)
    g.debug_prepare(dt)
    yield request.param, sc, dt, st, hz, g
    g.close()


def test_binning_permutation_bit_exact(prepared):
    hot = _hot()
    name, sc, dt, st, hz, g = prepared
    _, perm = O.bin_particles(sc)
    gp = g.debug_read(hot.DBG_PERM, dtype=np.int32)
    assert np.array_equal(gp, perm)


def test_levels_patterns_and_constraints_bit_exact(prepared):
    hot = _hot()
    name, sc, dt, st, hz, g = prepared
    for m, lev in enumerate(hz.levels):
        nodes = g.debug_read(hot.DBG_LEVEL_NODES, m, dtype=np.int32)
        assert np.array_equal(nodes.astype(np.int64), lev.lin), f"level {m} nodes"
        pat = unpack_pattern(g.debug_read(hot.DBG_LEVEL_PATTERN, m, dtype=np.uint32), lev.n)
        assert np.array_equal(pat, hz.patterns[m]), f"level {m} pattern"
        free = g.debug_read(hot.DBG_LEVEL_FREE, m, dtype=np.uint8)
        assert np.array_equal(free.astype(float), hz.free[m]), f"level {m} free DOFs"
    fixed = g.debug_read(hot.DBG_NODE_FIXED, dtype=np.int32)
    assert np.array_equal(fixed.astype(bool), st.fixed)


def test_p2g_fields(prepared):
    hot = _hot()
    name, sc, dt, st, hz, g = prepared
    assert rel(g.debug_read(hot.DBG_NODE_MASS), st.m) < 1e-13
    assert rel(g.debug_read(hot.DBG_NODE_VSTAR).reshape(-1, 3), st.vstar) < 1e-12
    assert rel(g.debug_read(hot.DBG_NODE_XI), st.xi) < 1e-13


def test_hierarchy_matrices(prepared):
    hot = _hot()
    name, sc, dt, st, hz, g = prepared
    for m, lev in enumerate(hz.levels):
        Hg = g.debug_read(hot.DBG_LEVEL_MATRIX, m).reshape(lev.n, 125, 3, 3)
        Ho = O.csr_to_slots(hz.A[m], lev)
        assert rel(Hg, Ho) < 1e-12, f"level {m}"


def test_gradient_energy_and_vcycle(prepared):
    name, sc, dt, st, hz, g = prepared
    n = st.lev0.n
    rng = np.random.Generator(np.random.PCG64(5))
    dv = rng.normal(size=(n, 3)) * 0.01 * st.free[:, None]
    go = O.gradient(st, dv)
    gg = g.debug_apply(1, dv.ravel()).reshape(n, 3)
    assert rel(gg, go) < 1e-11
    e = g.debug_apply(2, dv.ravel())[0]
    assert abs(e - O.energy(st, dv)) < 1e-12 * abs(O.energy(st, dv))
    Hx = g.debug_apply(3, dv.ravel())
    assert rel(Hx, hz.A[0] @ dv.ravel()) < 1e-12
    b = (rng.normal(size=3 * n) * hz.free[0])
    log = []
    uo = O.vcycle(hz, b, sweeps=sc.smoother_sweeps, log=log)
    ug = g.debug_apply(0, b)
    assert rel(ug, uo) < 1e-11


def assert_dt_matches(stats_dt, sc):
    """The library's own time step (hot_step with dt <= 0: CFL 0.6 on the
    largest particle or prescribed boundary speed, capped at 1/24 s) equals
    the oracle's, up to the rounding of the speed norm."""
    want = O.time_step(sc)
    assert abs(stats_dt - want) <= 4 * np.spacing(want), (stats_dt, want)


def _compare_step(sc, precision=0, tol_x=1e-10, tol_v=1e-10):
    """One step on both sides; the library picks its own time step."""
    hot = _hot()
    dt = O.time_step(sc)
    out, info = O.step(sc, dt=dt)
    g = hot.Scene.from_scene(sc, precision=precision)
    st = g.step(0.0)
    assert_dt_matches(g.stats["dt"], sc)
    res = g.read()
    logi = g.debug_read(hot.DBG_LOG_INT, dtype=np.int32).reshape(-1, 4)
    cn = g.debug_read(hot.DBG_LOG_CN)
    g.close()
    return out, info, res, logi, cn, st, g.stats


@pytest.fixture(params=["one_row", "run_form"])
def rows_per_wave(request):
    """Run the smoothing and residual sweeps with one row per wave on every
    level ("one_row"), or in the form that large levels use (work-groups over
    runs of 16 rows with the iterate window in LDS), forced onto every level
    ("run_form")."""
    hot = _hot()
    hot.debug_set(hot.SET_MULTIROW_MIN, 1 << 30 if request.param == "one_row" else 0)
    yield request.param
    hot.debug_set(hot.SET_MULTIROW_MIN, -1)


def test_vcycle_run_form(prepared):
    """The large-level form of the sweeps (x-runs, iterate window in LDS),
    forced onto every level, gives the one-row V-cycle bit for bit, and so
    matches the oracle's V-cycle."""
    hot = _hot()
    name, sc, dt, st, hz, g = prepared
    n = st.lev0.n
    b = np.random.Generator(np.random.PCG64(8)).normal(size=3 * n) * hz.free[0]
    try:
        hot.debug_set(hot.SET_MULTIROW_MIN, 1 << 30)
        u1 = g.debug_apply(0, b)
        hot.debug_set(hot.SET_MULTIROW_MIN, 0)
        u2 = g.debug_apply(0, b)
    finally:
        hot.debug_set(hot.SET_MULTIROW_MIN, -1)
    assert np.array_equal(u1, u2)
    assert rel(u2, O.vcycle(hz, b, sweeps=sc.smoother_sweeps)) < 1e-11


@pytest.mark.parametrize("name", list(SCENES))
def test_full_step_fp64(name, rows_per_wave):
    sc = _grip_scene() if name == "bars_small_grips" else SCENES[name]()
    out, info, res, logi, cn, status, stats = _compare_step(sc)
    log = info["log"]
    assert stats["iters"] == info["iters"]
    assert list(logi[:, 0]) == log["alpha_halvings"]
    assert list(logi[:, 2]) == log["fallback"]
    assert list(logi[: len(log["skipped"]), 1]) == log["skipped"]
    assert list(logi[:, 3]) == [sum(c) for c in log["cg"]]
    assert rel(cn, log["cn"]) < 1e-9
    assert rel(res["x"], out.x) < 1e-10
    assert rel(res["v"], out.v) < 1e-10
    assert rel(res["F"], out.F) < 1e-10
    assert rel(res["C"], out.C) < 1e-9


def test_rotating_cube_step_fp64():
    """The 32^3 rotating cube (32768 particles, FCR, 3 levels, history 5, CN
    tolerance 1e-6): one full step."""
    sc = hs.rotating_cube()
    out, info, res, logi, cn, status, stats = _compare_step(sc)
    log = info["log"]
    assert status == 0 and info["converged"]
    assert stats["iters"] == info["iters"]
    assert list(logi[:, 0]) == log["alpha_halvings"]
    assert list(logi[:, 3]) == [sum(c) for c in log["cg"]]
    assert rel(res["x"], out.x) < 1e-10
    assert rel(res["v"], out.v) < 1e-10
    assert rel(res["F"], out.F) < 1e-10
