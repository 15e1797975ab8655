"""Parity at the benchmark's full size: the 1,572,864-particle twisting bars
(256x64x64 grid, 5 levels), prepared exactly as the benchmark's first step.

Integer work is compared whole and bit for bit against the oracle:
binning permutation, the active node set of every level, constrained nodes.
Floating-point fields are compared at sampled nodes, each computed by the
oracle on the sub-scene of particles that can influence it (the particles
whose base node lies within [i - 4, i + 2] per axis of the sampled node i:
they hold every particle of i's stencil and every particle of the stencils
of those particles' nodes), so the oracle's value is exact for the full
scene:  node mass, v*, CN stiffness, the gradient at dv = 0 and the whole
125-block row of the level-0 Hessian.  Finally one full step at this size
must converge with a decreasing incremental potential, and its
grid-to-particle transfer must conserve momentum against the grid's own
final velocities and advance positions by dt times the new velocity.
"""
import math

import numpy as np
import pytest

import hot_scenes as hs
import oracle as O
from test_gpu_parity import _hot, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    hot = _hot()
    sc = hs.twisting_bars(side=16)
    dt = O.time_step(sc)
    g = hot.Scene.from_scene(sc)
    g.debug_prepare(dt)
    yield sc, dt, g
    g.close()


def test_binning_permutation_bit_exact(full):
    hot = _hot()
    sc, dt, g = full
    _, perm = O.bin_particles(sc)
    assert np.array_equal(g.debug_read(hot.DBG_PERM, dtype=np.int32), perm)


def test_level_node_sets_and_constraints_bit_exact(full):
    hot = _hot()
    sc, dt, g = full
    lev = O.active_fine_nodes(sc)
    fixed, _ = O.bc_nodes(sc, lev, dt)
    assert np.array_equal(g.debug_read(hot.DBG_NODE_FIXED, dtype=np.int32).astype(bool), fixed)
    counts = []
    for m in range(sc.mg_levels):
        nodes = g.debug_read(hot.DBG_LEVEL_NODES, m, dtype=np.int32).astype(np.int64)
        assert np.array_equal(nodes, lev.lin), f"level {m}"
        counts.append(lev.n)
        if m + 1 < sc.mg_levels:
            _, lev = O.prolongation(lev)
    # the closed-form counts of the 16x16-bar scene
    assert counts == [281580, 47916, 8619, 1323, 375]


def _subscene(sc, node, lo=-4, hi=2):
    base = O.bspline(sc.x, sc.origin, sc.dx)[0]
    sel = np.all((base >= node + lo) & (base <= node + hi), axis=1)
    out = sc.copy()
    for f in ("x", "v", "F", "C", "vol0", "mat_id"):
        setattr(out, f, getattr(sc, f)[sel].copy())
    return out


def _sample_nodes(sc, lev, fixed, k=6, seed=11):
    rng = np.random.Generator(np.random.PCG64(seed))
    free = np.nonzero(~fixed)[0]
    picks = list(rng.choice(free, size=k, replace=False))
    # two free nodes next to a gripped node, so the Dirichlet projection of
    # the Hessian is sampled too
    nb = lev.lookup(O.linear(lev.coords[:, None, :] + O.SLOT_OFFS[None], lev.dims))
    near = np.nonzero(~fixed & np.any((nb >= 0) & fixed[np.maximum(nb, 0)], axis=1))[0]
    picks += list(rng.choice(near, size=2, replace=False))
    return [int(p) for p in picks]


def test_sampled_nodes_p2g_gradient_and_hessian_rows(full):
    hot = _hot()
    sc, dt, g = full
    lev = O.active_fine_nodes(sc)
    fixed, _ = O.bc_nodes(sc, lev, dt)
    mass = g.debug_read(hot.DBG_NODE_MASS)
    vstar = g.debug_read(hot.DBG_NODE_VSTAR).reshape(-1, 3)
    xi = g.debug_read(hot.DBG_NODE_XI)
    grad = g.debug_apply(1, np.zeros(3 * lev.n)).reshape(-1, 3)
    H0 = g.debug_read(hot.DBG_LEVEL_MATRIX, 0).reshape(lev.n, 125, 3, 3)
    for i in _sample_nodes(sc, lev, fixed):
        node = lev.coords[i]
        sub = _subscene(sc, node)
        st = O.prepare(sub, dt)
        j = int(st.lev0.lookup(np.array([lev.lin[i]]))[0])
        assert j >= 0
        assert abs(mass[i] - st.m[j]) <= 1e-13 * st.m[j]
        assert rel(vstar[i], st.vstar[j]) < 1e-12
        assert abs(xi[i] - st.xi[j]) <= 1e-13 * st.xi[j]
        go = O.gradient(st, np.zeros((st.lev0.n, 3)))[j]
        # at dv = 0 the elastic forces nearly cancel away from the grips; the
        # node's momentum m_i |v*_i| sets the scale of a meaningful difference
        scale = max(np.abs(go).max(), st.m[j] * np.abs(st.vstar[j]).max())
        assert np.abs(grad[i] - go).max() <= 1e-10 * scale, (i, grad[i], go)
        Hs, _ = O.hessian_slots(st)
        assert rel(H0[i], Hs[j]) < 1e-12, f"row {i}"


def test_full_size_step_converges_and_decreases_energy():
    """One full step converges with a decreasing incremental potential, and
    its grid-to-particle transfer keeps the properties that hold at any size
    (Sec. 3): the B-spline weights sum to one and the node masses are the
    particles' weighted masses, so the particles' total momentum equals the
    grid's, sum_i m_i (v*_i + dv_i); positions advance by dt times the new
    particle velocity."""
    hot = _hot()
    sc = hs.twisting_bars(side=16)
    g = hot.Scene.from_scene(sc)
    try:
        status = g.step()
        st = g.stats
        out = g.read(F=False, Cm=False)
        m_i = g.debug_read(hot.DBG_NODE_MASS)
        v_i = g.debug_read(hot.DBG_NODE_VSTAR).reshape(-1, 3) + g.debug_read(hot.DBG_DV).reshape(-1, 3)
    finally:
        g.close()
    assert status == 0 and st["converged"]
    assert st["E"] < st["E0"]
    assert st["cn"] <= st["cn_tol"] < st["cn0"]
    dens = np.array([mt["density"] for mt in sc.materials])
    m_p = dens[sc.mat_id] * sc.vol0
    p_particles = m_p @ out["v"]
    p_grid = m_i @ v_i
    scale = float(m_p @ np.linalg.norm(out["v"], axis=1))
    assert np.max(np.abs(p_particles - p_grid)) <= 1e-11 * scale
    assert abs(m_i.sum() - m_p.sum()) <= 1e-12 * m_p.sum()
    xs = float(np.abs(sc.x).max())
    assert np.max(np.abs(out["x"] - (sc.x + st["dt"] * out["v"]))) <= 4e-16 * xs


def test_sphere_slab_full_size_mixed():
    """The 8,192,000-particle sphere slab (192^3 grid, dx = 1/192, 4 levels,
    von Mises FCR, rigid sphere at 3 m/s) in mixed precision, as the
    benchmark runs it: binning permutation and every level's node set
    bit-exact against the oracle; two steps converge with decreasing
    incremental potential, and every particle ends on or inside the yield
    surface."""
    hot = _hot()
    sc = hs.sphere_slab()
    _, perm = O.bin_particles(sc)
    lev = O.active_fine_nodes(sc)
    g = hot.Scene.from_scene(sc, precision=hot.HOT_MIXED)
    try:
        g.debug_prepare(O.time_step(sc))
        assert np.array_equal(g.debug_read(hot.DBG_PERM, dtype=np.int32), perm)
        counts = []
        for m in range(sc.mg_levels):
            nodes = g.debug_read(hot.DBG_LEVEL_NODES, m, dtype=np.int32).astype(np.int64)
            assert np.array_equal(nodes, lev.lin), f"level {m}"
            counts.append(lev.n)
            if m + 1 < sc.mg_levels:
                _, lev = O.prolongation(lev)
        assert counts == [1142467, 158447, 24037, 4232]
        for k in range(2):
            status = g.step()
            st = g.stats
            assert status == 0 and st["converged"], f"step {k}"
            assert st["E"] < st["E0"]
        F = g.read()["F"]
    finally:
        g.close()
    mu, lam = O.lame(sc.materials[0]["E"], sc.materials[0]["nu"])
    lim = math.sqrt(2.0 / 3.0) * sc.materials[0]["yield_stress"] / (2.0 * mu)
    s = np.linalg.svd(F[:: 16], compute_uv=False)
    eps = np.log(s)
    nd = np.linalg.norm(eps - eps.mean(axis=1, keepdims=True), axis=1)
    assert np.all(nd <= lim * (1.0 + 1e-9))


def test_run_form_sweeps_bit_identical_at_full_size(full):
    """Levels 0 and 1 of this scene (281,580 and 47,916 rows) run the sweeps
    over x-runs with the iterate staged in LDS.  The same V-cycle with one
    row per wave on every level (the form that the oracle-compared small
    scenes run by default) is bit-identical, in FP64 and in mixed precision,
    and so is a whole FP64 step."""
    hot = _hot()
    sc, dt, g = full
    n = g.debug_read(hot.DBG_LEVEL_NODES, 0, dtype=np.int32).size
    b = np.random.Generator(np.random.PCG64(12)).normal(size=3 * n)
    b *= g.debug_read(hot.DBG_LEVEL_FREE, 0, dtype=np.uint8).astype(float)
    u2 = g.debug_apply(0, b)
    try:
        hot.debug_set(hot.SET_MULTIROW_MIN, 1 << 30)
        u1 = g.debug_apply(0, b)
    finally:
        hot.debug_set(hot.SET_MULTIROW_MIN, -1)
    assert np.array_equal(u1, u2)
    m = hot.Scene.from_scene(sc, precision=hot.HOT_MIXED)
    try:
        m.debug_prepare(dt)
        v2 = m.debug_apply(0, b)
        try:
            hot.debug_set(hot.SET_MULTIROW_MIN, 1 << 30)
            v1 = m.debug_apply(0, b)
        finally:
            hot.debug_set(hot.SET_MULTIROW_MIN, -1)
    finally:
        m.close()
    assert np.array_equal(v1, v2)
    outs = []
    for forced in (None, 1 << 30):
        s = hot.Scene.from_scene(sc)
        try:
            if forced is not None:
                hot.debug_set(hot.SET_MULTIROW_MIN, forced)
            s.step()
            outs.append((s.read(F=False, Cm=False), dict(s.stats)))
        finally:
            hot.debug_set(hot.SET_MULTIROW_MIN, -1)
            s.close()
    (a, sa), (c, sc1) = outs
    assert sa["iters"] == sc1["iters"] and sa["cg_iters_total"] == sc1["cg_iters_total"]
    assert np.array_equal(a["x"], c["x"]) and np.array_equal(a["v"], c["v"])
