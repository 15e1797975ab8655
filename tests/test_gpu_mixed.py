"""Mixed-precision policy against the FP64 oracle, through the C ABI.

Under HOT_MIXED the V-cycle (smoothing, residual SpMV, restriction,
prolongation, coarsest Jacobi-PCG) runs on FP32 vectors over BF16-stored
3x3 blocks; energy, gradient, line search, CN test and the L-BFGS history stay
FP64.  The hierarchy itself is still built in FP64, so:

* the BF16 blocks must be the round-to-nearest-even BF16 of the FP32 rounding
  of the oracle's FP64 blocks (bit-exact);
* one mixed V-cycle differs from the oracle's FP64 V-cycle by the block
  rounding only (a few 1e-3 relative);
* once both sides run to a tolerance at which the step has converged, a mixed
  step lands within 1e-6 (relative to the largest position / velocity) of the
  FP64 oracle step: the outer quasi-Newton iteration removes the
  preconditioner's rounding;
* at the scene's own CN tolerance two runs of the method may stop anywhere
  inside the tolerance ball, so there the difference is reported as a
  measured figure.
"""
import numpy as np
import pytest

import oracle as O
from test_gpu_parity import SCENES, _grip_scene, _hot, oracle_prepare, rel

pytestmark = pytest.mark.gpu


def bf16_bits(a):
    """Round-to-nearest-even BF16 bit patterns of float32(a)."""
    u = np.asarray(a, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def _scene(name):
    return _grip_scene() if name == "bars_small_grips" else SCENES[name]()


@pytest.fixture(scope="module", params=list(SCENES))
def prepared_mixed(request):
    hot = _hot()
    sc = _scene(request.param)
    dt = O.time_step(sc)
    st, hz = oracle_prepare(sc, dt)
    g = hot.Scene.from_scene(sc, precision=hot.HOT_MIXED)
    g.debug_prepare(dt)
    yield request.param, sc, dt, st, hz, g
    g.close()


def test_bf16_blocks_bit_exact(prepared_mixed):
    hot = _hot()
    name, sc, dt, st, hz, g = prepared_mixed
    for m, lev in enumerate(hz.levels):
        hb = g.debug_read(hot.DBG_LEVEL_MATRIX_BF16, m, dtype=np.uint16).reshape(lev.n, 125, 3, 3)
        want = bf16_bits(O.csr_to_slots(hz.A[m], lev))
        assert np.array_equal(hb, want), f"level {m}: {np.count_nonzero(hb != want)} blocks differ"


def test_mixed_vcycle_close_to_fp64(prepared_mixed):
    name, sc, dt, st, hz, g = prepared_mixed
    n = st.lev0.n
    rng = np.random.Generator(np.random.PCG64(6))
    b = rng.normal(size=3 * n) * hz.free[0]
    uo = O.vcycle(hz, b, sweeps=sc.smoother_sweeps)
    ug = g.debug_apply(0, b)
    err = rel(ug, uo)
    print(f"{name}: mixed V-cycle relative error {err:.2e}")
    # BF16 keeps 8 significant bits (unit roundoff 2^-9); the cycle's
    # output error stays within a small multiple of it
    assert err < 2e-2
    # constrained DOFs stay exactly zero
    assert np.all(ug[hz.free[0] == 0] == 0.0)


def test_mixed_vcycle_run_form_bit_identical(prepared_mixed):
    """The BF16 sweeps' large-level form (work-groups over runs of 16 rows
    with the iterate window in LDS, and a memory gather where the rows are
    not one run), forced onto every level, gives the one-row V-cycle bit for
    bit."""
    hot = _hot()
    name, sc, dt, st, hz, g = prepared_mixed
    n = st.lev0.n
    b = np.random.Generator(np.random.PCG64(16)).normal(size=3 * n) * hz.free[0]
    try:
        hot.debug_set(hot.SET_MULTIROW_MIN, 1 << 30)
        u1 = g.debug_apply(0, b)
        hot.debug_set(hot.SET_MULTIROW_MIN, 0)
        u2 = g.debug_apply(0, b)
    finally:
        hot.debug_set(hot.SET_MULTIROW_MIN, -1)
    assert np.array_equal(u1, u2)


def _mixed_vs_oracle(sc, smoother="l1jacobi"):
    """The oracle's FP64 step and the library's mixed-precision step of the
    same scene at the scene's tolerance, with the same smoother."""
    hot = _hot()
    dt = O.time_step(sc)
    out, info = O.step(sc, dt=dt, smoother=smoother)
    g = hot.Scene.from_scene(sc, precision=hot.HOT_MIXED,
                             smoother=0 if smoother == "l1jacobi" else 1)
    try:
        status = g.step(dt)
        res = g.read()
        stats = dict(g.stats)
    finally:
        g.close()
    errs = dict(x=rel(res["x"], out.x), v=rel(res["v"], out.v), F=rel(res["F"], out.F))
    return status, stats, info, errs


# Tolerance and smoother at which each scene's FP64 step has converged far
# enough that two correct solves of it agree to better than 1e-6: the
# single-material box at eps = 1e-10 with the default smoother; the
# multi-material scenes (stiffness ratios 100 and 1000) at eps = 1e-11 with
# the paper's Gauss-Seidel smoother, since with l1 block-Jacobi the oracle
# needs over 1,000 iterations there (measured: 1,060 at eps = 1e-10 for the
# three-material box, whose l1 and Gauss-Seidel steps at that eps still differ
# by 1.2e-6 in v).
TIGHT = {"box_walls_fcr": (1e-10, "l1jacobi"), "box_nh_3mat": (1e-11, "sgs"),
         "bars_small_grips": (1e-11, "sgs")}


@pytest.mark.parametrize("name", list(SCENES))
def test_mixed_step_matches_fp64_oracle_at_tight_tolerance(name):
    """Mixed precision against the FP64 oracle at the same CN tolerance, once
    both have converged: x and v within 1e-6 relative (the outer L-BFGS
    iteration, run on FP64 gradients and energies, removes the BF16/FP32
    preconditioner's rounding)."""
    sc = _scene(name)
    sc.tol, smoother = TIGHT[name]
    status, stats, info, e = _mixed_vs_oracle(sc, smoother)
    print(f"{name} eps={sc.tol:g} {smoother}: iters mixed {stats['iters']} fp64 {info['iters']}; "
          f"mixed vs fp64 oracle: x {e['x']:.2e} v {e['v']:.2e} F {e['F']:.2e}")
    assert info["converged"] and status == 0 and stats["converged"]
    assert e["x"] <= 1e-6 and e["v"] <= 1e-6
    assert e["F"] <= 1e-6


@pytest.mark.parametrize("name", list(SCENES))
def test_mixed_step_at_scene_tolerance(name):
    """At the scenes' own eps = 1e-6 two correct runs of the method may stop
    anywhere inside the tolerance ball, so the mixed-vs-FP64 difference there
    is a measured figure rather than a parity bar (printed; measured 1e-4 to
    1e-3 relative in v on these scenes).  The assertion only rules out a
    broken step: both converge, and the difference stays below 1e-2."""
    sc = _scene(name)
    status, stats, info, e = _mixed_vs_oracle(sc)
    print(f"{name} eps={sc.tol:g}: iters mixed {stats['iters']} fp64 {info['iters']}; "
          f"mixed vs fp64 oracle: x {e['x']:.2e} v {e['v']:.2e} F {e['F']:.2e}")
    assert status == 0 and stats["converged"] and info["converged"]
    assert e["x"] < 1e-2 and e["v"] < 1e-2
