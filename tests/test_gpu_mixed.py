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
  inside the tolerance ball, so there the mixed step is held to the FP64
  step's own accuracy: its distance to a much tighter FP64 solve is at most
  twice the FP64 step's (or 1e-6 relative, whichever is larger).
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
    uo = O.vcycle(hz, b)
    ug = g.debug_apply(0, b)
    err = rel(ug, uo)
    print(f"{name}: mixed V-cycle relative error {err:.2e}")
    # BF16 keeps 8 significant bits (unit roundoff 2^-9); the cycle's
    # output error stays within a small multiple of it
    assert err < 2e-2
    # constrained DOFs stay exactly zero
    assert np.all(ug[hz.free[0] == 0] == 0.0)


def _mixed_vs_oracle(sc, keep=False):
    hot = _hot()
    dt = O.time_step(sc)
    out, info = O.step(sc, dt=dt)
    g = hot.Scene.from_scene(sc, precision=hot.HOT_MIXED)
    status = g.step(dt)
    res = g.read()
    stats = dict(g.stats)
    g.close()
    x0 = sc.x
    ex = rel(res["x"], out.x)
    ev = rel(res["v"], out.v)
    eF = rel(res["F"], out.F)
    disp = np.abs(res["x"] - out.x).max() / max(np.abs(out.x - x0).max(), 1e-300)
    if keep:
        return status, stats, info, ex, ev, eF, disp, out, dt, (res["x"], res["v"])
    return status, stats, info, ex, ev, eF, disp, out, dt


# CN tolerances at which the oracle's step is (close to) converged for each
# scene; the multi-material scenes converge slowly, so these differ
TIGHT = {"box_walls_fcr": 1e-10, "box_nh_3mat": 1e-8, "bars_small_grips": 1e-7}


@pytest.mark.parametrize("name", list(SCENES))
def test_mixed_step_at_scene_tolerance(name):
    sc = _scene(name)
    status, stats, info, ex, ev, eF, disp, out, dt, res_x_v = _mixed_vs_oracle(sc, keep=True)
    tight = _scene(name)
    tight.tol = TIGHT[name]
    ref, rinfo = O.step(tight, dt=dt)
    tx, tv = rel(out.x, ref.x), rel(out.v, ref.v)
    mx, mv = rel(res_x_v[0], ref.x), rel(res_x_v[1], ref.v)
    print(f"{name} eps={sc.tol:g}: iters mixed {stats['iters']} fp64 {info['iters']}; "
          f"mixed-vs-fp64 x {ex:.2e} v {ev:.2e} F {eF:.2e} (displacement-relative x "
          f"{disp:.2e}); vs the fp64 step at {TIGHT[name]:g} ({rinfo['iters']} iters): "
          f"fp64 x {tx:.2e} v {tv:.2e}, mixed x {mx:.2e} v {mv:.2e}")
    assert status == 0 and stats["converged"]
    assert mx <= max(1e-6, 2.0 * tx)
    assert mv <= max(1e-6, 2.0 * tv)


def test_mixed_step_tight_tolerance():
    sc = _scene("box_walls_fcr")
    sc.tol = 1e-10
    status, stats, info, ex, ev, eF, disp, out, dt = _mixed_vs_oracle(sc)
    print(f"box_walls_fcr eps=1e-10: iters mixed {stats['iters']} fp64 {info['iters']}; "
          f"x {ex:.2e} v {ev:.2e} F {eF:.2e} (displacement-relative x {disp:.2e})")
    assert status == 0 and stats["converged"] and info["converged"]
    assert ex < 1e-9
    assert ev < 1e-8
