"""Host-side validation of the C ABI (no device work happens for invalid
input, so this runs without a GPU): every malformed scene is refused with
HOT_E_INVALID and a message, and the footprint estimate behaves."""
import ctypes as C
import os

import numpy as np
import pytest

import hot_scenes as hs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1911_07913_amd", "libhot.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhot.so not built")


def _hot():
    from paper_1911_07913_amd import hot
    return hot


def _init(hot, sc, **over):
    """hot_init_scene on a possibly corrupted copy; returns (status, message)."""
    params = hot.params_of(sc, **{k: v for k, v in over.items() if k in ("tol", "mg_levels",
                                                                          "max_iters", "smoother")})
    L = hot.lib()
    x = np.ascontiguousarray(sc.x, dtype=np.float64)
    n = x.shape[0]
    mats = (hot.hot_material * len(sc.materials))()
    for k, m in enumerate(sc.materials):
        c2 = m.get("snow_clamp", (0.0, 0.0))
        mats[k] = hot.hot_material(int(m["model"]), m["E"], m["nu"], m["density"],
                                   m.get("yield_stress", 0.0), (C.c_double * 2)(*c2))
    bcs = (hot.hot_bc * max(len(sc.bcs), 1))()
    for k, b in enumerate(sc.bcs):
        bcs[k].kind = int(b["kind"])
        for j, val in enumerate(b["p"][:16]):
            bcs[k].p[j] = float(val)
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    v = np.ascontiguousarray(sc.v, dtype=np.float64)
    F = np.ascontiguousarray(sc.F, dtype=np.float64).reshape(n, 9)
    Cm = np.ascontiguousarray(sc.C, dtype=np.float64).reshape(n, 9)
    vol = np.ascontiguousarray(sc.vol0, dtype=np.float64)
    mid = np.ascontiguousarray(sc.mat_id, dtype=np.int32)
    h = C.c_void_p()
    st = L.hot_init_scene(C.byref(params), n, dp(x), dp(v), dp(F), dp(Cm), dp(vol),
                          mid.ctypes.data_as(C.POINTER(C.c_int32)), mats, len(sc.materials),
                          bcs, len(sc.bcs), None, None, C.byref(h))
    msg = L.hot_last_error().decode()
    if st == 0:
        L.hot_destroy_scene(h)
    return st, msg


def _box():
    return hs.small_box(seed=5, cells=(10, 10, 10), box_lo=(3, 3, 3), box_hi=(7, 7, 7), walls=2)


@pytest.mark.parametrize("case", ["nan_x", "outside", "E_zero", "nu_half", "bad_mat_id",
                                  "nan_v", "vol_zero", "nh_inverted", "snow_lo_above_1",
                                  "snow_with_yield", "empty"])
def test_invalid_scenes_are_refused(case):
    hot = _hot()
    sc = _box()
    if case == "nan_x":
        sc.x[3, 1] = np.nan
    elif case == "outside":
        sc.x[0, 0] = sc.origin[0] + 1.0 * sc.dx
    elif case == "E_zero":
        sc.materials[0]["E"] = 0.0
    elif case == "nu_half":
        sc.materials[0]["nu"] = 0.5
    elif case == "bad_mat_id":
        sc.mat_id[7] = 3
    elif case == "nan_v":
        sc.v[2, 2] = np.inf
    elif case == "vol_zero":
        sc.vol0[4] = 0.0
    elif case == "nh_inverted":
        sc.materials[0]["model"] = 1
        sc.F[5] = np.diag([1.0, 1.0, -1.0])
    elif case == "snow_lo_above_1":
        sc.materials[0]["snow_clamp"] = (1.01, 1.02)
    elif case == "snow_with_yield":
        sc.materials[0]["snow_clamp"] = (0.99, 1.001)
        sc.materials[0]["yield_stress"] = 100.0
    elif case == "empty":
        for f in ("x", "v", "F", "C", "vol0", "mat_id"):
            setattr(sc, f, np.ascontiguousarray(getattr(sc, f)[:0]))
    st, msg = _init(hot, sc)
    assert st == hot.HOT_E_INVALID, (case, st, msg)
    assert msg


@pytest.mark.parametrize("field,value", [("mg_levels", 0), ("mg_levels", 9), ("max_iters", 0),
                                         ("tol", -1.0), ("smoother", 2), ("smoother", -1)])
def test_invalid_parameters_are_refused(field, value):
    hot = _hot()
    st, msg = _init(hot, _box(), **{field: value})
    assert st == hot.HOT_E_INVALID and msg


def test_footprint_grows_with_the_scene_and_with_mixed_blocks():
    hot = _hot()
    small = hs.small_box(seed=6, cells=(12, 12, 12), box_lo=(3, 3, 3), box_hi=(6, 6, 6))
    large = hs.small_box(seed=6, cells=(12, 12, 12), box_lo=(3, 3, 3), box_hi=(9, 9, 9))
    fs = hot.footprint(hot.params_of(small), small.x)
    fl = hot.footprint(hot.params_of(large), large.x)
    fm = hot.footprint(hot.params_of(large, hot.HOT_MIXED), large.x)
    assert 0 < fs < fl < fm
    # the Gauss-Seidel colour lists and diagonal-block inverses are counted
    fg = hot.footprint(hot.params_of(large, smoother=hot.HOT_SMOOTH_SGS), large.x)
    assert fg > fl
    # at least the level-0 block rows: n0 rows of 1152 doubles
    import oracle as O
    n0 = O.active_fine_nodes(large).n
    assert fl > n0 * 1152 * 8


@pytest.mark.parametrize("slots", [0, -1, 65, 256])
def test_batch_slot_count_is_bounded(slots):
    """A batch holds 1 to 64 slots (the grid-barrier coarsest solves are
    limited separately, by the device's 16 tickets)."""
    hot = _hot()
    L = hot.lib()
    h = C.c_void_p()
    assert L.hot_batch_create(1 << 20, slots, C.byref(h)) == hot.HOT_E_INVALID
    assert not h.value
    assert b"64" in L.hot_last_error()
