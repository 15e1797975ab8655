"""hot_step_noalloc (the step for callers that cannot allocate device memory)
against hot_step, through the C ABI.

Both run the same kernels; the no-allocation step takes its per-call scratch
from the library's fixed device array instead of the scene's own buffers, so
its output must equal hot_step's bit for bit (FP64 and mixed alike: the
kernels are deterministic).  Two no-allocation calls run back to back on
different scenes, the second smaller, each against a twin scene stepped by
hot_step.  Also: a scene's first step (buffers not yet sized) is refused
with HOT_E_NOMEM and leaves the scene usable; a coarsest level too large for
the scratch, and tracing switched on, are refused with HOT_E_INVALID.
"""
import numpy as np
import pytest

import hot_scenes as hs
from test_gpu_parity import SCENES, _hot

pytestmark = pytest.mark.gpu


def _read_all(g):
    r = g.read()
    return np.concatenate([r["x"].ravel(), r["v"].ravel(), r["F"].ravel(), r["C"].ravel()])


def _same_step(make, precision, graph=0):
    hot = _hot()
    a = hot.Scene.from_scene(make(), precision=precision, graph=graph)
    b = hot.Scene.from_scene(make(), precision=precision, graph=graph)
    try:
        a.step(0.0)  # sizes both scenes' buffers
        b.step(0.0)
        sa = a.step_noalloc(0.0)
        stats_a = dict(a.stats)
        sb = b.step(0.0)
        stats_b = dict(b.stats)
        ra, rb = _read_all(a), _read_all(b)
    finally:
        a.close()
        b.close()
    print(f"n = {a.n}: status {sa}/{sb}, iters {stats_a['iters']}/{stats_b['iters']}")
    assert sa == sb
    for k in ("iters", "backtracks", "cg_iters_total", "converged", "fallbacks", "skipped_pairs",
              "n_nodes", "dt", "E", "cn"):
        assert stats_a[k] == stats_b[k], k
    assert np.array_equal(ra, rb)


def test_noalloc_step_equals_hot_step_twice_second_smaller():
    hot = _hot()
    big, small = SCENES["box_nh_3mat"], SCENES["box_walls_fcr"]
    assert big().n > small().n
    _same_step(big, hot.HOT_FP64)
    _same_step(small, hot.HOT_FP64)
    _same_step(small, hot.HOT_MIXED)
    # a scene set to capture its V-cycles runs them eagerly here
    _same_step(small, hot.HOT_FP64, graph=1)


def test_noalloc_first_step_refused_then_usable():
    hot = _hot()
    make = SCENES["box_walls_fcr"]
    a = hot.Scene.from_scene(make())
    b = hot.Scene.from_scene(make())
    try:
        with pytest.raises(hot.HotError) as e:
            a.step_noalloc(0.0)
        assert e.value.status == -2  # HOT_E_NOMEM
        n, t = a.info()
        assert t == 0.0
        a.step(0.0)
        b.step(0.0)
        assert np.array_equal(_read_all(a), _read_all(b))
    finally:
        a.close()
        b.close()


def test_noalloc_refuses_large_coarsest_level_and_tracing():
    hot = _hot()
    # one level: the coarsest PCG runs on all 23^3 = 12,167 fine rows, whose
    # vectors need 1.75 MB of scratch
    sc = hs.small_box(seed=17, cells=(28, 28, 28), box_lo=(4, 4, 4), box_hi=(24, 24, 24),
                      levels=1, walls=2)
    g = hot.Scene.from_scene(sc)
    try:
        g.step(0.0)
        x0 = _read_all(g)
        with pytest.raises(hot.HotError) as e:
            g.step_noalloc(0.0)
        assert e.value.status == -1 and "scratch" in str(e.value)
        assert np.array_equal(_read_all(g), x0)
        g.profile(True)
        with pytest.raises(hot.HotError) as e:
            g.step_noalloc(0.0)
        assert e.value.status == -1
    finally:
        g.close()
