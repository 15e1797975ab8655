"""The device-allocator hook of hot_init_scene: a caller's allocator carries
the same step bit for bit, and a block that breaks the 256-byte alignment
the kernels' vector accesses need is refused (and handed back)."""
import numpy as np
import pytest

import hot_scenes as hs

pytestmark = pytest.mark.gpu


def _hot():
    from paper_1911_07913_amd import hot
    return hot


class _Counting:
    """torch's caching allocator, shifted by `offset` bytes, counting live blocks."""

    def __init__(self, offset=0):
        import torch
        hot = _hot()
        self.torch, self.offset, self.live, self.calls = torch, offset, {}, 0
        self._alloc = hot.ALLOC_FN(self._a)
        self._free = hot.FREE_FN(self._f)
        self.struct = hot.hot_allocator(self._alloc, self._free, None)

    def _a(self, nbytes, ctx):
        self.calls += 1
        base = self.torch.cuda.caching_allocator_alloc(int(nbytes) + self.offset, 0)
        p = base + self.offset
        self.live[p] = base
        return p

    def _f(self, ptr, ctx):
        if ptr:
            self.torch.cuda.caching_allocator_delete(self.live.pop(ptr))


def test_caller_allocator_gives_the_same_step():
    import torch
    hot = _hot()
    torch.cuda.set_device(0)
    sc = hs.small_box(seed=7, cells=(12, 12, 12), box_lo=(3, 3, 3), box_hi=(9, 8, 8), levels=2)
    a = _Counting()
    g1 = hot.Scene.from_scene(sc, allocator=a)
    g2 = hot.Scene.from_scene(sc)
    try:
        g1.step()
        g2.step()
        r1, r2 = g1.read(), g2.read()
    finally:
        g1.close()
        g2.close()
    assert a.calls > 0 and not a.live
    for k in ("x", "v", "F", "C"):
        assert np.array_equal(r1[k], r2[k]), k


def test_misaligned_allocator_is_refused():
    import torch
    hot = _hot()
    torch.cuda.set_device(0)
    sc = hs.small_box(seed=8, cells=(12, 12, 12), box_lo=(3, 3, 3), box_hi=(9, 8, 8), levels=2)
    a = _Counting(offset=64)
    with pytest.raises(hot.HotError) as e:
        g = hot.Scene.from_scene(sc, allocator=a)
        g.close()
    assert e.value.status == hot.HOT_E_INVALID
    assert "256-byte aligned" in str(e.value)
    assert a.calls > 0 and not a.live
