"""ctypes binding of libhot (include/hot.h): argument marshalling only.

Every step of the implicit MPM solve runs inside the HIP library; this module
converts numpy arrays and small Python records to the C structs, and maps the
status codes to exceptions.  It fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhot.so")

HOT_OK = 0
HOT_W_NOT_CONVERGED = 1
HOT_E_INVALID = -1
HOT_E_NOMEM = -2
HOT_E_DEVICE = -3
HOT_E_NONFINITE = -4
HOT_FP64 = 0
HOT_MIXED = 1
HOT_SMOOTH_L1_JACOBI = 0
HOT_SMOOTH_SGS = 1
HOT_SOLVER_HOT = 0
HOT_SOLVER_PN_PCG = 1
HOT_SOLVER_PN_MGPCG = 2

DBG_PERM = 1
DBG_LEVEL_NODES = 10
DBG_LEVEL_PATTERN = 11
DBG_LEVEL_MATRIX = 12
DBG_LEVEL_FREE = 13
DBG_LEVEL_MATRIX_BF16 = 14
DBG_LEVEL_COLOR_ROWS = 15
DBG_NODE_MASS = 20
DBG_NODE_VSTAR = 21
DBG_NODE_XI = 22
DBG_NODE_FIXED = 23
DBG_DV = 30
DBG_LOG_INT = 40
DBG_LOG_CN = 41
DBG_COUNTS = 50
SET_MULTIROW_MIN = 1

EXPORTS = ["hot_scene_footprint", "hot_init_scene", "hot_step", "hot_read_particles",
           "hot_scene_info", "hot_scene_memory", "hot_destroy_scene", "hot_last_error",
           "hot_batch_create", "hot_batch_capacity", "hot_batch_add", "hot_batch_poll",
           "hot_batch_clock", "hot_batch_destroy", "hot_debug_read", "hot_debug_prepare",
           "hot_debug_apply", "hot_debug_set", "hot_profile_enable", "hot_profile_read",
           "hot_step_noalloc", "hot_batch_submit"]

BATCH_MAX_STEPS = 64

PROF_KERNELS = {0: "smooth0", 1: "residual0", 2: "assemble_h0", 3: "rap0", 4: "particle_eval",
                5: "gradient", 6: "particle_hessian", 7: "sgs0", 8: "vcycle"}


class hot_material(C.Structure):
    _fields_ = [("model", C.c_int32), ("E", C.c_double), ("nu", C.c_double),
                ("density", C.c_double), ("yield_stress", C.c_double),
                ("snow_clamp", C.c_double * 2)]


class hot_bc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("p", C.c_double * 16)]


class hot_batch_result(C.Structure):
    _fields_ = [("tag", C.c_int64), ("status", C.c_int32), ("steps", C.c_int32),
                ("iters", C.c_int32), ("reserved", C.c_int32), ("t_admit", C.c_double),
                ("t_step_end", C.c_double * BATCH_MAX_STEPS), ("message", C.c_char * 160),
                ("scene", C.c_void_p), ("t_created", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class hot_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class hot_scene_desc(C.Structure):
    _fields_ = [("params", C.c_void_p), ("n", C.c_int64), ("x", C.c_void_p), ("v", C.c_void_p),
                ("F", C.c_void_p), ("C", C.c_void_p), ("vol0", C.c_void_p), ("mat_id", C.c_void_p),
                ("mats", C.c_void_p), ("n_mats", C.c_int32), ("bcs", C.c_void_p),
                ("n_bcs", C.c_int32)]


class hot_params(C.Structure):
    _fields_ = [("dx", C.c_double), ("grid_cells", C.c_int32 * 3), ("origin", C.c_double * 3),
                ("gravity", C.c_double * 3), ("cfl", C.c_double), ("max_dt", C.c_double),
                ("tol", C.c_double), ("lbfgs_history", C.c_int32), ("mg_levels", C.c_int32),
                ("max_iters", C.c_int32), ("smoother_sweeps", C.c_int32),
                ("precision", C.c_int32), ("smoother", C.c_int32),
                ("graph", C.c_int32), ("solver", C.c_int32)]


class hot_step_stats(C.Structure):
    _fields_ = [("dt", C.c_double), ("t", C.c_double), ("E0", C.c_double), ("E", C.c_double),
                ("cn0", C.c_double), ("cn", C.c_double), ("cn_tol", C.c_double),
                ("iters", C.c_int32), ("backtracks", C.c_int32), ("cg_iters_total", C.c_int32),
                ("converged", C.c_int32), ("fallbacks", C.c_int32),
                ("skipped_pairs", C.c_int32), ("n_nodes", C.c_int32), ("n_levels", C.c_int32),
                ("ms_prepare", C.c_float), ("ms_hierarchy", C.c_float),
                ("ms_solve", C.c_float), ("ms_g2p", C.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class HotError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hot status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libhot.so (built by build.py).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1911_07913_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
    L.hot_scene_footprint.argtypes = [C.POINTER(hot_params), C.c_int64, dp, C.POINTER(C.c_size_t)]
    L.hot_init_scene.argtypes = [C.POINTER(hot_params), C.c_int64, dp, dp, dp, dp, dp, ip,
                                 C.POINTER(hot_material), C.c_int32, C.POINTER(hot_bc), C.c_int32,
                                 C.POINTER(hot_allocator), vp, C.POINTER(vp)]
    L.hot_step.argtypes = [vp, C.c_double, C.POINTER(hot_step_stats)]
    L.hot_step_noalloc.argtypes = [vp, C.c_double, C.POINTER(hot_step_stats)]
    L.hot_read_particles.argtypes = [vp, C.c_int64, dp, dp, dp, dp]
    L.hot_scene_info.argtypes = [vp, C.POINTER(C.c_int64), dp]
    L.hot_destroy_scene.argtypes = [vp]
    L.hot_destroy_scene.restype = None
    L.hot_last_error.restype = C.c_char_p
    L.hot_scene_memory.argtypes = [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
    L.hot_batch_create.argtypes = [C.c_size_t, C.c_int32, C.POINTER(vp)]
    L.hot_batch_capacity.argtypes = [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_int32)]
    L.hot_batch_add.argtypes = [vp, vp, C.c_int32, C.c_int64]
    L.hot_batch_submit.argtypes = [vp, C.POINTER(hot_scene_desc), C.c_int32, C.c_int64]
    L.hot_batch_poll.argtypes = [vp, C.POINTER(hot_batch_result), C.c_int32,
                                 C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32]
    L.hot_batch_clock.argtypes = [vp]
    L.hot_batch_clock.restype = C.c_double
    L.hot_batch_destroy.argtypes = [vp]
    L.hot_batch_destroy.restype = None
    L.hot_debug_read.argtypes = [vp, C.c_int32, C.c_int32, vp, C.c_size_t, C.POINTER(C.c_size_t)]
    L.hot_debug_prepare.argtypes = [vp, C.c_double]
    L.hot_debug_apply.argtypes = [vp, C.c_int32, dp, dp]
    L.hot_debug_set.argtypes = [C.c_int32, C.c_int64, C.POINTER(C.c_int64)]
    L.hot_profile_enable.argtypes = [vp, C.c_int32]
    L.hot_profile_read.argtypes = [vp, C.c_int32, dp, C.POINTER(C.c_int64), dp]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("hot_destroy_scene", "hot_batch_destroy", "hot_last_error",
                        "hot_batch_clock"):
            f.restype = C.c_int32
    _lib = L
    return L


def hip_runtimes():
    """Paths of the HIP runtime libraries mapped into this process."""
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(line.split()[-1])
    except OSError:
        pass
    return paths


def _require_single_runtime():
    rt = hip_runtimes()
    if len(rt) > 1:
        raise RuntimeError("two HIP runtimes are loaded (%s): import torch before the first call "
                           "into libhot when passing torch streams or allocators" % sorted(rt))


def _check(st, ok_warn=True):
    if st < 0 or (st > 0 and not ok_warn):
        raise HotError(st, lib().hot_last_error().decode())
    return st


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def make_params(dx, grid_cells, origin, gravity, cfl=0.6, max_dt=1.0 / 24.0, tol=1e-6,
                lbfgs_history=8, mg_levels=3, max_iters=500, smoother_sweeps=1,
                precision=HOT_FP64, smoother=HOT_SMOOTH_L1_JACOBI, graph=0, solver=0):
    p = hot_params()
    p.dx = dx
    for a in range(3):
        p.grid_cells[a] = int(grid_cells[a])
        p.origin[a] = origin[a]
        p.gravity[a] = gravity[a]
    p.cfl, p.max_dt, p.tol = cfl, max_dt, tol
    p.lbfgs_history, p.mg_levels, p.max_iters = int(lbfgs_history), int(mg_levels), int(max_iters)
    p.smoother_sweeps, p.precision = int(smoother_sweeps), int(precision)
    p.smoother = int(smoother)
    p.graph = int(graph)
    p.solver = int(solver)
    return p


def params_of(scene, precision=HOT_FP64, **over):
    """hot_params from any object with the scene attributes (dx, grid_cells,
    origin, gravity, cfl, max_dt, tol, lbfgs_history, mg_levels, max_iters,
    and optionally smoother_sweeps)."""
    kw = dict(cfl=scene.cfl, max_dt=scene.max_dt, tol=scene.tol,
              lbfgs_history=scene.lbfgs_history, mg_levels=scene.mg_levels,
              max_iters=scene.max_iters, precision=precision,
              smoother_sweeps=getattr(scene, "smoother_sweeps", 1))
    kw.update(over)
    return make_params(scene.dx, scene.grid_cells, scene.origin, scene.gravity, **kw)


class TorchAllocator:
    """Route the library's device allocations through torch's caching allocator."""

    def __init__(self, device=0):
        import torch
        self._torch = torch
        self.device = device
        self._alloc = ALLOC_FN(self._a)
        self._free = FREE_FN(self._f)
        self.struct = hot_allocator(self._alloc, self._free, None)

    def _a(self, nbytes, ctx):
        try:
            return self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device)
        except Exception:
            return None

    def _f(self, ptr, ctx):
        if ptr:
            self._torch.cuda.caching_allocator_delete(ptr)


class SceneArgs:
    """The host arrays of hot_init_scene in C layout (kept alive by this object)."""

    def __init__(self, params, x, v, F, Cm, vol0, mat_id, materials, bcs):
        self.params = params
        self.x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        n = self.n = self.x.shape[0]
        self.v = np.ascontiguousarray(v, dtype=np.float64).reshape(n, 3)
        self.F = None if F is None else np.ascontiguousarray(F, dtype=np.float64).reshape(n, 9)
        self.Cm = None if Cm is None else np.ascontiguousarray(Cm, dtype=np.float64).reshape(n, 9)
        self.vol0 = np.ascontiguousarray(vol0, dtype=np.float64).reshape(n)
        self.mat_id = np.ascontiguousarray(mat_id, dtype=np.int32).reshape(n)
        self.mats = (hot_material * len(materials))()
        for k, m in enumerate(materials):
            sc2 = m.get("snow_clamp", (0.0, 0.0))
            self.mats[k] = hot_material(int(m["model"]), m["E"], m["nu"], m["density"],
                                        m.get("yield_stress", 0.0),
                                        (C.c_double * 2)(float(sc2[0]), float(sc2[1])))
        self.n_mats = len(materials)
        self.nb = len(bcs)
        self.cb = (hot_bc * max(self.nb, 1))()
        for k, b in enumerate(bcs):
            self.cb[k].kind = int(b["kind"])
            for j, val in enumerate(np.asarray(b["p"], dtype=np.float64)[:16]):
                self.cb[k].p[j] = float(val)

    def desc(self):
        def addr(a):
            return None if a is None else a.ctypes.data
        return hot_scene_desc(C.addressof(self.params), self.n, addr(self.x), addr(self.v),
                              addr(self.F), addr(self.Cm), addr(self.vol0), addr(self.mat_id),
                              C.addressof(self.mats), self.n_mats, C.addressof(self.cb), self.nb)


class Scene:
    """Owner of one hot_scene handle."""

    def __init__(self, params, x, v, F, Cm, vol0, mat_id, materials, bcs, stream=None,
                 allocator=None):
        L = lib()
        a = SceneArgs(params, x, v, F, Cm, vol0, mat_id, materials, bcs)
        if stream or allocator is not None:
            _require_single_runtime()
        self.params = params
        self.n = a.n
        self._allocator = allocator
        h = C.c_void_p()
        _check(L.hot_init_scene(C.byref(params), a.n, _dp(a.x), _dp(a.v), _dp(a.F), _dp(a.Cm),
                                _dp(a.vol0), a.mat_id.ctypes.data_as(C.POINTER(C.c_int32)),
                                a.mats, a.n_mats, a.cb, a.nb,
                                C.byref(allocator.struct) if allocator else None,
                                C.c_void_p(stream) if stream else None, C.byref(h)))
        self.handle = h
        self.stats = None

    @classmethod
    def adopt(cls, handle, n, params):
        """Wrap a scene handle the library created (a submitted batch request)."""
        self = cls.__new__(cls)
        self.params = params
        self.n = n
        self._allocator = None
        self.handle = C.c_void_p(handle)
        self.stats = None
        return self

    @classmethod
    def from_scene(cls, sc, precision=HOT_FP64, stream=None, allocator=None, **over):
        return cls(params_of(sc, precision, **over), sc.x, sc.v, sc.F, sc.C, sc.vol0, sc.mat_id,
                   sc.materials, sc.bcs, stream=stream, allocator=allocator)

    def step(self, dt=0.0):
        """hot_step; returns the status (0 or HOT_W_NOT_CONVERGED) and keeps the stats."""
        s = hot_step_stats()
        st = _check(lib().hot_step(self.handle, dt, C.byref(s)))
        self.stats = s.as_dict()
        return st

    def step_noalloc(self, dt=0.0):
        """hot_step_noalloc: hot_step without device allocation (the scene's
        buffers must already be sized; per-call scratch from the library's
        fixed device array)."""
        s = hot_step_stats()
        st = _check(lib().hot_step_noalloc(self.handle, dt, C.byref(s)))
        self.stats = s.as_dict()
        return st

    def read(self, F=True, Cm=True):
        n = self.n
        x = np.empty((n, 3))
        v = np.empty((n, 3))
        Fa = np.empty((n, 3, 3)) if F else None
        Ca = np.empty((n, 3, 3)) if Cm else None
        _check(lib().hot_read_particles(self.handle, n, _dp(x), _dp(v), _dp(Fa), _dp(Ca)))
        return dict(x=x, v=v, F=Fa, C=Ca)

    def memory(self):
        """(device bytes held now, footprint estimate made at init)"""
        live = C.c_size_t()
        est = C.c_size_t()
        _check(lib().hot_scene_memory(self.handle, C.byref(live), C.byref(est)))
        return live.value, est.value

    def info(self):
        n = C.c_int64()
        t = C.c_double()
        _check(lib().hot_scene_info(self.handle, C.byref(n), C.byref(t)))
        return n.value, t.value

    def debug_read(self, what, level=0, dtype=np.float64):
        L = lib()
        need = C.c_size_t()
        _check(L.hot_debug_read(self.handle, what, level, None, 0, C.byref(need)))
        buf = np.empty(need.value // np.dtype(dtype).itemsize, dtype=dtype)
        _check(L.hot_debug_read(self.handle, what, level, buf.ctypes.data_as(C.c_void_p),
                                buf.nbytes, C.byref(need)))
        return buf

    def debug_prepare(self, dt=0.0):
        _check(lib().hot_debug_prepare(self.handle, dt))

    def debug_apply(self, op, vec):
        vec = np.ascontiguousarray(vec, dtype=np.float64)
        out = np.empty_like(vec)
        _check(lib().hot_debug_apply(self.handle, op, _dp(vec), _dp(out)))
        return out

    def profile(self, enable=True):
        _check(lib().hot_profile_enable(self.handle, 1 if enable else 0))

    def profile_read(self):
        """{kernel: (total_ms, launches, total_algorithmic_bytes)}"""
        out = {}
        for k, name in PROF_KERNELS.items():
            ms = C.c_double()
            n = C.c_int64()
            b = C.c_double()
            _check(lib().hot_profile_read(self.handle, k, C.byref(ms), C.byref(n), C.byref(b)))
            out[name] = (ms.value, n.value, b.value)
        return out

    def close(self):
        if self.handle:
            lib().hot_destroy_scene(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def footprint(params, x):
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    out = C.c_size_t()
    _check(lib().hot_scene_footprint(C.byref(params), x.shape[0], _dp(x), C.byref(out)))
    return out.value


class Batch:
    """Continuous batching of independent scenes (hot_batch_*): admission by
    HBM footprint, one host thread per slot, per-step completion times."""

    def __init__(self, budget_bytes, max_slots):
        h = C.c_void_p()
        _check(lib().hot_batch_create(budget_bytes, max_slots, C.byref(h)))
        self.handle = h

    def capacity(self):
        fb = C.c_size_t()
        fs = C.c_int32()
        _check(lib().hot_batch_capacity(self.handle, C.byref(fb), C.byref(fs)))
        return fb.value, fs.value

    def add(self, scene: Scene, n_steps: int, tag: int) -> bool:
        """Admit a scene; False when it does not fit now (HOT_E_NOMEM)."""
        st = lib().hot_batch_add(self.handle, scene.handle, n_steps, tag)
        if st == HOT_E_NOMEM:
            return False
        _check(st)
        return True

    def submit(self, args: SceneArgs, n_steps: int, tag: int) -> bool:
        """Admit a request as a scene description (the slot thread creates the
        scene); False when it does not fit now (HOT_E_NOMEM).  ``args`` must
        stay alive until the request is collected."""
        d = args.desc()
        st = lib().hot_batch_submit(self.handle, C.byref(d), n_steps, tag)
        if st == HOT_E_NOMEM:
            return False
        _check(st)
        return True

    def poll(self, wait_ms=0, cap=64):
        """Finished scenes as dicts (tag, status, steps, iters, t_admit,
        t_step_end list, message) and the number still resident."""
        res = (hot_batch_result * cap)()
        nd = C.c_int32()
        nr = C.c_int32()
        _check(lib().hot_batch_poll(self.handle, res, cap, C.byref(nd), C.byref(nr), wait_ms))
        out = []
        for k in range(nd.value):
            r = res[k]
            m = min(r.steps + (1 if r.status < 0 else 0), BATCH_MAX_STEPS)
            out.append(dict(tag=r.tag, status=r.status, steps=r.steps, iters=r.iters,
                            t_admit=r.t_admit, t_step_end=[r.t_step_end[i] for i in range(m)],
                            message=r.message.decode(errors="replace"), scene=r.scene,
                            t_created=r.t_created))
        return out, nr.value

    def clock(self):
        return lib().hot_batch_clock(self.handle)

    def close(self):
        if self.handle:
            lib().hot_batch_destroy(self.handle)
            self.handle = None


def debug_set(key, value):
    """Process-wide test setting (hot_debug_set); returns the previous value."""
    prev = C.c_int64()
    _check(lib().hot_debug_set(key, int(value), C.byref(prev)))
    return prev.value
