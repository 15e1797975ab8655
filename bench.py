"""Benchmark: implicit MPM steps/s on the 1.5M-particle twisting-bars scene,
FP64 and mixed precision, plus a served stream of independent scenes.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one full hot_step: CFL time step, binning, active grid and
hierarchy index sets, APIC P2G, level-0 Hessian, Galerkin hierarchy, the HOT
quasi-Newton solve (two-loop, V-cycle, line search, CN test) and G2P.  The
scene (4 Neo-Hookean bars of 192x16x16 cells, 8 particles per cell, E in
{1e5..1e8} Pa, grips twisting at +-2 rad/s, 256x64x64 grid, dx = 1/64, 5
Galerkin levels, L-BFGS window 8, CN tolerance 1e-6) is resident in HBM before
the timed region; the default K = 20 times the whole 20-step job from t = 0.
The served stream: 512 random spinning boxes (4k-256k particles, 10 steps
each) with Poisson arrivals at 0.7 of the closed-loop step rate.  Prints one
JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "implicit MPM steps/s @1.5M particles, FP64 vs mixed; served p50/p99 step latency"
HBM_PEAK_GBS = 8000.0
# FP64 vector peak: 256 CUs x 64 FP64 FMA lanes per clock x 2 flop x 2.4 GHz
FP64_PEAK_TFLOPS = 78.6

# What bounds each traced kernel, and the algorithmic FP64 flops of the
# ALU-bound ones per particle.  Level-0 assembly per particle, from the
# particle's C+ and a_ip = F^T grad w operands (formed with C+ in the
# stress-derivative pass): C+ a_jp for 27 nodes (27 x 81 FMA) and the 378
# distinct 3x3 blocks a_ip^T (C+ a_jp) of the symmetric 27 x 27 block pattern
# (378 x 27 FMA): 12,393 FMA = 24,786 flop.
BOUND = {"smooth0": "hbm", "residual0": "hbm", "sgs0": "hbm", "rap0": "hbm", "particle_eval": "hbm",
         "gradient": "hbm", "assemble_h0": "alu", "particle_hessian": "alu"}
# traced spans that hold several kernels (not candidates for the dominant kernel)
COMPOSITE = {"vcycle"}
FLOP_PER_PARTICLE = {"assemble_h0": 2.0 * (27 * 81 + 378 * 27)}

CSRC = os.path.join(ROOT, "paper_1911_07913_amd", "csrc")
# committed PMC summaries: per-launch HBM traffic of a kernel in the precision
# it was measured in, valid while the sources it was measured on are unchanged
_ASM_SRC = ["particles.hip", "mpm_math.h", "hot_internal.h"]
_SWEEP_SRC = ["matrix.hip", "mpm_math.h", "hot_internal.h"]
TRAFFIC = {(k, prec): (f"{stem}_twisting_bars_1p5M_{prec}_pmc.md", src)
           for prec in ("fp64", "mixed")
           for k, stem, src in (("assemble_h0", "assemble_h0", _ASM_SRC),
                                ("smooth0", "vcycle_level0", _SWEEP_SRC),
                                ("residual0", "vcycle_level0", _SWEEP_SRC))}

# CPU-baseline sample: the headline scene's particles in the cell slab
# x in [38, 42) of all four bars (32,768 particles), where the first grip's
# rotating nodes meet the free span, so that the sample's solve has work
SAMPLE_CELLS_X = (38, 42)
SAMPLE_ITERS = 3


def workload_name(side, smoother="l1 block-Jacobi"):
    n = 4 * 192 * side * side * 8
    return (f"twisting_bars: 4 Neo-Hookean bars 192x{side}x{side} cells, {n} particles, "
            f"256x64x64 grid dx=1/64, 5-level Galerkin MG with {smoother} smoothing, "
            f"L-BFGS w=8, CN eps=1e-6")


def hs_sweeps(side):
    """Smoothing sweeps the twisting-bars scene is stepped with."""
    import inspect

    import hot_scenes as hs
    return inspect.signature(hs.twisting_bars).parameters["sweeps"].default


def smoother_label(sgs, sweeps):
    return ("coloured symmetric Gauss-Seidel (1 forward-backward pair)" if sgs else
            f"l1 block-Jacobi ({sweeps} sweeps per level and direction)")


def cpu_worker(side):
    """Oracle timing on the bounded sample (run in a single-threaded child):
    the per-step set-up (binning, P2G, level-0 Hessian, Galerkin hierarchy)
    and the cost of one quasi-Newton iteration, on the headline scene's
    particles in a thin mid-span slab."""
    import numpy as np

    import hot_scenes as hs
    import oracle as O
    sc = hs.twisting_bars(side=side, n_steps=1)
    cell_x = np.floor(sc.x[:, 0] / sc.dx)
    keep = (cell_x >= SAMPLE_CELLS_X[0]) & (cell_x < SAMPLE_CELLS_X[1])
    for f in ("x", "v", "F", "C", "vol0", "mat_id"):
        setattr(sc, f, getattr(sc, f)[keep].copy())
    dt = O.time_step(sc)
    t0 = time.perf_counter()
    st = O.prepare(sc, dt)
    H0, nbr0 = O.hessian_slots(st)
    hz = O.build_hierarchy(st, H0, nbr0, sc.mg_levels)
    t1 = time.perf_counter()
    # the solve's own set-up (smoother inverses, first energy and gradient),
    # then exactly SAMPLE_ITERS iterations (tolerance 0)
    O.solve(st, hz, 0.0, sc.lbfgs_history, max_iters=0, sweeps=sc.smoother_sweeps)
    t2 = time.perf_counter()
    dv, info = O.solve(st, hz, 0.0, sc.lbfgs_history, max_iters=SAMPLE_ITERS,
                       sweeps=sc.smoother_sweeps)
    t3 = time.perf_counter()
    O.g2p(st, dv)
    t4 = time.perf_counter()
    it = max(info["iters"], 1)
    print(json.dumps(dict(setup=(t2 - t0) + (t4 - t3), per_iter=((t3 - t2) - (t2 - t1)) / it,
                          iters=info["iters"], n=sc.n, seconds=t4 - t0)))


def cpu_baseline(n_full, side, job_iters):
    """The oracle's steps/s on the whole timed job, from the bounded sample:
    each step costs the set-up plus its quasi-Newton iterations (the counts
    the GPU job took; the oracle takes the same decisions), both scaled from
    the sample to the full particle count."""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    env["HIP_VISIBLE_DEVICES"] = ""
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-worker",
                        "--side", str(side)], env=env, capture_output=True, text=True,
                       timeout=900)
    if r.returncode != 0:
        return dict(error=r.stderr[-500:])
    d = json.loads(r.stdout.strip().splitlines()[-1])
    scale = n_full / d["n"]
    sec = sum((d["setup"] + k * d["per_iter"]) * scale for k in job_iters)
    return {"value": len(job_iters) / sec, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle on the {d['n']} particles of the headline scene in cells "
                       f"x in [{SAMPLE_CELLS_X[0]}, {SAMPLE_CELLS_X[1]}) on 1 core: per-step "
                       f"set-up (binning, P2G, Hessian, hierarchy, G2P) {d['setup']:.2f} s, "
                       f"{d['per_iter']:.3f} s per quasi-Newton iteration ({d['iters']} "
                       f"timed); the job's {sum(job_iters)} iterations over "
                       f"{len(job_iters)} steps, both costs scaled by particle count to "
                       f"{n_full}: {sec:.0f} s")}


def mixed_step_errors(side, steps):
    """Per-step error of the mixed-precision step against the FP64 step from
    the same state.  Before each step of the FP64 job its state (x, v, F, C)
    seeds a mixed-precision scene; both take one step (the same CFL time step,
    from the same velocities) and the mixed positions and velocities are
    compared with the FP64 ones: max |dx| / max |x|, max |dv| / max |v|, and
    max |dx| over the largest FP64 displacement.  The FP64 GPU step stands in
    for the FP64 oracle at this size (it matches the oracle within 1e-10 at
    every size the tests compare).  A third step from the same state, FP64 at
    eps = 1e-9, gives each one's distance to a much tighter solve
    (tight_v_fp64, tight_v_mixed): at the config tolerance both stop inside
    the same tolerance ball."""
    import numpy as np

    import hot_scenes as hs
    from paper_1911_07913_amd import hot
    sc = hs.twisting_bars(side=side)
    g = hot.Scene.from_scene(sc)
    out = {"x": [], "v": [], "x_displacement": [], "iters_mixed": [], "iters_fp64": [],
           "tight_v_fp64": [], "tight_v_mixed": [], "iters_tight": []}

    def one_step(state, **kw):
        cur = sc.copy()
        cur.x, cur.v, cur.F, cur.C = state["x"], state["v"], state["F"], state["C"]
        h = hot.Scene.from_scene(cur, **kw)
        try:
            h.step()
            return h.read(F=False, Cm=False), h.stats["iters"]
        finally:
            h.close()

    def relv(a, b):
        return float(np.abs(a - b).max() / np.abs(b).max())
    try:
        for _ in range(steps):
            st = g.read()
            rm, im = one_step(st, precision=hot.HOT_MIXED)
            # a much tighter FP64 solve from the same state (Gauss-Seidel, one
            # pair, eps = 1e-9): how far each config-tolerance step lies from it
            rt, it_t = one_step(st, tol=1e-9, smoother=hot.HOT_SMOOTH_SGS, smoother_sweeps=1)
            g.step()
            r64 = g.read(F=False, Cm=False)
            out["x"].append(relv(rm["x"], r64["x"]))
            out["v"].append(relv(rm["v"], r64["v"]))
            out["x_displacement"].append(float(np.abs(rm["x"] - r64["x"]).max() /
                                               max(np.abs(r64["x"] - st["x"]).max(), 1e-300)))
            out["iters_mixed"].append(im)
            out["iters_fp64"].append(g.stats["iters"])
            out["tight_v_fp64"].append(relv(r64["v"], rt["v"]))
            out["tight_v_mixed"].append(relv(rm["v"], rt["v"]))
            out["iters_tight"].append(it_t)
    finally:
        g.close()
    out["max"] = {k: max(out[k]) for k in ("x", "v", "x_displacement", "tight_v_fp64",
                                            "tight_v_mixed")}
    return out


def run(precision, steps, warmup, side, profile=True, smoother=0, scene=None):
    """Warm up on a throwaway copy of the scene (kernels loaded, device memory
    in torch's cache), then time ``steps`` steps of a fresh scene from t = 0:
    with the default 20 steps, the whole twisting-bars job.  ``smoother`` is a
    hot_smoother (0: l1 block-Jacobi, 1: coloured symmetric Gauss-Seidel).
    ``scene``: another workload in place of the twisting bars."""
    import torch

    import hot_scenes as hs
    from paper_1911_07913_amd import hot

    sc = hs.twisting_bars(side=side) if scene is None else scene
    # the paper's smoothing is one symmetric Gauss-Seidel sweep pair per level
    over = {"smoother_sweeps": 1} if smoother == hot.HOT_SMOOTH_SGS else {}
    stream = torch.cuda.Stream()
    alloc = hot.TorchAllocator(0)
    if warmup > 0:
        w = hot.Scene.from_scene(sc, precision=precision, stream=stream.cuda_stream,
                                 allocator=alloc, smoother=smoother, **over)
        for _ in range(warmup):
            w.step()
        torch.cuda.synchronize()
        w.close()
    g = hot.Scene.from_scene(sc, precision=precision, stream=stream.cuda_stream, allocator=alloc,
                             smoother=smoother, **over)
    if profile:
        g.profile(True)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.step()
        stats.append(dict(g.stats))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = g.profile_read() if profile else {}
    g.profile(False)
    n = g.n
    g.close()
    return dict(seconds=t1 - t0, stats=stats, prof=prof, n=n)


class ServingRequests:
    """The serving request stream.  Every request's particle data is
    generated before the run starts (in parallel threads), as a client would
    hold it on arrival, so that generating inputs never counts as admission
    wait; host memory of a request is released once it is admitted."""

    def __init__(self, n, seed_base=4000, workers=8):
        import hot_scenes as hs
        from concurrent.futures import ThreadPoolExecutor
        self.n, self.seed_base = n, seed_base
        with ThreadPoolExecutor(max_workers=workers) as ex:
            scenes = list(ex.map(lambda k: hs.serving_scene(k, seed_base=seed_base), range(n)))
        self.cache = dict(enumerate(scenes))

    def __len__(self):
        return self.n

    def __getitem__(self, k):
        return self.cache[k]

    def release(self, k):
        self.cache.pop(k, None)


def run_serving(n_req, slots, budget_gb, precision, smoother, load=0.7, submit=True, graph=True,
                rate=None, sat=None):
    """Closed-loop run of the whole stream (every request arriving at t = 0)
    for the saturated step rate, then the stream with Poisson arrivals at
    ``load`` times it.  ``submit`` and ``graph``: the serving design (the
    batch creating each scene on its slot thread from its device pool, and
    captured V-cycle graphs), or the loop creating scenes itself and every
    kernel launched eagerly.  ``rate`` (requests/s) and ``sat`` (a summary of
    an earlier closed-loop run of the same design): use that arrival rate
    instead of ``load`` times this design's own saturated rate."""
    from paper_1911_07913_amd import hot, serving
    budget = int(budget_gb * (1 << 30))
    if sat is None:
        _, sat, _ = serving.serve(ServingRequests(n_req), [0.0] * n_req, budget, slots,
                                  precision, smoother=smoother, submit=submit, graph=graph)
    steps_per_req = 10
    if rate is None:
        rate = load * sat["steps_per_s"] / steps_per_req
    load = rate * steps_per_req / sat["steps_per_s"]
    arrivals = serving.poisson_arrivals(n_req, rate, seed=4000)
    records, summary, trace = serving.serve(ServingRequests(n_req), arrivals, budget, slots,
                                            precision, smoother=smoother, submit=submit,
                                            graph=graph)
    req_p50 = summary["request_latency_ms"]["p50"]
    summary.update(precision="fp64" if precision == hot.HOT_FP64 else "mixed",
                   smoother="l1jacobi" if smoother == hot.HOT_SMOOTH_L1_JACOBI else "sgs",
                   design=("slot threads create scenes from the batch's device pool; "
                           "V-cycles as captured HIP graphs") if submit and graph else
                          ("loop creates each scene and admits it; eager launches"),
                   admission_wait_share_p50=(summary["admission_wait_ms"]["p50"] / req_p50
                                             if req_p50 else None),
                   slots=slots,
                   budget_gb=budget_gb, load=load, arrival_rate_req_per_s=rate,
                   saturated_steps_per_s=sat["steps_per_s"],
                   saturated_step_latency_ms=sat["step_latency_ms"], **trace)
    summary["_sat"] = sat
    return summary


def source_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_of(kernel, precision):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) from
    the committed PMC summary, or None when there is none for this kernel in
    this precision or the kernel's sources changed since it was taken."""
    if (kernel, precision) not in TRAFFIC:
        return None
    fname, files = TRAFFIC[(kernel, precision)]
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as fh:
        for ln in fh:
            if ln.startswith("traffic-json: "):
                d = json.loads(ln[len("traffic-json: "):])
                if d.get("kernel") == kernel:
                    rec = d
    if rec is None or rec.get("source_sha256") != source_hash(files):
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def roofline_of(prof, n_particles, precision):
    """Roofline of the dominant traced kernel (largest summed launch time)."""
    name, (ms, launches, nbytes) = max(((k, v) for k, v in prof.items() if k not in COMPOSITE),
                                       key=lambda kv: kv[1][0])
    if launches == 0:
        return None
    avg_s = ms * 1e-3 / launches
    traffic = traffic_of(name, precision)
    if BOUND[name] == "alu":
        flops = FLOP_PER_PARTICLE[name] * n_particles
        achieved = flops / avg_s / 1e12
        return {"kernel": name, "bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                "avg_launch_ms": ms / launches, "launches": launches,
                "algorithmic_flop_per_launch": flops,
                "algorithmic_bytes_per_launch": nbytes / launches}
    achieved = nbytes / launches / avg_s / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "avg_launch_ms": ms / launches, "launches": launches,
            "algorithmic_bytes_per_launch": nbytes / launches}


def vcycle_roofline(prof, precision):
    """HBM roofline of the whole V-cycle (every level's smoothing, residual,
    restriction and prolongation, the coarsest Jacobi-PCG and the precision
    conversions, traced as one span per cycle), with the level-0 passes
    (smoothing, Gauss-Seidel or Jacobi, and the residual) broken out."""
    if "vcycle" not in prof or prof["vcycle"][1] == 0 or prof["vcycle"][0] <= 0:
        return None
    t, n, b = prof["vcycle"]
    achieved = b / (t * 1e-3) / 1e9
    out = {"span": "whole V-cycle", "bound": "hbm", "achieved": achieved,
           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
           "avg_cycle_ms": t / n, "cycles": n, "algorithmic_bytes_per_cycle": b / n}
    ks = [k for k in ("sgs0", "smooth0", "residual0") if k in prof and prof[k][1] > 0]
    ms = sum(prof[k][0] for k in ks)
    nbytes = sum(prof[k][2] for k in ks)
    if ms > 0:
        out["level0_passes"] = {"kernels": ks, "achieved": nbytes / (ms * 1e-3) / 1e9,
                                "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        for k in ks:
            t, n, b = prof[k]
            out["level0_passes"][k] = {"avg_launch_ms": t / n if n else None,
                                       "algorithmic_bytes_per_launch": b / n if n else None,
                                       "traffic": traffic_of(k, precision)}
    return out


def smoother_summary(r, steps, precision):
    """The same job with the paper's coloured symmetric Gauss-Seidel smoother:
    rate, iteration counts and the level-0 V-cycle passes' algorithmic
    bandwidth."""
    return {"value": steps / r["seconds"], "unit": "steps/s",
            "ms_per_step": 1000.0 * r["seconds"] / steps,
            "iters": [s["iters"] for s in r["stats"]],
            "cg_iters": [s["cg_iters_total"] for s in r["stats"]],
            "roofline": roofline_of(r["prof"], r["n"], precision),
            "vcycle_roofline": vcycle_roofline(r["prof"], precision)}


def stiffness_sweep(steps=3):
    """The varying-stiffness experiment (Sec. 7): a three-material bar (ends
    E = 1e5 Pa, middle E = 1e5 .. 1e10 Pa, 49,152 particles) twisted by its
    grips, stepped with HOT, LBFGS-H (HOT with one level: the level-0
    Jacobi-PCG as initial inverse Hessian), PN-PCG and PN-MGPCG; FP64, ms per
    step and iterations (quasi-Newton or Newton; CG iterations of the Newton
    solves, coarsest-PCG iterations of the quasi-Newton ones)."""
    import torch

    import hot_scenes as hs
    from paper_1911_07913_amd import hot
    out = []
    for E in (1e5, 1e6, 1e7, 1e8, 1e9, 1e10):
        row = {"E_mid": E}
        for name, kw in (("hot", {}), ("lbfgs_h", dict(mg_levels=1)),
                         ("pn_pcg", dict(solver=hot.HOT_SOLVER_PN_PCG)),
                         ("pn_mgpcg", dict(solver=hot.HOT_SOLVER_PN_MGPCG))):
            sc = hs.stiffness_bar(E_mid=E)
            g = hot.Scene.from_scene(sc, **kw)
            its, cgs = [], []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                g.step()
                its.append(g.stats["iters"])
                cgs.append(g.stats["cg_iters_total"])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            g.close()
            row[name] = {"ms_per_step": 1000.0 * (t1 - t0) / steps, "iters": its, "cg_iters": cgs}
        row["particles"] = sc.n
        out.append(row)
    return {"workload": "stiffness_bar: 3-material FCR bar 96x8x8 cells (ends 1e5 Pa), grips at "
                        "+-2 rad/s, 112x32x32 grid dx=1/64, 3 levels, eps=1e-6, "
                        f"{steps} steps per solver and stiffness", "rows": out}


def stretched_box_convergence():
    """The stretched-box convergence study (Sec. 8): a soft box that starts
    from a random diagonal deformation gradient relaxes; the
    quasi-Newton iterations to the CN tolerance 1e-7 in the first step, FP64,
    for HOT with three levels (the paper's smoothing, one coloured Gauss-Seidel
    sweep pair, and the headline job's five l1 block-Jacobi sweeps) and for
    LBFGS-H (one level: the level-0 Jacobi-PCG as initial inverse Hessian)."""
    import torch

    import hot_scenes as hs
    from paper_1911_07913_amd import hot
    sc = hs.stretched_box()
    out = {}
    for name, levels, kw in (("hot_sgs", 3, dict(smoother=hot.HOT_SMOOTH_SGS, smoother_sweeps=1)),
                             ("hot_l1jacobi", 3, dict(smoother_sweeps=5)),
                             ("lbfgs_h", 1, dict(smoother_sweeps=1))):
        g = hot.Scene.from_scene(sc, mg_levels=levels, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        status = g.step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out[name] = {"iters": g.stats["iters"], "coarse_cg_iters": g.stats["cg_iters_total"],
                     "converged": status == 0, "ms": 1000.0 * (t1 - t0)}
        g.close()
    return {"workload": f"stretched_box: FCR box 32^3 cells, {sc.n} particles, F = diag "
                        "U[0.7, 1.3] (one draw for the box), no gravity, no walls, 48^3 grid "
                        "dx=1/64, CN eps=1e-7, first step", **out}


def calibrate_copy(nbytes=1 << 30):
    """One plain device-to-device copy of a known size (for scaling HBM
    counters read under the profiler)."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--side", type=int, default=16, help="bar cross-section (16: 1.5M particles)")
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB device copy first (counter calibration under a profiler)")
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--serving-slots", type=int, default=12)
    ap.add_argument("--serving-budget-gb", type=float, default=64.0)
    ap.add_argument("--serving-precision", default="both", choices=["fp64", "mixed", "both"])
    ap.add_argument("--smoother", default="l1jacobi", choices=["l1jacobi", "sgs"],
                    help="smoother of the main job (profiling runs)")
    ap.add_argument("--no-sgs", action="store_true",
                    help="skip the same job with the coloured Gauss-Seidel smoother")
    ap.add_argument("--no-slab", action="store_true",
                    help="skip the 8.2M-particle sphere-slab job")
    ap.add_argument("--no-stiffness", action="store_true",
                    help="skip the varying-stiffness bar with the four solvers")
    ap.add_argument("--no-stretched", action="store_true",
                    help="skip the stretched-box convergence comparison")
    ap.add_argument("--no-mixed-error", action="store_true",
                    help="skip the per-step mixed-vs-FP64 error pass (untimed)")
    ap.add_argument("--sweep-run-min", type=int, default=None,
                    help="level size (rows) from which the V-cycle sweeps stage x-runs in LDS "
                         "(default: the library's; a huge value keeps every level one row per "
                         "wave, to profile that form)")
    ap.add_argument("--cpu-worker", action="store_true")
    a = ap.parse_args()
    if a.cpu_worker:
        cpu_worker(a.side)
        return 0
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {a.gpus} is not supported "
              "(the step is a single-GPU solver; sharding across GPUs is not built)",
              file=sys.stderr)
        return 2
    # torch first: libhot then binds to the HIP runtime torch already loaded,
    # so torch's streams and allocations are valid inside the library
    import torch
    from paper_1911_07913_amd import hot
    hot.lib()
    assert torch.cuda.is_available(), "no HIP device"
    if a.sweep_run_min is not None:
        hot.debug_set(hot.SET_MULTIROW_MIN, a.sweep_run_min)

    def prec_name(p):
        return "fp64" if p == hot.HOT_FP64 else "mixed"

    torch.cuda.set_device(0)
    if a.calibrate_copy:
        calibrate_copy()
    precs = {"fp64": [hot.HOT_FP64], "mixed": [hot.HOT_MIXED],
             "both": [hot.HOT_FP64, hot.HOT_MIXED]}[a.precision]
    main_sm = hot.HOT_SMOOTH_SGS if a.smoother == "sgs" else hot.HOT_SMOOTH_L1_JACOBI
    results = {}
    for p in precs:
        results[p] = run(p, a.steps, a.warmup, a.side, smoother=main_sm)
    main_p = precs[0]
    r = results[main_p]
    value = a.steps / r["seconds"]
    stats = r["stats"]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1000.0 * r["seconds"] / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_p == hot.HOT_FP64 else "f64+f32/bf16",
        "data": "synthetic",
        "config": {"workload": workload_name(a.side, smoother_label(
                       a.smoother == "sgs", hs_sweeps(a.side))),
                   "particles": r["n"],
                   "precision": prec_name(main_p),
                   "smoother": a.smoother},
        "roofline": roofline_of(r["prof"], r["n"], prec_name(main_p)),
        "vcycle_roofline": vcycle_roofline(r["prof"], prec_name(main_p)),
        "per_step": {
            "iters": [s["iters"] for s in stats],
            "cg_iters": [s["cg_iters_total"] for s in stats],
            "converged": [s["converged"] for s in stats],
            "dt": [s["dt"] for s in stats],
            "n_nodes": [s["n_nodes"] for s in stats],
            "ms_prepare": [round(s["ms_prepare"], 3) for s in stats],
            "ms_hierarchy": [round(s["ms_hierarchy"], 3) for s in stats],
            "ms_solve": [round(s["ms_solve"], 3) for s in stats],
            "ms_g2p": [round(s["ms_g2p"], 3) for s in stats],
        },
        "kernels": {k: {"total_ms": round(v[0], 3), "launches": v[1],
                        "gbs": round(v[2] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else None}
                    for k, v in r["prof"].items()},
    }
    if a.sweep_run_min is not None:
        line["config"]["sweep_run_min"] = a.sweep_run_min
    if hot.HOT_MIXED in results and main_p != hot.HOT_MIXED:
        rm = results[hot.HOT_MIXED]
        line["mixed"] = {"value": a.steps / rm["seconds"], "unit": "steps/s",
                         "ms_per_step": 1000.0 * rm["seconds"] / a.steps,
                         "iters": [s["iters"] for s in rm["stats"]],
                         "roofline": roofline_of(rm["prof"], rm["n"], "mixed"),
                         "vcycle_roofline": vcycle_roofline(rm["prof"], "mixed")}
        if not a.no_mixed_error:
            line["mixed"]["step_error_vs_fp64"] = mixed_step_errors(a.side, a.steps)
    if not a.no_sgs:
        line["smoother_sgs"] = {
            prec_name(p):
            smoother_summary(run(p, a.steps, a.warmup, a.side,
                                 smoother=hot.HOT_SMOOTH_SGS), a.steps, prec_name(p))
            for p in precs}
    if not a.no_slab:
        # the larger configuration: 8,192,000 particles, 30 steps, both precisions
        import hot_scenes as hs
        slab = {}
        for p in (hot.HOT_MIXED, hot.HOT_FP64):
            rs = run(p, 30, 1, a.side, profile=False, scene=hs.sphere_slab())
            slab["mixed" if p == hot.HOT_MIXED else "fp64"] = {
                "value": 30 / rs["seconds"], "unit": "steps/s",
                "ms_per_step": 1000.0 * rs["seconds"] / 30,
                "iters": [st["iters"] for st in rs["stats"]]}
        line["sphere_slab_8M"] = {"workload": "sphere_slab: FCR von Mises slab 160x40x160 cells, "
                                  "8192000 particles, 192^3 grid dx=1/192, 4-level Galerkin MG, "
                                  "rigid sphere at 3 m/s, 30 steps", **slab}
    if not a.no_stiffness:
        line["stiffness_sweep"] = stiffness_sweep()
    if not a.no_stretched:
        line["stretched_box"] = stretched_box_convergence()
    if a.serving_requests > 0:
        sp = {"fp64": [hot.HOT_FP64], "mixed": [hot.HOT_MIXED],
              "both": [hot.HOT_MIXED, hot.HOT_FP64]}[a.serving_precision]
        # the served scenes are small (4k-256k particles): there the single
        # fully parallel pass of l1 block-Jacobi beats the 53 colour passes of
        # Gauss-Seidel (measured: serving_sgs)
        l1 = hot.HOT_SMOOTH_L1_JACOBI
        args = (a.serving_requests, a.serving_slots, a.serving_budget_gb)
        line["serving"] = run_serving(*args, sp[0], l1)
        # the round-trip design for comparison: the loop creates each scene on
        # its own thread, every kernel is launched eagerly
        line["serving_thread_per_slot"] = run_serving(*args, sp[0], l1, submit=False,
                                                      graph=False)
        # the serving design at the comparison design's arrival rate
        line["serving_at_thread_per_slot_rate"] = run_serving(
            *args, sp[0], l1, rate=line["serving_thread_per_slot"]["arrival_rate_req_per_s"],
            sat=line["serving"]["_sat"])
        if len(sp) > 1:
            line["serving_fp64"] = run_serving(*args, sp[1], l1)
        line["serving_sgs"] = run_serving(*args, sp[0], hot.HOT_SMOOTH_SGS)
        for k in list(line):
            if k.startswith("serving") and isinstance(line[k], dict):
                line[k].pop("_sat", None)
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(r["n"], a.side, [s["iters"] for s in stats])
    print(json.dumps(line), flush=True)
    # hand the device memory back before the interpreter exits, so that the
    # process ends promptly
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return 0


if __name__ == "__main__":
    sys.exit(main())
