"""Request loop for serving implicit steps of many independent scenes on one GPU.

Requests (a scene plus a number of steps) arrive over time.  The loop admits
them in arrival order whenever the batch has a free slot and the scene's HBM
footprint fits in what resident scenes leave of the budget, creates the scene
on the device only then, and hands it to the native batch (hot_batch_*), whose
slot threads run each scene's steps on the scene's own stream so that the
GPU interleaves the kernels of everything resident.  Finished scenes are read
back (optionally) and destroyed; the batch frees a scene's slot when its last
step ends and its budget when the loop collects it.

Latencies follow the usual serving definitions: a step's latency runs from
the moment it became eligible (its scene admitted, or its previous step done)
to its completion; a request's latency runs from its arrival to the end of its
last step.
"""
from __future__ import annotations

import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import hot


def poisson_arrivals(n: int, rate: float, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of a Poisson process of ``rate`` requests/s."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if rate <= 0 or not np.isfinite(rate):
        return np.zeros(n)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def step_latencies(rec: dict) -> list:
    """Per-step latencies of one finished request record: the first step
    became eligible when its scene was ready (created on the device), each
    later step when the previous one ended."""
    ends = rec["t_step_end"][: rec["steps"]]
    out, prev = [], rec.get("t_created", rec["t_admit"])
    for t in ends:
        out.append(t - prev)
        prev = t
    return out


def summarize(records: list, t_begin: float) -> dict:
    """p50/p99 step and request latency (ms) and aggregate steps/s."""
    steps = [lat for r in records for lat in step_latencies(r)]
    req = [r["t_step_end"][r["steps"] - 1] - r["t_arrival"] for r in records if r["steps"] > 0]
    wait = [r["t_admit"] - r["t_arrival"] for r in records]
    create = [r.get("t_created", r["t_admit"]) - r["t_admit"] for r in records]
    t_end = max((r["t_step_end"][r["steps"] - 1] for r in records if r["steps"] > 0),
                default=t_begin)
    n_steps = sum(r["steps"] for r in records)
    span = max(t_end - t_begin, 1e-12)

    def pct(a, q):
        return float(np.percentile(np.asarray(a) * 1e3, q)) if len(a) else None

    return {
        "requests": len(records),
        "steps": n_steps,
        "steps_per_s": n_steps / span,
        "wall_s": span,
        "step_latency_ms": {"p50": pct(steps, 50), "p99": pct(steps, 99), "max": pct(steps, 100)},
        "request_latency_ms": {"p50": pct(req, 50), "p99": pct(req, 99)},
        "admission_wait_ms": {"p50": pct(wait, 50), "p99": pct(wait, 99)},
        "scene_creation_ms": {"p50": pct(create, 50), "p99": pct(create, 99)},
        "iters_per_step": (sum(r["iters"] for r in records) / n_steps) if n_steps else None,
        "failed": sum(1 for r in records if r["status"] < 0),
    }


def serve(requests, arrivals, budget_bytes: int, max_slots: int, precision=hot.HOT_MIXED,
          n_steps=None, collect=None, poll_ms: int = 20, smoother=hot.HOT_SMOOTH_L1_JACOBI,
          submit=True, graph=True):
    """Run a stream of requests through one batch.

    ``requests``: indexable scene descriptions (positions, velocities, F, C,
    volumes, material ids, materials, boundary conditions, parameters) as
    accepted by ``hot.Scene.from_scene``; a sequence with a ``release(k)``
    method is told when request k's host data is no longer needed;
    ``arrivals``: arrival time in seconds of each, non-decreasing; ``precision`` and
    ``smoother``: hot_precision and hot_smoother of every request; ``n_steps``: steps per request (default: each scene's
    ``n_steps``); ``collect(index, scene)``: called on each finished scene
    before it is destroyed (read its particles there); ``submit``: hand each
    request to the batch as a scene description, so that its slot thread
    creates the scene from the batch's device pool (False: the loop creates
    each scene itself and admits it); ``graph``: run every step's V-cycles as
    a captured HIP graph.

    Returns (records, summary, trace) where ``trace`` holds the largest number
    of resident scenes and of reserved bytes seen by the loop.
    """
    arrivals = np.asarray(arrivals, dtype=np.float64)
    assert len(arrivals) == len(requests) and np.all(np.diff(arrivals) >= 0)
    batch = hot.Batch(budget_bytes, max_slots)
    # finished scenes are destroyed off the admission path (destruction waits
    # for the scene's stream and releases its host resources; the batch has
    # already returned its budget when poll handed it out)
    reaper = ThreadPoolExecutor(max_workers=1)
    pending = deque(range(len(requests)))
    live, reserved, records = {}, {}, []
    peak_res, peak_bytes = 0, 0
    params, held = {}, {}
    try:
        t0 = batch.clock()
        while pending or live:
            now = batch.clock() - t0
            # admission, in arrival order
            while pending and arrivals[pending[0]] <= now:
                k = pending[0]
                sc = requests[k]
                if k not in params:
                    params[k] = hot.params_of(sc, precision, smoother=smoother,
                                              graph=1 if graph else 0)
                steps = int(n_steps if n_steps is not None else sc.n_steps)
                if submit:
                    # the batch computes the footprint and checks the budget
                    args = hot.SceneArgs(params[k], sc.x, sc.v, sc.F, sc.C, sc.vol0, sc.mat_id,
                                         sc.materials, sc.bcs)
                    if not batch.submit(args, steps, k):
                        if not live:
                            need = hot.footprint(params[k], sc.x)
                            if need > budget_bytes:
                                raise ValueError(f"request {k} needs {need} bytes, more than "
                                                 f"the whole budget {budget_bytes}")
                        break
                    held[k] = args
                    live[k] = None
                else:
                    if k not in reserved:
                        reserved[k] = hot.footprint(params[k], sc.x)
                    free_b, free_s = batch.capacity()
                    if free_s == 0 or reserved[k] > free_b:
                        if not live and reserved[k] > budget_bytes:
                            raise ValueError(f"request {k} needs {reserved[k]} bytes, more than "
                                             f"the whole budget {budget_bytes}")
                        break
                    scene = hot.Scene(params[k], sc.x, sc.v, sc.F, sc.C, sc.vol0, sc.mat_id,
                                      sc.materials, sc.bcs)
                    if not batch.add(scene, steps, k):
                        scene.close()
                        break
                    live[k] = scene
                pending.popleft()
                release = getattr(requests, "release", None)
                if release is not None:
                    release(k)
                peak_res = max(peak_res, len(live))
                peak_bytes = max(peak_bytes, budget_bytes - batch.capacity()[0])
            # completions
            if live:
                # wait for a completion, but no longer than the next arrival
                wait = poll_ms
                if pending:
                    dt_next = arrivals[pending[0]] - (batch.clock() - t0)
                    if dt_next > 0:
                        wait = int(min(poll_ms, dt_next * 1e3))
                done, _ = batch.poll(wait_ms=wait)
                for r in done:
                    k = int(r["tag"])
                    scene = live.pop(k)
                    if scene is None and r["scene"]:
                        scene = hot.Scene.adopt(r["scene"], held[k].n, params[k])
                    held.pop(k, None)
                    if scene is not None:
                        if collect is not None and r["status"] >= 0:
                            collect(k, scene)
                        if submit:
                            reaper.submit(scene.close)
                        else:
                            scene.close()
                    r["t_arrival"] = t0 + float(arrivals[k])
                    r["index"] = k
                    records.append(r)
            elif pending:
                time.sleep(max(arrivals[pending[0]] - (batch.clock() - t0), 0.0))
        summary = summarize(records, t0 + float(arrivals[0]) if len(arrivals) else t0)
    finally:
        # scenes the batch created come back only through poll: collect the
        # rest before the batch goes
        while any(v is None for v in live.values()):
            done, _ = batch.poll(wait_ms=100)
            for r in done:
                k = int(r["tag"])
                live.pop(k, None)
                if r["scene"]:
                    hot.Scene.adopt(r["scene"], held[k].n, params[k]).close()
        reaper.shutdown(wait=True)
        batch.close()
        for scene in live.values():
            if scene is not None:
                scene.close()
    return records, summary, {"peak_resident": peak_res, "peak_reserved_bytes": peak_bytes}
