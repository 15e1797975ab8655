"""Host-side logic of the serving loop (no GPU): arrivals and latency
bookkeeping."""
import numpy as np

from paper_1911_07913_amd import serving


def test_poisson_arrivals_rate_and_order():
    a = serving.poisson_arrivals(20000, rate=50.0, seed=3)
    assert np.all(np.diff(a) >= 0)
    # mean inter-arrival 1/rate within 3 standard errors
    gaps = np.diff(np.concatenate([[0.0], a]))
    assert abs(gaps.mean() - 0.02) < 3 * 0.02 / np.sqrt(len(gaps))
    assert np.array_equal(a, serving.poisson_arrivals(20000, rate=50.0, seed=3))


def test_step_latencies_chain_from_admission():
    rec = dict(t_admit=1.0, t_step_end=[1.5, 1.75, 3.0], steps=3, iters=9, status=0,
               t_arrival=0.5)
    assert serving.step_latencies(rec) == [0.5, 0.25, 1.25]


def test_first_step_latency_starts_when_the_scene_is_ready():
    # a scene the batch created: the first step became eligible at t_created,
    # and the creation time is reported on its own
    rec = dict(t_admit=1.0, t_created=1.2, t_step_end=[1.5, 1.75], steps=2, iters=5, status=0,
               t_arrival=0.5)
    lat = serving.step_latencies(rec)
    assert abs(lat[0] - 0.3) < 1e-12 and abs(lat[1] - 0.25) < 1e-12
    s = serving.summarize([rec], t_begin=0.5)
    assert abs(s["scene_creation_ms"]["p50"] - 200.0) < 1e-9
    assert abs(s["admission_wait_ms"]["p50"] - 500.0) < 1e-9
    assert abs(s["request_latency_ms"]["p50"] - 1250.0) < 1e-9


def test_summary_percentiles_and_throughput():
    recs = []
    for k in range(100):
        t0 = float(k)
        recs.append(dict(t_admit=t0 + 0.1, t_step_end=[t0 + 0.1 + 0.01 * (k + 1)], steps=1,
                         iters=4, status=0, t_arrival=t0))
    s = serving.summarize(recs, t_begin=0.0)
    assert s["steps"] == 100 and s["requests"] == 100 and s["failed"] == 0
    lat = np.arange(1, 101) * 10.0
    assert abs(s["step_latency_ms"]["p50"] - np.percentile(lat, 50)) < 1e-9
    assert abs(s["step_latency_ms"]["p99"] - np.percentile(lat, 99)) < 1e-9
    assert abs(s["request_latency_ms"]["p50"] - np.percentile(lat + 100.0, 50)) < 1e-9
    assert abs(s["steps_per_s"] - 100 / (99.0 + 0.1 + 1.0)) < 1e-9
    assert s["iters_per_step"] == 4
