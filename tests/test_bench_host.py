"""Host-side logic of bench.py: the one-GPU guard, the roofline arithmetic,
and the rule that HBM traffic is quoted from a committed counter summary only
while the kernel's sources are the ones it was measured on."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_assembly_flop_count():
    # C+ a_jp for 27 nodes (9x9 times 9-vector), and the 378 = 27 * 28 / 2
    # distinct blocks of the symmetric 27 x 27 block pattern, each a 9-long
    # contraction for 3 x 3 outputs (27 FMA); the a_ip themselves are formed
    # in the stress-derivative pass
    assert 27 * 28 // 2 == 378
    assert bench.FLOP_PER_PARTICLE["assemble_h0"] == 2 * (27 * 81 + 378 * 27) == 24786


def _fake_tree(tmp_path, monkeypatch, sources, fetch, write, sha=None):
    csrc = tmp_path / "csrc"
    csrc.mkdir()
    for name, text in sources.items():
        (csrc / name).write_text(text)
    monkeypatch.setattr(bench, "CSRC", str(csrc))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    files = list(sources)
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"kernel": "smooth0", "source_sha256": sha or bench.source_hash(files),
           "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write, "sources": files}
    (prof / "vcycle_level0_twisting_bars_1p5M_fp64_pmc.md").write_text(
        "# summary\n\ntraffic-json: " + json.dumps(rec) + "\n")
    monkeypatch.setitem(bench.TRAFFIC, ("smooth0", "fp64"),
                        ("vcycle_level0_twisting_bars_1p5M_fp64_pmc.md", files))
    return csrc


def test_traffic_quoted_while_sources_unchanged(tmp_path, monkeypatch):
    csrc = _fake_tree(tmp_path, monkeypatch, {"a.hip": "kernel A\n", "b.h": "header\n"},
                      fetch=3.0e9, write=1.5e9)
    assert bench.traffic_of("smooth0", "fp64") == pytest.approx(4.5e9)
    # no summary file for the other precision here, and no entry for an untraced kernel
    assert bench.traffic_of("smooth0", "mixed") is None
    assert bench.traffic_of("k_unknown", "fp64") is None
    # any change to a listed source withdraws the figure
    (csrc / "b.h").write_text("header, edited\n")
    assert bench.traffic_of("smooth0", "fp64") is None


def test_traffic_withdrawn_for_a_foreign_hash(tmp_path, monkeypatch):
    _fake_tree(tmp_path, monkeypatch, {"a.hip": "kernel A\n"}, fetch=1.0, write=1.0,
               sha="0" * 64)
    assert bench.traffic_of("smooth0", "fp64") is None


def test_committed_traffic_summaries_name_existing_sources():
    seen = 0
    for (kernel, prec), (fname, files) in bench.TRAFFIC.items():
        path = os.path.join(ROOT, "profiles", fname)
        assert os.path.exists(path), fname
        for f in files:
            assert os.path.exists(os.path.join(bench.CSRC, f)), f
        with open(path) as fh:
            recs = [json.loads(ln[len("traffic-json: "):]) for ln in fh
                    if ln.startswith("traffic-json: ")]
        rec = [r for r in recs if r["kernel"] == kernel]
        assert len(rec) == 1, (fname, kernel)
        assert rec[0]["sources"] == files
        assert rec[0]["fetch_bytes_per_launch"] > 0 and rec[0]["write_bytes_per_launch"] > 0
        seen += 1
    assert seen == 6


def test_roofline_of_picks_the_dominant_kernel(monkeypatch):
    monkeypatch.setattr(bench, "traffic_of", lambda k, p: None)
    n = 1_000_000
    prof = {"smooth0": (30.0, 100, 100 * 2.0e9),      # 0.3 ms per launch, 2 GB each
            "assemble_h0": (20.0, 4, 4 * 3.0e9),       # 5 ms per launch
            "vcycle": (500.0, 10, 10 * 2.5e10)}        # a span, never the dominant kernel
    r = bench.roofline_of(prof, n, "fp64")
    assert r["kernel"] == "smooth0" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(2.0e9 / 0.3e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    prof["assemble_h0"] = (40.0, 4, 4 * 3.0e9)         # now 10 ms per launch, dominant
    r = bench.roofline_of(prof, n, "fp64")
    assert r["kernel"] == "assemble_h0" and r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(24786 * n / 10e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6)
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(3.0e9)


def test_vcycle_roofline_spans_the_whole_cycle(monkeypatch):
    monkeypatch.setattr(bench, "traffic_of", lambda k, p: 7.0)
    prof = {"vcycle": (50.0, 10, 10 * 2.0e10), "smooth0": (36.0, 90, 90 * 2.0e9),
            "residual0": (4.0, 10, 10 * 2.0e9)}
    v = bench.vcycle_roofline(prof, "fp64")
    assert v["avg_cycle_ms"] == pytest.approx(5.0)
    assert v["achieved"] == pytest.approx(2.0e10 / 5e-3 / 1e9)
    lp = v["level0_passes"]
    assert lp["kernels"] == ["smooth0", "residual0"]
    assert lp["achieved"] == pytest.approx(100 * 2.0e9 / 40e-3 / 1e9)
    assert lp["smooth0"]["avg_launch_ms"] == pytest.approx(0.4)
    assert lp["residual0"]["traffic"] == 7.0
    assert bench.vcycle_roofline({"vcycle": (0.0, 0, 0.0)}, "fp64") is None
