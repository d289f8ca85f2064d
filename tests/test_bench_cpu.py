"""Host-side logic of bench.py (no GPU): the algorithmic byte counts behind
the roofline, the guard that drops a stored traffic figure once it no longer
describes the kernel, and the single-GPU refusal."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes():
    # 16x16x8 window, 17x17 grid: the Hermitian half of the spectrum is
    # 8 planes x 16 ky x 8 kz complex FP32 = 8 KB, read and written; the
    # smoothed R is 289 FP32, read and written; frame, delayed frame, output
    # (4 B each), velocity (8 B) and index (4 B)
    assert bench.algorithmic_bytes_per_pixel_frame((16, 16, 8), 289) == 2 * 8192 + 2 * 1156 + 24 == 18720
    # 8x8x4 window, 9x9 grid: 4 planes x 8 x 4 complex = 1 KB each way
    assert bench.algorithmic_bytes_per_pixel_frame((8, 8, 4), 81) == 2 * 1024 + 2 * 324 + 24 == 2720
    # ring of 2-D spectra: 7 slots of 8 x 16 complex read, 1 written
    assert bench.ring_bytes_per_pixel_frame((16, 16, 8), 289) == 8 * 1024 + 2312 + 24 == 10528


def test_measured_traffic_only_for_the_kernel_it_describes(tmp_path, monkeypatch):
    d = bench.kernel_source_digest()
    f = tmp_path / "traffic_pixel16_640x512.txt"
    f.write_text("# comment=ignored\nkernel=k_pixel16\nworkload=640x512\nsource_sha256=%s\n"
                 "hbm_bytes_per_launch=123456\n" % d)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic_pixel16_{workload}.txt"))
    assert bench.measured_traffic("k_pixel16", "640x512") == 123456.0
    assert bench.measured_traffic("k_pixel", "640x512") is None          # another kernel
    assert bench.measured_traffic("k_pixel16", "1280x1024") is None      # no summary for it
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0" * 16)
    assert bench.measured_traffic("k_pixel16", "640x512") is None        # sources changed


def test_committed_traffic_summaries_match_the_sources():
    """The committed counter summaries were taken on the current kernel
    sources (else bench.py would report traffic as null)."""
    for wl in ("640x512", "1280x1024"):
        assert bench.measured_traffic("k_pixel16", wl) is not None, wl
    assert bench.measured_traffic("k_pixel16<4>", "640x512", "ring") is not None
    assert bench.measured_traffic("k_pixel16<5>", "640x512", "direct") is not None
    assert bench.measured_traffic("k_pixel16<6>", "640x512", "pairs") is not None


def test_pair_bytes_model():
    """Frame pairs move the state and smoothed R once per two frames."""
    single = bench.algorithmic_bytes_per_pixel_frame((16, 16, 8), 289)
    pair = bench.pair_bytes_per_pixel_frame((16, 16, 8), 289)
    assert pair == (single - 24) / 2 + 18


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("wl", sorted(bench.WORKLOADS))
def test_workloads_are_well_formed(wl):
    w = bench.WORKLOADS[wl]
    assert w["H"] >= 1 and w["W"] >= 1 and len(w["M"]) == 3


def test_batch_cpu_baseline_aggregates_the_step(monkeypatch):
    """The batched workload's oracle rate: one strip per size class, combined
    as the step's pixel count over the summed per-stream times."""
    import numpy as np

    from paper_1408_3526_amd import scenes
    g8, g16 = scenes.grid(-1, 1, 1.0), scenes.grid(-1, 1, 1.0)
    rng = np.random.default_rng(0)
    specs = [dict(H=20, W=24, M=(8, 8, 4), gx=g8, gy=g8), dict(H=20, W=24, M=(8, 8, 4), gx=g8, gy=g8),
             dict(H=24, W=20, M=(16, 16, 8), gx=g16, gy=g16)]
    frames = [rng.normal(size=(2, sp["H"], sp["W"])).astype(np.float32) for sp in specs]
    r = bench.cpu_baseline_batch(frames, specs, strip_rows=8, n_frames=2)
    assert r["kind"] == "oracle" and r["cores"] >= 1
    # two size classes timed; the aggregate is px / (2 * 480 / rate8 + 480 / rate16)
    rates = {c["stream"]: c["rate"] for c in r["per_class"]}
    assert len(rates) == 2
    expect = 3 * 480 / (2 * 480 / rates["24x20 @8x8x4"] + 480 / rates["20x24 @16x16x8"])
    assert abs(r["value"] - expect) <= 1e-9 * expect
