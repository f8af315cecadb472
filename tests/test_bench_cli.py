"""Host-side checks of the benchmark script (no GPU): it refuses more than one
GPU with a message, and its measured-traffic lookup only accepts counters
taken from the current kernel sources."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_is_reported_only_for_matching_kernel_sources(tmp_path, monkeypatch):
    """The lookup reports a profiled tile's bytes only from a summary taken
    from the current kernel sources (same hash), for the same workload and
    tile shape; the committed summary is used as the template."""
    sys.path.insert(0, ROOT)
    import bench
    name = "headon_sinhcylindrical_128x2x256"
    counters = open(bench.COUNTERS).read()
    # the committed summary names its workload and the sources' hash
    assert f"workload: {name}" in counters and "source_sha256:" in counters

    def with_hash(h):
        f = tmp_path / f"counters_{h[:8]}.txt"
        lines = [("source_sha256: " + h) if l.startswith("source_sha256:") else l for l in counters.splitlines()]
        f.write_text("\n".join(lines) + "\n")
        return str(f)

    tiles = [l.split(":")[0].rsplit("_", 3)[1:] for l in counters.splitlines()
             if l.startswith("hbm_bytes_per_launch_tile_")]
    assert tiles
    # taken from the current sources: every profiled tile shape is reported
    fresh = with_hash(bench.kernel_source_hash())
    monkeypatch.setattr(bench, "COUNTERS", fresh)
    for t in tiles:
        assert bench.measured_traffic(name, [int(x) for x in t]) is not None
    # nor for another workload than the summary names, nor for a shape never profiled
    monkeypatch.setattr(bench, "COUNTERS_3D", fresh)
    assert bench.measured_traffic("vacuum3d_sinhspherical_256x128x64") is None
    assert bench.measured_traffic(name, [2, 0, 1]) is None
    # a summary whose hash does not match the sources gives no traffic
    monkeypatch.setattr(bench, "COUNTERS", with_hash("0" * 64))
    assert bench.measured_traffic(name) is None
    for t in tiles:
        assert bench.measured_traffic(name, [int(x) for x in t]) is None
