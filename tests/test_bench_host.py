"""Host-side parts of bench.py that run without a GPU: the one-GPU refusal,
the committed HBM-traffic record and the rule that its bytes are reported
only for the kernel source they were measured on."""

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RECORD = os.path.join(ROOT, "profiles", "k_star25_wave_1024x1024x512_traffic.json")
NPTS = 1024 * 1024 * 512


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr
    assert r.stdout.strip() == "" or not r.stdout.strip().startswith("{")


def test_traffic_record_is_plausible():
    with open(RECORD) as fh:
        rec = json.load(fh)
    reads, writes = rec["read_bytes"], rec["write_bytes"]
    assert rec["bytes_per_launch"] == reads + writes
    # the leapfrog reads u^n, u^{n-1}, v (12 B) and writes u^{n+1} (4 B) per
    # point: the counters can exceed that (halo re-reads) but not undercut it
    assert 12 * NPTS <= reads <= 1.25 * 12 * NPTS
    assert 4 * NPTS <= writes <= 1.05 * 4 * NPTS
    assert len(rec["source_hash"]) == 16
    assert os.path.exists(os.path.join(ROOT, rec["summary"]))


def test_traffic_is_reported_only_for_the_measured_source(monkeypatch):
    with open(RECORD) as fh:
        rec = json.load(fh)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: rec["source_hash"])
    assert bench.measured_traffic() == rec["bytes_per_launch"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic() is None


def test_kernel_source_hash_covers_the_kernel_sources(tmp_path, monkeypatch):
    # editing any of the hashed sources changes the hash
    h0 = bench.kernel_source_hash()
    csrc = tmp_path / "paper_2309_04671_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in ("star25.hip", "kcommon.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_2309_04671_amd", "csrc", name), "rb") as fh:
            (csrc / name).write_bytes(fh.read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == h0
    for name in ("star25.hip", "kcommon.h", "internal.h"):
        p = csrc / name
        data = p.read_bytes()
        p.write_bytes(data + b"\n")
        assert bench.kernel_source_hash() != h0, name
        p.write_bytes(data)


def test_committed_line_keeps_the_reporting_contract():
    # the latest full bench line kept under profiles/: keys, units and the
    # arithmetic that ties value, ms_per_step and the roofline together
    with open(os.path.join(ROOT, "profiles", "bench_1024x1024x512_full.json")) as fh:
        d = json.load(fh)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["unit"] == "GPts/s" and d["dtype"] == "f32" and d["data"] == "synthetic"
    assert d["higher_is_better"] is True and d["vs_baseline"] is None
    assert "workload" in d["config"] and d["config"]["grid"] == [1024, 1024, 512]
    steps = d["config"]["time_steps"]
    # value: points x time steps of one simulation over the wall time of one
    assert abs(d["value"] - NPTS * steps / (d["ms_per_step"] * 1e-3) / 1e9) <= 1e-3 * d["value"]
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["bytes_per_launch"] == 16 * NPTS
    assert abs(r["achieved"] - r["bytes_per_launch"] / (r["avg_launch_us"] * 1e-6) / 1e9) <= 0.1
    assert abs(r["frac"] - r["achieved"] / r["peak"]) <= 1e-3
    # the launches fit inside the wall time of a simulation
    assert steps * r["avg_launch_us"] * 1e-3 <= d["ms_per_step"]
    assert r["traffic"] is None or 16 * NPTS <= r["traffic"] <= 1.1 * 16 * NPTS
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["unit"] == "GPts/s" and c["cores"] >= 1 and c["value"] > 0
