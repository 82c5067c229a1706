"""Host logic of bench.py that runs without a GPU: the one-GPU refusal and the
reading of the committed counter profile (traffic is reported only while the
kernel sources are the ones the counters were taken with)."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def _profile(tmp_path, sources, sha):
    p = tmp_path / "traffic.txt"
    p.write_text("# header line: ignored\n"
                 "traffic_fetch_bytes: 5.0e+09\n"
                 "traffic_write_bytes: 1.0e+09\n"
                 "traffic_bytes: 6.0e+09\n"
                 f"kernel_sources_sha256: {sha}\n"
                 f"kernel_sources: {' '.join(sources)}\n")
    return str(p)


def _sha(sources):
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def test_traffic_read_while_sources_match(tmp_path, monkeypatch):
    src = ["paper_2311_07554_amd/csrc/common.h", "paper_2311_07554_amd/csrc/hook_kernels.h"]
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", _profile(tmp_path, src, _sha(src)))
    t = bench.sampling_kernel_traffic()
    assert t is not None
    assert t["bytes"] == 6.0e9 and t["fetch_bytes"] == 5.0e9 and t["write_bytes"] == 1.0e9


def test_traffic_dropped_when_sources_changed(tmp_path, monkeypatch):
    src = ["paper_2311_07554_amd/csrc/common.h", "paper_2311_07554_amd/csrc/hook_kernels.h"]
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", _profile(tmp_path, src, "0" * 64))
    assert bench.sampling_kernel_traffic() is None
    # a source list that no longer exists, and a missing profile
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", _profile(tmp_path, ["no/such/file.h"], _sha(src)))
    assert bench.sampling_kernel_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.txt"))
    assert bench.sampling_kernel_traffic() is None


def test_committed_profiles_name_their_command_and_calibration():
    for name in ("k_sample_hook_rmat20_traffic.txt", "k_sample_hook_rmat24_traffic.txt"):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            text = f.read()
        assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text
        assert "k_probe_copy" in text and "factor" in text


def test_fifo_latencies_of_the_plain_path():
    # one server, first come first served: a request waits for the one before it
    lat = bench.fifo_latencies([0.0, 1.0, 1.5, 10.0], [2.0, 2.0, 0.5, 1.0])
    assert lat == [2.0, 3.0, 3.0, 1.0]
    assert bench.fifo_latencies([], []) == []


def test_phase_frames_on_the_method_bytes():
    from types import SimpleNamespace
    g = SimpleNamespace(n=1 << 20, m_und=1 << 24)
    kern = {"sample_hook": {"launches": 4, "avg_ms": 2.0}, "bulk_keys": {"launches": 1, "avg_ms": 1.0}}
    f = bench.phase_frames(kern, True, g, 1 << 19, 64, 4, 256, g.n, 10.0)
    sk = f["phases"]["sketch"]
    # 4 passes of half-CSR plus E (8 R n bytes), over the 10 ms build
    want = 4 * (4.0 * g.m_und + 4.0 * g.n) + 8.0 * 256 * g.n
    assert sk["algorithmic_bytes_per_build"] == want
    assert abs(sk["GB_s"] - want / 1e-2 / 1e9) < 1e-6
    assert f["kernels"]["sample_hook"]["streaming_bytes_per_launch"] == 16.0 * g.m_und
    mb = f["phases"]["marginal_bulk"]
    assert mb["algorithmic_bytes_per_launch"] == 8.0 * 256 * g.n + 9.0 * g.n
