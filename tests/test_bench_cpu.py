"""Host-side parts of bench.py: the one-GPU contract, the per-launch byte models the roofline uses,
and the reading of committed counter summaries.  No GPU work."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_algorithmic_bytes_of_the_z_c2r_pass():
    n = 768
    G, C = n ** 3, n * n * (n // 2 + 1)
    assert bench.algorithmic_bytes("fft_z_c2r", n, n, 256) == 8 * C + 4 * G == 3628597248


def test_step_byte_models():
    floor, three = bench.floor_bytes(768, 256)
    assert 0 < floor < three
    # the three-pass model moves each 3D FFT's data three times
    G, C = 768 ** 3, 768 * 768 * 385
    fft = (4 * G + 8 * C) + 3 * (8 * C + 4 * G)
    assert three - floor == 2 * fft


def test_committed_counters_are_read_only_for_current_sources():
    got = bench.read_traffic("fft_z_c2r3", 768)
    path = os.path.join(ROOT, "profiles", "fft_z_c2r3_768_counters.txt")
    stamped = dict(line.split(":", 1) for line in open(path) if ":" in line and not line.startswith("#"))
    alg = bench.algorithmic_bytes("fft_z_c2r3", 768, 768, 256)
    assert alg == 24 * 768 * 768 * 385 + 12 * 768 ** 3
    if stamped["source_hash"].strip() == bench.source_hash("fft_z_c2r3"):
        # counter bytes within a few per cent of the algorithmic bytes (row padding and ghost
        # cells of the interleaved force mesh): no re-reads
        assert abs(got / alg - 1) < 0.08
    else:
        assert got is None
