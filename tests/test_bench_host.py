"""Host-side checks of bench.py's contract (no GPU): the multi-GPU refusal,
the algorithmic byte model of the step passes, and the measured-traffic
record tied to the kernel sources."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_padded_sizes():
    assert [bench.padded(n) for n in (1, 2, 3, 16, 17, 32, 125, 256, 500, 512)] == \
        [1, 4, 8, 32, 64, 64, 256, 512, 1024, 1024]


def test_byte_model_of_the_block_step():
    """Per-pass algorithmic bytes of the 256x256x32 step (complex64 spectra,
    FP32 state, real octant tensor): the a1-a4 figures and the 734.15 MB
    total of the fused step, and the 784.5 MB of the step with the
    x-inverse and the update as two kernels (H_demag written and read
    back)."""
    kb = bench.kernel_bytes((256, 256, 32), (512, 512, 64))
    mb = {k: v / 1e6 for k, v in kb.items()}
    assert abs(mb["xfwd"] - 75.7) < 0.1
    assert abs(mb["yfwd"] - 151.6) < 0.1
    assert abs(mb["zconv"] - 254.4) < 0.1
    assert abs(mb["yinv"] - 151.6) < 0.1
    assert abs(mb["xinv_local"] - 100.86) < 0.01
    unfused = ("xfwd", "yfwd", "zconv", "yinv", "xinv", "local")
    assert abs(sum(mb[k] for k in unfused) - 784.48) < 0.1
    # the fused tail does not write H_demag and read it back: 2 x 25.17 MB
    h_round_trip = 2 * 4 * 3 * 256 * 256 * 32
    assert abs(kb["xinv"] + kb["local"] - h_round_trip - kb["xinv_local"]) == 0
    # chaining the next step's x-forward into the fused pass saves that
    # x-forward's read of m (25.17 MB): 709.0 MB per step in steady state
    m_bytes = 4 * 3 * 256 * 256 * 32
    assert kb["xfwd"] + kb["xinv_local"] - kb["xinv_local_xfwd"] == m_bytes
    chained = kb["yfwd"] + kb["zconv"] + kb["yinv"] + kb["xinv_local_xfwd"]
    assert abs(chained / 1e6 - 708.98) < 0.01
    # the headline fraction of HBM peak is taken on that 734.15 MB model
    assert abs(bench.model_bytes((256, 256, 32), (512, 512, 64)) / 1e6 - 734.15) < 0.1


def test_measured_traffic_is_tied_to_the_sources():
    rec = bench.MEASURED_TRAFFIC["zconv"]
    assert rec["bytes_per_launch"] > bench.kernel_bytes((256, 256, 32), (512, 512, 64))["zconv"]
    got = bench.measured_traffic("zconv")
    assert got in (None, rec["bytes_per_launch"])
    if rec["source_sha"] == bench.kernel_source_sha():
        assert got == rec["bytes_per_launch"]
    assert bench.measured_traffic("no such kernel") is None
