"""Register budgets of the step kernels (host only: hipcc device assembly).

The z pass of long transforms is held to 3 waves per SIMD (at most 168
VGPRs); a spill there costs one scratch write and one read per wave and
showed up in the HBM counters as 2 x 101 MB per launch at 256^3.  The
64-point z pass must stay within 6 waves per SIMD (80 VGPRs) and the fused
x-inverse + update too (two 768-thread blocks per CU).
These are properties of the compiled code that the timing and traffic
figures rest on, so a change that breaks them fails here instead of
showing up as a slower profile.  Skipped without hipcc.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    from paper_1411_2565_amd import build
    out = str(tmp_path_factory.mktemp("asm") / "kernels.s")
    cmd = [HIPCC] + build.FLAGS + ["--cuda-device-only", "-S",
                                   os.path.join(build.CSRC, "kernels.hip"), "-o", out]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    text = open(out).read()
    res = {}
    for blk in text.split("  - .agpr_count")[1:]:
        name = re.search(r"\.name:\s+(\S+)", blk).group(1)
        get = lambda k: int(re.search(r"\." + k + r":\s+(\d+)", blk).group(1))  # noqa: E731
        res[name] = (get("vgpr_count"), get("vgpr_spill_count"))
    return res


def find(res, prefix):
    hits = {n: v for n, v in res.items() if n.startswith(prefix)}
    assert hits, prefix
    return hits


@pytest.mark.parametrize("L", [256, 512])
def test_long_z_pass_does_not_spill(kernels, L):
    # plain multiply, single sample and batch table
    for name, (vgpr, spill) in find(kernels, f"_ZN3mmk11k_zconv_seqILi{L}ELb0ELi0E").items():
        assert spill == 0 and vgpr <= 168, (name, vgpr, spill)


def test_short_z_pass_six_waves(kernels):
    # k_zconv64<COMP = false, TAB = false>: 6 waves per SIMD (<= 80 VGPRs)
    for name, (vgpr, spill) in find(kernels, "_ZN3mmk9k_zconv64ILb0ELb0E").items():
        assert spill == 0 and vgpr <= 80, (name, vgpr, spill)


def test_fused_pass_two_blocks_per_cu(kernels):
    # k_xinv_euler<256, 8, 4, TAB = false, XF = false, MAPPED = false>
    for name, (vgpr, spill) in find(kernels, "_ZN3mmk12k_xinv_eulerILi256ELi8ELi4ELb0ELb0ELb0E").items():
        assert spill == 0 and vgpr <= 80, (name, vgpr, spill)
