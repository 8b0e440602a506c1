"""The line-FFT device code run on the CPU.

`paper_2604_15796_amd/csrc/fft.hpp` is compiled with g++ against a host
stand-in for the HIP runtime header, one workgroup running as host threads
with a shared barrier, and every FFT length, plan family (radix 8/6/4/3 and
radix 16/32), line layout and precision is compared with a direct DFT:
forward transforms of zero-padded lines, inverse transforms cropped to half a
line, and the fused convolution (forward, multiply, inverse), with the
twiddle powers built per butterfly and read from a per-stage power table.
This checks the index arithmetic of the Stockham stages without a GPU; the
build uses the address sanitizer, and every array (the LDS image and the
power table included) is sized exactly, so an access out of bounds fails.
"""
import os
import pathlib
import shutil
import subprocess

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
EMU = ROOT / "tests" / "host_emu"
CSRC = ROOT / "paper_2604_15796_amd" / "csrc"


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_line_fft_plans_on_host(tmp_path):
    # four quarters of the configurations, built and run in parallel
    parts = range(4)
    exes = [tmp_path / f"fft_plans_{k}" for k in parts]
    builds = [subprocess.Popen(["g++", "-std=c++20", "-O1", "-fsanitize=address", f"-DFWI_EMU_PART={k}",
                                f"-I{EMU}", f"-I{CSRC}", str(EMU / "fft_plans.cpp"), "-o", str(exes[k]), "-lpthread"])
              for k in parts]
    assert all(b.wait(timeout=900) == 0 for b in builds)
    runs = [subprocess.Popen([str(e)], stdout=subprocess.PIPE, text=True) for e in exes]
    outs = [r.communicate(timeout=900)[0] for r in runs]
    assert all(r.returncode == 0 for r in runs)
    out = "".join(outs)
    lines = [l for l in out.splitlines() if l.strip()]
    assert len(lines) == 43, out
    bad = [l for l in lines if not l.endswith(" ok")]
    assert not bad, "\n".join(bad)
    assert sum(" BIG=1 " in l for l in lines) >= 10  # the radix-32/16/12 plans are exercised
    assert sum(" L= 192 " in l and " BIG=1 " in l for l in lines) == 2  # 16 x 12, both precisions


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_fused_lateral_elevation_passes_on_host(tmp_path):
    """The fused 3D lateral-elevation passes (csrc/xy_passes.hpp) on one
    z-plane, one workgroup as host threads, built with the address sanitizer:
    class-major forward spectrum against a direct 2D DFT of the padded
    operand, the inverse against a direct inverse DFT, the Gram-Schmidt and
    start operands with their per-row norms, and the operator epilogue."""
    exes = [tmp_path / f"xy_plans_{k}" for k in (0, 1)]  # the two shapes, in parallel
    builds = [subprocess.Popen(["g++", "-std=c++20", "-O1", "-fsanitize=address", f"-DFWI_XY_PART={k}",
                                f"-I{EMU}", f"-I{CSRC}", str(EMU / "xy_plans.cpp"), "-o", str(e), "-lpthread"])
              for k, e in enumerate(exes)]
    assert all(b.wait(timeout=900) == 0 for b in builds)
    runs = [subprocess.Popen([str(e)], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True) for e in exes]
    res = [r.communicate(timeout=900) for r in runs]
    out = "".join(o for o, _ in res)
    lines = [l for l in out.splitlines() if l.strip()]
    assert all(r.returncode == 0 for r in runs), out + "".join(e for _, e in res)
    assert len(lines) == 22, out
    bad = [l for l in lines if not l.endswith(" ok")]
    assert not bad, "\n".join(bad)
