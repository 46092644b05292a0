"""The launch-parameter block passed by value to every kernel stays within
512 bytes: builds whose block had grown past that hung in the cooperative fit
launch on the GPU (three runs), while every run at 512 bytes passed.  Device
buffers added later belong in the device state, reached through a pointer."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_launch_parameters_fit_in_512_bytes(tmp_path):
    src = tmp_path / "size.hip"
    src.write_text('#include "asp_device.h"\n'
                   "static_assert(sizeof(asp::Params) <= 512, \"launch parameters\");\n")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    res = subprocess.run([hipcc, "--offload-arch=gfx950", "-fsyntax-only", "-I",
                          os.path.join(ROOT, "include"), "-I",
                          os.path.join(ROOT, "paper_1606_07872_amd", "csrc"), str(src)],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
