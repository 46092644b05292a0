"""Resources of the kernels whose work-groups wait for one another (the
cooperative fit kernel and the persistent batched kernel), read from the
compiler's resource-usage remarks of a gfx950 build (CPU only).

Every work-group of such a launch must be resident at once, or a wait between
work-groups never ends.  A private segment (scratch) breaks that guarantee:
the waves of a dispatch can be held back until scratch is free.  The library
refuses such a launch at run time too (fit_grid_size / batch_grid_size); this
test keeps a build with scratch from getting that far."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1606_07872_amd", "csrc")

WAITING_KERNELS = {"_ZN3asp5k_fitENS_6ParamsE": "k_fit", "_ZN3asp7k_batchENS_9BatchArgsE": "k_batch"}


def resource_remarks(source):
    from paper_1606_07872_amd import build
    cmd = ["/opt/rocm/bin/hipcc", *[f for f in build.HIPCC_FLAGS if f != "-shared"],
           "--cuda-device-only", "-c", "-o", os.devnull, "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, os.path.join(CSRC, source), "-Rpass-analysis=kernel-resource-usage"]
    out = subprocess.run(cmd, capture_output=True, text=True, check=True).stderr
    kernels, cur = {}, None
    for line in out.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = kernels.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([A-Za-z][A-Za-z /\[\]]*?):\s+(\S+) \[", line)
        if m and cur is not None:
            cur[m.group(1).strip()] = m.group(2)
    return kernels


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_waiting_kernels_have_no_private_segment():
    k = resource_remarks("fit.hip")
    for sym, name in WAITING_KERNELS.items():
        assert sym in k, (name, sorted(k))
        r = k[sym]
        print(name, {key: r[key] for key in ("VGPRs", "AGPRs", "ScratchSize [bytes/lane]",
                                             "Occupancy [waves/SIMD]", "LDS Size [bytes/block]")})
        assert r["ScratchSize [bytes/lane]"] == "0", (name, r)
        assert r["Dynamic Stack"] == "False", (name, r)
        assert int(r["Occupancy [waves/SIMD]"]) >= 1, (name, r)
