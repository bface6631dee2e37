"""Register budget of the FP32 lattice kernels (no GPU needed: hipcc reports
each kernel's resources when it compiles cfust_estep.hip for gfx950).

The E-step's time is the FP32 lattice loop, bound by VALU issue; its speed
depends on enough resident waves per SIMD, so the kernels that read the
lattice coordinate table (k_estep_qmc<m, FP32, 1 point per lane, table>) must
stay within their register budgets and use no scratch beyond the fixed call
frame.  A refactor that stops the integrand from being inlined (it once took
the m = 7 / 8 kernels from 122 / 116 to 197 / 229 VGPRs) fails here."""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "paper_1606_02054_amd", "csrc", "cfust_estep.hip")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# VGPR budget per m: 8 waves per SIMD up to m = 4 (at most 64 VGPRs), then the
# occupancy the kernels are held to (fp32_min_blocks) or reach.
BUDGET = {2: 64, 3: 64, 4: 64, 5: 80, 6: 96, 7: 128, 8: 128}
FRAME_BYTES = 32      # the out-of-line FP64 prologue/epilogue calls' frame


def _resources():
    out = subprocess.run(
        [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-fno-fast-math", "--cuda-device-only", "-c", "-Rpass-analysis=kernel-resource-usage",
         SRC, "-o", os.devnull], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    res, cur = {}, None
    for line in out.stderr.splitlines():
        mm = re.search(r"Function Name: (\S+)", line)
        if mm:
            cur = mm.group(1)
            res[cur] = {}
            continue
        mm = re.search(r"remark:\s+(VGPRs|ScratchSize \[bytes/lane\]): (\d+)", line)
        if cur and mm:
            res[cur][mm.group(1)] = int(mm.group(2))
    return res


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not available")
def test_lattice_kernel_register_budget():
    res = _resources()
    for m, budget in BUDGET.items():
        name = f"_ZN5cfust11k_estep_qmcILi{m}ELb1ELi1ELb1EEEvNS_12EstepQmcArgsE"
        assert name in res, f"kernel k_estep_qmc<{m}, FP32, 1, table> not found"
        r = res[name]
        assert r["VGPRs"] <= budget, f"m = {m}: {r['VGPRs']} VGPRs > {budget}"
        assert r.get("ScratchSize [bytes/lane]", 0) <= FRAME_BYTES, f"m = {m}: scratch {r}"
