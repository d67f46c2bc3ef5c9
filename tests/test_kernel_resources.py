"""Register budget of the element kernels on the hot path (no GPU: the
compiler's resource report for gfx950).

The element operator is latency-bound, so its speed rests on how many waves a
SIMD holds: the kernels that the benchmark and the junction solves launch
must not spill and must keep the occupancy they were tuned for (the Picard
tangent three waves in FP64 and four in FP32; the Newton tangent at K = 3
three in FP64 and four in FP32, at K = 6 two in FP64).  A source change that
pushes one of them over its register budget fails here rather than as a
slowdown on the GPU.
"""
import os
import re
import subprocess
import tempfile

import pytest

from paper_2311_09465_amd import build as B

# (K, mode, type) -> fewest waves per SIMD; mode 0 Picard, 2 Newton,
# 16 Picard with tau in bf16, 18 Newton with tau in bf16, 32 the work-list
# instantiation of the Picard tangent used by segmented solves
EXPECT = {
    (6, 0, "d"): 3, (6, 0, "f"): 4, (6, 16, "f"): 4,
    (3, 0, "d"): 3, (3, 0, "f"): 4,
    (3, 2, "d"): 3, (3, 2, "f"): 4, (3, 18, "f"): 4,
    (6, 2, "f"): 3, (6, 2, "d"): 2, (7, 32, "d"): 3,
}


def _report():
    src = os.path.join(B.SRC, "elemop.hip")
    with tempfile.TemporaryDirectory() as d:
        cmd = [B.HIPCC] + B.COMMON + ["-x", "hip", "--offload-device-only", "-c", src,
                                      "-o", os.path.join(d, "elemop.o"),
                                      "-Rpass-analysis=kernel-resource-usage"]
        res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    out, cur = {}, None
    for line in res.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            out[cur] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z \[\]/]+): (\d+)", line)
        if m and cur:
            out[cur][m.group(1).strip()] = int(m.group(2))
    return out


@pytest.mark.slow
def test_hot_element_kernels_keep_their_occupancy_without_spilling():
    if not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not found")
    rep = _report()
    for (K, mode, t), waves in EXPECT.items():
        prefix = f"_ZN5tsgls4k_opILi{K}ELi{mode}E{t}E"
        hits = [v for k, v in rep.items() if k.startswith(prefix)]
        assert len(hits) == 1, f"k_op<{K}, {mode}, {t}> not found in the resource report"
        r = hits[0]
        assert r["ScratchSize [bytes/lane]"] == 0 and r["VGPRs Spill"] == 0, (K, mode, t, r)
        assert r["Occupancy [waves/SIMD]"] >= waves, (K, mode, t, r)
