"""The library build refuses kernels that use scratch memory.

Launch shapes that spilled registers were the only ones that ever computed
wrong values (the cross-lane column exchange reads a neighbour's register
whatever that lane's state; a spill inside a divergent region restores only
the active lanes), and a private array kept in scratch turns register reads
into memory traffic inside the march; the build reads the compiler's
resource report of every kernel and fails on scratch, on spills and on
accumulation registers (with no matrix-core code, they only hold spills).
"""
import os

import pytest

from paper_1206_0270_amd.csrc import build as libbuild

SAMPLE = """\
x.hip:10:1: remark: Function Name: _Z6k_goodv [-Rpass-analysis=kernel-resource-usage]
x.hip:10:1: remark:     VGPRs: 120 [-Rpass-analysis=kernel-resource-usage]
x.hip:10:1: remark:     AGPRs: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:10:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:10:1: remark:     Occupancy [waves/SIMD]: 4 [-Rpass-analysis=kernel-resource-usage]
x.hip:10:1: remark:     VGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:20:1: remark: Function Name: _Z5k_badv [-Rpass-analysis=kernel-resource-usage]
x.hip:20:1: remark:     VGPRs: 256 [-Rpass-analysis=kernel-resource-usage]
x.hip:20:1: remark:     ScratchSize [bytes/lane]: 48 [-Rpass-analysis=kernel-resource-usage]
x.hip:20:1: remark:     Occupancy [waves/SIMD]: 2 [-Rpass-analysis=kernel-resource-usage]
x.hip:20:1: remark:     VGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]
"""


def test_resource_report_is_parsed_per_kernel():
    r = libbuild.kernel_resources(SAMPLE)
    assert set(r) == {"_Z6k_goodv", "_Z5k_badv"}
    assert r["_Z6k_goodv"] == {"VGPRs": 120, "AGPRs": 0, "ScratchSize": 0, "Occupancy": 4, "VGPRs Spill": 0}
    assert r["_Z5k_badv"]["ScratchSize"] == 48


def test_built_kernels_use_no_scratch():
    path = os.path.join(libbuild.BUILD, "kernel_resources.txt")
    if not os.path.exists(path):
        pytest.skip("library not built here (build() writes the report)")
    with open(path) as f:
        lines = [ln for ln in f if ln.strip()]
    assert len(lines) >= 20  # every compiled kernel variant is listed
    for ln in lines:
        assert "'ScratchSize': 0" in ln and "'VGPRs Spill': 0" in ln and "'AGPRs': 0" in ln, ln
