"""The build's guard against vector-register spills (the per-lane loops
keep every per-cell value in registers): the remark parser finds the
kernels that spill and only those."""
from paper_2604_21438_amd.build import vgpr_spills

REMARKS = """\
k.hip:10:1: remark: Function Name: _Z4goodv [-Rpass-analysis=kernel-resource-usage]
k.hip:10:1: remark:     VGPRs: 120 [-Rpass-analysis=kernel-resource-usage]
k.hip:10:1: remark:     SGPRs Spill: 3 [-Rpass-analysis=kernel-resource-usage]
k.hip:10:1: remark:     VGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]
k.hip:20:1: remark: Function Name: _Z3badv [-Rpass-analysis=kernel-resource-usage]
k.hip:20:1: remark:     SGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]
k.hip:20:1: remark:     VGPRs Spill: 47 [-Rpass-analysis=kernel-resource-usage]
"""


def test_vgpr_spill_parser():
    assert vgpr_spills(REMARKS) == {"_Z3badv": 47}
    assert vgpr_spills("") == {}
