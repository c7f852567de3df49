"""The measured FP32 vector ceiling (tm_probe_fp32_fma) against the chip's unit counts.

Without packed FP32 instructions an MI355X compute unit retires 64 FMA lanes per clock:
256 CUs x 64 x 2 flops x 2.4 GHz = 78.6 TFLOP/s.  The probe must land below that
(it cannot beat the hardware) and well above half of it (the loop is pure FMA).
"""
import pytest

import paper_1610_02370_amd as tm

from gpu_util import announce

pytestmark = pytest.mark.gpu


def test_fp32_fma_probe_against_unit_counts():
    import torch

    # the device and its runtime come up through torch, as in every caller of the library
    torch.cuda.set_device(0)
    torch.zeros(1, device="cuda")
    announce("FP32 FMA probe")
    t = tm.tm_probe_fp32_fma()
    print(f"measured FP32 vector FMA rate: {t:.1f} TFLOP/s", flush=True)
    assert 39.3 < t < 78.6 * 1.02
