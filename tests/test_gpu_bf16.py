"""The network kernels round to bfloat16 with the hardware conversion
(v_cvt_pk_bf16_f32): its result must be round-to-nearest-even, the rounding
the network's definition takes at every stored tensor, for every float32
bit pattern but the NaNs (2^32 - 2^24 + 2 inputs, on the device)."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_hardware_bf16_rounding_is_round_to_nearest_even():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_00558_amd as m
    m.lib()
    print("[gpu] bfloat16 rounding over all float32 patterns", flush=True)
    sys.stdout.flush()
    assert m.check_bf16(0) == 0
