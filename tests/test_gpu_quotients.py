"""The kernels' reciprocal of a projected depth (hardware estimate, one
Newton step, the all-ones-significand correction) and the quotients derived
from it, against correctly rounded division on the device: every
significand of the binades 2^-7 .. 2^20 (projected depths from the 0.01 m
clip plane to a million metres), two dividends per divisor."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_reciprocal_and_quotients_match_division_on_device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_00558_amd as m
    m.lib()
    print("[gpu] reciprocal check over 28 binades", flush=True)
    sys.stdout.flush()
    assert m.check_reciprocal(0, -7, 20) == 0
