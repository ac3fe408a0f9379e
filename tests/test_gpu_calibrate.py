"""The integer-VALU calibration kernel (pa_calibrate_philox) returns a
finite rate of Philox calls per second below what the issue rate allows:
each call is 40 VALU operations, so at most 256 CUs x 64 lanes x 2.4 GHz / 40
= 9.8e11 calls/s on an MI355X (the bound below leaves a margin for clocks).
Longer chains amortise the launch, so the longest is close to the best."""
import math

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2207_05535_amd as pa  # noqa: E402


def test_calibration_rate_is_plausible():
    rates = [pa.pa_calibrate_philox(n) for n in (256, 1024, 4096)]
    for r in rates:
        assert math.isfinite(r) and 1e10 < r < 1.2e12, rates
    assert rates[-1] >= 0.5 * max(rates), rates
