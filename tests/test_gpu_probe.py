"""Ceiling probes (bfm_debug_probe): every instruction mix runs and reports a
rate below the published peak of its arithmetic (with a 10% allowance for
the clock), and bad arguments are rejected."""
import pytest

from paper_1905_01341_amd import bfm

pytestmark = pytest.mark.gpu

# published MI355X peaks (TFLOP/s): FP64 MFMA and vector 78.6, FP32 vector
# 157.3 (packed; these builds issue unpacked FP32 at half of it), BF16 MFMA 2500
PEAKS = {0: 78.6, 1: 78.6, 2: 157.3, 3: 78.6, 4: 157.3, 5: 2500.0}


@pytest.mark.parametrize("kind,iters", [(0, 20), (1, 2000), (2, 2000), (3, 5), (4, 10), (5, 50)])
def test_probe_rates(kind, iters):
    ms, ops = bfm.debug_probe(kind, iters)
    rate = ops / (ms * 1e-3) / 1e12
    print(f"probe {bfm.PROBE_KINDS[kind]}: {rate:.1f} TFLOP/s ({ms:.3f} ms)")
    assert ms > 0 and 0.0 < rate < 1.1 * PEAKS[kind]


def test_probe_errors():
    for kind, iters in ((6, 1), (-1, 1), (0, 0), (0, (1 << 16) + 1)):
        with pytest.raises(bfm.BfmError):
            bfm.debug_probe(kind, iters)
