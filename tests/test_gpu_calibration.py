"""Matrix-core peak probe: the measured rates of the register-only MFMA loops
are positive and within the device's datasheet peaks (dense FP32 157.3, BF16
2500, FP64 78.6 TFLOP/s, int8 5000 TOP/s) and above a fifth of them."""

import pytest

from paper_2305_13925_amd import binding as bd

pytestmark = pytest.mark.gpu

DATASHEET = {"fp32": 157.3, "bf16": 2500.0, "fp64": 78.6, "int8": 5000.0}


def test_mfma_peaks_are_plausible():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    with bd.Session(0) as s:
        peaks = bd.mfma_peaks(s)
    print("measured matrix-core peaks:", peaks)
    for k, ds in DATASHEET.items():
        assert 0.2 * ds < peaks[k] <= 1.05 * ds, (k, peaks[k])
