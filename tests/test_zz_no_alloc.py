"""rzf_precoder_noalloc (the entry point that allocates nothing, on the
library's fixed device workspace) gives rzf_precoder's results: two calls in a
row, the second on a smaller input, each bitwise equal to the allocating entry
point on the same channels, with the per-instance status reduced."""

import numpy as np
import pytest

import oracle
from channelgen import device_pool
from paper_2305_13925_amd import binding as bd

pytestmark = pytest.mark.gpu


def test_noalloc_matches_rzf_precoder_two_calls_second_smaller():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    cases = [
        # (M, S, K, n, xi, tol, max_iter, precision, flags, gain)
        (1024, 8, 64, 96, 6.4, 0.0, 8, bd.GRAM_BF16X6, bd.PRECOND_JACOBI, "normalised"),
        (300, 4, 37, 5, 0.9, 1e-6, 16, bd.GRAM_FP32, bd.EPILOGUE_FP32, "normalised"),
    ]
    with bd.Session(0) as s:
        for M, S, K, n, xi, tol, mi, prec, flags, gain in cases:
            print(f"noalloc case M={M} K={K} n={n} prec={prec} flags={flags}", flush=True)
            H = device_pool(M, S, K, 0.5, (2, 4), n, 100 + K, gain=gain)
            W_ref, st, rc = bd.rzf_precoder(s, H, xi, tol=tol, max_iter=mi, precision=prec, flags=flags,
                                            stats=True)
            W = torch.full_like(H, float("nan"))
            status = torch.full((n,), -77, dtype=torch.int32, device=H.device)
            bd.rzf_precoder_noalloc(s, H, xi, tol=tol, max_iter=mi, precision=prec, flags=flags, W=W,
                                    status=status)
            torch.cuda.synchronize()
            assert torch.equal(W, W_ref), (M, K)
            assert rc in (bd.OK, bd.NOT_CONVERGED)
            assert int(status.max()) in (0, 1) and int(status.min()) >= 0
            if rc == bd.OK:
                assert int(status.max()) == 0
            if tol == 0.0:  # fixed T: within the FP32 bar of the oracle's T-th iterate
                Hn = H[0].cpu().numpy().T.astype(np.complex128)
                ref = oracle.rzf(Hn, xi, tol=0.0, max_iter=mi)
                e = np.linalg.norm(W[0].cpu().numpy().T - ref["W"]) / np.linalg.norm(ref["W"])
                assert e <= 1e-5, e
