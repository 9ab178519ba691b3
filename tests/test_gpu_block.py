"""Subarray-block RZF (eqs. 2, 6, 7) through rzf_block_precoder, against the
complex128 oracle. Bar: relative Frobenius error <= 1e-5 per instance at the
same iteration count; the zero blocks exactly zero; eq. 9's SINR of the block
precoder through rzf_sinr."""

import numpy as np
import pytest

import oracle
from channelgen import block_channel_batch
from paper_2305_13925_amd import binding as bd

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a HIP device"
    return t


@pytest.fixture(scope="module")
def sess(torch):
    s = bd.Session(0)
    yield s
    s.close()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.mark.parametrize("shape,n,T,precision,flags", [
    ((48, 32, 40, 6, 5), 3, 6, bd.GRAM_FP32, bd.PRECOND_JACOBI),
    ((64, 0, 64, 8, 8), 2, 8, bd.GRAM_FP32, bd.EPILOGUE_FP32),
    ((30, 50, 20, 4, 7), 2, 5, bd.GRAM_BF16X6, bd.PRECOND_JACOBI),
    ((384, 256, 384, 32, 32), 4, 8, bd.GRAM_BF16X6, bd.PRECOND_JACOBI),
    ((1024, 1024, 1024, 64, 64), 2, 8, bd.GRAM_FP32, bd.PRECOND_JACOBI),
])
def test_block_precoder_matches_oracle(torch, sess, shape, n, T, precision, flags):
    M1, Mc, M2, K1, K2 = shape
    H = block_channel_batch(M1, Mc, M2, K1, K2, 0.6, n, seed=9)
    xi = (K1 + K2) / 10.0
    G = torch.full(H.shape, float("nan"), dtype=torch.complex64, device="cuda")   # every entry must be written
    G, st, rc = bd.rzf_block_precoder(sess, torch.from_numpy(H).cuda(), xi, M1, Mc, M2, K1, K2, power=1.5,
                                      max_iter=T, precision=precision, flags=flags, G=G, stats=True)
    assert rc == bd.OK, st
    Gn = G.cpu().numpy()
    assert np.isfinite(Gn).all()
    for b in range(n):
        Hb = H[b].T.astype(np.complex128)
        ref, _ = oracle.block_rzf(Hb, xi, M1, Mc, M2, K1, K2, max_iter=st["max_iters"], P_tx=1.5)
        direct, _ = oracle.block_rzf(Hb, xi, M1, Mc, M2, K1, K2, direct=True, P_tx=1.5)
        Gb = Gn[b].T
        e = rel(Gb, ref)
        print(f"block {shape} prec={precision} flags={flags} b={b}: err {e:.2e} (vs FP64 direct {rel(Gb, direct):.2e})")
        assert e <= TOL
        assert np.all(Gb[:M1, K1:] == 0) and np.all(Gb[M1 + Mc:, :K1] == 0)


def test_block_sinr_is_eq9(torch, sess):
    M1, Mc, M2, K1, K2 = 96, 64, 80, 12, 10
    H = block_channel_batch(M1, Mc, M2, K1, K2, 0.6, 2, seed=4)
    Hd = torch.from_numpy(H).cuda()
    G = bd.rzf_block_precoder(sess, Hd, 2.2, M1, Mc, M2, K1, K2, max_iter=10)
    sinr, se = bd.rzf_sinr(sess, Hd, G, 0.1)
    torch.cuda.synchronize()
    for b in range(2):
        ref = oracle.sinr(H[b].T.astype(np.complex128), G[b].cpu().numpy().T.astype(np.complex128), 0.1)
        assert rel(sinr[b].cpu().numpy(), ref) <= TOL
        assert abs(se[b].item() - np.sum(np.log2(1 + ref))) <= TOL * np.sum(np.log2(1 + ref))


def test_block_refined_reaches_direct(torch, sess):
    M1, Mc, M2, K1, K2 = 256, 128, 256, 24, 20
    H = block_channel_batch(M1, Mc, M2, K1, K2, 0.8, 2, seed=6)
    G, st, rc = bd.rzf_block_precoder(sess, torch.from_numpy(H).cuda(), 0.05, M1, Mc, M2, K1, K2, tol=1e-5,
                                      max_iter=64, precision=bd.GRAM_FP32 | bd.REFINE_FP64, stats=True)
    assert rc == bd.OK and st["max_refine_residual"] <= 1e-10
    for b in range(2):
        direct, _ = oracle.block_rzf(H[b].T.astype(np.complex128), 0.05, M1, Mc, M2, K1, K2, direct=True)
        assert rel(G[b].cpu().numpy().T, direct) <= 1e-6          # G is complex64: its rounding remains
