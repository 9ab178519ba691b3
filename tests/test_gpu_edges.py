"""Edge cases of every entry point: empty batches, extreme shapes, singular and
zero systems, padded leading dimensions through the raw C ABI."""

import ctypes as C

import numpy as np
import pytest

import oracle
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


def crandn(rng, *shape):
    return ((rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)).astype(np.complex64)


def test_empty_batches(torch, sess):
    H = torch.empty((0, 8, 64), dtype=torch.complex64, device="cuda")
    assert bd.rzf_precoder(sess, H, 1.0).shape == (0, 8, 64)
    assert bd.rzf_precoder_vr(sess, H, 1.0).shape == (0, 8, 64)
    assert bd.rzf_block_precoder(sess, H, 1.0, 16, 32, 16, 4, 4).shape == (0, 8, 64)
    S = torch.empty((0, 3, 8), dtype=torch.complex64, device="cuda")
    assert bd.rzf_transmit(sess, H, S, 1.0).shape == (0, 3, 64)
    sinr, se = bd.rzf_sinr(sess, H, H, 0.1)
    assert sinr.shape == (0, 8) and se.shape == (0,)
    torch.cuda.synchronize()


@pytest.mark.parametrize("M,K,xi,T", [(100000, 3, 0.5, 3), (128, 256, 1.0, 12), (1, 1, 0.25, 1), (33, 200, 4.0, 6)])
def test_extreme_shapes(torch, sess, M, K, xi, T):
    rng = np.random.default_rng(M + K)
    H = crandn(rng, 2, K, M) / np.float32(np.sqrt(M))
    W, st, rc = bd.rzf_precoder(sess, torch.from_numpy(H).cuda(), xi, max_iter=T, stats=True)
    assert rc == bd.OK, st
    for b in range(2):
        ref = oracle.rzf(H[b].T.astype(np.complex128), xi, tol=0.0, max_iter=st["max_iters"])
        e = rel(W[b].cpu().numpy().T, ref["W"])
        print(f"M={M} K={K}: err {e:.2e}")
        assert e <= TOL


def test_singular_system_ends_with_a_status(torch, sess):
    # xi = 0 and K > M: A = H^H H is singular. The solve must end (breakdown
    # or not converged), report it, and leave finite outputs where it did not
    # break down.
    rng = np.random.default_rng(3)
    H = crandn(rng, 2, 48, 16)
    try:
        W, st, rc = bd.rzf_precoder(sess, torch.from_numpy(H).cuda(), 0.0, tol=1e-6, max_iter=200, stats=True)
    except bd.JacpcgError as e:  # negative statuses raise in the binding
        print("singular: breakdown reported:", e)
        assert e.code == bd.E_BREAKDOWN
        return
    print("singular:", rc, st)
    assert rc in (bd.OK, bd.NOT_CONVERGED) and rc == st["worst_status"]
    assert torch.isfinite(torch.view_as_real(W)).all()


def test_zero_channel_gives_zero_precoder(torch, sess):
    # H = 0: A = xi I, X = I / xi after one iteration, H X = 0, so beta_pow is
    # taken as 0 and W = 0 exactly (no NaN from 0/0).
    H = torch.zeros((3, 8, 128), dtype=torch.complex64, device="cuda")
    X = torch.empty((3, 8, 8), dtype=torch.complex64, device="cuda")
    W, st, rc = bd.rzf_precoder(sess, H, 2.0, max_iter=4, X_out=X, stats=True)
    assert rc == bd.OK and st["max_iters"] <= 1
    assert torch.equal(W, torch.zeros_like(W))
    eye = torch.eye(8, dtype=torch.complex64, device="cuda").expand(3, 8, 8)
    assert torch.allclose(X, eye / 2.0, rtol=1e-6, atol=0)


def test_padded_leading_dimensions_through_the_c_abi(torch, sess):
    # ldh > M, stride_h > ldh * K, ldw > M: the same precoder as the packed layout.
    rng = np.random.default_rng(9)
    batch, M, K, ldh, sh, ldw, sw = 3, 200, 20, 213, 213 * 20 + 40, 205, 205 * 20 + 8
    H = crandn(rng, batch, K, M)
    Hp = torch.zeros(batch * sh, dtype=torch.complex64, device="cuda")
    view = Hp.as_strided((batch, K, M), (sh, ldh, 1))
    view.copy_(torch.from_numpy(H))
    Wp = torch.full((batch * sw,), complex(7.0, 7.0), dtype=torch.complex64, device="cuda")
    rc = bd.lib().rzf_precoder(sess.handle, C.c_void_p(torch.cuda.current_stream().cuda_stream), batch, M, K,
                               C.c_void_p(Hp.data_ptr()), ldh, sh, 1.1, 1.0, 0.0, 6, bd.GRAM_FP32, 0, 1e-10,
                               C.c_void_p(Wp.data_ptr()), ldw, sw, None, None, None)
    assert rc == bd.OK
    Wd = bd.rzf_precoder(sess, torch.from_numpy(H).cuda(), 1.1, max_iter=6)
    torch.cuda.synchronize()
    Wv = Wp.as_strided((batch, K, M), (sw, ldw, 1))
    assert rel(Wv.cpu().numpy(), Wd.cpu().numpy()) <= 1e-6
    # the padding between columns and instances is untouched
    pad = Wp.as_strided((batch, K, ldw - M), (sw, ldw, 1), M)
    assert torch.all(pad == complex(7.0, 7.0))


def test_calls_on_two_streams_share_the_workspace_safely(torch, sess):
    # A long call on stream a, then at once a short one on stream b, with the
    # same session (workspace): b's call waits for a's, so both results equal
    # the ones computed alone.
    from channelgen import device_pool
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    H1 = device_pool(1024, 8, 64, 0.5, (3, 6), 512, 21)
    H2 = device_pool(1024, 8, 64, 0.5, (3, 6), 64, 22)
    torch.cuda.synchronize()
    ref1 = bd.rzf_precoder(sess, H1, 6.4, max_iter=8)
    ref2 = bd.rzf_precoder(sess, H2, 6.4, max_iter=8)
    torch.cuda.synchronize()
    W1, W2 = torch.empty_like(H1), torch.empty_like(H2)
    for _ in range(3):
        bd.rzf_precoder(sess, H1, 6.4, max_iter=8, W=W1, stream=a)
        bd.rzf_precoder(sess, H2, 6.4, max_iter=8, W=W2, stream=b)
    torch.cuda.synchronize()
    assert torch.equal(W1, ref1) and torch.equal(W2, ref2)
