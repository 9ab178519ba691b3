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


@pytest.mark.parametrize("prec", [bd.GRAM_FP32, bd.GRAM_BF16X6])
def test_non_finite_channel_is_isolated(torch, sess, prec):
    # A NaN in one instance's channel and an Inf in another make their Gram
    # matrices non-finite. Their solves must end with a breakdown status within
    # max_iter, and every other instance must come out bitwise as in the same
    # call with clean channels (instances are independent). Ragged K and M.
    rng = np.random.default_rng(11)
    n, K, M, xi, T = 6, 40, 200, 4.0, 8
    Hc = torch.from_numpy(crandn(rng, n, K, M)).cuda()
    Hb = Hc.clone()
    Hb[2, 5, 17] = complex(float("nan"), 0.0)
    Hb[4, 0, 0] = complex(float("inf"), 0.0)
    good, bad = [0, 1, 3, 5], [2, 4]

    W_clean = bd.rzf_precoder(sess, Hc, xi, max_iter=T, precision=prec)
    W_bad = bd.rzf_precoder(sess, Hb, xi, max_iter=T, precision=prec)
    torch.cuda.synchronize()
    assert torch.equal(W_bad[good], W_clean[good])
    assert torch.isfinite(torch.view_as_real(W_clean)).all()
    with pytest.raises(bd.JacpcgError) as ei:  # synchronising call: the worst status is an error code
        bd.rzf_precoder(sess, Hb, xi, max_iter=T, precision=prec, stats=True)
    assert ei.value.code == bd.E_BREAKDOWN

    # per-instance statuses and iteration counts through the solver entry point
    A = bd.jacpcg_gram(sess, Hb, xi, precision=prec)
    status = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    its = torch.full((n, K), -1, dtype=torch.int32, device="cuda")
    bd.jacpcg_solve(sess, A, None, tol=1e-6, max_iter=T, iters=its, status=status)
    torch.cuda.synchronize()
    st = status.cpu().tolist()
    print("non-finite: statuses", st, "max iters", int(its.max()))
    assert [st[b] for b in bad] == [bd.E_BREAKDOWN] * 2
    assert all(st[b] in (bd.OK, bd.NOT_CONVERGED) for b in good)
    assert int(its.min()) >= 0 and int(its.max()) <= T

    # the session is unaffected: the clean call repeats bitwise
    W_again = bd.rzf_precoder(sess, Hc, xi, max_iter=T, precision=prec)
    torch.cuda.synchronize()
    assert torch.equal(W_again, W_clean)


def test_non_finite_channel_refined_path(torch, sess):
    # The FP64-refined path with one NaN instance: the call reports the
    # breakdown, and the other instances still reach the FP64 direct precoder
    # (their refinement stops on their own residuals; a NaN residual does not
    # count towards the stopping test).
    rng = np.random.default_rng(12)
    n, K, M, xi = 3, 24, 160, 2.0
    H = crandn(rng, n, K, M)
    Hb = torch.from_numpy(H).cuda()
    Hb[1, 3, 3] = complex(float("nan"), float("nan"))
    W = torch.empty_like(Hb)
    with pytest.raises(bd.JacpcgError) as ei:
        bd.rzf_precoder(sess, Hb, xi, tol=1e-6, max_iter=64, precision=bd.GRAM_FP32 | bd.REFINE_FP64,
                        refine_tol=1e-10, W=W, stats=True)
    assert ei.value.code == bd.E_BREAKDOWN
    Wn = W.cpu().numpy()
    for b in (0, 2):
        _, Ws, _ = oracle.direct_rzf(H[b].T.astype(np.complex128), xi)
        err = rel(Wn[b].T, Ws)
        print(f"non-finite refined: instance {b} W err {err:.2e}")
        assert err <= 1e-6  # W is complex64: only its rounding remains
