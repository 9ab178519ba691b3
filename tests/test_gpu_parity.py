"""GPU path (libjacpcg through its C ABI) against the complex128 oracle.

Bar (relative Frobenius error per instance): 1e-5 for every FP32 result. FP32
fixed-iteration results are compared with the oracle at the same iteration
count; tolerance-stopped results with the oracle replaying each column for the
GPU's reported iteration count. The error against the exact (FP64 direct
inverse) precoder is printed for every case.
"""

import numpy as np
import pytest

import oracle
from channelgen import channel_batch, workload
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


def dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def crandn(rng, *shape):
    return ((rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)).astype(np.complex64)


def chan(rng, batch, K, M, spread=10.0):
    """Random channel [batch, K, M] with per-user gains spanning `spread`."""
    g = np.geomspace(1.0, spread, K).astype(np.float32)
    return (crandn(rng, batch, K, M) * g[None, :, None]).astype(np.complex64)


# ---------------------------------------------------------------------------
GRAM_SHAPES = [(256, 16, 1), (100, 37, 3), (1024, 64, 4), (333, 70, 2), (64, 256, 1), (1000, 130, 2),
               (7, 5, 3), (64, 1, 2), (4100, 96, 1)]


@pytest.mark.parametrize("M,K,batch", GRAM_SHAPES)
def test_gram_parity(torch, sess, M, K, batch):
    rng = np.random.default_rng(M * 1000 + K)
    H = chan(rng, batch, K, M)
    xi = 0.37
    diag = torch.empty((batch, K), dtype=torch.float32, device="cuda")
    A = bd.jacpcg_gram(sess, dev(torch, H), xi, diag=diag)
    torch.cuda.synchronize()
    A = A.cpu().numpy().astype(np.complex128)
    d = diag.cpu().numpy()
    for b in range(batch):
        ref = oracle.gram(H[b].T, xi)
        assert rel(A[b], ref) <= TOL, (b, rel(A[b], ref))
        assert np.array_equal(A[b], A[b].conj().T)          # exactly Hermitian
        assert np.all(A[b].diagonal().imag == 0)
        np.testing.assert_array_equal(d[b], A[b].diagonal().real.astype(np.float32))


@pytest.mark.parametrize("prec", [bd.GRAM_BF16X6, bd.GRAM_BF16X3])
@pytest.mark.parametrize("M,K,batch", [(1024, 64, 2), (333, 70, 2), (4100, 96, 1), (64, 256, 1), (7, 5, 3),
                                       (1000, 130, 1), (4096, 128, 2), (512, 192, 1), (256, 250, 1)])
def test_gram_split_bf16_parity(torch, sess, prec, M, K, batch):
    # Split-BF16 Gram: three exact parts / six products is FP32-class; hi+lo
    # with three products carries ~2^-16 relative product error.
    rng = np.random.default_rng(M + 31 * K)
    H = chan(rng, batch, K, M)
    xi = 0.37
    diag = torch.empty((batch, K), dtype=torch.float32, device="cuda")
    A = bd.jacpcg_gram(sess, dev(torch, H), xi, precision=prec, diag=diag)
    torch.cuda.synchronize()
    A = A.cpu().numpy().astype(np.complex128)
    for b in range(batch):
        ref = oracle.gram(H[b].T, xi)
        e = rel(A[b], ref)
        print(f"gram precision {prec} M={M} K={K} b={b}: rel err {e:.2e}")
        assert e <= (2e-6 if prec == bd.GRAM_BF16X6 else TOL)
        assert np.array_equal(A[b], A[b].conj().T)
        assert np.all(A[b].diagonal().imag == 0)
    np.testing.assert_array_equal(diag.cpu().numpy(), A.diagonal(axis1=1, axis2=2).real.astype(np.float32))


def test_gram_batch_zero_is_noop(torch, sess):
    H = torch.zeros((0, 4, 8), dtype=torch.complex64, device="cuda")
    A = bd.jacpcg_gram(sess, H, 1.0)
    assert A.shape == (0, 4, 4)


# ---------------------------------------------------------------------------
def _system(rng, batch, K, M, xi, spread=10.0):
    H = chan(rng, batch, K, M, spread)
    A64 = np.stack([oracle.gram(H[b].T, xi) for b in range(batch)])
    return A64.astype(np.complex64)


SOLVE_CASES = [(16, 16, 16, 2, True), (37, 37, 10, 2, True), (64, 64, 8, 3, True), (64, 20, 8, 2, False),
               (100, 100, 12, 1, True), (130, 40, 10, 1, False), (256, 256, 6, 1, True), (5, 3, 5, 2, False),
               (1, 1, 3, 2, True), (200, 33, 7, 2, False)]


@pytest.mark.parametrize("K,n,T,batch,identity", SOLVE_CASES)
def test_solve_fixed_iterations(torch, sess, K, n, T, batch, identity):
    rng = np.random.default_rng(K * 100 + n)
    A = _system(rng, batch, K, 2 * K + 7, xi=0.3)
    B = None if identity else crandn(rng, batch, n, K)
    iters = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    relres = torch.empty((batch, n), dtype=torch.float32, device="cuda")
    status = torch.empty((batch,), dtype=torch.int32, device="cuda")
    X = bd.jacpcg_solve(sess, dev(torch, A), None if B is None else dev(torch, B), tol=0.0, max_iter=T,
                        iters=iters, relres=relres, status=status)
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    it, rr = iters.cpu().numpy(), relres.cpu().numpy()
    # exactly T iterations, unless the FP32 residual fell below the 2^-40 range guard
    assert np.all((it == T) | ((it < T) & (rr <= 2.0 ** -40 * 1.01)))
    assert np.all(status.cpu().numpy() == bd.OK)
    for b in range(batch):
        Bm = None if B is None else B[b].T.astype(np.complex128)
        ref = oracle.jacpcg(A[b].astype(np.complex128), Bm, tol=0.0, max_iter=T)
        assert rel(X[b].T, ref["X"]) <= TOL, (b, rel(X[b].T, ref["X"]))
        # recurrence residual: equal where it is above the FP32 rounding floor
        np.testing.assert_allclose(relres.cpu().numpy()[b], ref["relres"], rtol=1e-2, atol=5e-5)


@pytest.mark.parametrize("K,snr_spread", [(64, 30.0), (128, 10.0), (32, 100.0)])
def test_solve_tolerance_replay(torch, sess, K, snr_spread):
    rng = np.random.default_rng(K + 7)
    batch, tol = 2, 1e-5
    A = _system(rng, batch, K, 4 * K, xi=0.05, spread=snr_spread)
    iters = torch.empty((batch, K), dtype=torch.int32, device="cuda")
    relres = torch.empty((batch, K), dtype=torch.float32, device="cuda")
    status = torch.empty((batch,), dtype=torch.int32, device="cuda")
    X = bd.jacpcg_solve(sess, dev(torch, A), None, tol=tol, max_iter=500, iters=iters, relres=relres,
                        status=status)
    torch.cuda.synchronize()
    X, it, rr = X.cpu().numpy(), iters.cpu().numpy(), relres.cpu().numpy()
    assert np.all(status.cpu().numpy() == bd.OK)
    assert np.all(rr <= tol)
    for b in range(batch):
        Ab = A[b].astype(np.complex128)
        cols = []
        for j in range(K):
            cols.append(oracle.jacpcg(Ab, np.eye(K)[:, j], tol=0.0, max_iter=int(it[b, j]))["X"][:, 0])
        ref = np.stack(cols, axis=1)
        assert rel(X[b].T, ref) <= TOL, (b, rel(X[b].T, ref))
        own = oracle.jacpcg(Ab, None, tol=tol, max_iter=500)["iters"]
        assert np.max(np.abs(own - it[b])) <= 1


def test_solve_breakdown_zero_column_and_plain_cg(torch, sess):
    K = 8
    bad = np.eye(K, dtype=np.complex64)
    bad[0, 1] = bad[1, 0] = 3.0                                   # indefinite
    Bm = np.zeros((1, 2, K), np.complex64)
    Bm[0, 1, 0], Bm[0, 1, 1] = 1.0, -1.0
    status = torch.empty((1,), dtype=torch.int32, device="cuda")
    iters = torch.empty((1, 2), dtype=torch.int32, device="cuda")
    X = bd.jacpcg_solve(sess, dev(torch, bad[None]), dev(torch, Bm), tol=0.0, max_iter=4, iters=iters,
                        status=status)
    torch.cuda.synchronize()
    ref = oracle.jacpcg(bad.astype(np.complex128), Bm[0].T.astype(np.complex128), tol=0.0, max_iter=4)
    assert status.item() == bd.E_BREAKDOWN and ref["instance_status"] == oracle.BREAKDOWN
    assert iters.cpu().numpy()[0, 0] == 0 and np.all(X.cpu().numpy()[0, 0] == 0)   # zero RHS column
    np.testing.assert_array_equal(iters.cpu().numpy()[0], ref["iters"])
    # plain CG flag (preconditioner = identity)
    rng = np.random.default_rng(3)
    A = _system(rng, 1, 24, 40, xi=0.2, spread=20.0)
    X = bd.jacpcg_solve(sess, dev(torch, A), None, tol=0.0, max_iter=6, flags=bd.PRECOND_NONE)
    torch.cuda.synchronize()
    ref = oracle.jacpcg(A[0].astype(np.complex128), None, tol=0.0, max_iter=6, precond="none")
    assert rel(X.cpu().numpy()[0].T, ref["X"]) <= TOL


# ---------------------------------------------------------------------------
RZF_CASES = [("single", "literal", 1), ("single", "normalised", 1), ("batched", "literal", 3),
             ("batched", "normalised", 3)]


@pytest.mark.parametrize("prec,flags", [(bd.GRAM_FP32, 0), (bd.GRAM_FP32, bd.EPILOGUE_FP32),
                                        (bd.GRAM_BF16X6, 0)])
@pytest.mark.parametrize("name,gain,n", RZF_CASES)
def test_rzf_fixed_iterations(torch, sess, name, gain, n, prec, flags):
    w = workload(name, gain=gain)
    H = channel_batch(w, n=n)
    T = 8 if name == "batched" else 16
    for xi in w.xi_values():
        X = torch.empty((n, w.K, w.K), dtype=torch.complex64, device="cuda")
        W, st, rc = bd.rzf_precoder(sess, dev(torch, H), xi, power=1.0, tol=0.0, max_iter=T, X_out=X, stats=True,
                                    precision=prec, flags=flags)
        # T iterations unless the FP32 recurrence residual reached exactly zero earlier
        assert rc == bd.OK and 1 <= st["max_iters"] <= T
        Wn, Xn = W.cpu().numpy(), X.cpu().numpy()
        for b in range(n):
            Hb = H[b].T.astype(np.complex128)
            ref = oracle.rzf(Hb, xi, tol=0.0, max_iter=T)
            ex, ew = rel(Xn[b].T, ref["X"]), rel(Wn[b].T, ref["W"])
            _, Wstar, _ = oracle.direct_rzf(Hb, xi)
            print(f"{name}/{gain} prec={prec} flags={flags} xi={xi:g} b={b}: err X {ex:.2e} W {ew:.2e}; "
                  f"W vs FP64 direct {rel(Wn[b].T, Wstar):.2e}")
            assert ex <= TOL and ew <= TOL
            assert abs(np.linalg.norm(Wn[b]) ** 2 - 1.0) <= 1e-5


@pytest.mark.parametrize("M,K", [(512, 96), (500, 80), (1024, 128), (384, 100), (256, 72)])
def test_split_epilogue_across_user_tiles(torch, sess, M, K):
    # The split-BF16 epilogue for 64 < K <= 128 (three and four 32-user tiles,
    # whole and ragged antenna blocks and user tiles) against the oracle at
    # the same iteration count.
    rng = np.random.default_rng(M * 7 + K)
    H = chan(rng, 2, K, M)
    xi, T = K / 10.0, 8
    W, st, rc = bd.rzf_precoder(sess, dev(torch, H), xi, tol=0.0, max_iter=T, stats=True,
                                precision=bd.GRAM_BF16X6)
    assert rc == bd.OK
    Wn = W.cpu().numpy()
    for b in range(2):
        ref = oracle.rzf(H[b].T.astype(np.complex128), xi, tol=0.0, max_iter=st["max_iters"])
        e = rel(Wn[b].T, ref["W"])
        print(f"split epilogue M={M} K={K} b={b}: err W {e:.2e}")
        assert e <= TOL


def test_rzf_tolerance_mode_and_plain_path_agree(torch, sess):
    w = workload("batched", gain="normalised")
    H = dev(torch, channel_batch(w, n=3))
    for xi in w.xi_values():
        X1 = torch.empty((3, 64, 64), dtype=torch.complex64, device="cuda")
        X2 = torch.empty_like(X1)
        W1, s1, _ = bd.rzf_precoder(sess, H, xi, tol=1e-5, max_iter=64, X_out=X1, stats=True)
        W2, s2, _ = bd.rzf_precoder_plain(sess, H, xi, tol=1e-5, max_iter=64, X_out=X2, stats=True)
        torch.cuda.synchronize()
        assert torch.equal(X1, X2) and torch.equal(W1, W2)     # same arithmetic, bitwise
        assert s1["max_iters"] == s2["max_iters"] and s1["worst_status"] == bd.OK
        assert s1["max_rel_residual"] <= 1e-5
        Hn = H.cpu().numpy()
        for b in range(3):
            _, Wstar, _ = oracle.direct_rzf(Hn[b].T.astype(np.complex128), xi)
            e = rel(W1.cpu().numpy()[b].T, Wstar)
            print(f"tol 1e-5 xi={xi:g} b={b}: iters {s1['max_iters']} W vs FP64 direct {e:.2e}")
            assert e <= 1e-3


@pytest.mark.parametrize("prec", [bd.GRAM_FP32, bd.GRAM_BF16X6])
def test_rzf_tolerance_mode_column_replay(torch, sess, prec):
    # The tolerance-stopped precoder end to end at the FP32 bar: its X equals
    # the solver's on the same Gram bit for bit (which reports each column's
    # iteration count), X matches the oracle replaying every column for that
    # many iterations, and W matches the oracle's precoder of that X.
    w = workload("batched", gain="normalised")
    n, tol = 3, 1e-5
    Hn = channel_batch(w, n=n)
    H = dev(torch, Hn)
    for xi in w.xi_values():
        X = torch.empty((n, w.K, w.K), dtype=torch.complex64, device="cuda")
        W, st, rc = bd.rzf_precoder(sess, H, xi, tol=tol, max_iter=64, precision=prec, X_out=X, stats=True)
        assert rc == bd.OK
        A = bd.jacpcg_gram(sess, H, xi, precision=prec)
        it = torch.zeros((n, w.K), dtype=torch.int32, device="cuda")
        Xs = bd.jacpcg_solve(sess, A, None, tol=tol, max_iter=64, iters=it)
        torch.cuda.synchronize()
        assert torch.equal(X, Xs)
        itn, Xn, Wn = it.cpu().numpy(), X.cpu().numpy(), W.cpu().numpy()
        assert int(itn.max()) == st["max_iters"]
        for b in range(n):
            Hb = Hn[b].T.astype(np.complex128)
            Ab = oracle.gram(Hb, xi)
            cols = [oracle.jacpcg(Ab, np.eye(w.K)[:, j], tol=0.0, max_iter=int(itn[b, j]))["X"][:, 0]
                    for j in range(w.K)]
            Xref = np.stack(cols, axis=1)
            Wref, _ = oracle.precoder(Hb, Xref)
            ex, ew = rel(Xn[b].T, Xref), rel(Wn[b].T, Wref)
            print(f"tol {tol:g} prec={prec} xi={xi:g} b={b}: iters {itn[b].min()}-{itn[b].max()} "
                  f"err X {ex:.2e} W {ew:.2e}")
            assert ex <= TOL and ew <= TOL


def test_rzf_fixed_plain_equals_batched(torch, sess):
    rng = np.random.default_rng(11)
    H = dev(torch, chan(rng, 4, 70, 300))
    W1 = bd.rzf_precoder(sess, H, 0.2, tol=0.0, max_iter=5)
    W2 = bd.rzf_precoder_plain(sess, H, 0.2, tol=0.0, max_iter=5)
    torch.cuda.synchronize()
    assert torch.equal(W1, W2)


def test_rzf_deterministic(torch, sess):
    w = workload("batched")
    H = dev(torch, channel_batch(w, n=8))
    a = bd.rzf_precoder(sess, H, 6.4, max_iter=8).clone()
    b = bd.rzf_precoder(sess, H, 6.4, max_iter=8)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_rzf_closed_forms(torch, sess):
    # K = 1: W = sqrt(P) h / ||h|| for every xi > 0
    rng = np.random.default_rng(5)
    h = crandn(rng, 2, 1, 50)
    W = bd.rzf_precoder(sess, dev(torch, h), 0.7, power=2.0, tol=0.0, max_iter=3)
    torch.cuda.synchronize()
    for b in range(2):
        want = np.sqrt(2.0) * h[b, 0] / np.linalg.norm(h[b, 0])
        assert rel(W.cpu().numpy()[b, 0], want) <= TOL
    # H = 0: A = xi I, X = I / xi after one iteration; H X = 0, so W = 0
    Z = torch.zeros((1, 6, 40), dtype=torch.complex64, device="cuda")
    X = torch.empty((1, 6, 6), dtype=torch.complex64, device="cuda")
    W, st, rc = bd.rzf_precoder(sess, Z, 1.6, tol=1e-6, max_iter=16, X_out=X, stats=True)
    assert rc == bd.OK and st["max_iters"] == 1
    np.testing.assert_allclose(X.cpu().numpy()[0], np.eye(6) / 1.6, rtol=1e-6)
    assert torch.count_nonzero(W).item() == 0


def test_rzf_ragged_shapes(torch, sess):
    rng = np.random.default_rng(21)
    for (M, K) in [(37, 5), (129, 33), (500, 97), (77, 160)]:
        H = chan(rng, 2, K, M, spread=3.0)
        xi = 0.5
        W = bd.rzf_precoder(sess, dev(torch, H), xi, tol=0.0, max_iter=6).cpu().numpy()
        for b in range(2):
            ref = oracle.rzf(H[b].T.astype(np.complex128), xi, tol=0.0, max_iter=6)
            assert rel(W[b].T, ref["W"]) <= TOL, (M, K, b)


@pytest.mark.parametrize("M,K", [(40, 150), (129, 150), (1000, 256), (4100, 200)])
def test_fp32_gram_antenna_chunks(torch, sess, M, K):
    # Above K = 128 the precoder's FP32 Gram splits each 64 x 64 block's
    # antennas into four chunks of whole 16-antenna stages and sums the partial
    # blocks afterwards; at M = 40 and M = 129 the last chunk is empty, at
    # M = 4100 the last stage is partial. X (no cancellation in the product
    # over users) and W against the oracle at the same iteration count.
    rng = np.random.default_rng(M + 7 * K)
    H = chan(rng, 2, K, M, spread=3.0)
    xi, T = K / 10.0, 6
    X = torch.empty((2, K, K), dtype=torch.complex64, device="cuda")
    W, st, rc = bd.rzf_precoder(sess, dev(torch, H), xi, tol=0.0, max_iter=T, precision=bd.GRAM_FP32, X_out=X,
                                stats=True)
    assert rc == bd.OK, st
    Xn, Wn = X.cpu().numpy(), W.cpu().numpy()
    for b in range(2):
        ref = oracle.rzf(H[b].T.astype(np.complex128), xi, tol=0.0, max_iter=T)
        ex, ew = rel(Xn[b].T, ref["X"]), rel(Wn[b].T, ref["W"])
        print(f"fp32 gram chunks M={M} K={K} b={b}: X err {ex:.2e} W err {ew:.2e}")
        assert ex <= TOL
        if M >= K:
            assert ew <= TOL


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,T,samples", [("batched", 8, (0, 1, 513, 1023)), ("precision", 16, (0, 255)),
                                              ("stress", 16, (0, 63))])
def test_full_size_sampled(torch, sess, name, T, samples):
    """Full workload sizes in the benchmark's launch configuration; sampled
    instances against the oracle, the power constraint on every instance."""
    w = workload(name)
    H = channel_batch(w)
    xi = w.xi_values()[-1] if name == "batched" else w.xi_values()[0]
    Hd = dev(torch, H)
    W, st, rc = bd.rzf_precoder(sess, Hd, xi, tol=0.0, max_iter=T, stats=True)
    assert rc == bd.OK
    Wn = W.cpu().numpy()
    p = np.sum(np.abs(Wn) ** 2, axis=(1, 2))
    assert np.all(np.isfinite(p)) and np.max(np.abs(p - 1.0)) <= 1e-5
    for b in samples:
        ref = oracle.rzf(H[b].T.astype(np.complex128), xi, tol=0.0, max_iter=T)
        e = rel(Wn[b].T, ref["W"])
        print(f"{name} b={b}: W err {e:.2e}")
        assert e <= TOL


# ---------------------------------------------------------------------------
# FP64-residual iterative refinement: X64 against the exact (FP64 Cholesky)
# inverse at 1e-10.
REFINE_TOL = 1e-10


REFINED_PRECISIONS = [bd.GRAM_FP32, bd.GRAM_BF16X3, bd.GRAM_BF16X6, bd.GRAM_FP64_ROUNDED]


@pytest.mark.parametrize("prec", REFINED_PRECISIONS)
@pytest.mark.parametrize("name,gain,n,tol,T", [("precision", "normalised", 2, 1e-6, 64),
                                               ("precision", "literal", 2, 0.0, 16),
                                               ("batched", "normalised", 3, 1e-5, 32)])
def test_refined_reaches_fp64(torch, sess, prec, name, gain, n, tol, T):
    w = workload(name, gain=gain)
    H = channel_batch(w, n=n)
    xi = w.xi_values()[-1]
    X64 = torch.empty((n, w.K, w.K), dtype=torch.complex128, device="cuda")
    W, st, rc = bd.rzf_precoder(sess, dev(torch, H), xi, tol=tol, max_iter=T, precision=prec | bd.REFINE_FP64,
                                refine_tol=REFINE_TOL, X64_out=X64, stats=True)
    assert rc == bd.OK, st
    assert st["max_refine_residual"] <= REFINE_TOL and st["refine_steps"] >= 1
    Xn, Wn = X64.cpu().numpy(), W.cpu().numpy()
    for b in range(n):
        Xs, Ws, _ = oracle.direct_rzf(H[b].T.astype(np.complex128), xi)
        ex, ew = rel(Xn[b].T, Xs), rel(Wn[b].T, Ws)
        print(f"refined {name}/{gain} prec={prec} b={b}: steps {st['refine_steps']} X64 err {ex:.2e} W err {ew:.2e}")
        assert ex <= REFINE_TOL
        assert ew <= 1e-6          # W is complex64: only its rounding remains


@pytest.mark.parametrize("gram", [bd.GRAM_FP32, bd.GRAM_FP64_ROUNDED])
def test_refined_stress_sampled(torch, sess, gram):
    # Near-ZF regularisation, strong correlation: ill-conditioned systems. The
    # solves on the FP32 Gram or on the FP64 Gram rounded to FP32.
    w = workload("stress")
    H = channel_batch(w, n=2)
    X64 = torch.empty((2, w.K, w.K), dtype=torch.complex128, device="cuda")
    W, st, rc = bd.rzf_precoder(sess, dev(torch, H), w.xi, tol=1e-6, max_iter=1024,
                                precision=gram | bd.REFINE_FP64, refine_tol=REFINE_TOL, X64_out=X64,
                                stats=True)
    assert rc == bd.OK, st
    Xn = X64.cpu().numpy()
    for b in range(2):
        A = oracle.gram(H[b].T.astype(np.complex128), w.xi)
        Xs = oracle.chol_inverse(A)
        e = rel(Xn[b].T, Xs)
        print(f"stress b={b}: cond {np.linalg.cond(A):.1e} PCG iters {st['max_iters']} refine steps "
              f"{st['refine_steps']} X64 err {e:.2e}")
        assert e <= REFINE_TOL


def test_refined_full_size_precision_sampled(torch, sess):
    w = workload("precision")
    H = channel_batch(w)
    xi = w.xi_values()[0]
    X64 = torch.empty((w.batch, w.K, w.K), dtype=torch.complex128, device="cuda")
    W, st, rc = bd.rzf_precoder(sess, dev(torch, H), xi, tol=1e-6, max_iter=64,
                                precision=bd.GRAM_BF16X3 | bd.REFINE_FP64, refine_tol=REFINE_TOL, X64_out=X64,
                                stats=True)
    assert rc == bd.OK and st["max_refine_residual"] <= REFINE_TOL
    Xn = X64.cpu().numpy()
    for b in (0, 97, 255):
        Xs, _, _ = oracle.direct_rzf(H[b].T.astype(np.complex128), xi)
        assert rel(Xn[b].T, Xs) <= REFINE_TOL


@pytest.mark.parametrize("prec", REFINED_PRECISIONS)
@pytest.mark.parametrize("M,K", [(333, 100), (344, 100), (333, 200), (37, 40), (40, 150), (1000, 256)])
def test_refined_ragged_shapes(torch, sess, prec, M, K):
    # The FP64 Gram works in 64 x 64 blocks of A and stages 16 antennas at a
    # time: K off a multiple of 64 leaves rows past K in the last block, and M
    # off a multiple of 16 leaves a partial last stage (and rows of H whose
    # length is not a multiple of two complex entries). Above K = 128 the
    # antennas are split into four chunks summed afterwards; at M = 40 the last
    # chunk is empty. The refined result must still reach the FP64 direct
    # precoder.
    rng = np.random.default_rng(K + M)
    n, xi = 2, K / 10.0
    H = chan(rng, n, K, M)
    X64 = torch.empty((n, K, K), dtype=torch.complex128, device="cuda")
    W, st, rc = bd.rzf_precoder(sess, dev(torch, H), xi, tol=1e-6, max_iter=200, precision=prec | bd.REFINE_FP64,
                                refine_tol=REFINE_TOL, X64_out=X64, stats=True)
    assert rc == bd.OK, st
    assert st["max_refine_residual"] <= REFINE_TOL
    Xn, Wn = X64.cpu().numpy(), W.cpu().numpy()
    for b in range(n):
        Xs, Ws, _ = oracle.direct_rzf(H[b].T.astype(np.complex128), xi)
        ex, ew = rel(Xn[b].T, Xs), rel(Wn[b].T, Ws)
        # W = beta H X is formed in complex64 from X64 rounded to complex64.
        # With more users than antennas (K > M) the sum over users cancels
        # (||H|| ||X|| / ||H X|| reaches about 1600 at M = 40, K = 150), so the
        # W bar is the larger of 1e-6 and twice the error of that same product
        # taken from the exact X and H rounded to complex64.
        Hb = H[b].T.astype(np.complex128)
        W32 = (Hb.astype(np.complex64) @ Xs.astype(np.complex64)).astype(np.complex128)
        W32 *= np.linalg.norm(Ws) / np.linalg.norm(W32)
        w_bar = max(1e-6, 2.0 * rel(W32, Ws))
        print(f"refined ragged M={M} K={K} prec={prec} b={b}: steps {st['refine_steps']} X64 err {ex:.2e} "
              f"W err {ew:.2e} (bar {w_bar:.2e})")
        assert ex <= REFINE_TOL
        assert ew <= w_bar


def test_refined_solves_use_the_requested_gram(torch, sess):
    # With a refinement tolerance no column misses, the refined call's X is the
    # first FP32 solve's: it must equal the unrefined call's X for the same
    # Gram precision bit for bit, and differ between precisions (the FP32
    # solves run on the Gram the precision bits name; A64 feeds only the
    # FP64 residual).
    w = workload("precision", gain="normalised")
    H = dev(torch, channel_batch(w, n=2))
    xi = w.xi_values()[-1]
    Xs = {}
    for prec in REFINED_PRECISIONS:
        X_ref = torch.empty((2, w.K, w.K), dtype=torch.complex64, device="cuda")
        _, st, rc = bd.rzf_precoder(sess, H, xi, tol=1e-6, max_iter=64, precision=prec | bd.REFINE_FP64,
                                    refine_tol=1e30, X_out=X_ref, stats=True)
        assert rc == bd.OK and st["refine_steps"] == 0, st
        if prec != bd.GRAM_FP64_ROUNDED:
            X_plain = torch.empty_like(X_ref)
            bd.rzf_precoder(sess, H, xi, tol=1e-6, max_iter=64, precision=prec, X_out=X_plain)
            torch.cuda.synchronize()
            assert torch.equal(X_ref, X_plain), prec
        Xs[prec] = X_ref
    for i, a in enumerate(REFINED_PRECISIONS):
        for b in REFINED_PRECISIONS[i + 1:]:
            assert not torch.equal(Xs[a], Xs[b]), (a, b)
    # the two-part split Gram is the least accurate: it needs the most corrections
    steps = {}
    for prec in REFINED_PRECISIONS:
        _, st, rc = bd.rzf_precoder(sess, H, xi, tol=1e-6, max_iter=64, precision=prec | bd.REFINE_FP64,
                                    refine_tol=REFINE_TOL, stats=True)
        assert rc == bd.OK and st["max_refine_residual"] <= REFINE_TOL
        steps[prec] = st["refine_steps"]
    print("refinement steps by Gram precision:", steps)
    assert steps[bd.GRAM_BF16X3] >= max(steps[bd.GRAM_FP32], steps[bd.GRAM_FP64_ROUNDED]) >= 1


def test_refined_not_converged_status(torch, sess):
    # A tolerance below what FP64 can reach leaves columns above it after the
    # 16 corrections: NOT_CONVERGED, with X64 still at the FP64 solution.
    w = workload("precision", gain="normalised")
    Hn = channel_batch(w, n=1)
    xi = w.xi_values()[-1]
    X64 = torch.empty((1, w.K, w.K), dtype=torch.complex128, device="cuda")
    _, st, rc = bd.rzf_precoder(sess, dev(torch, Hn), xi, tol=1e-6, max_iter=64,
                                precision=bd.GRAM_FP32 | bd.REFINE_FP64, refine_tol=1e-30, X64_out=X64, stats=True)
    assert rc == bd.NOT_CONVERGED and st["refine_steps"] == 16, st
    Xs, _, _ = oracle.direct_rzf(Hn[0].T.astype(np.complex128), xi)
    assert rel(X64[0].cpu().numpy().T, Xs) <= REFINE_TOL
