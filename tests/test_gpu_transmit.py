"""Per-symbol transmission (eqs. 15-16) through rzf_transmit, and Jac-PCG against
plain CG on the same systems. Bar: relative Frobenius error <= 1e-5 per
instance against the complex128 oracle at the GPU's iteration count."""

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


def symbols(rng, batch, nsym, K):
    """QPSK symbol vectors, [batch, nsym, K] (column-major K x nsym per instance)."""
    re = rng.choice([-1.0, 1.0], size=(batch, nsym, K))
    im = rng.choice([-1.0, 1.0], size=(batch, nsym, K))
    return ((re + 1j * im) / np.sqrt(2.0)).astype(np.complex64)


@pytest.mark.parametrize("name,gain,nsym,T,precision,flags,xi", [
    ("single", "literal", 1, 6, bd.GRAM_FP32, bd.PRECOND_JACOBI, None),
    # Plain CG on systems where its FP32 iterates track the FP64 ones (0 dB,
    # cond <= 11). On the gain-normalised channels at 10-20 dB, unpreconditioned
    # CG in FP32 drifts from FP64 by up to 3e-4 within 6 iterations (a complex64
    # CG on the CPU shows the same), while Jacobi-PCG stays at 1e-7.
    ("batched", "normalised", 5, 8, bd.GRAM_FP32, bd.PRECOND_NONE, 64.0),
    ("batched", "normalised", 1, 8, bd.GRAM_BF16X6, bd.PRECOND_JACOBI, None),
    ("batched", "normalised", 40, 8, bd.GRAM_FP32, bd.EPILOGUE_FP32, None),
    ("precision", "normalised", 3, 16, bd.GRAM_FP32, bd.PRECOND_JACOBI, None),
])
def test_transmit_matches_oracle(torch, sess, name, gain, nsym, T, precision, flags, xi):
    w = workload(name, gain=gain)
    n = 3 if name != "precision" else 2
    H = channel_batch(w, n=n)
    xi = w.xi_values()[-1] if xi is None else xi
    S = symbols(np.random.default_rng(nsym), n, nsym, w.K)
    Hd = torch.from_numpy(H).cuda()
    Sd = torch.from_numpy(S).cuda()
    w_out = torch.empty((n, nsym, w.K), dtype=torch.complex64, device="cuda")
    x, st, rc = bd.rzf_transmit(sess, Hd, Sd, xi, power=2.0, max_iter=T, precision=precision, flags=flags,
                                w_out=w_out, stats=True)
    assert rc == bd.OK, st
    xn, wn = x.cpu().numpy(), w_out.cpu().numpy()
    pre = "none" if flags & bd.PRECOND_NONE else "jacobi"
    for b in range(n):
        Hb = H[b].T.astype(np.complex128)
        ref = oracle.rzf(Hb, xi, B=S[b].T.astype(np.complex128), tol=0.0, max_iter=st["max_iters"], P_tx=2.0,
                         precond=pre)
        ex, ew = rel(xn[b].T, ref["W"]), rel(wn[b].T, ref["X"])
        Xs, Ws, _ = oracle.direct_rzf(Hb, xi, B=S[b].T.astype(np.complex128), P_tx=2.0)
        print(f"{name}/{gain} nsym={nsym} prec={precision} flags={flags} b={b}: x err {ex:.2e} w err {ew:.2e} "
              f"(vs FP64 direct {rel(xn[b].T, Ws):.2e})")
        assert ex <= TOL and ew <= TOL
        assert abs(np.linalg.norm(xn[b]) ** 2 - 2.0) <= 1e-5 * 2.0   # the block carries the stated power


def test_transmit_identity_block_is_the_precoder(torch, sess):
    w = workload("batched", gain="normalised")
    H = torch.from_numpy(channel_batch(w, n=4)).cuda()
    I = torch.eye(w.K, dtype=torch.complex64, device="cuda").expand(4, w.K, w.K).contiguous()
    x = bd.rzf_transmit(sess, H, I, 6.4, max_iter=8, precision=bd.GRAM_BF16X6)
    W = bd.rzf_precoder(sess, H, 6.4, max_iter=8, precision=bd.GRAM_BF16X6)
    torch.cuda.synchronize()
    assert torch.equal(x, W)


def test_transmit_tolerance_mode_per_instance(torch, sess):
    # One instance per call, so the reported iteration count is its own.
    w = workload("batched", gain="normalised")
    H = channel_batch(w, n=3)
    S = symbols(np.random.default_rng(7), 3, 1, w.K)
    for b in range(3):
        x, st, rc = bd.rzf_transmit(sess, torch.from_numpy(H[b:b + 1]).cuda(), torch.from_numpy(S[b:b + 1]).cuda(),
                                    0.64, tol=1e-6, max_iter=64, stats=True)
        assert rc == bd.OK and st["max_rel_residual"] <= 1e-6
        ref = oracle.rzf(H[b].T.astype(np.complex128), 0.64, B=S[b].T.astype(np.complex128), tol=0.0,
                         max_iter=st["max_iters"])
        assert rel(x[0].cpu().numpy().T, ref["W"]) <= TOL
        o = oracle.rzf(H[b].T.astype(np.complex128), 0.64, B=S[b].T.astype(np.complex128), tol=1e-6, max_iter=64)
        print(f"b={b}: GPU {st['max_iters']} iterations, oracle {int(o['iters'][0])}")
        assert abs(st["max_iters"] - int(o["iters"][0])) <= 1


def test_jacobi_vs_cg_iterations(torch, sess):
    # The paper's convergence claim (Sec. IV, Fig. 2): on channels whose Gram
    # diagonal spreads over users, Jacobi preconditioning needs fewer
    # iterations than plain CG. Per-instance counts from jacpcg_solve, against
    # the oracle's counts on the same systems.
    w = workload("batched", gain="normalised")
    n = 16
    H = channel_batch(w, n=n)
    S = symbols(np.random.default_rng(3), n, 1, w.K)
    A = bd.jacpcg_gram(sess, torch.from_numpy(H).cuda(), 0.64)
    counts = {}
    for name, fl in (("jacobi", bd.PRECOND_JACOBI), ("cg", bd.PRECOND_NONE)):
        it = torch.zeros((n, 1), dtype=torch.int32, device="cuda")
        st = torch.zeros((n,), dtype=torch.int32, device="cuda")
        bd.jacpcg_solve(sess, A, torch.from_numpy(S).cuda(), tol=1e-6, max_iter=256, flags=fl, iters=it, status=st)
        torch.cuda.synchronize()
        assert (st.cpu().numpy() == bd.OK).all()
        counts[name] = it.cpu().numpy()[:, 0]
        An = A.cpu().numpy().astype(np.complex128)
        for b in range(0, n, 5):
            o = oracle.jacpcg(An[b], S[b].T.astype(np.complex128), tol=1e-6, max_iter=256,
                              precond="none" if fl else "jacobi")
            g, f = int(counts[name][b]), int(o["iters"][0])
            print(f"{name} b={b}: GPU {g} iterations, oracle (FP64) {f}")
            if name == "jacobi":
                assert abs(g - f) <= 2, (name, b, g, f)
            else:
                # plain CG in FP32 loses orthogonality and needs more iterations
                # than in FP64 (54 -> 78 on these systems), never fewer
                assert g >= f - 2, (name, b, g, f)
    print("iterations to 1e-6: jacobi", counts["jacobi"].tolist(), "cg", counts["cg"].tolist())
    assert counts["jacobi"].mean() < counts["cg"].mean()
