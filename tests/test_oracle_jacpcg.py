"""Pins of the oracle's Jacobi-preconditioned CG (Algorithm 1 / eq. 21, standard
PCG reading of Step 3)."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from tests import _exact as ex
from tests.test_oracle_gram_inverse import _crandn, _golden


def _hpd(rng, M, K, xi, spread=1.0):
    H = _crandn(rng, M, K) * (np.geomspace(1.0, spread, K)[None, :])
    return oracle.gram(H, xi)


def test_golden_worked_iterates():
    g = _golden()
    A = g["A"].reshape(2, 2)
    b = np.array([1.0, 0.0])
    x1 = oracle.jacpcg(A, b, tol=0.0, max_iter=1)["X"][:, 0]
    x2 = oracle.jacpcg(A, b, tol=0.0, max_iter=2)["X"][:, 0]
    np.testing.assert_allclose(x1, g["x1_col0"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(x2, g["x2_col0"], rtol=0, atol=1e-15)


def _exact_case():
    H = np.array([[1, 2j, 0, 1 - 1j], [1j, 1, 2, 0], [0, 1 + 1j, 1, 1], [2, 0, -1j, 1],
                  [1, 1, 1, 1j], [0, -1, 1j, 2]])
    return H, 0.5


@pytest.mark.parametrize("t", [1, 2, 3, 4])
def test_iterates_equal_exact_krylov_optimum(t):
    # The t-th Jacobi-PCG iterate is the minimiser of the A-norm error over
    # span{z0, N z0, ..., N^{t-1} z0} with N = D^{-1} A, z0 = D^{-1} b.
    # Computed here exactly in rationals, without any CG recurrence.
    H, xi = _exact_case()
    A = oracle.gram(H, xi)
    K = A.shape[0]
    Aq = [[ex.QC(A[i, j].real, A[i, j].imag) for j in range(K)] for i in range(K)]
    dinv = [ex.QC(1) / Aq[i][i] for i in range(K)]
    for col in range(K):
        b = [[ex.QC(1 if i == col else 0)] for i in range(K)]
        want = np.array([complex(v[0]) for v in ex.krylov_optimal_iterate(Aq, b, t, dinv)])
        got = oracle.jacpcg(A, np.eye(K)[:, col], tol=0.0, max_iter=t)["X"][:, 0]
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_exact_termination_after_K_steps():
    # CG on an HPD K x K system reaches A^{-1} b after K steps (exact arithmetic).
    H, xi = _exact_case()
    A = oracle.gram(H, xi)
    K = A.shape[0]
    Aq = [[ex.QC(A[i, j].real, A[i, j].imag) for j in range(K)] for i in range(K)]
    Ainv = np.array([[complex(v) for v in row] for row in ex.solve(Aq, ex.identity(K))])
    res = oracle.jacpcg(A, None, tol=0.0, max_iter=K)
    np.testing.assert_allclose(res["X"], Ainv, rtol=0, atol=1e-12)
    assert np.all(res["true_relres"] < 1e-12)


@pytest.mark.parametrize("T", [1, 3, 6])
def test_matches_scipy_pcg_iterates(rng, T):
    A = _hpd(rng, 30, 12, 0.2, spread=8.0)
    d = A.diagonal().real
    Minv = spla.LinearOperator(A.shape, matvec=lambda v: v / d, dtype=complex)
    for j in range(3):
        b = _crandn(rng, 12)
        x_sp, _ = spla.cg(A, b, x0=np.zeros(12, complex), rtol=0.0, atol=0.0, maxiter=T, M=Minv)
        x_or = oracle.jacpcg(A, b, tol=0.0, max_iter=T)["X"][:, 0]
        np.testing.assert_allclose(x_or, x_sp, rtol=0, atol=1e-13 * np.abs(x_sp).max())


def test_plain_cg_flag_matches_scipy_cg(rng):
    A = _hpd(rng, 30, 10, 0.2, spread=4.0)
    b = _crandn(rng, 10)
    x_sp, _ = spla.cg(A, b, x0=np.zeros(10, complex), rtol=0.0, atol=0.0, maxiter=4)
    x_or = oracle.jacpcg(A, b, tol=0.0, max_iter=4, precond="none")["X"][:, 0]
    np.testing.assert_allclose(x_or, x_sp, rtol=0, atol=1e-13 * np.abs(x_sp).max())


def test_zero_channel_one_iteration():
    # H = 0 -> A = xi I; Jacobi-PCG is exact after one iteration: X = B / xi.
    xi = 1.6
    A = oracle.gram(np.zeros((8, 5), complex), xi)
    res = oracle.jacpcg(A, None, tol=1e-12, max_iter=16)
    assert np.all(res["iters"] == 1)
    np.testing.assert_allclose(res["X"], np.eye(5) / xi, rtol=0, atol=1e-15)


def test_disjoint_users_one_iteration(rng):
    # Users on disjoint antennas (disjoint visibility regions) -> diagonal A:
    # the Jacobi preconditioner is exact and one iteration solves the system.
    M, K = 12, 4
    H = np.zeros((M, K), complex)
    for k in range(K):
        H[3 * k:3 * k + 3, k] = _crandn(rng, 3)
    A = oracle.gram(H, 0.3)
    res = oracle.jacpcg(A, None, tol=1e-13, max_iter=10)
    assert np.all(res["iters"] == 1)
    np.testing.assert_allclose(res["X"], np.diag(1.0 / A.diagonal().real), rtol=1e-14, atol=0)


def test_single_user_closed_form(rng):
    h = _crandn(rng, 9, 1)
    xi = 0.7
    res = oracle.jacpcg(oracle.gram(h, xi), None, tol=1e-14, max_iter=3)
    assert res["iters"][0] == 1
    np.testing.assert_allclose(res["X"][0, 0], 1.0 / (np.linalg.norm(h) ** 2 + xi), rtol=1e-15)


def test_tolerance_stop_is_first_crossing(rng):
    # Right-hand sides far from unit norm: the rule is relative to ||b_j||.
    A = _hpd(rng, 40, 16, 0.05, spread=10.0)
    tol = 1e-6
    B = _crandn(rng, 16, 1) * np.array([1e-4, 1e-2, 1.0, 1e2, 1e4, 1e6])   # one direction, six scales
    res = oracle.jacpcg(A, B, tol=tol, max_iter=200)
    assert res["instance_status"] == oracle.OK
    for j in range(6):
        t = res["iters"][j]
        r = B[:, j] - A @ res["X"][:, j]
        assert res["relres"][j] <= tol
        assert np.linalg.norm(r) <= 10 * tol * np.linalg.norm(B[:, j])
        if t > 1:
            prev = oracle.jacpcg(A, B[:, j], tol=0.0, max_iter=t - 1)
            assert prev["relres"][0] > tol
    assert len(set(res["iters"].tolist())) == 1   # scale-invariant iteration count


def test_a_norm_error_nonincreasing(rng):
    A = _hpd(rng, 25, 12, 0.01, spread=20.0)
    b = _crandn(rng, 12)
    xs = np.linalg.solve(A, b)
    errs = []
    for t in range(1, 13):
        x = oracle.jacpcg(A, b, tol=0.0, max_iter=t)["X"][:, 0]
        e = x - xs
        errs.append(np.vdot(e, A @ e).real)
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-9) + 1e-25 for i in range(len(errs) - 1))


def test_not_converged_and_breakdown_status():
    A = oracle.gram(np.eye(6, 6, dtype=complex) * np.arange(1, 7), 1e-3)
    res = oracle.jacpcg(A + 0.5 * (np.ones((6, 6)) - np.eye(6)), None, tol=1e-14, max_iter=1)
    assert res["instance_status"] == oracle.NOT_CONVERGED
    bad = np.array([[1.0, 3.0], [3.0, 1.0]], complex)   # indefinite
    res = oracle.jacpcg(bad, np.array([1.0, -1.0]), tol=0.0, max_iter=4)
    assert res["status"][0] == oracle.BREAKDOWN
    assert res["instance_status"] == oracle.BREAKDOWN


def test_zero_rhs_column():
    A = oracle.gram(np.ones((4, 3), complex), 1.0)
    B = np.zeros((3, 2), complex)
    B[0, 1] = 1.0
    res = oracle.jacpcg(A, B, tol=0.0, max_iter=5)
    assert res["iters"][0] == 0 and np.all(res["X"][:, 0] == 0)
    assert res["iters"][1] >= 1


def test_literal_algorithm1_coincides_only_for_constant_diagonal(rng):
    # Reading of Algorithm 1 (Euclidean products on C^{-1} A) vs standard
    # Jacobi-PCG: identical when diag(A) is constant, different otherwise.
    A = _hpd(rng, 30, 8, 0.1, spread=1.0)
    dh = 1.0 / np.sqrt(A.diagonal().real)
    Aunit = dh[:, None] * A * dh[None, :]            # unit diagonal
    b = _crandn(rng, 8)
    for T in (1, 3, 5):
        np.testing.assert_allclose(oracle.cg_on_jacobi_scaled_operator(Aunit, b, T),
                                   oracle.jacpcg(Aunit, b, tol=0.0, max_iter=T)["X"][:, 0],
                                   rtol=0, atol=1e-12)
    Avar = _hpd(rng, 30, 8, 0.01, spread=30.0)
    lit = oracle.cg_on_jacobi_scaled_operator(Avar, b, 8)
    std = oracle.jacpcg(Avar, b, tol=0.0, max_iter=8)["X"][:, 0]
    assert np.linalg.norm(lit - std) > 1e-6 * np.linalg.norm(std)
    assert np.linalg.norm(std - np.linalg.solve(Avar, b)) < 1e-9 * np.linalg.norm(std)


def test_jacobi_needs_fewer_iterations_than_cg():
    # The paper's convergence comparison (Sec. IV, Fig. 2): Jacobi
    # preconditioning (eq. 21) beats plain CG when the users' gains -- the
    # diagonal of A -- are spread, as in the gain-normalised channels.
    from channelgen import channel_batch, workload
    w = workload("single", gain="normalised")
    H = channel_batch(w, n=6)
    jac, cg = [], []
    for b in range(6):
        A = oracle.gram(H[b].T.astype(np.complex128), w.xi_values()[0])
        s = np.ones((w.K, 1), np.complex128)
        jac.append(int(oracle.jacpcg(A, s, tol=1e-6, max_iter=500)["iters"][0]))
        cg.append(int(oracle.jacpcg(A, s, tol=1e-6, max_iter=500, precond="none")["iters"][0]))
    assert all(j < c for j, c in zip(jac, cg)), (jac, cg)
