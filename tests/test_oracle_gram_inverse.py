"""Pins of the oracle's Gram matrix (eq. 7) and direct inverses (Appendix A)."""

import os

import numpy as np
import pytest

import oracle
from tests import _exact as ex

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rzf_2x2_worked.txt")


def _golden():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *rest = line.split()
            nums = []
            for tok in rest:
                if "," in tok:
                    re, im = tok.split(",")
                    nums.append(complex(float(re), float(im)))
                else:
                    nums.append(float(tok))
            vals[key] = np.array(nums)
    return vals


def _crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def test_gram_golden_worked_example():
    g = _golden()
    H = g["H"].reshape(2, 2)
    A = oracle.gram(H, g["xi"][0])
    np.testing.assert_allclose(A, g["A"].reshape(2, 2), rtol=0, atol=1e-15)


@pytest.mark.parametrize("M,K", [(7, 3), (16, 16), (64, 24), (5, 9)])
def test_gram_bilinear_form(rng, M, K):
    # u^H A v = (H u)^H (H v) + xi u^H v for all u, v determines A uniquely
    # (polarisation); a transposed index or a missing conjugate breaks it.
    H = _crandn(rng, M, K)
    xi = 0.37
    A = oracle.gram(H, xi)
    for _ in range(5):
        u = _crandn(rng, K)
        v = _crandn(rng, K)
        lhs = np.vdot(u, A @ v)
        rhs = np.vdot(H @ u, H @ v) + xi * np.vdot(u, v)
        assert abs(lhs - rhs) <= 1e-12 * (abs(rhs) + np.linalg.norm(H) ** 2)


def test_gram_exactly_hermitian_and_real_diagonal(rng):
    H = _crandn(rng, 33, 17)
    A = oracle.gram(H, 0.1)
    assert np.array_equal(A, A.conj().T)
    assert np.all(A.diagonal().imag == 0)


def test_gram_zero_channel_gives_xi_identity():
    A = oracle.gram(np.zeros((10, 4), complex), 2.5)
    assert np.array_equal(A, 2.5 * np.eye(4))


def test_gram_eigenvalue_bounds(rng):
    # eq. 18 argument: A - xi I = H^H H is PSD, so xi <= lambda_min and
    # lambda_max <= xi + ||H||_F^2.
    H = _crandn(rng, 20, 12)
    xi = 0.05
    lam = np.linalg.eigvalsh(oracle.gram(H, xi))
    assert lam.min() >= xi * (1 - 1e-12)
    assert lam.max() <= xi + np.linalg.norm(H) ** 2 + 1e-9


def test_gram_exact_gaussian_integers(rng):
    # Gaussian-integer channel: every entry of H^H H is an exact integer sum,
    # checked against exact rational matrix multiplication.
    H = rng.integers(-3, 4, size=(6, 4)) + 1j * rng.integers(-3, 4, size=(6, 4))
    A = oracle.gram(H, 0.5)
    Hq = ex.mat(H.tolist())
    G = ex.matmul(ex.adjoint(Hq), Hq)
    for i in range(4):
        for j in range(4):
            want = complex(G[i][j]) + (0.5 if i == j else 0.0)
            assert A[i, j] == want


def test_cholesky_matches_lapack(rng):
    H = _crandn(rng, 40, 20)
    A = oracle.gram(H, 0.3)
    L = oracle.cholesky_lower(A)
    np.testing.assert_allclose(L, np.linalg.cholesky(A), rtol=0, atol=1e-12)
    np.testing.assert_allclose(L @ L.conj().T, A, rtol=0, atol=1e-12)


def test_chol_inverse_matches_lapack_and_identity(rng):
    H = _crandn(rng, 50, 24)
    A = oracle.gram(H, 0.02)
    Ai = oracle.chol_inverse(A)
    cond = np.linalg.cond(A)
    np.testing.assert_allclose(Ai, np.linalg.inv(A), rtol=0, atol=1e-13 * cond * np.abs(Ai).max())
    np.testing.assert_allclose(A @ Ai, np.eye(24), rtol=0, atol=1e-12 * cond)


@pytest.mark.parametrize("K", [1, 2, 5, 8])
def test_gauss_jordan_agrees_with_cholesky(rng, K):
    H = _crandn(rng, K + 3, K)
    A = oracle.gram(H, 0.4)
    np.testing.assert_allclose(oracle.gauss_jordan_inverse(A), oracle.chol_inverse(A),
                               rtol=0, atol=1e-12)


def test_inverse_exact_rational():
    # Gaussian-integer H, xi = 1/2: exact inverse by rational elimination.
    H = np.array([[1, 2j, 0, 1 - 1j], [1j, 1, 2, 0], [0, 1 + 1j, 1, 1], [2, 0, -1j, 1],
                  [1, 1, 1, 1j], [0, -1, 1j, 2]])
    A = oracle.gram(H, 0.5)
    Aq = [[ex.QC(complex(A[i, j]).real, complex(A[i, j]).imag) for j in range(4)] for i in range(4)]
    Ainv = ex.solve(Aq, ex.identity(4))
    want = np.array([[complex(v) for v in row] for row in Ainv])
    np.testing.assert_allclose(oracle.chol_inverse(A), want, rtol=0, atol=1e-14)
    np.testing.assert_allclose(oracle.gauss_jordan_inverse(A), want, rtol=0, atol=1e-14)


def test_inverse_golden():
    g = _golden()
    A = g["A"].reshape(2, 2)
    np.testing.assert_allclose(oracle.chol_inverse(A), g["Ainv"].reshape(2, 2), rtol=0, atol=1e-15)


def test_cholesky_rejects_non_hpd():
    with pytest.raises(ValueError):
        oracle.chol_inverse(np.array([[1.0, 2.0], [2.0, 1.0]], complex))
