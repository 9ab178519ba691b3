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


def test_gram_zero_for_disjoint_visibility_regions():
    # eq. 4: D_k is binary, so users whose visibility regions share no subarray
    # have exactly orthogonal channels and A_ij = 0; in VR order A is banded.
    from channelgen import channel_instance, vr_order, vr_spans
    h, meta = channel_instance(1024, 32, 48, 0.9, (1, 3), 5, 0)
    order = vr_order(meta)
    spans = vr_spans(meta, 1024, 32)[order]
    A = oracle.gram(h[order].T.astype(np.complex128), 1e-3)
    disjoint = (np.minimum(spans[:, None, 1], spans[None, :, 1]) <= np.maximum(spans[:, None, 0], spans[None, :, 0]))
    assert disjoint.any() and np.all(A[disjoint] == 0)
    assert np.all(np.abs(A[~disjoint & ~np.eye(48, dtype=bool)]) > 0)
    # H is zero outside each user's span
    Hs = h[order]
    for k in range(48):
        assert np.all(Hs[k, :spans[k, 0]] == 0) and np.all(Hs[k, spans[k, 1]:] == 0)
    # envelope: in VR order (by start), every user j that starts at or after
    # user i's region ends is disjoint from i, and those users form a suffix
    for i in range(48):
        later = np.flatnonzero(spans[:, 0] >= spans[i, 1])
        if later.size:
            assert np.array_equal(later, np.arange(later[0], 48)) and np.all(A[i, later[0]:] == 0)
