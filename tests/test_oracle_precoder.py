"""Pins of the oracle's power-normalised RZF precoder (eq. 7, beta after eq. 7,
eq. 15) and the SINR / sum-rate evaluation (eqs. 9-10)."""

import numpy as np

import oracle
from tests.test_oracle_gram_inverse import _crandn, _golden


def test_golden_worked_precoder():
    g = _golden()
    H = g["H"].reshape(2, 2)
    Xs, W, beta = oracle.direct_rzf(H, g["xi"][0])
    np.testing.assert_allclose(beta, g["beta_pow"][0], rtol=1e-15)
    np.testing.assert_allclose(W * 4 * np.sqrt(13), g["W_times_4sqrt13"].reshape(2, 2), rtol=0, atol=1e-13)


def test_power_constraint(rng):
    H = _crandn(rng, 32, 8)
    for P in (1.0, 3.5):
        res = oracle.rzf(H, 0.3, tol=1e-10, max_iter=50, P_tx=P)
        np.testing.assert_allclose(np.linalg.norm(res["W"]) ** 2, P, rtol=1e-13)


def test_single_user_is_matched_filter(rng):
    h = _crandn(rng, 16, 1)
    for xi in (1e-3, 1.0, 100.0):
        _, W, _ = oracle.direct_rzf(h, xi, P_tx=2.0)
        np.testing.assert_allclose(W, np.sqrt(2.0) * h / np.linalg.norm(h), rtol=1e-13)


def test_effective_channel_identity(rng):
    # With X = A^{-1}: H^H W = beta (H^H H) A^{-1} = beta (I - xi A^{-1}).
    H = _crandn(rng, 24, 6)
    xi = 0.8
    Xs, W, beta = oracle.direct_rzf(H, xi)
    np.testing.assert_allclose(H.conj().T @ W, beta * (np.eye(6) - xi * Xs), rtol=0, atol=1e-12)


def test_matches_numpy_solve_closed_form(rng):
    H = _crandn(rng, 20, 7)
    xi = 0.25
    F = H @ np.linalg.solve(H.conj().T @ H + xi * np.eye(7), np.eye(7))
    want = F / np.linalg.norm(F)
    _, W, _ = oracle.direct_rzf(H, xi)
    np.testing.assert_allclose(W, want, rtol=0, atol=1e-13)


def test_invariances(rng):
    H = _crandn(rng, 18, 5)
    xi = 0.6
    _, W, _ = oracle.direct_rzf(H, xi)
    c = 3.7
    _, Wc, _ = oracle.direct_rzf(c * H, c * c * xi)            # (cH, c^2 xi) -> same W
    np.testing.assert_allclose(Wc, W, rtol=0, atol=1e-12)
    phi = np.exp(1j * rng.uniform(0, 2 * np.pi, 5))
    _, Wp, _ = oracle.direct_rzf(H * phi[None, :], xi)         # per-user phases
    np.testing.assert_allclose(Wp, W * phi[None, :], rtol=0, atol=1e-12)
    Q, _ = np.linalg.qr(_crandn(rng, 18, 18))                  # antenna unitary
    np.testing.assert_allclose(oracle.gram(Q @ H, xi), oracle.gram(H, xi), rtol=0, atol=1e-12)
    _, Wu, _ = oracle.direct_rzf(Q @ H, xi)
    np.testing.assert_allclose(Wu, Q @ W, rtol=0, atol=1e-12)


def test_pcg_precoder_converges_to_direct(rng):
    H = _crandn(rng, 64, 12)
    res = oracle.rzf(H, 0.5, tol=1e-12, max_iter=100)
    _, W, _ = oracle.direct_rzf(H, 0.5)
    np.testing.assert_allclose(res["W"], W, rtol=0, atol=1e-10)


def test_sinr_zero_forcing_limit(rng):
    # xi -> 0 with K <= M full rank: RZF -> ZF, inter-user leakage vanishes and
    # every user sees the same SINR beta^2 / sigma2.
    H = _crandn(rng, 40, 6)
    _, W, beta = oracle.direct_rzf(H, 1e-12)
    s = oracle.sinr(H, W, sigma2=0.01)
    np.testing.assert_allclose(s, beta ** 2 / 0.01, rtol=1e-8)
    np.testing.assert_allclose(oracle.sum_rate(H, W, 0.01), 6 * np.log2(1 + beta ** 2 / 0.01), rtol=1e-8)


def test_sinr_brute_force(rng):
    H = _crandn(rng, 8, 3)
    W = _crandn(rng, 8, 3)
    s = oracle.sinr(H, W, 0.5)
    for k in range(3):
        sig = abs(np.sum(H[:, k].conj() * W[:, k])) ** 2
        intf = sum(abs(np.sum(H[:, k].conj() * W[:, j])) ** 2 for j in range(3) if j != k)
        np.testing.assert_allclose(s[k], sig / (intf + 0.5), rtol=1e-13)
