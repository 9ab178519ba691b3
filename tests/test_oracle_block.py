"""Pins of the subarray-block RZF oracle (Sec. II, eqs. 2, 6, 7, 9)."""

import numpy as np
import pytest

import oracle
from channelgen import block_channel_batch, block_channel_instance

SHAPES = [(48, 32, 40, 6, 5), (64, 0, 64, 8, 8), (30, 50, 20, 4, 7), (16, 16, 16, 1, 1)]


def _H(shape, index=0, gain="normalised"):
    M1, Mc, M2, K1, K2 = shape
    return block_channel_instance(M1, Mc, M2, K1, K2, 0.6, 3, index, gain).T.astype(np.complex128)


@pytest.mark.parametrize("shape", SHAPES)
def test_channel_has_the_block_form_of_eq2(shape):
    M1, Mc, M2, K1, K2 = shape
    H = _H(shape)
    assert H.shape == (M1 + Mc + M2, K1 + K2)
    assert np.all(H[:M1, K1:] == 0) and np.all(H[M1 + Mc:, :K1] == 0)
    assert np.all(np.abs(H[:M1, :K1]).sum(axis=0) > 0) and np.all(np.abs(H[M1 + Mc:, K1:]).sum(axis=0) > 0)
    B = block_channel_batch(M1, Mc, M2, K1, K2, 0.6, 2, seed=3)
    assert np.array_equal(B[0], block_channel_instance(M1, Mc, M2, K1, K2, 0.6, 3, 0))


@pytest.mark.parametrize("shape", SHAPES)
def test_block_structure_and_power_per_block(shape):
    M1, Mc, M2, K1, K2 = shape
    H = _H(shape)
    G, betas = oracle.block_rzf(H, 0.7, M1, Mc, M2, K1, K2, max_iter=12, P_tx=2.0)
    assert np.all(G[:M1, K1:] == 0) and np.all(G[M1 + Mc:, :K1] == 0)        # eq. 6's zero blocks
    for name, (rows, cols) in oracle.block_slices(M1, Mc, M2, K1, K2).items():
        if G[rows, cols].size:
            assert abs(np.sum(np.abs(G[rows, cols]) ** 2) - 2.0) < 1e-12          # tr(G_i^H G_i) = P
            assert betas[name] > 0


@pytest.mark.parametrize("shape", SHAPES)
def test_direct_blocks_match_numpy_solve(shape):
    # Each block is the RZF of its own sub-channel (eq. 7), with its own beta.
    M1, Mc, M2, K1, K2 = shape
    H = _H(shape, 1)
    xi = 0.3
    G, _ = oracle.block_rzf(H, xi, M1, Mc, M2, K1, K2, direct=True)
    for rows, cols in oracle.block_slices(M1, Mc, M2, K1, K2).values():
        Hi = H[rows, cols]
        if Hi.size == 0:
            continue
        F = Hi @ np.linalg.solve(Hi.conj().T @ Hi + xi * np.eye(Hi.shape[1]), np.eye(Hi.shape[1]))
        Gi = F * np.sqrt(1.0 / np.sum(np.abs(F) ** 2))
        assert np.allclose(G[rows, cols], Gi, rtol=0, atol=1e-12 * np.abs(Gi).max())


@pytest.mark.parametrize("shape", SHAPES[:3])
def test_iterative_blocks_converge_to_direct(shape):
    M1, Mc, M2, K1, K2 = shape
    H = _H(shape, 2)
    Gd, _ = oracle.block_rzf(H, 0.9, M1, Mc, M2, K1, K2, direct=True)
    Gi, _ = oracle.block_rzf(H, 0.9, M1, Mc, M2, K1, K2, max_iter=K1 + K2)
    assert np.linalg.norm(Gi - Gd) <= 1e-9 * np.linalg.norm(Gd)


def test_no_common_subarray_decouples_the_groups():
    # Mc = 0: the two groups share no antennas, so the block precoder is
    # blockdiag(G_1, G_2) and each group's SINR equals that of its own RZF.
    shape = (64, 0, 64, 8, 8)
    H = _H(shape, 4)
    G, _ = oracle.block_rzf(H, 0.5, *shape, direct=True)
    s = oracle.sinr(H, G, 0.05)
    _, G1, _ = oracle.direct_rzf(H[:64, :8], 0.5)
    _, G2, _ = oracle.direct_rzf(H[64:, 8:], 0.5)
    assert np.allclose(s[:8], oracle.sinr(H[:64, :8], G1, 0.05), rtol=1e-12)
    assert np.allclose(s[8:], oracle.sinr(H[64:, 8:], G2, 0.05), rtol=1e-12)


def _eq9(H, G, M1, Mc, M2, K1, K2, sigma2):
    """Eq. 9 written out with the paper's blocks and sums (groups i, m; users k, j)."""
    sl = {"1": slice(0, M1), "c": slice(M1, M1 + Mc), "2": slice(M1 + Mc, M1 + Mc + M2)}
    users = {1: range(0, K1), 2: range(K1, K1 + K2)}
    own = {1: "1", 2: "2"}
    out = np.zeros(K1 + K2)
    for i in (1, 2):
        m = 2 if i == 1 else 1
        for k in users[i]:
            h_ik, h_cik = H[sl[own[i]], k], H[sl["c"], k]

            def eff(j):  # h_{i,k}^H g_{i,j} + h_{ci,k}^H g_{ci,j}
                return np.vdot(h_ik, G[sl[own[i]], j]) + np.vdot(h_cik, G[sl["c"], j])

            sig = abs(eff(k)) ** 2
            intra = sum(abs(eff(j)) ** 2 for j in users[i] if j != k)
            inter = sum(abs(np.vdot(h_cik, G[sl["c"], j])) ** 2 for j in users[m])
            out[k] = sig / (intra + inter + sigma2)
    return out


@pytest.mark.parametrize("shape", SHAPES)
def test_generic_sinr_is_eq9_on_the_block_model(shape):
    M1, Mc, M2, K1, K2 = shape
    H = _H(shape, 5)
    G, _ = oracle.block_rzf(H, 0.4, M1, Mc, M2, K1, K2, max_iter=5)
    assert np.allclose(oracle.sinr(H, G, 0.02), _eq9(H, G, M1, Mc, M2, K1, K2, 0.02), rtol=1e-12, atol=0)
