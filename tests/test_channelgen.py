"""Statistics and determinism of the seeded channel generator."""

import numpy as np

from channelgen import channel_batch, channel_instance, workload, xi_from_snr, serving_requests


def test_instance_regenerates_bit_identically():
    w = workload("batched")
    batch = channel_batch(w, n=4, start=10)
    one, _ = channel_instance(w.M, w.S, w.K, w.r, w.vr, w.seed, 12)
    assert np.array_equal(batch[2], one)
    assert batch.dtype == np.complex64 and batch.shape == (4, 64, 1024)


def test_visibility_regions_contiguous_and_sized():
    w = workload("batched")
    for i in range(5):
        H, meta = channel_instance(w.M, w.S, w.K, w.r, w.vr, 3, i)
        Ms = w.M // w.S
        for k in range(w.K):
            active = np.abs(H[k].reshape(w.S, Ms)).sum(axis=1) > 0
            idx = np.flatnonzero(active)
            assert w.vr[0] <= len(idx) <= w.vr[1]
            assert np.all(np.diff(idx) == 1)
            assert len(idx) == meta["vr_len"][k]


def test_exponential_correlation_within_subarray():
    # Empirical correlation of antenna pairs (i, i+lag) inside visible subarrays
    # approaches r^lag; gains are divided out.
    M, S, K, r = 256, 4, 32, 0.7
    acc = np.zeros(4)
    cnt = 0
    for i in range(40):
        H, meta = channel_instance(M, S, K, r, (4, 4), 7, i, gain="normalised")
        Y = H.reshape(K, S, M // S) / np.sqrt(meta["beta"])[:, None, None]
        for lag in range(4):
            acc[lag] += np.mean((Y[:, :, lag:] * Y[:, :, :Y.shape[2] - lag].conj()).real)
        cnt += 1
    est = acc / cnt
    np.testing.assert_allclose(est, r ** np.arange(4), atol=0.03)


def test_path_loss_models():
    w = workload("single")
    _, m = channel_instance(w.M, w.S, w.K, w.r, w.vr, 0, 0)
    np.testing.assert_allclose(m["beta"], m["distance"] ** -3.7)
    assert np.all((m["distance"] >= 10) & (m["distance"] <= 100))
    _, mn = channel_instance(w.M, w.S, w.K, w.r, w.vr, 0, 0, gain="normalised")
    np.testing.assert_allclose(mn["beta"], (mn["distance"] / 10) ** -3.7)


def test_xi_rule_and_serving_stream():
    assert xi_from_snr(64, 10.0) == 6.4
    assert abs(xi_from_snr(64, 20.0) - 0.64) < 1e-15
    reqs = serving_requests(rate_hz=2000.0, duration_s=0.5, seed=1)
    assert 800 < len(reqs) < 1200
    for q in reqs:
        assert q["M"] in (256, 512, 1024, 2048, 4096)
        assert q["K"] in (8, 16, 32, 64, 128, 256) and q["K"] <= q["M"] // 8
        assert 1 <= q["n_sub"] <= 64 and 0.3 <= q["r"] <= 0.9
    gaps = np.diff([q["t"] for q in reqs])
    assert abs(gaps.mean() - 1 / 2000) < 0.15 / 2000


def test_device_pool_r_draws_each_instance_at_its_own_r():
    # per-instance correlation: the lag-1 antenna correlation of an instance
    # drawn at r is r (one subarray, every user visible, many users)
    import torch
    from channelgen import device_pool_r
    H, rs = device_pool_r(512, 1, 64, (0.3, 0.9), (1, 1), 4, 5, device="cpu", gain="normalised", chunk=3)
    assert H.shape == (4, 64, 512) and H.dtype == torch.complex64
    r = rs.numpy()
    assert np.all((r >= 0.3) & (r <= 0.9)) and np.ptp(r) > 0.05
    for b in range(4):
        x = H[b].numpy().astype(np.complex128)
        c = np.sum(x[:, 1:] * np.conj(x[:, :-1])) / np.sum(np.abs(x[:, :-1]) ** 2)
        assert abs(c.real - r[b]) < 0.03 and abs(c.imag) < 0.03, (b, c, r[b])
