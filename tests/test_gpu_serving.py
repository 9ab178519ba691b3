"""Request API (continuous batching): results equal the direct call, a request's
result is the same alone and in a mix, cancellation, budget and timeouts."""

import time

import numpy as np
import pytest

import oracle
from channelgen import device_pool
from paper_2305_13925_amd import binding as bd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a HIP device"
    return t


@pytest.fixture(scope="module")
def sess(torch):
    s = bd.Session(0, hbm_budget_bytes=8 << 30)
    yield s
    s.close()


def test_request_matches_direct_call_and_oracle(torch, sess):
    H = device_pool(512, 4, 32, 0.5, (2, 4), 5, 1)
    W_req = torch.empty_like(H)
    t = bd.jacpcg_submit(sess, H, W_req, 3.2, tol=1e-6, max_iter=16, user_tag=77)
    res = bd.jacpcg_wait(sess, t, 10000)
    assert res["status"] == bd.OK and res["user_tag"] == 77
    assert res["t_submit_us"] <= res["t_admit_us"] <= res["t_done_us"]
    W_dir = bd.rzf_precoder(sess, H, 3.2, tol=1e-6, max_iter=16)
    torch.cuda.synchronize()
    assert torch.equal(W_req, W_dir)
    Hn = H.cpu().numpy()
    for b in range(5):
        ref = oracle.rzf(Hn[b].T.astype(np.complex128), 3.2, tol=0.0, max_iter=res["max_iters"])
        Wb = W_req[b].cpu().numpy().T
        assert np.linalg.norm(Wb - ref["W"]) / np.linalg.norm(ref["W"]) <= 1e-5


def test_alone_equals_in_mix(torch, sess):
    # The same request computed alone, then in a burst of other requests of the
    # same and of other shapes (so it is batched with them): bitwise equal.
    H = device_pool(1024, 8, 64, 0.7, (2, 4), 7, 2, gain="normalised")
    W_alone = torch.empty_like(H)
    t = bd.jacpcg_submit(sess, H, W_alone, 6.4, tol=1e-6, max_iter=16)
    assert bd.jacpcg_wait(sess, t, 10000)["status"] == bd.OK
    others = [device_pool(1024, 8, 64, 0.5, (2, 4), 3 + i, 10 + i) for i in range(6)]
    others += [device_pool(512, 4, 16, 0.5, (2, 4), 4, 20 + i) for i in range(4)]
    outs = [torch.empty_like(o) for o in others]
    W_mix = torch.empty_like(H)
    tickets = []
    for i, (o, w) in enumerate(zip(others, outs)):
        xi = 6.4 if o.shape[1] == 64 else 1.6
        tickets.append(bd.jacpcg_submit(sess, o, w, xi, tol=1e-6, max_iter=16))
        if i == 2:
            tickets.append(bd.jacpcg_submit(sess, H, W_mix, 6.4, tol=1e-6, max_iter=16))
    for t in tickets:
        assert bd.jacpcg_wait(sess, t, 20000)["status"] == bd.OK
    assert torch.equal(W_alone, W_mix)


def test_poll_cancel_and_unknown_ticket(torch, sess):
    H = device_pool(2048, 4, 128, 0.5, (2, 4), 48, 3)
    Ws = [torch.empty_like(H) for _ in range(6)]
    tickets = [bd.jacpcg_submit(sess, H, W, 12.8, tol=1e-6, max_iter=16) for W in Ws]
    bd.jacpcg_cancel(sess, tickets[-1])
    final = {}
    deadline = time.time() + 30
    while len(final) < len(tickets) and time.time() < deadline:
        for t in tickets:
            if t in final:
                continue
            rc, res = bd.jacpcg_poll(sess, t)
            if rc == bd.OK:
                final[t] = res
        time.sleep(0.001)
    assert len(final) == len(tickets)
    assert final[tickets[-1]]["status"] in (bd.E_CANCELLED,)
    assert all(final[t]["status"] == bd.OK for t in tickets[:-1])
    with pytest.raises(bd.JacpcgError) as ei:
        bd.jacpcg_poll(sess, tickets[0])          # already collected
    assert ei.value.code == bd.E_INVALID_ARG


def test_budget_rejection_and_timeout(torch):
    with bd.Session(0, hbm_budget_bytes=1 << 20) as small:
        H = device_pool(1024, 4, 64, 0.5, (2, 4), 4, 4)
        W = torch.empty_like(H)
        with pytest.raises(bd.JacpcgError) as ei:
            bd.jacpcg_submit(small, H, W, 6.4)     # 4 MiB of H + W: never fits 1 MiB
        assert ei.value.code == bd.E_BUDGET
    with bd.Session(0) as s:
        H = device_pool(4096, 4, 256, 0.5, (2, 4), 64, 5)
        W = torch.empty_like(H)
        t = bd.jacpcg_submit(s, H, W, 25.6, tol=0.0, max_iter=64)
        try:
            bd.jacpcg_wait(s, t, 0)
        except bd.JacpcgError as e:
            assert e.code == bd.E_TIMEOUT
        assert bd.jacpcg_wait(s, t, 60000)["status"] == bd.OK


def test_short_poisson_stream(torch, sess):
    from paper_2305_13925_amd.serve import run_serving
    out = run_serving(sess, rate_hz=1000.0, warmup_s=0.1, measure_s=0.4, seed=3)
    print(out)
    assert out["requests"] > 100
    assert out["statuses"].get(str(bd.OK), 0) + out["statuses"].get(str(bd.NOT_CONVERGED), 0) == out["requests"]
    assert out["p99_ms"] < 1000.0


def test_request_waits_for_the_stream_that_produces_H(torch, sess):
    # H is written on a side stream, with extra work queued behind its
    # generation, and submitted without any synchronisation: the request must
    # read the finished H (the ready event recorded on that stream at submission).
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        H = device_pool(2048, 4, 64, 0.5, (2, 4), 32, 11)
        for _ in range(50):
            H.mul_(1.0)
        W = torch.empty_like(H)
        t = bd.jacpcg_submit(sess, H, W, 6.4, tol=0.0, max_iter=8, stream=side)
    res = bd.jacpcg_wait(sess, t, 20000)
    assert res["status"] == bd.OK
    torch.cuda.synchronize()
    W_dir = bd.rzf_precoder(sess, H, 6.4, tol=0.0, max_iter=8)
    torch.cuda.synchronize()
    assert torch.equal(W, W_dir)


def test_requests_differing_in_one_setting_never_share_a_batch(torch, sess):
    # Requests queued together are grouped into one batch only when shape and
    # every solve setting match. These pairs differ in M alone (42 / 43 at
    # K = 59) and in max_iter alone (468 / 502): each must come out exactly as
    # its own direct call. Long requests occupy the slots first, so the pairs
    # wait in the queue and are admitted in one pass.
    blockers = [device_pool(4096, 4, 256, 0.5, (2, 4), 32, 40 + i) for i in range(4)]
    bouts = [torch.empty_like(h) for h in blockers]
    cases = [(42, 59, 16, 3), (43, 59, 16, 3), (4096, 8, 468, 2), (4096, 8, 502, 2)]
    Hs, Ws = [], []
    for i, (M, K, _, n) in enumerate(cases):
        Hs.append(device_pool(M, 1, K, 0.5, (1, 1), n, 60 + i))
        Ws.append(torch.empty_like(Hs[-1]))
    torch.cuda.synchronize()
    tb = [bd.jacpcg_submit(sess, h, w, 25.6, tol=0.0, max_iter=64) for h, w in zip(blockers, bouts)]
    tickets = [bd.jacpcg_submit(sess, H, W, 1.6, tol=1e-6, max_iter=mi) for H, W, (_, _, mi, _) in zip(Hs, Ws, cases)]
    for t in tb + tickets:
        assert bd.jacpcg_wait(sess, t, 60000)["status"] in (bd.OK, bd.NOT_CONVERGED)
    for H, W, (M, K, mi, _) in zip(Hs, Ws, cases):
        W_dir = bd.rzf_precoder(sess, H, 1.6, tol=1e-6, max_iter=mi)
        torch.cuda.synchronize()
        assert torch.equal(W, W_dir), (M, K, mi)


@pytest.mark.parametrize("prec,M,K", [(bd.GRAM_BF16X6, 1024, 64), (bd.GRAM_BF16X6, 1024, 128),
                                      (bd.GRAM_BF16X3, 512, 96)])
def test_split_gram_requests_equal_direct_calls(torch, sess, prec, M, K):
    # Split-BF16 requests of one key (the K <= 64 Gram and the block-pair Gram
    # above it, channels read through per-instance pointers when batched):
    # each result equals the direct call on its own channels bit for bit.
    Ha = device_pool(M, 4, K, 0.6, (2, 4), 3, 31)
    Hb = device_pool(M, 4, K, 0.6, (2, 4), 5, 32)
    Wa, Wb = torch.empty_like(Ha), torch.empty_like(Hb)
    xi = K / 10.0
    ta = bd.jacpcg_submit(sess, Ha, Wa, xi, tol=0.0, max_iter=8, precision=prec)
    tb = bd.jacpcg_submit(sess, Hb, Wb, xi, tol=0.0, max_iter=8, precision=prec)
    for t in (ta, tb):
        assert bd.jacpcg_wait(sess, t, 20000)["status"] == bd.OK
    for H, W in ((Ha, Wa), (Hb, Wb)):
        Wd = bd.rzf_precoder(sess, H, xi, tol=0.0, max_iter=8, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(W, Wd)
