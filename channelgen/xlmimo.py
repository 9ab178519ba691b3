"""Non-stationary, spatially correlated XL-MIMO channels (paper Sec. II, eqs. 2-4).

Model, per user k and instance (subcarrier):

    h_k = sqrt(beta_k) * D_k * R^{1/2} g_k,     g_k ~ CN(0, I_M)

  * R is block diagonal over the S subarrays of M/S antennas, with entries
    r^|i-j| inside a subarray (exponential correlation). R^{1/2} g is realised
    by the AR(1) recursion y_0 = g_0, y_i = r y_{i-1} + sqrt(1 - r^2) g_i, whose
    matrix is the exact Cholesky factor of r^|i-j|.
  * D_k is the binary visibility-region (VR) mask (eq. 4: Theta = D^1/2 R D^1/2);
    the VR is a contiguous run of L_k subarrays, L_k uniform on the stated
    range and its first subarray uniform over the valid positions.
  * beta_k = d_k^-3.7 with d_k ~ U[10, 100] m ("literal" gain). The "normalised"
    gain (d_k / 10 m)^-3.7 makes H^H H comparable to xi, so the solves are not
    trivially well conditioned.

The paper's per-antenna near-field path loss (eq. 3) and log-normal VR lengths
are replaced by this per-user model, which is what the workloads specify.

Every instance i of a workload draws from its own PCG64 stream seeded with
SeedSequence([seed, i]), so any instance can be regenerated alone and
bit-identically. Values are drawn in complex128 and rounded once to complex64;
both the GPU path and the oracle consume the same complex64 values.

Layout: a batch is returned as a complex64 array of shape [n, K, M]; row k of
instance b is user k's channel over the M antennas, i.e. each instance is the
column-major M x K matrix H (``instance_matrix`` gives the M x K view).
"""

from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    M: int
    S: int
    K: int
    r: float
    vr: tuple            # (min, max) number of visible subarrays, inclusive
    batch: int
    snr_db: tuple = (10.0,)
    xi: float | None = None   # fixed xi overrides the K/SNR rule
    gain: str = "literal"     # "literal" or "normalised"
    seed: int = 0
    tol: float = 0.0
    max_iter: int = 16
    extra: dict = field(default_factory=dict)

    def xi_values(self):
        if self.xi is not None:
            return [float(self.xi)]
        return [xi_from_snr(self.K, s) for s in self.snr_db]


def xi_from_snr(K, snr_db):
    """Regularisation xi = K / SNR (SNR in dB), the workloads' rule."""
    return float(K) / (10.0 ** (float(snr_db) / 10.0))


WORKLOADS = {
    # one plain instance: M=256 in 4 subarrays of 64, K=16, r=0.5, VR of 2-4
    # subarrays, 10 dB, Jac-PCG to relative residual 1e-6 or 16 iterations
    "single": Workload("single", M=256, S=4, K=16, r=0.5, vr=(2, 4), batch=1,
                       snr_db=(10.0,), tol=1e-6, max_iter=16),
    # 1024 subcarriers of M=1024 (8 x 128) and K=64, r=0.5, VR of 3-6,
    # SNR 0/10/20 dB, 8 fixed iterations (plus a tolerance-1e-5 variant)
    "batched": Workload("batched", M=1024, S=8, K=64, r=0.5, vr=(3, 6), batch=1024,
                        snr_db=(0.0, 10.0, 20.0), tol=0.0, max_iter=8),
    # 256 instances of M=4096 (16 x 256) and K=128, r=0.7, 10 dB; the VR
    # length is not stated for this workload: 6-12 of 16 subarrays keeps the
    # 3/8-6/8 visible fraction of the batched workload
    "precision": Workload("precision", M=4096, S=16, K=128, r=0.7, vr=(6, 12),
                          batch=256, snr_db=(10.0,), tol=1e-6, max_iter=64),
    # 64 instances of M=8192 (32 x 256) and K=256, r=0.95, VR of 1-3,
    # near-ZF regularisation xi = 1e-3
    "stress": Workload("stress", M=8192, S=32, K=256, r=0.95, vr=(1, 3), batch=64,
                       xi=1e-3, tol=1e-6, max_iter=1024),
}


def workload(name, **overrides):
    w = WORKLOADS[name]
    return replace(w, **overrides) if overrides else w


def _rng(seed, index):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(index)])))


def _ar1_factor(Ms, r):
    """Lower-triangular L with L L^T = [r^|i-j|] (the AR(1) recursion as a matrix)."""
    i = np.arange(Ms)
    expo = i[:, None] - i[None, :]
    L = np.where(expo >= 0, np.power(float(r), np.maximum(expo, 0)), 0.0)
    L[:, 1:] *= np.sqrt(1.0 - float(r) ** 2)
    return L


def channel_instance(M, S, K, r, vr, seed, index, gain="literal"):
    """Draw one instance. Returns (H as complex64 [K, M], meta dict)."""
    if M % S:
        raise ValueError("M must be a multiple of S")
    Ms = M // S
    lo, hi = int(vr[0]), int(vr[1])
    hi = min(hi, S)
    lo = max(1, min(lo, hi))
    rng = _rng(seed, index)
    d = rng.uniform(10.0, 100.0, size=K)
    vr_len = rng.integers(lo, hi + 1, size=K)
    vr_start = np.array([rng.integers(0, S - L + 1) for L in vr_len])
    g = (rng.standard_normal((K, S, Ms)) + 1j * rng.standard_normal((K, S, Ms))) / np.sqrt(2.0)
    y = g @ _ar1_factor(Ms, r).T                      # correlate along antennas
    mask = np.zeros((K, S), dtype=bool)
    for k in range(K):
        mask[k, vr_start[k]:vr_start[k] + vr_len[k]] = True
    y = y * mask[:, :, None]
    if gain == "literal":
        beta = d ** -3.7
    elif gain == "normalised":
        beta = (d / 10.0) ** -3.7
    else:
        raise ValueError(gain)
    h = (np.sqrt(beta)[:, None, None] * y).reshape(K, M)
    meta = dict(distance=d, beta=beta, vr_start=vr_start, vr_len=vr_len, mask=mask)
    return h.astype(np.complex64), meta


def vr_order(meta):
    """User order by visibility region (start subarray, then length): a
    permutation under which A = H^H H + xi I is banded, since users with
    disjoint regions have A_ij = 0 (eq. 4, D_k binary)."""
    return np.lexsort((meta["vr_len"], meta["vr_start"]))


def vr_spans(meta, M, S):
    """Per-user antenna span [first, end) of the visibility region: int32 [K, 2]."""
    Ms = M // S
    first = meta["vr_start"] * Ms
    return np.stack([first, first + meta["vr_len"] * Ms], axis=1).astype(np.int32)


def sorted_channel_batch(w: Workload, n=None, start=0, seed=None, gain=None):
    """Instances of workload w with each instance's users put in VR order.
    Returns (complex64 [n, K, M], int32 spans [n, K, 2])."""
    n = w.batch if n is None else int(n)
    seed = w.seed if seed is None else seed
    gain = w.gain if gain is None else gain
    H = np.empty((n, w.K, w.M), dtype=np.complex64)
    spans = np.empty((n, w.K, 2), dtype=np.int32)
    for b in range(n):
        h, meta = channel_instance(w.M, w.S, w.K, w.r, w.vr, seed, start + b, gain)
        order = vr_order(meta)
        H[b] = h[order]
        spans[b] = vr_spans(meta, w.M, w.S)[order]
    return H, spans


def channel_batch(w: Workload, n=None, start=0, seed=None, gain=None):
    """Instances start .. start+n-1 of workload w as complex64 [n, K, M]."""
    n = w.batch if n is None else int(n)
    seed = w.seed if seed is None else seed
    gain = w.gain if gain is None else gain
    out = np.empty((n, w.K, w.M), dtype=np.complex64)
    for b in range(n):
        out[b], _ = channel_instance(w.M, w.S, w.K, w.r, w.vr, seed, start + b, gain)
    return out


def instance_matrix(Hb):
    """The M x K matrix H (complex128) of one instance stored as [K, M]."""
    return np.asarray(Hb).T.astype(np.complex128)


def block_channel_instance(M1, Mc, M2, K1, K2, r, seed, index, gain="normalised"):
    """One channel of the subarray-block form of eq. 2 (three subarrays, two
    user groups): group 1 (K1 users) sees subarray 1 (M1 antennas) and the
    common subarray (Mc), group 2 (K2 users) sees the common subarray and
    subarray 2 (M2); every other block is zero (outside the users' visibility
    regions). Within a subarray the antennas are exponentially correlated with
    coefficient r (AR(1) recursion); the per-user gain follows ``gain`` as in
    ``channel_instance``. Returns complex64 [K1 + K2, M1 + Mc + M2].
    """
    K, M = K1 + K2, M1 + Mc + M2
    rng = _rng(seed, index)
    d = rng.uniform(10.0, 100.0, size=K)
    beta = d ** -3.7 if gain == "literal" else (d / 10.0) ** -3.7
    h = np.zeros((K, M), dtype=np.complex128)
    spans = {"1": (0, M1), "c": (M1, M1 + Mc), "2": (M1 + Mc, M)}
    for k in range(K):
        for sub in (("1", "c") if k < K1 else ("c", "2")):
            a, b = spans[sub]
            if b == a:
                continue
            g = (rng.standard_normal(b - a) + 1j * rng.standard_normal(b - a)) / np.sqrt(2.0)
            h[k, a:b] = _ar1_factor(b - a, r) @ g
    h *= np.sqrt(beta)[:, None]
    return h.astype(np.complex64)


def block_channel_batch(M1, Mc, M2, K1, K2, r, n, seed=0, gain="normalised"):
    """Instances 0 .. n-1 of the block channel model as complex64 [n, K1 + K2, M]."""
    return np.stack([block_channel_instance(M1, Mc, M2, K1, K2, r, seed, i, gain) for i in range(n)])


def serving_requests(rate_hz=2000.0, duration_s=11.0, seed=0, max_requests=None):
    """Poisson request stream of the serving workload.

    Each request: arrival time (exponential gaps at ``rate_hz``), M from
    {256, 512, 1024, 2048, 4096}, K uniform on {8, 16, 32, 64, 128, 256} with
    K <= M/8, 1-64 subcarriers, r ~ U[0.3, 0.9]; channels follow the
    single-instance model (4 subarrays of M/4, VR of 2-4) at xi = K/10 (10 dB).
    Channels are not drawn here -- ``request_channels`` draws them on demand.
    """
    rng = _rng(seed, 10 ** 9)
    t = 0.0
    reqs = []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t > duration_s:
            break
        M = int(rng.choice([256, 512, 1024, 2048, 4096]))
        ks = [k for k in (8, 16, 32, 64, 128, 256) if k <= M // 8]
        K = int(rng.choice(ks))
        n_sub = int(rng.integers(1, 65))
        r = float(rng.uniform(0.3, 0.9))
        reqs.append(dict(t=t, M=M, K=K, n_sub=n_sub, r=r, S=4, vr=(2, 4),
                         xi=xi_from_snr(K, 10.0), seed=int(seed) * 1000003 + len(reqs)))
        if max_requests is not None and len(reqs) >= max_requests:
            break
    return reqs


def request_channels(req):
    """complex64 [n_sub, K, M] channels of one serving request."""
    out = np.empty((req["n_sub"], req["K"], req["M"]), dtype=np.complex64)
    for b in range(req["n_sub"]):
        out[b], _ = channel_instance(req["M"], req["S"], req["K"], req["r"], req["vr"],
                                     req["seed"], b)
    return out


def device_pool(M, S, K, r, vr, n, seed, device="cuda", gain="literal"):
    """n instances of the same channel model drawn with torch on a device
    (complex64 [n, K, M]), for workloads too large to draw on the host (the
    serving stream). Same law as ``channel_instance``; a different stream of
    random numbers (torch's generator seeded with `seed`)."""
    import torch
    if M % S:
        raise ValueError("M must be a multiple of S")
    Ms = M // S
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    d = torch.rand((n, K), generator=g, device=device, dtype=torch.float64) * 90.0 + 10.0
    lo, hi = int(vr[0]), min(int(vr[1]), S)
    lo = max(1, min(lo, hi))
    vr_len = torch.randint(lo, hi + 1, (n, K), generator=g, device=device)
    start = (torch.rand((n, K), generator=g, device=device, dtype=torch.float64)
             * (S - vr_len + 1).to(torch.float64)).floor().to(torch.int64)
    sub = torch.arange(S, device=device)
    mask = (sub[None, None, :] >= start[..., None]) & (sub[None, None, :] < (start + vr_len)[..., None])
    re = torch.randn((n, K, S, Ms), generator=g, device=device, dtype=torch.float64)
    im = torch.randn((n, K, S, Ms), generator=g, device=device, dtype=torch.float64)
    L = torch.as_tensor(_ar1_factor(Ms, r), device=device)
    y = torch.complex(re @ L.T, im @ L.T) / (2.0 ** 0.5)
    y = y * mask[..., None]
    beta = d ** -3.7 if gain == "literal" else (d / 10.0) ** -3.7
    h = (beta.sqrt()[..., None, None] * y).reshape(n, K, M)
    return h.to(torch.complex64).contiguous()


def device_pool_r(M, S, K, r_range, vr, n, seed, device="cuda", gain="literal", chunk=16):
    """Like ``device_pool``, but every instance draws its own correlation
    coefficient r ~ U[r_range] (the serving workload's per-request r), so the
    AR(1) factor differs per instance. Drawn in chunks of ``chunk`` instances
    to bound the temporary memory. Returns (complex64 [n, K, M], r per instance)."""
    import torch
    if M % S:
        raise ValueError("M must be a multiple of S")
    Ms = M // S
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    lo_r, hi_r = float(r_range[0]), float(r_range[1])
    rs = torch.rand((n,), generator=g, device=device, dtype=torch.float64) * (hi_r - lo_r) + lo_r
    out = torch.empty((n, K, M), dtype=torch.complex64, device=device)
    i = torch.arange(Ms, device=device)
    expo = (i[:, None] - i[None, :]).to(torch.float64)
    lo, hi = int(vr[0]), min(int(vr[1]), S)
    lo = max(1, min(lo, hi))
    sub = torch.arange(S, device=device)
    for c0 in range(0, n, chunk):
        m = min(chunk, n - c0)
        r = rs[c0:c0 + m]
        # lower-triangular AR(1) factors, one per instance: L[i, j] = r^(i-j) (i >= j),
        # columns after the first scaled by sqrt(1 - r^2)
        L = torch.where(expo[None] >= 0, r[:, None, None] ** expo.clamp(min=0)[None], torch.zeros((), device=device,
                                                                                           dtype=torch.float64))
        L[:, :, 1:] *= torch.sqrt(1.0 - r * r)[:, None, None]
        d = torch.rand((m, K), generator=g, device=device, dtype=torch.float64) * 90.0 + 10.0
        vr_len = torch.randint(lo, hi + 1, (m, K), generator=g, device=device)
        start = (torch.rand((m, K), generator=g, device=device, dtype=torch.float64)
                 * (S - vr_len + 1).to(torch.float64)).floor().to(torch.int64)
        mask = (sub[None, None, :] >= start[..., None]) & (sub[None, None, :] < (start + vr_len)[..., None])
        re = torch.randn((m, K * S, Ms), generator=g, device=device, dtype=torch.float64)
        im = torch.randn((m, K * S, Ms), generator=g, device=device, dtype=torch.float64)
        Lt = L.transpose(1, 2).contiguous()
        y = torch.complex(torch.bmm(re, Lt), torch.bmm(im, Lt)).reshape(m, K, S, Ms) / (2.0 ** 0.5)
        y = y * mask[..., None]
        beta = d ** -3.7 if gain == "literal" else (d / 10.0) ** -3.7
        out[c0:c0 + m] = (beta.sqrt()[..., None, None] * y).reshape(m, K, M).to(torch.complex64)
        del L, Lt, re, im, y
    return out, rs

