"""Benchmark of the batched Jac-PCG RZF precoder on one MI355X.

    python bench.py [--gpus 1] [--steps 100] [--warmup 10] [--snr-db 10] [--gain literal]

One step = the whole path (regularised Gram -> persistent Jacobi-PCG with
B = I_K -> power-normalised precoder) over one batch of 1024 subcarrier
instances of M = 1024 antennas (8 subarrays of 128) and K = 64 users, 8 fixed
PCG iterations, synthetic seeded channels already resident in HBM.

Prints ONE JSON line: precoders/s of the batched path, the plain
one-instance-at-a-time path on the same GPU, p50/p99 batch latency, the error
against the FP64 direct precoder, the roofline of the dominant kernel (timed
with HIP events on its launch stream) and the CPU oracle's throughput.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3     # MI355X dense FP32 matrix peak
PEAK_HBM_GBS = 8000.0             # MI355X HBM3E peak


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--snr-db", type=float, default=10.0)
    ap.add_argument("--gain", default="literal", choices=["literal", "normalised"])
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--gram", default="bf16x6", choices=["fp32", "bf16x3", "bf16x6"],
                    help="Gram precision (bf16x6: exact 3-part split, six products, FP32 accumulation)")
    ap.add_argument("--epilogue", default="split", choices=["split", "fp32"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="measured seconds of the Poisson serving stream (0: skip)")
    ap.add_argument("--no-rows", action="store_true", help="skip the adjacent rows (transmit, block, SINR)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch choices (no autotuning)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of launch choices: shapes found there are not tuned again, new ones are "
                         "added (counter passes reuse the choices of an unprofiled run: the profiler's "
                         "serialised dispatches would skew the tuner's timings)")
    ap.add_argument("--rows-only", default=None, choices=["precision", "stress"],
                    help="only run one workload's rows (for per-workload profiles) and print them as JSON")
    ap.add_argument("--calibrate-peaks", action="store_true",
                    help="only measure the matrix-core peaks (FP32, BF16, FP64, int8) with register-only loops")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for the HBM traffic counters)")
    return ap.parse_args()


PEAK_BF16_MFMA_TFLOPS = 2500.0    # MI355X dense BF16 matrix peak
TUNE_CACHE = None                 # --tune-cache
SETTLE_STEPS = 100                # untimed steps before the timed ones, at least (warmup included)


def session(bd, **kw):
    return bd.Session(0, tune_cache_path=TUNE_CACHE, **kw)


def autotune(sess, batch, M, K, prec, flags, stream):
    """The session's autotuner for one shape, unless the tune cache already
    holds that shape's choices."""
    if TUNE_CACHE and sess.tune_get("gram_waves", M, K, prec):
        return
    sess.autotune(batch, M, K, prec, flags, stream=stream)


def algorithmic(M, K, n, T, batch, gram, epilogue, T_exec=None):
    """Per launch: algorithmic flops and HBM bytes of each kernel, and the work
    its instructions actually execute on the matrix cores.

    T is the mean number of solver iterations per column (useful work);
    T_exec (default T) the mean over 32-column blocks of the block's largest
    count, which is what the solver executes. Split-BF16 kernels execute
    `products` bf16 MFMA products per FP32 product (3 for hi+lo, 6 for the
    exact three-part split)."""
    T_exec = T if T_exec is None else T_exec
    kp = -(-K // 32) * 32
    gram_products = {"fp32": 1, "bf16x3": 3, "bf16x6": 6}[gram]
    ep_products = 6 if epilogue == "split" else 1
    return {
        "gram": dict(flops=batch * 4.0 * M * K * (K + 1), bytes=batch * (8.0 * M * K + 8.0 * K * K),
                     exec_flops=batch * 8.0 * M * kp * (kp + 32) / 2 * gram_products,
                     dtype="fp32" if gram == "fp32" else "bf16"),
        "solve": dict(flops=batch * T * 8.0 * K * K * n, bytes=batch * (8.0 * K * K + 8.0 * K * n),
                      exec_flops=batch * (T_exec + 1) * 8.0 * kp * kp * n, dtype="fp32"),
        "epilogue": dict(flops=batch * 8.0 * M * K * n, bytes=batch * (8.0 * M * K + 8.0 * K * n + 8.0 * M * n),
                         exec_flops=batch * 8.0 * M * kp * n * ep_products,
                         dtype="fp32" if epilogue == "fp32" else "bf16"),
    }


def binding_roof(k):
    """The roof that bounds a kernel: HBM time of its algorithmic bytes or the
    matrix-core time of the work it executes, whichever is longer."""
    peak = PEAK_FP32_MFMA_TFLOPS if k["dtype"] == "fp32" else PEAK_BF16_MFMA_TFLOPS
    t_hbm = k["bytes"] / (PEAK_HBM_GBS * 1e9)
    t_mma = k["exec_flops"] / (peak * 1e12)
    return ("hbm", t_hbm) if t_hbm >= t_mma else ("mfma", t_mma)


def traffic_for(kernel_phase):
    """Measured HBM bytes per launch from committed rocprofv3 counter runs,
    valid only while the kernel sources are unchanged."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_batched_M1024_K64_T8_split.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = rec.get("sources", {})
    for f, digest in src.items():
        p = os.path.join(ROOT, f)
        if not os.path.exists(p) or hashlib.sha256(open(p, "rb").read()).hexdigest() != digest:
            return None
    v = rec.get("per_launch_bytes", {}).get(kernel_phase)
    return float(v) if v is not None else None


def stream_ceiling(torch, nbytes, reps=20):
    """What plain device streaming reaches on this GPU for the bytes of one
    batch of H: a copy (torch's copy kernel, read + write of nbytes each), in
    GB/s of bytes moved."""
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    out = {}
    for name, fn, moved in (("copy_GBs", lambda: y.copy_(x), 2 * nbytes),):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(moved / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9, 1)
    del x, y
    return out


def cpu_baseline(H_host, xi, T, W_gpu, budget_s):
    """The oracle (plain complex128 CPU implementation) on a bounded sample of
    the same workload, plus the error of the GPU precoders of that sample
    against the FP64 direct inverse and against the oracle at the same T."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    n_done, t0 = 0, time.perf_counter()
    errs_T, errs_64 = [], []
    while n_done < H_host.shape[0] and (time.perf_counter() - t0) < budget_s:
        Hb = H_host[n_done].T.astype(np.complex128)
        ref = oracle.rzf(Hb, xi, tol=0.0, max_iter=T)
        n_done += 1
        Wg = W_gpu[n_done - 1].T
        errs_T.append(np.linalg.norm(Wg - ref["W"]) / np.linalg.norm(ref["W"]))
    elapsed = time.perf_counter() - t0
    for b in range(min(8, n_done)):
        _, Wstar, _ = oracle.direct_rzf(H_host[b].T.astype(np.complex128), xi)
        errs_64.append(np.linalg.norm(W_gpu[b].T - Wstar) / np.linalg.norm(Wstar))
    return dict(value=n_done / elapsed, unit="precoders/s", cores=int(threads), kind="oracle",
                host_cpu_count=os.cpu_count(), host_cpu_model=cpu_model(),
                sample=f"first {n_done} of the batch's instances through oracle.rzf (complex128 Gram, "
                       f"Jacobi-PCG T={T}, precoder), {elapsed:.1f} s"), \
        float(np.max(errs_T)), float(np.max(errs_64)) if errs_64 else None


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_other_workloads():
    """The oracle on small subsets of the precision (4 instances) and stress (2
    instances) workloads, as precoders/s, with the solve settings of those
    workloads (tolerance 1e-6)."""
    import oracle
    from channelgen import channel_batch, workload
    out = {}
    for name, n in (("precision", 4), ("stress", 2)):
        w = workload(name)
        H = channel_batch(w, n=n)
        xi = w.xi_values()[0]
        t0 = time.perf_counter()
        for b in range(n):
            oracle.rzf(H[b].T.astype(np.complex128), xi, tol=1e-6, max_iter=w.max_iter)
        out[name] = {"precoders_per_s": round(n / (time.perf_counter() - t0), 3),
                     "sample": f"{n} instances of M={w.M}, K={w.K}, tol 1e-6"}
    return out


def cpu_best(H_host, xi, n=64):
    """A vectorised direct CPU path (batched Gram, LAPACK LU solve, power
    normalisation) on n instances, in complex64 and complex128, with all BLAS
    threads and with one: a CPU throughput figure beside the oracle's."""
    from threadpoolctl import threadpool_info, threadpool_limits
    out = {}
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    for dt, prefix in ((np.complex64, ""), (np.complex128, "c128_")):
        Hm = np.ascontiguousarray(np.transpose(H_host[:n], (0, 2, 1))).astype(dt)            # [n, M, K]
        K = Hm.shape[2]

        def run():
            A = np.matmul(np.conj(np.transpose(Hm, (0, 2, 1))), Hm) + xi * np.eye(K, dtype=dt)
            X = np.linalg.solve(A, np.broadcast_to(np.eye(K, dtype=dt), A.shape))
            F = np.matmul(Hm, X)
            return F / np.sqrt(np.sum(np.abs(F) ** 2, axis=(1, 2)))[:, None, None]

        for label, lim in (("all_cores", None), ("one_core", 1)):
            with threadpool_limits(limits=lim):
                run()
                reps, t0 = 0, time.perf_counter()
                while reps < 3 or time.perf_counter() - t0 < 2.0:
                    run()
                    reps += 1
                out[prefix + label] = round(n * reps / (time.perf_counter() - t0), 1)
    out.update(unit="precoders/s", threads=int(threads),
               kind="numpy direct (batched LU solve): complex64, and complex128 under c128_",
               sample=f"{n} instances")
    return out


def progress(msg):
    """One progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def sample_errors(samples, rows):
    """CPU leg: the accuracy checks of the GPU results kept in `samples`
    (relative Frobenius error against the oracle's FP64 direct precoder, or
    against the oracle's Jacobi-PCG at the same iteration count), the maximum
    per (row, field) written into `rows`."""
    import oracle
    worst = {}
    for smp in samples:
        Hb = np.asarray(smp["H"]).T.astype(np.complex128)
        direct = oracle.direct_rzf(Hb, smp["xi"]) if any(k != "W_oracle_T" for _, k, _ in smp["checks"]) else None
        for field, kind, val in smp["checks"]:
            if kind == "W_fp64":
                e = _rel(val, direct[1])
            elif kind == "X_fp64":
                e = _rel(val, direct[0])
            else:
                e = _rel(val, oracle.rzf(Hb, smp["xi"], tol=0.0, max_iter=smp["T"])["W"])
            key = (smp["path"], field)
            worst[key] = max(worst.get(key, 0.0), e)
    for (path, field), e in worst.items():
        d = rows
        for p in path:
            d = d[p]
        d[field] = e


def headline_variants(bd, torch, sess, H, H_host, stream, samples, reps=20):
    """The headline shape at every SNR of the workload (0, 10, 20 dB; xi =
    K/SNR), for literal and gain-normalised channels: time per batch at T = 8
    and at relative residual 1e-5, and the iterations run. Two instances of
    each are kept in `samples` for the CPU leg's accuracy checks (against the
    FP64 direct precoder, and against the oracle at T = 8)."""
    from channelgen import channel_batch, workload
    batch, K, M = H.shape
    out = {}
    for gain in ("literal", "normalised"):
        if gain == "literal":
            Hd, Hh = H, H_host
        else:
            Hh = channel_batch(workload("batched", gain="normalised"))
            Hd = torch.from_numpy(Hh).to("cuda")
        W = torch.empty_like(Hd)
        for snr in (0.0, 10.0, 20.0):
            xi = K / 10 ** (snr / 10.0)
            rec = {"xi": xi}
            for mode, kw in (("T8", dict(tol=0.0, max_iter=8)), ("tol_1e-5", dict(tol=1e-5, max_iter=64))):
                run = lambda: bd.rzf_precoder(sess, Hd, xi, precision=bd.GRAM_BF16X6, W=W, stream=stream, **kw)
                run()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    run()
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3 / reps
                _, st, _ = bd.rzf_precoder(sess, Hd, xi, precision=bd.GRAM_BF16X6, W=W, stats=True, stream=stream,
                                           **kw)
                torch.cuda.synchronize()
                rec[mode] = {"ms": round(ms, 4), "precoders_per_s": round(batch / (ms / 1e3), 1),
                             "max_iters": st["max_iters"]}
                for b in (0, batch - 1):
                    checks = [("sampled_err_vs_fp64", "W_fp64", W[b].cpu().numpy().T)]
                    if mode == "T8":
                        checks.append(("sampled_err_vs_oracle_same_T", "W_oracle_T", checks[0][2]))
                    samples.append(dict(path=("headline_variants", f"{gain}_{snr:g}dB", mode), H=Hh[b], xi=xi,
                                        T=8, checks=checks))
            out[f"{gain}_{snr:g}dB"] = rec
        del W
    return out


def single_call_latency(bd, torch, sess, reps=200):
    """One instance of M=256, K=16 (4 subarrays of 64, 10 dB), Jacobi-PCG to
    relative residual 1e-6 or 16 iterations: per-call latency of rzf_precoder
    (graph replayed), p50 / p99 over reps, host-synchronised per call."""
    from channelgen import channel_batch, workload
    w = workload("single")
    Hd = torch.from_numpy(channel_batch(w)).to("cuda")
    xi = w.xi_values()[0]
    W = torch.empty_like(Hd)
    run = lambda: bd.rzf_precoder(sess, Hd, xi, tol=w.tol, max_iter=w.max_iter, precision=bd.GRAM_FP32, W=W)
    for _ in range(5):
        run()
    torch.cuda.synchronize()
    lat = []
    for _ in range(reps):
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    lat = np.array(lat)
    return {"p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
            "config": f"1 x (M={w.M}, K={w.K}), 10 dB, tol {w.tol:g} or {w.max_iter} iterations, FP32 Gram"}


def two_sessions(bd, torch, H, xi, T, prec, flags, steps=120):
    """The headline batch with two sessions on two streams of default priority,
    calls alternating between them with no join in between: consecutive
    batches overlap (one batch's solve beside the other's Gram or epilogue).
    Same arguments as the headline; each session replays its own graph."""
    sessions = [session(bd) for _ in range(2)]
    streams = [torch.cuda.Stream() for _ in range(2)]
    Hs = [H, H.clone(), H.clone(), H.clone()]
    Ws = [torch.empty_like(H) for _ in range(2)]
    M, K = H.shape[2], H.shape[1]
    for s in sessions:
        autotune(s, H.shape[0], M, K, prec, flags, torch.cuda.current_stream())
    torch.cuda.synchronize()

    def step(i):
        j = i % 2
        bd.rzf_precoder(sessions[j], Hs[2 * ((i // 2) % 2) + j], xi, power=1.0, tol=0.0, max_iter=T, precision=prec,
                        flags=flags, W=Ws[j], stream=streams[j])

    for i in range(8):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for s in sessions:
        s.close()
    del Hs, Ws
    torch.cuda.empty_cache()
    batch = H.shape[0]
    return {"ms_per_batch": round(dt * 1e3 / steps, 4), "precoders_per_s": round(steps * batch / dt, 1),
            "config": "headline batches alternating between two sessions on two streams, no join between calls"}


def next_rows(bd, torch, sess, H, xi, stream, samples, reps=20):
    """Throughput of the adjacent rows on the headline channels: per-symbol
    transmission (one symbol vector per instance), the subarray-block
    precoder, the SINR / sum-rate evaluator, and Jacobi-PCG vs plain CG
    iteration counts."""
    batch, K, M = H.shape
    out = {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    g = torch.Generator(device="cuda").manual_seed(1)
    S = (torch.randint(0, 2, (batch, 1, K), generator=g, device="cuda") * 2 - 1).to(torch.complex64)
    x = torch.empty((batch, 1, M), dtype=torch.complex64, device="cuda")
    ms = timed(lambda: bd.rzf_transmit(sess, H, S, xi, max_iter=8, precision=bd.GRAM_BF16X6, x=x, stream=stream))
    # HBM: the Gram and the epilogue each read H; x is M x 1 per instance
    out["transmit_nsym1"] = {"ms": round(ms, 4), "symbol_vectors_per_s": round(batch / (ms / 1e3), 1),
                             "hbm_GBs": round(batch * (16.0 * M * K + 8.0 * M) / (ms / 1e3) / 1e9, 1),
                             "config": f"{batch} x (M={M}, K={K}), one QPSK vector each, T=8, split-BF16 Gram"}
    M1, Mc, M2, K1 = 3 * M // 8, M // 4, 3 * M // 8, K // 2
    G = torch.empty_like(H)
    ms = timed(lambda: bd.rzf_block_precoder(sess, H, xi, M1, Mc, M2, K1, K - K1, max_iter=8,
                                             precision=bd.GRAM_BF16X6, G=G, stream=stream))
    out["block_precoder"] = {"ms": round(ms, 4), "precoders_per_s": round(batch / (ms / 1e3), 1),
                             "config": f"{batch} x (M1={M1}, Mc={Mc}, M2={M2}, K1={K1}, K2={K - K1}), T=8"}
    W = bd.rzf_precoder(sess, H, xi, max_iter=8, stream=stream)
    sinr = torch.empty((batch, K), dtype=torch.float32, device="cuda")
    se = torch.empty((batch,), dtype=torch.float32, device="cuda")
    ms = timed(lambda: bd.rzf_sinr(sess, H, W, 0.1, sinr=sinr, se=se, stream=stream))
    t_hbm = batch * 16.0 * M * K / (PEAK_HBM_GBS * 1e9)
    t_mma = batch * 8.0 * M * K * (-(-K // 32) * 32) / (PEAK_FP32_MFMA_TFLOPS * 1e12)
    out["sinr"] = {"ms": round(ms, 4), "instances_per_s": round(batch / (ms / 1e3), 1),
                   "bound": "hbm" if t_hbm >= t_mma else "mfma",
                   "frac_of_roof": round(max(t_hbm, t_mma) / (ms / 1e3), 4)}
    # Jacobi-PCG vs plain CG on the gain-normalised channels at 20 dB, where
    # the users' gains (the diagonal of A) spread and the systems are not ~xi I
    from channelgen import channel_batch, workload
    n = 64
    Hn = torch.from_numpy(channel_batch(workload("batched", gain="normalised"), n=n)).to("cuda")
    A = bd.jacpcg_gram(sess, Hn, K / 100.0)
    counts = {}
    for name, fl in (("jacobi", bd.PRECOND_JACOBI), ("cg", bd.PRECOND_NONE)):
        it = torch.zeros((n, 1), dtype=torch.int32, device="cuda")
        bd.jacpcg_solve(sess, A, S[:n].contiguous(), tol=1e-6, max_iter=512, flags=fl, iters=it, stream=stream)
        torch.cuda.synchronize()
        c = it.cpu().numpy()[:, 0]
        counts[name] = {"mean": round(float(c.mean()), 2), "max": int(c.max())}
    out["iterations_to_1e-6"] = dict(counts, instances=n, rhs="one QPSK vector",
                                     channels="batched workload, gain-normalised, 20 dB (xi = K/100)")
    return out


def _timed_ms(torch, stream, fn, reps):
    """Mean milliseconds of fn over reps back-to-back calls (HIP events on the
    launch stream), after one untimed call."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _phases_us(sess, fn, reps):
    """Per-kernel microseconds per call from a separate pass with per-kernel
    HIP events (eager launches)."""
    sess.phase_times(reset=True)
    sess.set_profiling(True)
    for _ in range(reps):
        fn()
    sess.set_profiling(False)
    ph = sess.phase_times(reset=True)
    return {k: round(v[0] / reps * 1e3, 1) for k, v in ph.items() if v[1]}


def _column_iters(bd, torch, sess, H, xi, tol, max_iter, precision, stream):
    """Per-column PCG iteration counts of the first solve (mean, max)."""
    A = bd.jacpcg_gram(sess, H, xi, precision=precision, stream=stream)
    batch, K = A.shape[0], A.shape[1]
    its = torch.zeros((batch, K), dtype=torch.int32, device="cuda")
    bd.jacpcg_solve(sess, A, None, tol=tol, max_iter=max_iter, iters=its, stream=stream)
    torch.cuda.synchronize()
    c = its.cpu().numpy()
    del A
    return {"mean": round(float(c.mean()), 2), "max": int(c.max())}


REFINE_TOL = 1e-10


def precision_rows(bd, torch, sess, stream, keep, reps=5):
    """Precision workload: 256 x (M=4096 in 16 subarrays of 256, K=128), r=0.7,
    regions of 6-12 subarrays, 10 dB (xi = 12.8), FP32 Jacobi-PCG to relative
    residual 1e-6 (at most 64 iterations) and FP64-residual refinement to
    1e-10 per column. One row per Gram precision of the FP32 solves: two-part
    split BF16 (hi+lo, the workload as stated), FP32, the three-part split, and
    the FP64 Gram rounded to FP32. Timed on the default path (graph replay);
    per-kernel times from a separate profiled pass. X of every instance comes
    back for the CPU leg's check against the FP64 direct inverse, before and
    after refinement."""
    from channelgen import device_pool, workload
    wp = workload("precision")
    xi = wp.xi_values()[0]
    Hp = device_pool(wp.M, wp.S, wp.K, wp.r, wp.vr, wp.batch, 7)
    Wp = torch.empty_like(Hp)
    X64 = torch.empty((wp.batch, wp.K, wp.K), dtype=torch.complex128, device="cuda")
    X32 = torch.empty((wp.batch, wp.K, wp.K), dtype=torch.complex64, device="cuda")
    out = {"config": f"{wp.batch} x (M={wp.M} = {wp.S} x {wp.M // wp.S}, K={wp.K}), r={wp.r}, regions of "
                     f"{wp.vr[0]}-{wp.vr[1]}, xi={xi:g}, FP32 PCG to 1e-6 (<= 64 iterations), FP64 refinement "
                     f"to {REFINE_TOL:g} per column", "before_refinement": {}}
    kept = {"H": Hp.cpu().numpy(), "xi": xi, "X64": {}, "X32": {}}
    for gp in (bd.GRAM_BF16X3, bd.GRAM_FP32, bd.GRAM_BF16X6):  # the session's launch choices for this shape
        autotune(sess, wp.batch, wp.M, wp.K, gp, 0, stream)
    for name, gp in (("bf16x3_gram", bd.GRAM_BF16X3), ("fp32_gram", bd.GRAM_FP32)):
        bd.rzf_precoder(sess, Hp, xi, tol=1e-6, max_iter=64, precision=gp, W=Wp, X_out=X32, stream=stream)
        torch.cuda.synchronize()
        kept["X32"][name] = X32.cpu().numpy()
        out["before_refinement"][name] = {"pcg_iters": _column_iters(bd, torch, sess, Hp, xi, 1e-6, 64, gp, stream)}
    for name, gp in (("bf16x3", bd.GRAM_BF16X3), ("fp32", bd.GRAM_FP32), ("bf16x6", bd.GRAM_BF16X6),
                     ("fp64_rounded", bd.GRAM_FP64_ROUNDED)):
        prec = gp | bd.REFINE_FP64
        run = lambda: bd.rzf_precoder(sess, Hp, xi, tol=1e-6, max_iter=64, precision=prec,
                                      refine_tol=REFINE_TOL, W=Wp, X64_out=X64, stream=stream)
        ms = _timed_ms(torch, stream, run, reps)
        _, st, rc = bd.rzf_precoder(sess, Hp, xi, tol=1e-6, max_iter=64, precision=prec, refine_tol=REFINE_TOL,
                                    W=Wp, X64_out=X64, stats=True, stream=stream)
        kept["X64"][name] = X64.cpu().numpy()
        out[name] = {"ms": round(ms, 3), "precoders_per_s": round(wp.batch / (ms / 1e3), 1), "status": rc,
                     "max_pcg_iters": st["max_iters"], "refine_steps": st["refine_steps"],
                     "max_refine_residual": st["max_refine_residual"],
                     "phases_us": _phases_us(sess, run, 3)}
    keep["precision"] = kept
    del Hp, Wp, X64, X32
    return out


def stress_rows(bd, torch, sess, stream, keep, reps=3):
    """Stress workload: 64 x (M=8192 in 32 subarrays of 256, K=256), r=0.95,
    regions of 1-3 subarrays, near-ZF xi = 1e-3, users in region order.
    Complex64 Jacobi-PCG to relative residual 1e-6 (at most 4K = 1024
    iterations) on the FP64 Gram that the refinement forms anyway, rounded
    once to FP32, then FP64-residual refinement to 1e-10 per column; dense
    path and visibility-region sparse path, literal and gain-normalised
    channels (the normalised gain is the literal one times 10^3.7 for every
    user). The same with a separate FP32 Gram for the solves under
    *_fp32_gram. Per-column iteration counts of the first solve (FP32 Gram);
    two instances per row come back for the CPU leg's check against the FP64
    direct inverse."""
    from channelgen import sorted_channel_batch, workload
    ws = workload("stress")
    Hs_np, spans_np = sorted_channel_batch(ws)
    spans = torch.from_numpy(spans_np).to("cuda")
    out = {"config": f"{ws.batch} x (M={ws.M} = {ws.S} x {ws.M // ws.S}, K={ws.K}), r={ws.r}, regions of "
                     f"{ws.vr[0]}-{ws.vr[1]}, xi={ws.xi:g}, users in region order, PCG to 1e-6 (<= 1024 "
                     f"iterations) on the FP64 Gram rounded to FP32 (a separate FP32 Gram under *_fp32_gram), "
                     f"FP64 refinement to {REFINE_TOL:g} per column"}
    picks = (0, ws.batch - 1)
    prec = bd.GRAM_FP64_ROUNDED | bd.REFINE_FP64
    autotune(sess, ws.batch, ws.M, ws.K, bd.GRAM_FP32, 0, stream)
    for gain in ("literal", "normalised"):
        H = torch.from_numpy(Hs_np).to("cuda")
        if gain == "normalised":
            H = (H.to(torch.complex128) * 10.0 ** 1.85).to(torch.complex64)
        W = torch.empty_like(H)
        X64 = torch.empty((ws.batch, ws.K, ws.K), dtype=torch.complex128, device="cuda")
        rec = {"pcg_iters": _column_iters(bd, torch, sess, H, ws.xi, 1e-6, 1024, bd.GRAM_FP32, stream)}
        for path in ("dense", "vr"):
            if path == "dense":
                run = lambda: bd.rzf_precoder(sess, H, ws.xi, tol=1e-6, max_iter=1024, precision=prec,
                                              refine_tol=REFINE_TOL, W=W, X64_out=X64, stream=stream)
            else:
                run = lambda: bd.rzf_precoder_vr(sess, H, ws.xi, user_span=spans, tol=1e-6, max_iter=1024,
                                                 precision=prec, refine_tol=REFINE_TOL, W=W, stream=stream)
            ms = _timed_ms(torch, stream, run, reps)
            if path == "dense":
                _, st, rc = bd.rzf_precoder(sess, H, ws.xi, tol=1e-6, max_iter=1024, precision=prec,
                                            refine_tol=REFINE_TOL, W=W, X64_out=X64, stats=True, stream=stream)
                keep.setdefault("stress", []).append(dict(H={b: H[b].cpu().numpy() for b in picks}, xi=ws.xi,
                                                          X64={b: X64[b].cpu().numpy() for b in picks},
                                                          row=(gain, path)))
            else:
                _, st, rc = bd.rzf_precoder_vr(sess, H, ws.xi, user_span=spans, tol=1e-6, max_iter=1024,
                                               precision=prec, refine_tol=REFINE_TOL, W=W, stats=True,
                                               stream=stream)
            rec[path] = {"ms": round(ms, 3), "precoders_per_s": round(ws.batch / (ms / 1e3), 1), "status": rc,
                         "max_pcg_iters": st["max_iters"], "refine_steps": st["refine_steps"],
                         "max_refine_residual": st["max_refine_residual"],
                         "phases_us": _phases_us(sess, run, 2)}
        # The same with a separate FP32 Gram for the solves.
        p32 = bd.GRAM_FP32 | bd.REFINE_FP64
        for path in ("dense", "vr"):
            if path == "dense":
                run = lambda: bd.rzf_precoder(sess, H, ws.xi, tol=1e-6, max_iter=1024, precision=p32,
                                              refine_tol=REFINE_TOL, W=W, stream=stream)
                _, st, rc = bd.rzf_precoder(sess, H, ws.xi, tol=1e-6, max_iter=1024, precision=p32,
                                            refine_tol=REFINE_TOL, W=W, stats=True, stream=stream)
            else:
                run = lambda: bd.rzf_precoder_vr(sess, H, ws.xi, user_span=spans, tol=1e-6, max_iter=1024,
                                                 precision=p32, refine_tol=REFINE_TOL, W=W, stream=stream)
                _, st, rc = bd.rzf_precoder_vr(sess, H, ws.xi, user_span=spans, tol=1e-6, max_iter=1024,
                                               precision=p32, refine_tol=REFINE_TOL, W=W, stats=True,
                                               stream=stream)
            ms = _timed_ms(torch, stream, run, reps)
            rec[path + "_fp32_gram"] = {"ms": round(ms, 3), "status": rc, "max_pcg_iters": st["max_iters"],
                                        "refine_steps": st["refine_steps"],
                                        "max_refine_residual": st["max_refine_residual"]}
        rec["vr_speedup"] = round(rec["dense"]["ms"] / rec["vr"]["ms"], 2)
        out[gain] = rec
        del H, W, X64
    return out


def refined_cpu_checks(keep, rows):
    """CPU leg of the refined rows: relative Frobenius error of X against the
    oracle's FP64 direct inverse, for every instance of the precision workload
    (before and after refinement) and for the sampled stress instances."""
    import oracle
    if "precision" in keep and "precision" in rows:
        kp = keep["precision"]
        errs = {name: [] for name in list(kp["X64"]) + list(kp["X32"])}
        for b in range(kp["H"].shape[0]):
            Xs, _, _ = oracle.direct_rzf(kp["H"][b].T.astype(np.complex128), kp["xi"])
            for name, X in kp["X64"].items():
                errs[name].append(_rel(X[b].T, Xs))
            for name, X in kp["X32"].items():
                errs[name].append(_rel(X[b].T.astype(np.complex128), Xs))
        for name, e in errs.items():
            row = rows["precision"]["before_refinement"][name] if name in kp["X32"] else rows["precision"][name]
            row["err_X_vs_fp64"] = {"max": float(np.max(e)), "median": float(np.median(e)), "instances": len(e)}
    for rec in keep.get("stress", []):
        gain, path = rec["row"]
        worst = 0.0
        for b, Hb in rec["H"].items():
            Xs, _, _ = oracle.direct_rzf(Hb.T.astype(np.complex128), rec["xi"])
            worst = max(worst, _rel(rec["X64"][b].T, Xs))
        rows["stress"][gain][path]["sampled_err_X64_vs_fp64"] = worst



def calibrate_copy():
    """One plain device-to-device copy of 1 GiB, three times: the counter
    reference for FETCH_SIZE / WRITE_SIZE."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": src.numel() * 4}), flush=True)
    return 0


def main():
    a = parse()
    if a.calibrate_copy:
        return calibrate_copy()
    if a.calibrate_peaks:
        import torch
        from paper_2305_13925_amd import binding as bd
        with bd.Session(0) as s:
            print(json.dumps({"mfma_peaks": bd.mfma_peaks(s, torch.cuda.current_stream()),
                              "unit": "TFLOP/s (int8: TOP/s)"}), flush=True)
        return 0
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}): instances are independent and a "
              "multi-GPU run would shard them without communication.", file=sys.stderr)
        return 2
    import torch
    from channelgen import workload, channel_batch
    from paper_2305_13925_amd import binding as bd

    global TUNE_CACHE
    TUNE_CACHE = a.tune_cache
    if a.rows_only:
        sess = session(bd)
        stream = torch.cuda.current_stream()
        keep = {}
        fn = precision_rows if a.rows_only == "precision" else stress_rows
        rows = {a.rows_only: fn(bd, torch, sess, stream, keep)}
        if not a.no_cpu:
            refined_cpu_checks(keep, rows)
        print(json.dumps(rows), flush=True)
        sess.close()
        return 0

    w = workload("batched", gain=a.gain)
    M, K, T, batch = w.M, w.K, w.max_iter, w.batch
    xi = (K / 10 ** (a.snr_db / 10.0))
    H_host = channel_batch(w)
    H = torch.from_numpy(H_host).to("cuda")
    # Timed steps alternate two copies of the channel batch at different
    # addresses, so no step starts on channels the previous step left in the
    # 256 MB Infinity Cache (a new channel per step, as in a real stream).
    Hs = (H, H.clone())
    W = torch.empty_like(H)
    sess = session(bd)
    stream = torch.cuda.current_stream()

    prec = {"fp32": bd.GRAM_FP32, "bf16x3": bd.GRAM_BF16X3, "bf16x6": bd.GRAM_BF16X6}[a.gram]
    flags = 0 if a.epilogue == "split" else bd.EPILOGUE_FP32

    def step(i=0):
        bd.rzf_precoder(sess, Hs[i % 2], xi, power=1.0, tol=0.0, max_iter=T, precision=prec, flags=flags, W=W,
                        stream=stream)

    # Launch choices for the headline shape from the session's autotuner.
    tuned = None
    if not a.no_tune:
        autotune(sess, H.shape[0], M, K, prec, flags, stream)
        split = 0 if flags & bd.EPILOGUE_FP32 else 3
        tuned = {"gram_waves": sess.tune_get("gram_waves", M, K, prec),
                 "pcg_a_source": sess.tune_get("pcg_a_source", 0, K, 0),
                 "precoder_nj": sess.tune_get("precoder_nj", M, K, split),
                 "precoder_mtiles": sess.tune_get("precoder_mtiles", M, K, split)}
        progress(f"autotuned launch choices: {tuned}")

    # Timed region: the product's default launch path. Repeated calls with the
    # same arguments replay the session's captured HIP graph; profiling is off.
    # The first ~50 ms of steps after the tuner and the first touches of the
    # buffers run 7-8% slower (measured: 1.90 M/s after 5 warmup steps, 2.03-2.06
    # M/s after 100 or more); untimed settle steps bring the warmup to at least
    # SETTLE_STEPS so the timed steps see the steady state a calling loop sees.
    settle = max(0, SETTLE_STEPS - a.warmup)
    for i in range(settle + a.warmup):
        step(i)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(a.steps):
        step(i)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    progress(f"{a.steps} timed steps (graph replay): {wall * 1e3 / a.steps:.4f} ms per step")
    lat = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(a.steps)])
    ms_per_step = wall * 1e3 / a.steps
    value = batch / (wall / a.steps)

    # Per-kernel times: the same steps again, launched kernel by kernel with HIP
    # events around every kernel on its launch stream (the events add a little
    # host time per launch, so this pass is not the headline).
    sess.phase_times(reset=True)
    sess.set_profiling(True)
    torch.cuda.synchronize()
    tg = time.perf_counter()
    for i in range(a.steps):
        step(i)
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - tg) * 1e3 / a.steps
    sess.set_profiling(False)
    phases = sess.phase_times(reset=True)

    # tolerance variant: relative residual 1e-5 per column (at most 64 iterations)
    bd.rzf_precoder(sess, H, xi, tol=1e-5, max_iter=64, precision=prec, flags=flags, W=W, stream=stream)
    torch.cuda.synchronize()
    tt = time.perf_counter()
    nt = max(10, a.steps // 5)
    for _ in range(nt):
        bd.rzf_precoder(sess, H, xi, tol=1e-5, max_iter=64, precision=prec, flags=flags, W=W, stream=stream)
    torch.cuda.synchronize()
    tol_ms = (time.perf_counter() - tt) * 1e3 / nt
    _, tol_stats, _ = bd.rzf_precoder(sess, H, xi, tol=1e-5, max_iter=64, precision=prec, flags=flags, W=W,
                                      stats=True, stream=stream)
    # back to the fixed-T result for the accuracy checks below
    step()
    torch.cuda.synchronize()

    progress("graph replay and tolerance variant done")
    # plain path: one instance at a time, one launch per iteration
    plain_value, same = None, None
    if a.plain_steps > 0:
        W_plain = torch.empty_like(H)
        bd.rzf_precoder_plain(sess, H[:8], xi, tol=0.0, max_iter=T, flags=flags, W=W_plain[:8], stream=stream)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for _ in range(a.plain_steps):
            bd.rzf_precoder_plain(sess, H, xi, tol=0.0, max_iter=T, flags=flags, W=W_plain, stream=stream)
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - tp) * 1e3 / a.plain_steps
        plain_value = batch / (plain_ms / 1e3)
        same = float(torch.linalg.vector_norm(W - W_plain) / torch.linalg.vector_norm(W_plain))

    # Iterations the solver runs on these channels: a column stops before T
    # once its residual is below 2^-40 of its right-hand side (FP32 range
    # guard), and a 32-column block runs until its last column stops.
    A_h = bd.jacpcg_gram(sess, H, xi, precision=prec, stream=stream)
    its = torch.zeros((batch, K), dtype=torch.int32, device="cuda")
    bd.jacpcg_solve(sess, A_h, None, tol=0.0, max_iter=T, iters=its, stream=stream)
    torch.cuda.synchronize()
    itn = its.cpu().numpy()
    nb = -(-K // 32)
    blocks = np.zeros((batch, nb * 32), dtype=itn.dtype)
    blocks[:, :K] = itn
    t_alg, t_exec = float(itn.mean()), float(blocks.reshape(batch, nb, 32).max(axis=2).mean())
    del A_h, its

    # roofline of the dominant kernel (and the binding roof of every kernel)
    alg = algorithmic(M, K, K, t_alg, batch, a.gram, a.epilogue, T_exec=t_exec)
    per_launch = {k: (phases[k][0] / phases[k][1]) if phases[k][1] else 0.0 for k in ("gram", "solve", "epilogue")}
    kernels = {}
    for k in ("gram", "solve", "epilogue"):
        d = per_launch[k] / 1e3
        if d <= 0:
            continue
        bound, t_roof = binding_roof(alg[k])
        kernels[k] = {"us": round(per_launch[k] * 1e3, 2), "bound": bound,
                      "roof_us": round(t_roof * 1e6, 1), "frac_of_roof": round(t_roof / d, 4),
                      "alg_tflops": round(alg[k]["flops"] / d / 1e12, 2),
                      "alg_GBs": round(alg[k]["bytes"] / d / 1e9, 1),
                      "mfma_dtype": alg[k]["dtype"]}
        if k == "solve":
            kernels[k].update(iters_mean=round(t_alg, 3), iters_per_block=round(t_exec, 3))
    dom = max(per_launch, key=per_launch.get)
    dur_s = per_launch[dom] / 1e3
    bound, _ = binding_roof(alg[dom])
    if bound == "hbm":
        achieved, peak, unit = alg[dom]["bytes"] / dur_s / 1e9, PEAK_HBM_GBS, "GB/s"
    else:
        pk = PEAK_FP32_MFMA_TFLOPS if alg[dom]["dtype"] == "fp32" else PEAK_BF16_MFMA_TFLOPS
        achieved, peak, unit = alg[dom]["flops"] / dur_s / 1e12, pk, "TFLOP/s"
    roofline = {"bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": traffic_for(dom), "kernel": dom,
                "avg_launch_us": round(per_launch[dom] * 1e3, 2)}
    # Context for the HBM-bound kernels: plain device streaming of one batch of H
    ceiling = stream_ceiling(torch, batch * M * K * 8)
    roofline["stream_ceiling"] = ceiling
    if "epilogue" in kernels:
        kernels["epilogue"]["frac_of_copy"] = round(kernels["epilogue"]["alg_GBs"] / ceiling["copy_GBs"], 4)

    W_host = W.cpu().numpy()
    rows, samples, keep = None, [], {}
    if not a.no_rows:
        progress("adjacent rows")
        rows = next_rows(bd, torch, sess, H, xi, stream, samples)
        progress("headline variants (SNR, gain)")
        rows["headline_variants"] = headline_variants(bd, torch, sess, H, H_host, stream, samples)
        rows["single_call"] = single_call_latency(bd, torch, sess)
        progress("two sessions on two streams")
        rows["two_sessions"] = two_sessions(bd, torch, H, xi, T, prec, flags)
        progress("precision workload (refined)")
        rows["precision"] = precision_rows(bd, torch, sess, stream, keep)
        progress("stress workload (refined, dense and visibility-region sparse)")
        rows["stress"] = stress_rows(bd, torch, sess, stream, keep)

    # The serving stream runs before the CPU leg: the host's numeric thread pools
    # that the CPU leg leaves behind would compete with the scheduler's threads.
    serving = None
    if a.serve_seconds > 0:
        from paper_2305_13925_amd.serve import run_serving
        serving = {}
        for gain in ("literal", "normalised"):
            progress(f"serving stream ({gain} gain)")
            sv = bd.Session(0, hbm_budget_bytes=64 << 30)
            rec = run_serving(sv, rate_hz=2000.0, warmup_s=1.0, measure_s=a.serve_seconds, seed=0, gain=gain)
            sv.close()
            torch.cuda.empty_cache()
            serving[gain] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in rec.items()}
        serving["config"] = ("Poisson 2000 requests/s, M in {256..4096}, K in {8..256} (K <= M/8), 1-64 "
                             "subcarriers, per-request r ~ U[0.3, 0.9], 4 subarrays with regions of 2-4, 10 dB, "
                             "tol 1e-6 or 16 iterations, FP32 Gram, 64 GB budget")

    # CPU leg: the oracle timed on a bounded sample, a vectorised CPU path, and
    # the accuracy checks of sampled GPU results against the oracle
    cpu, err_T, err_64, best = (None, None, None, None)
    if not a.no_cpu:
        progress("CPU leg: oracle timing, CPU direct path, accuracy checks")
        cpu, err_T, err_64 = cpu_baseline(H_host, xi, T, W_host, a.cpu_seconds)
        cpu["other_workloads"] = oracle_other_workloads()
        best = cpu_best(H_host, xi)
        if rows is not None:
            sample_errors(samples, rows)
            progress("CPU leg: refined results against the FP64 direct inverse")
            refined_cpu_checks(keep, rows)

    out = {
        "metric": "RZF precoders/s (M=1024,K=64) batched vs plain Jac-PCG; p99 latency; err vs FP64",
        "value": round(value, 1),
        "unit": "precoders/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "settle_steps": settle,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"batched: {batch} x (M={M}, K={K}), 8 subarrays of 128, r=0.5, VR 3-6, "
                               f"{a.gain} gain, SNR {a.snr_db:g} dB (xi={xi:g}), B=I_K, T={T} (a column stops "
                               f"earlier once its residual is below 2^-40 of its right-hand side)",
                   "batch": batch, "M": M, "K": K, "iterations": T, "gram": a.gram, "epilogue": a.epilogue},
        "plain_value": round(plain_value, 1) if plain_value else None,
        "speedup_vs_plain": round(value / plain_value, 2) if plain_value else None,
        "plain_vs_batched_rel_diff": same,
        "launch_path": "graph replay (the default for repeated calls), profiling off",
        "tuned_choices": tuned,
        "eager_profiled_ms_per_step": round(eager_ms, 4),
        "eager_profiled_value": round(batch / (eager_ms / 1e3), 1),
        "tol_1e-5": {"ms_per_step": round(tol_ms, 4), "value": round(batch / (tol_ms / 1e3), 1),
                     "max_iters": tol_stats["max_iters"], "max_rel_residual": tol_stats["max_rel_residual"]},
        "p50_ms": round(float(np.percentile(lat, 50)), 4),
        "p99_ms": round(float(np.percentile(lat, 99)), 4),
        "err_vs_fp64": err_64,
        "err_vs_oracle_same_T": err_T,
        "kernels": kernels,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_best": best,
        "serving": serving,
        "rows": rows,
    }
    print(json.dumps(out), flush=True)
    sess.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
