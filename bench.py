"""Benchmark of the CROSS hot path on one MI355X.

Workload (one "step"): forward + inverse NTT of a CKKS-shaped batch,
N = 2^16, L = 24 limbs of 28-bit primes, 8 ciphertexts x 2 polynomials = 384
limb-NTTs each way, through the BAT int8-MFMA path with the library's default
factoring of 2^16 (three factors, 64 x 32 x 32; the 256 x 256 two-factor form
is timed beside it).  Inputs are resident in HBM before timing starts.
Reported beside it: the same step through the plain radix-2 butterfly kernels
(bit-identical results, checked), the roofline of the dominant kernel from
live HIP-event timings, HE-Mult / Rotate / Rescale / HE-Add at N = 2^16,
L = 24, dnum = 3 (HE-Mult also with its NTTs on the butterfly kernels), the
uneven batch, the request loop, and the CPU oracle timed on bounded samples
(before the GPU is touched; its HE-Mult results also check the GPU's batch-8
HE-Mult bit for bit).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import gc
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "N=2^16 NTTs/sec and HE-Mult/s, int8-MFMA vs butterfly, bit-exact"
INT8_PEAK_TOPS = 5000.0      # MI355X dense int8 MFMA, TOP/s
HBM_PEAK_GBS = 8000.0

LOG_N, L, POLYS = 16, 24, 16
PROFILE_EVERY = 4      # one timed step in this many brackets the dominant kernel's launches with HIP events


def gemm_ops_per_launch(log_n, log_r, nlimb_polys, kind):
    # algorithmic int8 ops of one BAT GEMM step: 2 * (4U) * (4U) * V per limb-polynomial
    R, C = 1 << log_r, 1 << (log_n - log_r)
    U, V = (R, C) if kind == "left" else (C, R)
    return 2.0 * (4 * U) * (4 * U) * V * nlimb_polys


def rows_bytes_per_launch(log_n, log_r, log_c1, nlimbs, npolys):
    """Algorithmic HBM bytes of one row-kernel launch, averaged over forward and inverse:
    every residue read and written once, per prime the BAT-expanded C1 x C1 and C2 x C2
    tables (one when C1 = C2) and the C inner twiddle pairs, and on inverse launches (half
    of them) the N inverse step-2 twiddle pairs."""
    n, c = 1 << log_n, 1 << (log_n - log_r)
    c1, c2 = 1 << log_c1, c >> log_c1
    tables = 16 * c1 * c1 if c1 == c2 else 16 * c1 * c1 + 16 * c2 * c2
    return nlimbs * npolys * n * 8 + nlimbs * (tables + 8 * c) + nlimbs * n * 8 // 2


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2501_07047_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel, kernel_hash):
    """HBM bytes per launch from committed rocprofv3 counter runs, if still current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != kernel_hash:
        return None
    return rec.get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def pool_size():
    """Worker processes for the multi-process oracle leg: the CPUs this process may run
    on, at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n, os.cpu_count() or 1))


_POOL_ARGS = None         # inputs handed to forked oracle workers


def _ntt_limb_job(limb):
    import numpy as np
    from oracle.ntt import ntt_ct, intt_gs
    from oracle.primes import psi
    primes, x = _POOL_ARGS
    q = primes[limb]
    p = psi(q, 1 << LOG_N)
    y = ntt_ct(x[:, limb].astype(np.uint64), q, p)
    intt_gs(y, q, p)
    return 2 * x.shape[0]


def _he_mult_job(k):
    from oracle import ckks as CK
    qs, ps, a, b, key = _POOL_ARGS
    return k, CK.he_mult(a[k], b[k], key, qs, ps, 3).astype("uint32")


def cpu_baseline(he_inputs, budget_s=6.0):
    """The oracle on bounded samples of the workloads, on the host cores (run before the
    GPU is touched, so the worker pool is a plain fork):
      * the NTT step: oracle.ntt.ntt_ct / intt_gs, forward + inverse of the 16
        polynomials of one limb per task, single process and over a process pool;
      * HE-Mult at N=2^16, L=24, dnum=3, K=8 (oracle.ckks.he_mult) on ciphertexts of the
        GPU benchmark's own batch-8 input: one in a single process, then every one of
        the eight over the pool (those results are compared with the GPU's later);
      * the N=4096 single-prime case by definition (O(N^2) ntt_def / intt_def, schoolbook
        negacyclic product).
    Returns (baseline dict, {ciphertext: oracle HE-Mult})."""
    global _POOL_ARGS
    import multiprocessing as mp
    import numpy as np
    import synthetic
    from oracle.ntt import ntt_def, intt_def
    from oracle.poly import negacyclic_mul
    from oracle.primes import psi

    primes, x = synthetic.ntt_batch(0, LOG_N, L, POLYS)
    _POOL_ARGS = (primes, x)
    done, t0 = 0, time.perf_counter()
    for limb in range(len(primes)):
        done += _ntt_limb_job(limb)
        if time.perf_counter() - t0 > budget_s:
            break
    dt1 = time.perf_counter() - t0
    single = {"value": round(done / dt1, 2), "unit": "limb-NTT/s", "cores": 1,
              "sample": "%d limb-NTTs (forward+inverse of %d polys for each of %d limbs) in %.1f s"
                        % (done, POLYS, done // (2 * POLYS), dt1)}
    P = pool_size()
    ctx = mp.get_context("fork")
    per_limb = dt1 / max(1, done // (2 * POLYS))
    nlimbs = int(P * max(1, budget_s // max(per_limb, 1e-3)))      # whole rounds of the pool
    with ctx.Pool(P) as pool:
        t0 = time.perf_counter()
        done_p = sum(pool.map(_ntt_limb_job, [i % len(primes) for i in range(nlimbs)], chunksize=1))
        dtp = time.perf_counter() - t0
    # HE-Mult, single process (ciphertext 0), then the whole batch over the pool
    qs, ps, a, b, key = he_inputs
    _POOL_ARGS = he_inputs
    t0 = time.perf_counter()
    _, he0 = _he_mult_job(0)
    dth = time.perf_counter() - t0
    nct = a.shape[0]
    with ctx.Pool(min(P, nct)) as pool:
        t0 = time.perf_counter()
        he_all = dict(pool.map(_he_mult_job, range(nct), chunksize=1))
        dthp = time.perf_counter() - t0
    _POOL_ARGS = None
    # N = 4096, one prime, by definition
    q = synthetic.primes(1)[0]
    _, y = synthetic.ntt_batch(1, 12, 1, 2)
    w = psi(q, 4096)
    c1 = {}
    t0 = time.perf_counter()
    f = ntt_def(y[0, 0], q, w)
    c1["ntt_us"] = round((time.perf_counter() - t0) * 1e6, 1)
    t0 = time.perf_counter()
    intt_def(f, q, w)
    c1["intt_us"] = round((time.perf_counter() - t0) * 1e6, 1)
    t0 = time.perf_counter()
    negacyclic_mul(y[0, 0], y[1, 0], q)
    c1["polymul_schoolbook_us"] = round((time.perf_counter() - t0) * 1e6, 1)
    base = {"value": round(done_p / dtp, 2), "unit": "limb-NTT/s", "cores": P, "kind": "oracle",
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "sample": "%d limb-NTTs (forward+inverse, N=2^16, 16 polys per limb task) over a pool of %d "
                      "processes in %.1f s, oracle.ntt.ntt_ct/intt_gs" % (done_p, P, dtp),
            "single_process": single,
            "he_mult": {"config": "N=2^16, L=24, dnum=3, K=8, oracle.ckks.he_mult",
                        "single_process_per_s": round(1.0 / dth, 4), "single_process_s": round(dth, 2),
                        "pool_per_s": round(nct / dthp, 4), "pool_processes": min(P, nct),
                        "sample": "ciphertext 0, then all %d of the batch-8 input" % nct},
            "config1_n4096": dict(c1, note="O(N^2) definitions, one prime, batch 1")}
    return base, he_all


def he_mult_model(log_n, L_, K, dnum, batch, log_r, log_c1):
    """Algorithmic work of one HE-Mult (tensor + relinearisation) at (N, L, K, dnum), per
    ciphertext pair in a call of `batch` pairs sharing one key:
      int8 ops: every limb-(I)NTT at 32 N (R + C1 + C2) ops (three factors; 32 N (R + C)
      for two), INTT(d2) L + ModUp dnum x (L + K - alpha) NTTs + ModDown 2 x (K INTT + L NTT),
      and the BConv GEMMs 2 (4 l)(4 l') N per conversion (ModUp: alpha -> L + K - alpha per
      digit; ModDown: K -> L, twice);
      HBM bytes: both input ciphertexts read, the output written, the key read once per call."""
    n = 1 << log_n
    alpha = -(-L_ // dnum)
    c = 1 << (log_n - log_r)
    inner = (1 << log_c1) + (c >> log_c1) if log_c1 else c
    per_ntt = 32.0 * n * ((1 << log_r) + inner)
    n_ntt = L_ + dnum * (L_ + K - alpha) + 2 * (K + L_)
    bconv = dnum * 2.0 * (4 * alpha) * (4 * (L_ + K - alpha)) * n + 2 * 2.0 * (4 * K) * (4 * L_) * n
    ct = 2 * L_ * n * 4
    key = dnum * 2 * (L_ + K) * n * 4
    return {"int8_ops": per_ntt * n_ntt + bconv, "limb_ntts": n_ntt, "hbm_bytes": 3 * ct + key / batch}


def he_mult_bench(B, steps, warmup, batch, ops=("he_mult", "rotate", "rescale", "he_add"), engine="mfma"):
    """HE-Mult + relinearisation at N=2^16, L=24, dnum=3, K=8 (and Rotate, Rescale, HE-Add at
    the same shape); `ops` selects which, `engine` the NTT kernels (MFMA or butterfly).
    The HE-Mult output of the last call is returned under "_out" (host array)."""
    import numpy as np
    import torch
    import synthetic
    qs, ps, a, b, key = synthetic.ckks_pair(0, 16, 24, 3, 8, batch)
    da = torch.from_numpy(a.view(np.int32)).cuda()
    db = torch.from_numpy(b.view(np.int32)).cuda()
    dk = torch.from_numpy(key.view(np.int32)).cuda()
    out = torch.empty_like(da)
    out_rs = torch.empty((batch, 2, 23, 1 << 16), dtype=torch.int32, device="cuda")
    res = {}
    B.set_ntt_engine(engine)
    try:
        for name, fn in (("he_mult", lambda: B.he_mult(da, db, dk, out, qs, ps, 3)),
                         ("rotate", lambda: B.rotate(da, 1, dk, out, qs, ps, 3)),
                         ("rescale", lambda: B.rescale(da, out_rs, qs, 1)),
                         ("he_add", lambda: B.he_add(da, db, out, qs))):
            if name not in ops:
                continue
            for _ in range(warmup):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if name == "he_mult":
                res["_out"] = out.cpu().numpy().view(np.uint32).copy()
            # per-kernel breakdown from a second, event-timed pass (kept out of the timing)
            B.profile_report()
            B.profile_enable(True)
            for _ in range(steps):
                fn()
            prof = B.profile_report()
            B.profile_enable(False)
            res[name] = {"per_s": round(batch * steps / dt, 1), "us_per_op": round(dt / steps / batch * 1e6, 1),
                         "batch": batch, "calls_timed": steps,
                         "event_us_per_op_by_kernel": {k: round(v[1] * 1e3 / steps / batch, 1)
                                                       for k, v in prof.items()}}
    finally:
        B.set_ntt_engine("mfma")
    return res


def he_mult_roofline(B, us_per_op, batch):
    """HE-Mult against both peaks: algorithmic int8 ops / time vs the dense int8 MFMA peak
    and algorithmic HBM bytes / time vs the HBM peak; `bound` is the one whose time at
    peak is longer."""
    log_r, log_c1 = B.get_ntt_split(16)
    m = he_mult_model(16, 24, 8, 3, batch, log_r, log_c1)
    t = us_per_op * 1e-6
    t_mfma, t_hbm = m["int8_ops"] / (INT8_PEAK_TOPS * 1e12), m["hbm_bytes"] / (HBM_PEAK_GBS * 1e9)
    tops, gbs = m["int8_ops"] / t / 1e12, m["hbm_bytes"] / t / 1e9
    if t_mfma >= t_hbm:
        r = {"bound": "mfma", "achieved": round(tops, 1), "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
             "frac": round(tops / INT8_PEAK_TOPS, 4)}
    else:
        r = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(gbs / HBM_PEAK_GBS, 4)}
    r.update({"int8_ops_per_op": m["int8_ops"], "limb_ntts_per_op": m["limb_ntts"],
              "hbm_bytes_per_op": m["hbm_bytes"], "int8_tops": round(tops, 1), "hbm_gbs": round(gbs, 1),
              "us_at_int8_peak": round(t_mfma * 1e6, 2), "us_at_hbm_peak": round(t_hbm * 1e6, 2),
              "us_per_op": us_per_op})
    return r


def two_factor_bench(B, data, primes, reps):
    """Config 2 as the paper writes it: N=2^16 as 256 x 256 (two factors, both steps BAT
    int8 GEMMs), forward + inverse of the 384 limb-polynomials; the library default is
    restored afterwards."""
    import torch
    B.set_ntt_split(LOG_N, 8)
    try:
        for _ in range(3):
            B.ntt_forward(data, primes)
            B.ntt_inverse(data, primes)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            B.ntt_forward(data, primes)
            B.ntt_inverse(data, primes)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        B.profile_report()
        B.profile_enable(True)
        for _ in range(reps):
            B.ntt_forward(data, primes)
            B.ntt_inverse(data, primes)
        prof = B.profile_report()
        B.profile_enable(False)
    finally:
        B.set_ntt_split3(LOG_N, 0, 0)
    npolys = L * POLYS
    ops = gemm_ops_per_launch(LOG_N, 8, npolys, "left")      # 256 x 256: both steps alike
    gemm = {k: v for k, v in prof.items() if k.startswith("bat_gemm")}
    launches = sum(v[0] for v in gemm.values())
    avg_s = sum(v[1] for v in gemm.values()) / 1e3 / max(1, launches)
    return {"config": "N=2^16 as R x C = 256 x 256, L=24, 16 polys, forward + inverse",
            "us_per_step": round(dt * 1e6, 1), "limb_ntt_per_s": round(2 * npolys / dt, 1),
            "gemm_launch_us_avg": round(avg_s * 1e6, 2), "int8_ops_per_gemm_launch": ops,
            "gemm_int8_tops": round(ops / avg_s / 1e12, 1),
            "gemm_frac_of_int8_peak": round(ops / avg_s / 1e12 / INT8_PEAK_TOPS, 4)}


def config1_bench(B, reps=200):
    """Config 1: N=4096, one 28-bit prime, batch 1: NTT, INTT and the negacyclic product
    (NTT a, NTT b, pointwise, INTT); median microseconds over individually event-timed calls."""
    import numpy as np
    import torch
    import synthetic
    primes, x = synthetic.ntt_batch(1, 12, 1, 2)
    d = torch.from_numpy(np.ascontiguousarray(x[:1]).view(np.int32)).cuda()
    e = torch.from_numpy(np.ascontiguousarray(x[1:]).view(np.int32)).cuda()
    out = torch.empty_like(d)
    calls = {"ntt_us": lambda: B.ntt_forward(d, primes), "intt_us": lambda: B.ntt_inverse(d, primes),
             "polymul_us": lambda: B.poly_mul(d, e, out, primes)}
    res = {}
    for name, fn in calls.items():
        for _ in range(20):
            fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e3)
        res[name] = round(float(np.median(ts)), 2)
    return dict(res, config="N=4096, one prime (268042241), batch 1; median of %d event-timed calls" % reps)


def modred_bench(B, reps):
    """VecModMul a * w mod q (w pre-known, one vector per limb shared by every polynomial) at
    N=2^16, L=24 under each modular reduction, for 1..64 polynomials (Fig. diff_modred analog)."""
    import numpy as np
    import torch
    import synthetic
    primes, a = synthetic.ntt_batch(5, 16, 24, 64)
    _, w = synthetic.ntt_batch(6, 16, 24, 1)
    da = torch.from_numpy(a.view(np.int32)).cuda()
    dw = torch.from_numpy(np.ascontiguousarray(w[0]).view(np.int32)).cuda()
    limb_words = 24 << 16
    res = {}
    for method in ("barrett", "montgomery", "shoup", "bat_lazy"):
        prep = B.vec_modmul_prepare(dw, primes, method)
        row = {}
        for npoly in (1, 4, 16, 64):
            x = da[:npoly]
            out = torch.empty_like(x)
            for _ in range(3):
                B.vec_modmul(x, prep, out, primes, method)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                B.vec_modmul(x, prep, out, primes, method)
            e1.record()
            e1.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / reps
            nbytes = 4 * limb_words * (2 * npoly + (2 if method == "shoup" else 1))
            row[str(npoly)] = {"us": round(us, 2), "gbs": round(nbytes / us / 1e3, 1),
                               "elements_per_s": round(npoly * limb_words / us * 1e6, 1)}
        res[method] = row
    return res


def wide_prime_bench(B, reps):
    """Forward + inverse NTT at N=2^16, L=24, 16 polynomials with the largest primes below
    2^28 (narrow form) and below 2^31 (wide form: byte operands, signed-digit tables);
    microseconds per pair, both measured in the same run."""
    import numpy as np
    import torch
    import synthetic
    res = {}
    for name, primes in (("narrow_28bit", synthetic.primes(L)), ("wide_31bit", synthetic.wide_primes(L))):
        x = synthetic.residues(synthetic.rng(12), (16,), primes, 1 << LOG_N)
        d = torch.from_numpy(x.view(np.int32)).cuda()
        for _ in range(3):
            B.ntt_forward(d, primes)
            B.ntt_inverse(d, primes)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            B.ntt_forward(d, primes)
            B.ntt_inverse(d, primes)
        e1.record()
        e1.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        res[name] = {"us_fwd_inv": round(us, 2), "limb_ntt_per_s": round(2 * L * 16 / us * 1e6),
                     "bits_per_limb": max(primes).bit_length()}
    return res


def ntt_reduction_bench(B, reps):
    """Forward + inverse NTT at N=2^16, L=24 (64 x 32 x 32) with every step's epilogue
    reduction Montgomery vs Barrett, for 1, 4 and 16 polynomials (the NTT side of
    Fig. diff_modred); microseconds per pair and the row-kernel and row-side-step shares."""
    import numpy as np
    import torch
    import synthetic
    primes, x = synthetic.ntt_batch(11, LOG_N, L, 16)
    res = {}
    try:
        for method in ("montgomery", "barrett"):
            B.set_ntt_reduction(method)
            row = {}
            for npoly in (1, 4, 16):
                d = torch.from_numpy(np.ascontiguousarray(x[:npoly]).view(np.int32)).cuda()
                for _ in range(3):
                    B.ntt_forward(d, primes)
                    B.ntt_inverse(d, primes)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    B.ntt_forward(d, primes)
                    B.ntt_inverse(d, primes)
                e1.record()
                e1.synchronize()
                B.profile_report()
                B.profile_enable(True)             # a second, event-bracketed pass for the row kernels
                for _ in range(reps):
                    B.ntt_forward(d, primes)
                    B.ntt_inverse(d, primes)
                prof = B.profile_report()
                B.profile_enable(False)
                rows = prof.get("ntt_rows", (1, 0.0))
                left = prof.get("bat_gemm_left", (1, 0.0))
                row[str(npoly)] = {"us_fwd_inv": round(e0.elapsed_time(e1) * 1e3 / reps, 2),
                                   "row_kernel_us_avg": round(rows[1] * 1e3 / max(1, rows[0]), 2),
                                   "row_side_step_us_avg": round(left[1] * 1e3 / max(1, left[0]), 2)}
            res[method] = row
    finally:
        B.set_ntt_reduction("montgomery")
    return res


def stream_bench(B, reps):
    """Key-switching streams in both forms at the HE-Mult shape (N=2^16, L=24, K=8,
    dnum=3): the inner product with the plain and the BAT-expanded evaluation key, and
    the tensor product with 32-bit products and with byte-convolution products, for
    1 and 8 ciphertexts; microseconds per call and algorithmic HBM rate."""
    import numpy as np
    import torch
    import synthetic
    n, L, LK, dnum = 1 << 16, 24, 32, 3
    p = synthetic.primes(LK)
    g = synthetic.rng(9)
    ext = torch.from_numpy(synthetic.residues(g, (8, dnum), p, n).view(np.int32)).cuda()
    key = torch.from_numpy(synthetic.residues(g, (dnum, 2), p, n).view(np.int32)).cuda()
    kbat = B.evk_bat_prepare(key, p)
    ct = torch.from_numpy(synthetic.residues(g, (8, 2), p[:L], n).view(np.int32)).cuda()
    ct2 = torch.from_numpy(synthetic.residues(g, (8, 2), p[:L], n).view(np.int32)).cuda()

    def timed(fn):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps

    res = {"inner_product": {}, "tensor": {}}
    for form in ("valu", "chunked"):
        k = kbat if form == "chunked" else key
        row = {}
        for b in (1, 8):
            out = torch.empty((b, 2, LK, n), dtype=torch.int32, device="cuda")
            us = timed(lambda: B.keyswitch_inner_product(ext[:b], k, out, p, form))
            nbytes = 4 * LK * n * (b * dnum + dnum * 2 * (4 if form == "chunked" else 1) + b * 2)
            row[str(b)] = {"us": round(us, 2), "gbs": round(nbytes / us / 1e3, 1)}
        res["inner_product"][form] = row
        row = {}
        for b in (1, 8):
            out = torch.empty((b, 2, L, n), dtype=torch.int32, device="cuda")
            d2 = torch.empty((b, L, n), dtype=torch.int32, device="cuda")
            us = timed(lambda: B.tensor(ct[:b], ct2[:b], out, d2, p[:L], form))
            nbytes = 4 * L * n * b * 7
            row[str(b)] = {"us": round(us, 2), "gbs": round(nbytes / us / 1e3, 1)}
        res["tensor"][form] = row
    return res


def uneven_batch_bench(B, replays):
    """Config C4: 64 ciphertexts, N in {2^13..2^16}, L in [4, 36], HE-Mult (p = 0.5) else
    NTT of both polynomials; one captured graph per pass vs. the per-job calls (timed first,
    with the library's default splits), then the autotuner's choices (per-call splits and
    the batch runtime's work-list tiles) for the batch."""
    import torch
    import synthetic
    pool = synthetic.DevicePool(4)
    jobs, calls = [], []
    for k, (op, log_n, L) in enumerate(synthetic.uneven_jobs(4, 64)):
        qs, ps, _ = pool.params(L)
        a, b = pool.ciphertexts(log_n, L, k)
        if op == "he_mult":
            key = pool.key(log_n, L, "relin")
            out = torch.empty((1,) + tuple(a.shape), dtype=torch.int32, device="cuda")
            scratch_out = torch.empty_like(out)
            j = {"op": "he_mult", "a": a.unsqueeze(0), "b": b.unsqueeze(0), "key": key, "out": out,
                 "qs": qs, "ps": ps, "dnum": 3}
            calls.append(lambda j=j, o=scratch_out: B.he_mult(j["a"], j["b"], j["key"], o, j["qs"], j["ps"], 3))
        else:
            data = a.clone()
            j = {"op": "ntt_forward", "data": data, "primes": qs}
            scratch = a.clone()
            calls.append(lambda s=scratch, q=qs: B.ntt_forward(s, q))
        jobs.append(j)
    torch.cuda.synchronize()
    # warm-up: the first pass builds tables and job lists on the host (the GPU idles and
    # its clocks drop); keep passing for about half a second before timing
    t_w = time.perf_counter()
    while time.perf_counter() - t_w < 0.5:
        for c in calls:
            c()
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    eager_reps = max(3, replays // 2)
    for _ in range(eager_reps):
        for c in calls:
            c()
    torch.cuda.synchronize()
    t_eager = (time.perf_counter() - t0) / eager_reps
    tuned = {log_n: B.autotune(log_n, L=8, batch=4) for log_n in (13, 14, 15, 16)}
    bt = B.Batch(jobs, use_graph=True)
    info = bt.info()
    t_w = time.perf_counter()
    while time.perf_counter() - t_w < 0.3:
        bt.run()
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(replays):
        bt.run()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / replays
    bt.close()
    n_he = sum(1 for j in jobs if j["op"] == "he_mult")
    return {"config": "64 ciphertexts, N in {2^13..2^16}, L in [4,36], dnum=3, K=alpha; "
                      "%d HE-Mult + %d NTT(2 polys)" % (n_he, 64 - n_he),
            "graph_ms_per_pass": round(t_graph * 1e3, 3), "per_job_calls_ms_per_pass": round(t_eager * 1e3, 3),
            "speedup_vs_per_job_calls": round(t_eager / t_graph, 3),
            "ciphertexts_per_s": round(64 / t_graph, 1), "launches_per_pass_eager": info["launches"],
            "gemm_tiles_per_pass": info["gemm_tiles"], "replays": replays,
            "batch_ntt_form": {"2^13": "two factors", "2^14": "16 x 32 x 32", "2^15": "32 x 32 x 32",
                               "2^16": "64 x 32 x 32"},
            "batch_list_tiles": {str(k): {d: B.get_batch_tile(k, d == "inverse")[0] for d in ("forward", "inverse")}
                                 for k in (13, 14, 15, 16)},
            "autotuned": {str(k): {"R": 1 << v["log_r"], "C": 1 << (k - v["log_r"]),
                                   "C1": (1 << v["log_c1"]) if v["log_c1"] else None, "tile": v["tile"],
                                   "ntt_fwd_inv_us_L8_b4": round(v["us"], 1)} for k, v in tuned.items()}}


def serving_bench(n_req, budget_gb=4.0):
    """Config C5: Poisson arrivals of HE-Mult / Rotate requests, N in {2^14..2^16}, L in [8, 36]."""
    import torch
    import synthetic
    from paper_2501_07047_amd import serving as S
    pool = synthetic.DevicePool(5)
    budget = int(budget_gb * (1 << 30))

    def run(rate, seed):
        specs = synthetic.poisson_requests(seed, n_req, rate)
        reqs = S.build_requests(specs, pool)
        torch.cuda.synchronize()
        return S.Server(S.GpuExecutor(slots=4), hbm_budget=budget, slots=4, max_group=8).run(reqs)

    run(1e9, 99)                                   # warm keys, tables and clocks
    sat = run(1e9, 7)                              # closed loop: every request waiting at t = 0
    out = {"config": "%d requests per point, HE-Mult p=0.5 else Rotate r in {1..64}, N in {2^14,2^15,2^16}, "
                     "L in [8,36], dnum=3, K=alpha, HBM budget %.1f GiB, 4 stream slots, at most 8 requests "
                     "per admitted group; every shape's tables built before the arrival clock starts"
                     % (n_req, budget_gb),
           "saturation_per_s": round(sat["throughput_per_s"], 1),
           "saturation_groups": sat.get("groups"), "saturation_host_us_per_group": sat.get("host_us_per_group"),
           "points": []}
    for f in (0.5, 0.8, 0.95):
        r = run(f * sat["throughput_per_s"], 8)
        out["points"].append({"load": f, "rate_per_s": round(f * sat["throughput_per_s"], 1),
                              "throughput_per_s": round(r["throughput_per_s"], 1),
                              "p50_ms": round(r["p50_ms"], 3), "p99_ms": round(r["p99_ms"], 3),
                              "peak_hbm_gib": round(r["peak_hbm_bytes"] / (1 << 30), 2),
                              "groups": r.get("groups"), "host_us_per_group": r.get("host_us_per_group")})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--warmup-seconds", type=float, default=1.0,
                    help="keep warming up until this much wall time has passed (0 under a profiler)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", choices=["all", "ntt", "copy", "he_mult", "uneven"], default="all",
                    help="ntt: time only the NTT step; copy: a plain 256 MiB device copy "
                         "(calibrates rocprofv3 FETCH_SIZE/WRITE_SIZE against known bytes); "
                         "he_mult: only HE-Mult at batch 8 (for a kernel trace of its kernels); "
                         "uneven: only the 64-ciphertext uneven batch (for a trace of the batch runtime)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the hot path shards by ciphertext with no "
              "exchange between GPUs, so one MI355X's throughput is the figure (use --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import synthetic

    cpu, he_oracle = None, None
    if not args.no_cpu and args.only == "all":
        # the oracle first, before anything touches the GPU (its worker pool forks)
        cpu, he_oracle = cpu_baseline(synthetic.ckks_pair(0, 16, 24, 3, 8, 8))

    # a full collection of the interpreter's objects takes tens of milliseconds, longer
    # than most timed regions here: collect once now and time with automatic collection
    # off (as timeit does)
    gc.collect()
    gc.disable()

    import torch
    from paper_2501_07047_amd import binding as B

    torch.cuda.set_device(0)
    if args.only == "copy":
        src = torch.ones(1 << 26, dtype=torch.int32, device="cuda")     # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                          "launches": args.steps}))
        return
    if args.only == "he_mult":
        r = he_mult_bench(B, args.steps, args.warmup, 8, ("he_mult",))
        print(json.dumps({"he_mult_batch8": r["he_mult"]}))
        return
    if args.only == "uneven":
        print(json.dumps({"uneven_batch": uneven_batch_bench(B, max(4, args.steps // 2))}))
        return
    log_r, log_c1 = B.get_ntt_split(LOG_N)       # the library's default factoring of 2^16
    primes, x = synthetic.ntt_batch(0, LOG_N, L, POLYS)
    host = torch.from_numpy(x.view(np.int32))
    data = host.cuda()
    ref = host.cuda()
    stream = torch.cuda.current_stream()

    def step_mfma():
        B.ntt_forward(data, primes)
        B.ntt_inverse(data, primes)

    def step_bf():
        B.ntt_forward_butterfly(ref, primes)
        B.ntt_inverse_butterfly(ref, primes)

    # bit-exactness of the timed configuration: MFMA forward == butterfly forward, round trip == input
    B.ntt_forward(data, primes)
    B.ntt_forward_butterfly(ref, primes)
    torch.cuda.synchronize()
    exact = bool(torch.equal(data, ref))
    B.ntt_inverse(data, primes)
    B.ntt_inverse_butterfly(ref, primes)
    torch.cuda.synchronize()
    exact = exact and bool(torch.equal(data, host.cuda())) and bool(torch.equal(ref, data))

    # warm up: at least W steps and about a second of work, so clocks have settled
    t_w = time.perf_counter()
    n_w = 0
    while n_w < args.warmup or (time.perf_counter() - t_w < args.warmup_seconds and n_w < 6000):
        step_mfma()
        n_w += 1
        if n_w % 10 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    # the dominant kernel family, from a few event-timed steps before the timed region
    B.profile_report()
    B.profile_enable(True)
    for _ in range(5):
        step_mfma()
    pre = B.profile_report()
    B.profile_enable(False)
    fam = max((k for k in pre if k in ("bat_gemm_left", "bat_gemm_right", "ntt_rows")),
              key=lambda k: pre[k][1])
    # timed region: events bracket the dominant family's launches (one forward and one
    # inverse per step) in one step of every PROFILE_EVERY; each bracketed launch costs a
    # few microseconds of queue time, and the other families run unbracketed
    B.profile_only(fam)
    t0 = time.perf_counter()
    for i in range(args.steps):
        B.profile_enable(i % PROFILE_EVERY == 0)
        step_mfma()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = B.profile_report()
    B.profile_enable(False)
    B.profile_only(None)

    for _ in range(max(1, args.warmup // 2)):
        step_bf()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bf_steps = max(2, args.steps // 4)
    for _ in range(bf_steps):
        step_bf()
    torch.cuda.synchronize()
    dt_bf = time.perf_counter() - t1

    limb_ntts = 2 * L * POLYS
    value = limb_ntts * args.steps / dt
    bf_value = limb_ntts * bf_steps / dt_bf

    launches, total_ms = prof[fam]
    avg_s = total_ms / 1e3 / max(1, launches)
    npolys = L * POLYS
    n = 1 << LOG_N
    measured_peak = {"mfma_i8_tops": round(B.measure_peak("mfma_i8_32x32"), 1),
                     "hbm_copy_gbs": round(B.measure_peak("hbm_copy"), 1)}
    if fam == "ntt_rows":
        # row transform of every row (C1 x C2 split): HBM-bound.  Per launch: every residue
        # read and written once, the row tables (one matrix when C1 = C2) and the C-entry
        # twiddle pairs per prime, and (inverse launches, half of them) the N-entry inverse
        # step-2 twiddle pairs.
        c = 1 << (LOG_N - log_r)
        c1, c2 = 1 << log_c1, c // (1 << log_c1)
        nbytes = rows_bytes_per_launch(LOG_N, log_r, log_c1, L, POLYS)
        ops = 32.0 * n * (c1 + c2) * npolys
        achieved = nbytes / avg_s / 1e9
        khash = source_hash("ntt_rows.hip")
        roof = {"bound": "hbm", "kernel": fam, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_for(fam, khash),
                "bytes_per_launch": nbytes, "int8_ops_per_launch": ops,
                "int8_tops": round(ops / avg_s / 1e12, 1),
                "frac_of_measured_copy": round(achieved / measured_peak["hbm_copy_gbs"], 4)}
    else:
        ops = gemm_ops_per_launch(LOG_N, log_r, npolys, "left" if fam.endswith("left") else "right")
        achieved = ops / avg_s / 1e12
        khash = source_hash("ntt_mfma.hip")
        roof = {"bound": "mfma", "kernel": fam, "achieved": round(achieved, 2), "peak": INT8_PEAK_TOPS,
                "unit": "TOP/s", "frac": round(achieved / INT8_PEAK_TOPS, 4), "traffic": traffic_for(fam, khash),
                "ops_per_launch": ops,
                "frac_of_measured_mfma_peak": round(achieved / measured_peak["mfma_i8_tops"], 4)}
    roof.update({"avg_launch_us": round(avg_s * 1e6, 2), "launches_timed": launches,
                 "timed_steps_with_events": f"1 of every {PROFILE_EVERY}",
                 "measured_peaks": measured_peak,
                 "event_ms_by_kernel_5_steps": {k: [v[0], round(v[1], 3)] for k, v in pre.items()}})

    line = {"metric": METRIC, "value": round(value, 1), "unit": "limb-NTT/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i8",
            "data": "synthetic",
            "config": {"workload": "NTT+INTT, N=2^16, L=24 28-bit primes, 8 ciphertexts x 2 polys "
                                   "(384 limb-NTTs each way)",
                       "log_n": LOG_N, "R": 1 << log_r, "C1": 1 << log_c1 if log_c1 else None,
                       "C2": (1 << (LOG_N - log_r - log_c1)) if log_c1 else None,
                       "C": 1 << (LOG_N - log_r), "L": L, "polys": POLYS},
            "poly_ntt_per_s": round(value / L, 1),
            "butterfly_limb_ntt_per_s": round(bf_value, 1),
            "speedup_vs_butterfly": round(value / bf_value, 3),
            "bit_exact": exact,
            "roofline": roof}
    if args.only == "ntt":
        print(json.dumps(line))
        return
    line["config2_two_factor_256x256"] = two_factor_bench(B, data, primes, max(5, args.steps // 2))
    line["config1"] = config1_bench(B)
    he1 = he_mult_bench(B, max(10, args.steps), 2, 1)
    he8 = he_mult_bench(B, max(20, args.steps), 3, 8)
    he8_bf = he_mult_bench(B, 5, 1, 8, ("he_mult",), engine="butterfly")
    out8 = he8.pop("_out")
    he1.pop("_out", None)
    he8_bf.pop("_out", None)
    he8["he_mult"]["roofline"] = he_mult_roofline(B, he8["he_mult"]["us_per_op"], 8)
    he1["he_mult"]["roofline"] = he_mult_roofline(B, he1["he_mult"]["us_per_op"], 1)
    line["he_mult_per_s"] = he8["he_mult"]["per_s"]
    line["he_mult"] = {"config": "N=2^16, L=24, dnum=3 (alpha=8), K=8 special primes, tensor + relinearisation",
                       "batch1": he1["he_mult"], "batch8": he8["he_mult"],
                       "batch8_butterfly_ntt": he8_bf["he_mult"],
                       "speedup_vs_butterfly_ntt": round(he8["he_mult"]["per_s"] / he8_bf["he_mult"]["per_s"], 3)}
    if he_oracle is not None:
        line["he_mult"]["bit_exact_vs_oracle"] = all(np.array_equal(out8[k], he_oracle[k]) for k in range(8))
        line["he_mult"]["oracle_checked"] = "all 8 ciphertexts of the batch-8 call (oracle.ckks.he_mult)"
    line["rotate"] = {"config": "same parameters, 1 slot", "batch1": he1["rotate"], "batch8": he8["rotate"]}
    line["rescale"] = {"config": "N=2^16, L=24 -> 23 (divide by the last prime), per ciphertext",
                       "batch1": he1["rescale"], "batch8": he8["rescale"]}
    line["modred_ablation"] = {"config": "VecModMul a*w mod q, w pre-known per limb, N=2^16, L=24; "
                                         "key = polynomials per call; us per call and HBM GB/s "
                                         "(a read + out written + w read once)",
                               "methods": modred_bench(B, max(10, args.steps))}
    line["ntt_reduction_ablation"] = {"config": "NTT+INTT at N=2^16, L=24 (64 x 32 x 32); epilogue of "
                                               "every step Montgomery (tables x 2^32, REDC) vs Barrett "
                                               "(plain tables); key = polynomials per call",
                                     "methods": ntt_reduction_bench(B, max(10, args.steps))}
    line["wide_prime_ntt"] = {"config": "NTT+INTT at N=2^16, L=24, 16 polynomials, default split; "
                                        "largest primes < 2^28 vs < 2^31 (1 mod 2^17)",
                              "forms": wide_prime_bench(B, max(10, args.steps))}
    line["stream_ablation"] = {"config": "key-switch inner product (N=2^16, L+K=32, dnum=3; key plain vs "
                                         "BAT-expanded, 16 B per residue) and tensor product (N=2^16, L=24; "
                                         "32-bit vs byte-convolution products), per call for 1 and 8 "
                                         "ciphertexts: us and algorithmic HBM GB/s",
                               "forms": stream_bench(B, max(10, args.steps))}
    add_bytes = 3 * 2 * 24 * (1 << 16) * 4        # a, b read, out written: one ciphertext pair
    line["he_add"] = {"config": "N=2^16, L=24, per ciphertext pair", "batch1": he1["he_add"],
                      "batch8": he8["he_add"], "bytes_per_op": add_bytes,
                      "hbm_gbs_batch8": round(add_bytes * he8["he_add"]["per_s"] / 1e9, 1)}
    line["uneven_batch"] = uneven_batch_bench(B, max(4, args.steps // 2))
    line["serving"] = serving_bench(2000)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line))


if __name__ == "__main__":
    main()
