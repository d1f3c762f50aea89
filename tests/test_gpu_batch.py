"""GPU tests of the batch runtime: every job of a mixed batch (uneven N, limb
count and kind) is bit-identical to the per-call entry points and to the
oracle, eagerly and through repeated hipGraph replays."""
import numpy as np
import pytest

import synthetic
from oracle import ckks as CK
from oracle.ntt import ntt_ct, intt_gs
from oracle.primes import psi as psi_of
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def _mixed_jobs(seed, specs):
    """specs: list of (op, log_n, L, dnum, batch). Returns jobs (device) and host inputs."""
    import torch
    jobs, host = [], []
    for k, (op, log_n, L, dnum, batch) in enumerate(specs):
        if op.startswith("ntt"):
            primes, x = synthetic.ntt_batch(seed * 100 + k, log_n, L, batch)
            jobs.append({"op": op, "data": to_dev(x), "primes": primes})
            host.append({"x": x, "primes": primes})
        else:
            qs, ps, a, b, key = synthetic.ckks_pair(seed * 100 + k, log_n, L, dnum, None, batch)
            j = {"op": op, "key": to_dev(key), "qs": qs, "ps": ps, "dnum": dnum,
                 "out": torch.empty(a.shape, dtype=torch.int32, device="cuda")}
            if op == "he_mult":
                j.update(a=to_dev(a), b=to_dev(b))
            else:
                j.update(ct=to_dev(a), steps=k + 1)
            jobs.append(j)
            host.append({"a": a, "b": b, "key": key, "qs": qs, "ps": ps})
    return jobs, host


def _reference(B, j, h):
    """Per-call entry points on fresh copies (already pinned to the oracle elsewhere)."""
    import torch
    if j["op"].startswith("ntt"):
        d = to_dev(h["x"])
        (B.ntt_forward if j["op"] == "ntt_forward" else B.ntt_inverse)(d, h["primes"])
        return to_host(d)
    out = torch.empty(h["a"].shape, dtype=torch.int32, device="cuda")
    if j["op"] == "he_mult":
        B.he_mult(to_dev(h["a"]), to_dev(h["b"]), to_dev(h["key"]), out, h["qs"], h["ps"], j["dnum"])
    else:
        B.rotate(to_dev(h["a"]), j["steps"], to_dev(h["key"]), out, h["qs"], h["ps"], j["dnum"])
    return to_host(out)


def _result(j):
    return to_host(j["data"] if j["op"].startswith("ntt") else j["out"])


def _reset(jobs, host):
    import torch
    for j, h in zip(jobs, host):
        if j["op"].startswith("ntt"):
            j["data"].copy_(torch.from_numpy(h["x"].view(np.int32)))
        else:
            j["out"].fill_(0)


SPECS = [("he_mult", 12, 5, 3, 2), ("ntt_forward", 14, 3, 1, 3), ("rotate", 12, 4, 3, 1),
         ("he_mult", 13, 7, 1, 1), ("ntt_inverse", 12, 2, 1, 2), ("he_mult", 14, 4, 3, 1),
         ("ntt_forward", 16, 2, 1, 1), ("rotate", 13, 6, 2, 2)]


@pytest.mark.parametrize("use_graph", [False, True])
def test_mixed_batch_matches_per_call_and_oracle(use_graph):
    import torch
    from paper_2501_07047_amd import binding as B
    jobs, host = _mixed_jobs(1, SPECS)
    refs = [_reference(B, j, h) for j, h in zip(jobs, host)]
    bt = B.Batch(jobs, use_graph=use_graph)
    info = bt.info()
    # 7 vector phases + 4 NTT phases of two halves, each half at most one GEMM launch per
    # list tile (3) and packed-input layout (2) plus one row-kernel launch
    assert info["launches"] <= 7 + 4 * (2 * 3 * 2 + 2)
    replays = 3 if use_graph else 1
    for r in range(replays):
        _reset(jobs, host)
        torch.cuda.synchronize()
        bt.run()
        torch.cuda.synchronize()
        for k, (j, ref) in enumerate(zip(jobs, refs)):
            assert np.array_equal(_result(j), ref), "job %d (%s) replay %d" % (k, j["op"], r)
        # unrelated eager work between replays
        x = torch.arange(1 << 20, device="cuda", dtype=torch.int32)
        assert int(x.sum().item()) == (1 << 20) * ((1 << 20) - 1) // 2
    bt.close()
    # oracle spot checks on two small jobs
    h = host[0]
    assert np.array_equal(refs[0][1], CK.he_mult(h["a"][1], h["b"][1], h["key"], h["qs"], h["ps"], 3))
    h = host[1]
    n = 1 << 14
    for i, q in enumerate(h["primes"]):
        assert np.array_equal(refs[1][:, i], ntt_ct(h["x"][:, i].astype(np.uint64), q, psi_of(q, n)))
    h = host[4]
    for i, q in enumerate(h["primes"]):
        assert np.array_equal(refs[4][:, i], intt_gs(h["x"][:, i].astype(np.uint64), q, psi_of(q, 1 << 12)))


def test_config4_uneven_batch_64_ciphertexts():
    """64 ciphertexts, N in {2^13..2^16}, L in [4, 36], HE-Mult with p = 0.5 else NTT of both polys."""
    import torch
    from paper_2501_07047_amd import binding as B
    spec = synthetic.uneven_jobs(4, 64)
    specs = [("he_mult" if op == "he_mult" else "ntt_forward", log_n, L, 3, 1 if op == "he_mult" else 2)
             for op, log_n, L in spec]
    jobs, host = _mixed_jobs(2, specs)
    refs = [_reference(B, j, h) for j, h in zip(jobs, host)]
    bt = B.Batch(jobs, use_graph=True)
    for r in range(2):
        _reset(jobs, host)
        torch.cuda.synchronize()
        bt.run()
        torch.cuda.synchronize()
        bad = [k for k, (j, ref) in enumerate(zip(jobs, refs)) if not np.array_equal(_result(j), ref)]
        assert not bad, "mismatching jobs %s in replay %d" % (bad, r)
    got = {k: _result(jobs[k]) for k in range(len(jobs))}
    bt.close()
    # oracle checks of the batch's own results: the smallest and the largest HE-Mult
    # job (N = 2^16, L = 36, K = 12 with this seed) and the largest N = 2^16 NTT job
    he = [k for k, s in enumerate(specs) if s[0] == "he_mult"]
    for k in (min(he, key=lambda i: (specs[i][1], specs[i][2])), max(he, key=lambda i: (specs[i][1], specs[i][2]))):
        h = host[k]
        assert np.array_equal(got[k][0], CK.he_mult(h["a"][0], h["b"][0], h["key"], h["qs"], h["ps"], 3)), \
            "HE-Mult job %d %s" % (k, specs[k])
    nt = [k for k, s in enumerate(specs) if s[0] != "he_mult" and s[1] == 16]
    k = max(nt, key=lambda i: specs[i][2])
    h = host[k]
    for i, q in enumerate(h["primes"]):
        ref = ntt_ct(h["x"][:, i].astype(np.uint64), q, psi_of(q, 1 << 16))
        assert np.array_equal(got[k][:, i], ref), "NTT job %d %s limb %d" % (k, specs[k], i)


def test_group_workspace_within_the_sum_of_its_jobs_alone():
    # the request loop sizes a group's workspace as the sum of its requests' sizes alone:
    # a batch's scratch is the sum of its jobs' and its merged task lists take no more
    # room than theirs apart.  Sizing only, nothing runs.
    from paper_2501_07047_amd import binding as B
    jobs, _ = _mixed_jobs(5, SPECS)
    alone = [B.batch_workspace_bytes([j]) for j in jobs]
    for k in range(1, len(jobs) + 1):
        assert B.batch_workspace_bytes(jobs[:k]) <= sum(alone[:k])
    # in reverse order too (the phases' lists are filled in job order)
    assert B.batch_workspace_bytes(jobs[::-1]) <= sum(alone)


def test_batch_rejects_bad_jobs():
    import torch
    from paper_2501_07047_amd import binding as B
    primes, x = synthetic.ntt_batch(0, 10, 2, 1)       # log_n 10 is below the batch runtime's range
    with pytest.raises(B.CrossError) as e:
        B.Batch([{"op": "ntt_forward", "data": to_dev(x), "primes": primes}])
    assert e.value.code == -7


def test_batch_rejects_wide_primes():
    # the work-list kernels are narrow-only: a wide prime (2^28 <= q < 2^31) in a
    # CKKS job is refused with CROSS_ERANGE before anything is planned
    from paper_2501_07047_amd import binding as B
    wp = synthetic.wide_primes(6)
    qs, ps = wp[:4], wp[4:]
    n = 1 << 14
    a = synthetic.residues(synthetic.rng(5), (1, 2), qs, n)
    key = synthetic.residues(synthetic.rng(6), (2, 2), qs + ps, n)
    out = to_dev(np.zeros_like(a))
    with pytest.raises(B.CrossError) as e:
        B.Batch([{"op": "he_mult", "a": to_dev(a), "b": to_dev(a), "key": to_dev(key), "out": out,
                  "qs": qs, "ps": ps, "dnum": 2}])
    assert e.value.code == -4


def test_tuned_list_tiles_keep_batch_results():
    """After the autotuner has chosen the batch runtime's work-list tiles for N = 2^13
    and 2^14 (two- and three-factor forms), a mixed batch still equals the per-call
    entry points, and the chosen tiles are reported."""
    import torch
    from paper_2501_07047_amd import binding as B
    for log_n in (13, 14):
        B.autotune(log_n, L=3, batch=2)
        for inv in (False, True):
            name, tuned = B.get_batch_tile(log_n, inv)
            assert tuned and name in ("256x128", "128x64", "64x64")
    specs = [("ntt_forward", 14, 3, 1, 2), ("ntt_inverse", 13, 2, 1, 2), ("he_mult", 14, 5, 3, 1),
             ("rotate", 13, 4, 3, 1)]
    jobs, host = _mixed_jobs(5, specs)
    refs = [_reference(B, j, h) for j, h in zip(jobs, host)]
    bt = B.Batch(jobs, use_graph=True)
    _reset(jobs, host)
    torch.cuda.synchronize()
    bt.run()
    torch.cuda.synchronize()
    for k, (j, ref) in enumerate(zip(jobs, refs)):
        assert np.array_equal(_result(j), ref), "job %d (%s)" % (k, j["op"])
    bt.close()
    h = host[0]
    for i, q in enumerate(h["primes"]):
        assert np.array_equal(refs[0][:, i], ntt_ct(h["x"][:, i].astype(np.uint64), q, psi_of(q, 1 << 14)))
