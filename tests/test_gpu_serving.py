"""GPU test of the request loop: every request's result is bit-identical whether it
runs alone or in the continuously batched mix, and the loop respects its HBM budget."""
import numpy as np
import pytest

import synthetic
from tests.gpu_util import to_host

pytestmark = pytest.mark.gpu


def test_alone_vs_mixed_identity_and_budget():
    import torch
    from paper_2501_07047_amd import binding as B
    from paper_2501_07047_amd import serving as S
    pool = synthetic.DevicePool(11)
    specs = synthetic.poisson_requests(5, 24, rate=20000.0, log_ns=(12, 13), L_range=(4, 10))
    reqs = S.build_requests(specs, pool)
    budget = 3 * max(r.footprint for r in reqs)
    srv = S.Server(S.GpuExecutor(slots=3), hbm_budget=budget, slots=3, max_group=4)
    res = srv.run(reqs)
    torch.cuda.synchronize()
    assert res["requests"] == 24 and res["peak_hbm_bytes"] <= budget
    assert all(r.t_done is not None for r in reqs)
    for r in reqs:
        alone = torch.empty_like(r.out)
        x = r.inputs
        if r.op == "he_mult":
            B.he_mult(x["a"], x["b"], x["key"], alone, r.qs, r.ps, r.dnum)
        else:
            B.rotate(x["a"], r.steps, x["key"], alone, r.qs, r.ps, r.dnum)
        assert np.array_equal(to_host(alone), to_host(r.out)), "request %d (%s) differs" % (r.rid, r.op)


def _oracle(CK, r):
    a = to_host(r.inputs["a"])[0]
    key = to_host(r.inputs["key"])
    if r.op == "he_mult":
        return CK.he_mult(a, to_host(r.inputs["b"])[0], key, r.qs, r.ps, r.dnum)
    return CK.rotate(a, r.steps, key, r.qs, r.ps, r.dnum)


def test_request_loop_at_full_scale_matches_oracle():
    """Request-loop workload at its own sizes (N in {2^14, 2^16}, L in [8, 36], dnum = 3,
    K = alpha): every result equals the request run alone, and the largest HE-Mult and
    the largest Rotate request equal the oracle."""
    import torch
    from oracle import ckks as CK
    from paper_2501_07047_amd import binding as B
    from paper_2501_07047_amd import serving as S
    pool = synthetic.DevicePool(12)
    specs = synthetic.poisson_requests(6, 12, rate=5000.0, log_ns=(14, 16), L_range=(8, 36))
    reqs = S.build_requests(specs, pool)
    # each request alone first (per-call entry points), then the same requests served
    alone = {}
    for r in reqs:
        x = r.inputs
        o = torch.empty_like(x["a"])
        if r.op == "he_mult":
            B.he_mult(x["a"], x["b"], x["key"], o, r.qs, r.ps, r.dnum)
        else:
            B.rotate(x["a"], r.steps, x["key"], o, r.qs, r.ps, r.dnum)
        alone[r.rid] = to_host(o)
    budget = 4 << 30
    srv = S.Server(S.GpuExecutor(slots=3), hbm_budget=budget, slots=3, max_group=4)
    res = srv.run(reqs)
    torch.cuda.synchronize()
    assert res["requests"] == len(reqs) and res["peak_hbm_bytes"] <= budget
    served = {r.rid: to_host(r.out) for r in reqs}
    for r in reqs:
        if not np.array_equal(alone[r.rid], served[r.rid]):
            ref = _oracle(CK, r)
            pytest.fail("request %d (%s, N=2^%d, L=%d) differs alone / served; oracle equals alone: %s, served: %s"
                        % (r.rid, r.op, r.log_n, r.L, np.array_equal(alone[r.rid][0], ref),
                           np.array_equal(served[r.rid][0], ref)))
    for op in ("he_mult", "rotate"):
        mine = [r for r in reqs if r.op == op]
        assert mine, "workload has no %s request" % op
        r = max(mine, key=lambda q: (q.log_n, q.L))
        ref = _oracle(CK, r)
        assert np.array_equal(to_host(r.out)[0], ref), "request %d (%s, N=2^%d, L=%d) vs oracle" % (
            r.rid, op, r.log_n, r.L)
