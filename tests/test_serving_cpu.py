"""CPU tests of the request loop's admission and accounting, with a simulated executor."""
import heapq

from paper_2501_07047_amd.serving import Request, Server, footprint_bytes
import synthetic


class FakeExecutor:
    """Each batch takes `cost` seconds per request after it is launched (simulated clock)."""

    def __init__(self, clock, cost=0.01):
        self.clock = clock
        self.cost = cost
        self.launched = []

    def start(self, t0):
        self.t0 = t0

    def launch(self, group, slot):
        t_end = self.clock.t + self.cost * len(group)
        self.launched.append((slot, [r.rid for r in group]))
        return {"end": t_end, "rids": [r.rid for r in group]}

    def done(self, h):
        return self.clock.t >= h["end"]

    def wait_any(self, hs):
        self.clock.t = max(self.clock.t, min(h["end"] for h in hs))

    def finish(self, h):
        return {rid: h["end"] - self.t0 for rid in h["rids"]}


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4          # every poll advances simulated time a little
        return self.t


def _reqs(n, fp, spacing):
    return [Request(i, "he_mult", 14, 8, 3, i * spacing, None, [], [], footprint=fp) for i in range(n)]


def test_budget_is_never_exceeded_and_all_complete():
    clk = Clock()
    ex = FakeExecutor(clk)
    srv = Server(ex, hbm_budget=1000, slots=3, max_group=4)
    reqs = _reqs(40, 300, 0.001)
    res = srv.run(reqs, clock=clk)
    assert res["requests"] == 40
    assert res["peak_hbm_bytes"] <= 1000
    assert all(r.t_done is not None and r.t_done >= r.arrival for r in reqs)
    assert all(len(g) <= 3 for _, g in ex.launched)          # 3 x 300 <= 1000


def test_requests_admitted_while_others_run():
    # a request that arrives while a batch is in flight is launched on another slot before that batch ends
    clk = Clock()
    ex = FakeExecutor(clk, cost=0.05)
    srv = Server(ex, hbm_budget=10 ** 9, slots=2, max_group=8)
    reqs = _reqs(2, 1, 0.01)
    srv.run(reqs, clock=clk)
    assert [g for _, g in ex.launched] == [[0], [1]]
    assert reqs[1].t_admit < reqs[0].t_done


def test_oversized_request_is_rejected():
    import pytest
    srv = Server(FakeExecutor(Clock()), hbm_budget=10, slots=1)
    with pytest.raises(ValueError):
        srv.run(_reqs(1, 11, 0.0))


def test_poisson_workload_is_seeded():
    a = synthetic.poisson_requests(3, 50, 100.0)
    b = synthetic.poisson_requests(3, 50, 100.0)
    assert a == b
    assert all(8 <= r["L"] <= 36 and r["log_n"] in (14, 15, 16) for r in a)
    assert all(x["arrival"] < y["arrival"] for x, y in zip(a, a[1:]))


def test_footprint_grows_with_size():
    assert footprint_bytes(16, 24, 8, 3, "he_mult") > footprint_bytes(14, 24, 8, 3, "he_mult")
    assert footprint_bytes(16, 24, 8, 3, "he_mult") > footprint_bytes(16, 24, 8, 3, "rotate")


def test_automatic_collection_is_off_while_serving_and_restored():
    # a full collection of the interpreter's objects would stall the loop: it runs once
    # before the clock starts, automatic collection stays off during the loop, and the
    # caller's setting comes back afterwards, also when the executor raises
    import gc

    class Recording(FakeExecutor):
        def launch(self, group, slot):
            self.gc_states = getattr(self, "gc_states", []) + [gc.isenabled()]
            return super().launch(group, slot)

    class Failing(FakeExecutor):
        def launch(self, group, slot):
            raise RuntimeError("launch failed")

    was = gc.isenabled()
    try:
        for caller_setting in (True, False):
            (gc.enable if caller_setting else gc.disable)()
            clk = Clock()
            ex = Recording(clk)
            Server(ex, hbm_budget=1000, slots=2, max_group=4).run(_reqs(12, 300, 0.001), clock=clk)
            assert ex.gc_states and not any(ex.gc_states)
            assert gc.isenabled() == caller_setting
            try:
                Server(Failing(Clock()), hbm_budget=1000, slots=2, max_group=4).run(_reqs(3, 300, 0.0),
                                                                                    clock=Clock())
                assert False, "the executor's error must propagate"
            except RuntimeError:
                pass
            assert gc.isenabled() == caller_setting
    finally:
        (gc.enable if was else gc.disable)()
