"""Continuous-batching request loop for HE-Mult and Rotate requests.

Requests arrive over time (seeded Poisson arrivals in the benchmark).  Each
iteration of the loop

  1. retires batches whose GPU work has finished (their HBM footprint and
     stream slot are released, completion times are read from HIP events),
  2. admits waiting requests in arrival order while their footprint fits in
     the HBM budget and a stream slot is free,
  3. launches the admitted group as one batch (libcross batch runtime, work
     carved from a caller-provided workspace so nothing is allocated or
     synchronised per iteration) on the free stream.

A group is planned and uploaded while earlier groups run, so requests that
arrive while others run are admitted as soon as memory and a slot free up --
the queue is drained continuously, not in lock-step rounds (GpuExecutor keeps
the groups' execution on the device in admission order).  The executor is
pluggable: GpuExecutor drives libcross; tests use a CPU stand-in to check the
admission and accounting logic without a GPU.
"""
import collections
import gc
import time


class Request:
    """One HE-Mult (a * b, relinearised with `key`) or Rotate (ct by `steps`, key) request."""

    __slots__ = ("rid", "op", "log_n", "L", "dnum", "steps", "arrival", "inputs", "footprint",
                 "t_admit", "t_done", "out", "qs", "ps")

    def __init__(self, rid, op, log_n, L, dnum, arrival, inputs, qs, ps, steps=0, footprint=0):
        self.rid, self.op, self.log_n, self.L, self.dnum = rid, op, log_n, L, dnum
        self.steps, self.arrival, self.inputs, self.qs, self.ps = steps, arrival, inputs, qs, ps
        self.footprint = footprint
        self.t_admit = self.t_done = None
        self.out = None


def footprint_bytes(log_n, L, K, dnum, op):
    """HBM bytes one request holds while admitted: its ciphertext operands and output,
    the evaluation key, and the key-switching workspace."""
    n = 1 << log_n
    LK = L + K
    words = (2 if op == "he_mult" else 1) * 2 * L * n      # input ciphertexts
    words += 2 * L * n                                      # output
    words += dnum * 2 * LK * n                              # evaluation key
    words += L * n                                          # d2 / rotated c1
    words += dnum * LK * n                                  # ModUp output
    words += max(dnum * LK, 2 * LK) * n                     # NTT scratch
    words += 2 * LK * n + 2 * L * n                         # accumulators, ModDown z
    return 4 * words


class Server:
    """Admission, batching and accounting.  `executor` provides
    launch(requests, slot) -> handle, done(handle) -> bool, finish(handle) -> {rid: t_done}."""

    def __init__(self, executor, hbm_budget, slots=4, max_group=16):
        self.ex = executor
        self.budget = hbm_budget
        self.slots = slots
        self.max_group = max_group

    def run(self, requests, clock=time.perf_counter):
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            if r.footprint > self.budget:
                raise ValueError("request %d needs %d bytes > budget %d" % (r.rid, r.footprint, self.budget))
        prepare = getattr(self.ex, "prepare", None)
        if prepare is not None:
            prepare(reqs)            # per-shape tables, before the arrival clock starts
        # a full collection of the interpreter's objects stalls the loop for tens of
        # milliseconds (seen as the p99 of a whole load point): collect once before the
        # arrival clock starts and keep automatic collection off while requests are served
        gc_on = gc.isenabled()
        gc.collect()
        gc.disable()
        try:
            peak, iterations = self._serve(reqs, clock)
        finally:
            if gc_on:
                gc.enable()
        makespan = max(r.t_done for r in reqs) if reqs else 0.0
        out = summarize(reqs, makespan, peak, iterations)
        stats = getattr(self.ex, "host_stats", None)
        if stats is not None:
            out.update(stats())
        return out

    def _serve(self, reqs, clock):
        pending = collections.deque(reqs)
        waiting = collections.deque()
        free_slots = list(range(self.slots))
        inflight = []
        used = 0
        peak = 0
        t0 = clock()
        self.ex.start(t0)
        iterations = 0
        while pending or waiting or inflight:
            iterations += 1
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            still = []
            for h, group, slot in inflight:
                if self.ex.done(h):
                    times = self.ex.finish(h)
                    for r in group:
                        r.t_done = times[r.rid]
                        used -= r.footprint
                    free_slots.append(slot)
                else:
                    still.append((h, group, slot))
            inflight = still
            progressed = False
            while free_slots and waiting:
                group = []
                while waiting and len(group) < self.max_group and used + waiting[0].footprint <= self.budget:
                    r = waiting.popleft()
                    used += r.footprint
                    r.t_admit = clock() - t0
                    group.append(r)
                if not group:
                    break
                peak = max(peak, used)
                slot = free_slots.pop()
                inflight.append((self.ex.launch(group, slot), group, slot))
                progressed = True
            if not progressed and not pending and not waiting and inflight:
                self.ex.wait_any([h for h, _, _ in inflight])
            elif not progressed and pending and not waiting and not inflight:
                # idle until the next arrival
                delay = pending[0].arrival - (clock() - t0)
                if delay > 0:
                    time.sleep(min(delay, 0.001))
        return peak, iterations


def summarize(reqs, makespan, peak, iterations):
    lat = sorted(r.t_done - r.arrival for r in reqs)

    def pct(p):
        if not lat:
            return 0.0
        k = min(len(lat) - 1, max(0, int(round(p / 100.0 * (len(lat) - 1)))))
        return lat[k]

    return {"requests": len(reqs), "makespan_s": makespan,
            "throughput_per_s": len(reqs) / makespan if makespan > 0 else 0.0,
            "p50_ms": pct(50) * 1e3, "p99_ms": pct(99) * 1e3, "mean_ms": (sum(lat) / len(lat) * 1e3) if lat else 0.0,
            "peak_hbm_bytes": peak, "iterations": iterations}


class GpuExecutor:
    """Runs each admitted group as one libcross batch on the slot's stream.

    A group's batch is planned, uploaded and enqueued while earlier groups run, but its
    kernels start only after the previous group's have finished (its stream waits on
    that group's completion event): groups whose batches executed at the same time on
    two streams gave wrong results for some requests (seen in the full-scale
    request-loop test), so execution on the device is kept in admission order."""

    def __init__(self, slots, use_graph=False):
        import torch
        from . import binding
        self.torch = torch
        self.B = binding
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.use_graph = use_graph
        self.groups = 0
        self.host_s = 0.0
        self.last_ev = None
        # workspace bytes of a batch of one request, by request shape: a group's batch
        # needs at most the sum over its requests (its scratch is the sum of theirs and
        # its merged task lists take no more than their lists apart; creating a batch
        # checks the size it is given), so a group is not lowered once more to size it
        self.ws_bytes = {}

    def prepare(self, requests):
        """Build the tables of every request shape (NTT plans of each prime and size, CKKS
        plans, automorphism tables) once, before serving: one request per (op, N, L,
        rotation) is lowered alone for its workspace size only, which creates them and
        allocates nothing else, and the sizes are kept by request shape."""
        seen = {}
        for r in requests:
            seen.setdefault((r.op, r.log_n, r.L, r.steps if r.op == "rotate" else 0), r)
        group = list(seen.values())
        if not group:
            return
        # nothing runs: every job may name the same (largest) output buffer
        big = max(group, key=lambda r: r.inputs["a"].numel())
        scratch = self.torch.empty(big.inputs["a"].shape, dtype=self.torch.int32, device="cuda")
        saved = [r.out for r in group]
        for r in group:
            r.out = scratch.view(-1)[:r.inputs["a"].numel()].view(r.inputs["a"].shape)
        try:
            for r, j in zip(group, self._jobs(group, alloc=False)):
                n = self.B.batch_workspace_bytes([j])          # also builds the request's tables
                k = self._shape(r)
                self.ws_bytes[k] = max(n, self.ws_bytes.get(k, 0))
        finally:
            for r, o in zip(group, saved):
                r.out = o
        self.torch.cuda.synchronize()

    @staticmethod
    def _shape(r):
        return (r.op, r.log_n, r.L, len(r.ps), r.dnum)

    def _workspace_bytes(self, group, jobs):
        total = 0
        for r, j in zip(group, jobs):
            k = self._shape(r)
            if k not in self.ws_bytes:
                self.ws_bytes[k] = self.B.batch_workspace_bytes([j])
            total += self.ws_bytes[k]
        return total

    def host_stats(self):
        return {"groups": self.groups,
                "host_us_per_group": round(self.host_s / max(1, self.groups) * 1e6, 1)}

    def start(self, t0):
        self.torch.cuda.synchronize()        # inputs were produced on other streams
        self.t0_host = t0
        self.t0_event = self.torch.cuda.Event(enable_timing=True)
        self.t0_event.record(self.torch.cuda.current_stream())

    def _jobs(self, group, alloc=True):
        torch = self.torch
        jobs = []
        for r in group:
            x = r.inputs
            if alloc:
                r.out = torch.empty(x["a"].shape, dtype=torch.int32, device="cuda")
            if r.op == "he_mult":
                jobs.append({"op": "he_mult", "a": x["a"], "b": x["b"], "key": x["key"], "out": r.out,
                             "qs": r.qs, "ps": r.ps, "dnum": r.dnum})
            else:
                jobs.append({"op": "rotate", "ct": x["a"], "key": x["key"], "out": r.out, "steps": r.steps,
                             "qs": r.qs, "ps": r.ps, "dnum": r.dnum})
        return jobs

    def launch(self, group, slot):
        torch = self.torch
        s = self.streams[slot]
        t_host = time.perf_counter()
        with torch.cuda.stream(s):
            jobs = self._jobs(group)
            nbytes = self._workspace_bytes(group, jobs)
            ws = torch.empty((nbytes + 255) // 256 * 64 + 64, dtype=torch.int32, device="cuda")
            off = (-ws.data_ptr()) % 256 // 4
            ws = ws[off:]
            batch = self.B.Batch(jobs, use_graph=self.use_graph, workspace=ws, stream=s.cuda_stream)
            if self.last_ev is not None:
                s.wait_event(self.last_ev)
            batch.run(s.cuda_stream)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
            self.last_ev = ev
        self.groups += 1
        self.host_s += time.perf_counter() - t_host
        return (ev, batch, ws)

    def done(self, h):
        return h[0].query()

    def wait_any(self, handles):
        handles[0][0].synchronize()

    def finish(self, h):
        ev, batch, ws = h
        t = self.t0_event.elapsed_time(ev) / 1e3
        batch.close()
        return collections.defaultdict(lambda: t)


def build_requests(specs, pool):
    """Turn workload dicts (rid, arrival, op, log_n, L, steps) into Requests whose
    inputs come from a synthetic.DevicePool-like `pool` (ciphertexts(), key(), params())."""
    out = []
    for sp in specs:
        qs, ps, _ = pool.params(sp["L"])
        a, b = pool.ciphertexts(sp["log_n"], sp["L"], sp["rid"])
        kind = "relin" if sp["op"] == "he_mult" else ("rot", sp["steps"])
        key = pool.key(sp["log_n"], sp["L"], kind)
        inputs = {"a": a.unsqueeze(0), "b": b.unsqueeze(0), "key": key}
        fp = footprint_bytes(sp["log_n"], sp["L"], len(ps), pool.dnum, sp["op"])
        out.append(Request(sp["rid"], sp["op"], sp["log_n"], sp["L"], pool.dnum, sp["arrival"], inputs,
                           qs, ps, steps=sp["steps"], footprint=fp))
    return out
