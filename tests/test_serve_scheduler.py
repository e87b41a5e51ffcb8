"""Serving loop on the CPU: scheduler logic with an oracle-backed stand-in backend.

The stand-in implements the backend interface with the oracle at tiny N and a
simulated single device (work completes at max(device free, now) + cost), so
admission, continuous batching, failure isolation and latency accounting are
tested without a GPU, and every result is checked bit for bit against the
oracle evaluating that request alone.
"""
import numpy as np
import pytest

from oracle import ckks, params, plan
from paper_2104_09164_amd import serve, synth


class SimClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class OracleBackend(serve.Backend):
    def __init__(self, name, o, keys, layers, clock, slots=8, max_batch=4, base=1e-3, per_item=2e-4,
                 fail_payload=None):
        self.name, self.o, self.keys, self.layers, self.clock = name, o, keys, layers, clock
        self.stages = []
        for li in range(len(layers)):
            self.stages += [("dense", li), ("rescale", li)]
            if li + 1 < len(layers):
                self.stages += [("square", li), ("rescale", li)]
        self.max_batch, self.base, self.per_item = max_batch, base, per_item
        self.free = list(range(slots))[::-1]
        self.cts = {}
        self.busy_until = 0.0
        self.slot_bytes = 1000
        self.fail_payload = fail_payload
        self.max_seen_batch = 0

    def _finish_at(self, n):
        t = max(self.busy_until, self.clock.now()) + self.base + self.per_item * n
        self.busy_until = t
        return t

    def acquire_slot(self):
        return self.free.pop() if self.free else None

    def release_slot(self, slot):
        self.cts.pop(slot, None)
        self.free.append(slot)

    def load(self, slot, payload):
        if payload is self.fail_payload:
            raise ValueError("corrupt input")
        self.cts[slot] = payload.copy()
        return self._finish_at(1)

    def run(self, stage, slots):
        kind, li = self.stages[stage]
        self.max_seen_batch = max(self.max_seen_batch, len(slots))
        for s in slots:
            ct = self.cts[s]
            if kind == "dense":
                ct = self.o.dense(ct, self.layers[li], self.keys)
            elif kind == "rescale":
                ct = self.o.rescale(ct)
            else:
                ct = self.o.square(ct, self.keys)
            self.cts[s] = ct
        return self._finish_at(len(slots))

    def export(self, slot):
        return (self._finish_at(0), self.cts[slot].copy())

    def done(self, handle):
        t = handle[0] if isinstance(handle, tuple) else handle
        return self.clock.now() >= t

    def result(self, handle):
        return handle[1]


@pytest.fixture(scope="module")
def net(oracle_lib):
    pr = params.make(6, [50, 40, 40, 40, 40], [50, 50], 2, 30)
    o = ckks.Oracle(pr)
    shapes = [(4, 16, 2), (2, 4, 2)]
    keys = o.keygen(1, ckks.network_steps(shapes))
    Ws, bs = synth.network_weights(shapes, 0.1)
    layers = o.prepare_network(Ws, bs, [s[2] for s in shapes])
    return pr, o, keys, layers, shapes


def requests(net, count, times, name="small"):
    pr, o, keys, _, shapes = net
    reqs = []
    for r in range(count):
        x = synth.request_input(shapes[0][1], r)
        ct = o.encrypt(plan.input_slots(x, pr.slots), keys.pk, synth.request_seed(r))
        reqs.append(serve.Request(r, name, ct, float(times[r])))
    return reqs


def expected(net, ct):
    pr, o, keys, layers, _ = net
    return o.eval_network(ct, layers, keys)


def test_results_bit_identical_alone_and_in_mix(net):
    clock = SimClock()
    pr, o, keys, layers, _ = net
    be = OracleBackend("small", o, keys, layers, clock)
    sched = serve.Scheduler({"small": be}, budget_bytes=10 ** 9, clock=clock.now)
    times = serve.poisson_arrivals(rate=2000.0, count=10, seed=5)
    reqs = requests(net, 10, times)
    inputs = {r.rid: r.payload.copy() for r in reqs}
    serve.run_arrivals(sched, reqs, clock=clock.now, sleep=clock.sleep)
    assert len(sched.done) == 10 and all(r.error is None for r in sched.done)
    for r in sched.done:
        want = expected(net, inputs[r.rid])
        assert np.array_equal(r.result.data, want.data) and r.result.scale == want.scale
        assert r.arrival <= r.admit <= r.start <= r.finish
    assert be.max_seen_batch > 1                       # requests shared launches
    m = sched.metrics()
    assert m["completed"] == 10 and m["p99_ms"] >= m["p50_ms"] > 0


def test_low_rate_runs_one_at_a_time(net):
    clock = SimClock()
    pr, o, keys, layers, _ = net
    be = OracleBackend("small", o, keys, layers, clock)
    sched = serve.Scheduler({"small": be}, budget_bytes=10 ** 9, clock=clock.now)
    reqs = requests(net, 3, [0.0, 1.0, 2.0])
    serve.run_arrivals(sched, reqs, clock=clock.now, sleep=clock.sleep)
    assert be.max_seen_batch == 1
    assert all(r.error is None for r in sched.done)


def test_admission_respects_memory_budget(net):
    clock = SimClock()
    pr, o, keys, layers, _ = net
    be = OracleBackend("small", o, keys, layers, clock, slots=16)
    sched = serve.Scheduler({"small": be}, budget_bytes=2 * be.slot_bytes, clock=clock.now)
    peak = []
    orig = sched._admit

    def admit():
        orig()
        peak.append(sched.used_bytes)
    sched._admit = admit
    reqs = requests(net, 6, np.zeros(6))
    serve.run_arrivals(sched, reqs, clock=clock.now, sleep=clock.sleep)
    assert max(peak) <= 2 * be.slot_bytes
    assert sum(r.error is None for r in sched.done) == 6
    assert sched.used_bytes == 0 and len(be.free) == 16


def test_failure_is_isolated(net):
    clock = SimClock()
    pr, o, keys, layers, _ = net
    reqs = requests(net, 4, [0.0, 0.0, 0.001, 0.001])
    be = OracleBackend("small", o, keys, layers, clock, fail_payload=reqs[1].payload)
    sched = serve.Scheduler({"small": be}, budget_bytes=10 ** 9, clock=clock.now)
    inputs = {r.rid: r.payload.copy() for r in reqs}
    serve.run_arrivals(sched, reqs, clock=clock.now, sleep=clock.sleep)
    by = {r.rid: r for r in sched.done}
    assert by[1].error and "corrupt" in by[1].error
    for rid in (0, 2, 3):
        assert by[rid].error is None
        assert np.array_equal(by[rid].result.data, expected(net, inputs[rid]).data)
    assert sched.metrics()["failed"] == 1 and len(be.free) == 8


def test_unknown_network_rejected(net):
    clock = SimClock()
    pr, o, keys, layers, _ = net
    sched = serve.Scheduler({"small": OracleBackend("small", o, keys, layers, clock)}, 10 ** 9, clock=clock.now)
    sched.submit(serve.Request(0, "huge", None, 0.0))
    assert sched.done[0].error and sched.idle()


def test_two_networks_interleave(net):
    clock = SimClock()
    pr, o, keys, layers, _ = net
    a = OracleBackend("small", o, keys, layers, clock, max_batch=3)
    b = OracleBackend("large", o, keys, layers, clock, max_batch=3)
    sched = serve.Scheduler({"small": a, "large": b}, budget_bytes=10 ** 9, clock=clock.now)
    times = serve.poisson_arrivals(rate=3000.0, count=8, seed=9)
    reqs = requests(net, 8, times)
    for r in reqs[::3]:
        r.net = "large"
    inputs = {r.rid: r.payload.copy() for r in reqs}
    serve.run_arrivals(sched, reqs, clock=clock.now, sleep=clock.sleep)
    assert len(sched.done) == 8 and all(r.error is None for r in sched.done)
    for r in sched.done:
        assert np.array_equal(r.result.data, expected(net, inputs[r.rid]).data)
    assert {n for n, _, _ in sched.batches} == {"small", "large"}
    assert max(s for _, _, s in sched.batches) <= 3


def test_late_retirement_exports_once(net):
    """With zero-cost work and a wide window, several stages of one request are
    enqueued before any dispatch retires; only the dispatch of its last stage
    may trigger the export, so every request finishes exactly once."""
    clock = SimClock()
    pr, o, keys, layers, _ = net
    be = OracleBackend("small", o, keys, layers, clock, base=0.0, per_item=0.0)
    sched = serve.Scheduler({"small": be}, budget_bytes=10 ** 9, window=8, clock=clock.now)
    reqs = requests(net, 3, [0.0, 0.0, 0.0])
    inputs = {r.rid: r.payload.copy() for r in reqs}
    serve.run_arrivals(sched, reqs, clock=clock.now, sleep=clock.sleep, timeout_s=5.0)
    assert sorted(r.rid for r in sched.done) == [0, 1, 2]
    for r in sched.done:
        assert np.array_equal(r.result.data, expected(net, inputs[r.rid]).data)


@pytest.mark.parametrize("per_network", [False, True])
def test_dispatch_window_global_or_per_network(net, per_network):
    """window = 1: over all networks, one dispatch in flight at a time; per
    network, each network (its own stream, here its own simulated device) keeps
    one in flight, so both run at once.  Results bit for bit either way."""
    clock = SimClock()
    pr, o, keys, layers, _ = net
    a = OracleBackend("small", o, keys, layers, clock, max_batch=2)
    b = OracleBackend("large", o, keys, layers, clock, max_batch=2)
    sched = serve.Scheduler({"small": a, "large": b}, budget_bytes=10 ** 9, window=1, clock=clock.now,
                            per_network=per_network)
    seen = []
    step = sched.step

    def recording_step():
        n = step()
        seen.append([d.backend for d in sched.inflight])
        return n

    sched.step = recording_step
    reqs = requests(net, 6, [0.0] * 6)
    for r in reqs[1::2]:
        r.net = "large"
    inputs = {r.rid: r.payload.copy() for r in reqs}
    serve.run_arrivals(sched, reqs, clock=clock.now, sleep=clock.sleep)
    assert len(sched.done) == 6 and all(r.error is None for r in sched.done)
    for r in sched.done:
        assert np.array_equal(r.result.data, expected(net, inputs[r.rid]).data)
    if per_network:
        assert max(len(s) for s in seen) == 2
        assert all(s.count("small") <= 1 and s.count("large") <= 1 for s in seen)
    else:
        assert max(len(s) for s in seen) == 1


def test_check_payload_rejects_what_fails_a_batch():
    """A request input at another level, scale or shape is refused at
    admission (it would make the batched launch fail for every request in
    it); a valid one passes."""
    from paper_2104_09164_amd import netplan
    pr = params.make(10, [50, 40, 40, 40, 40], [50, 50], 2, 30)
    npl = netplan.plan_network(pr.log_n, pr.q, pr.p, pr.alpha, 30, [(8, 64, 4), (2, 8, 2)])
    N, L = pr.n, pr.L
    good = np.zeros((2, L + 1, N), dtype=np.uint64)
    serve.check_payload(npl, (good, L, npl.scale))
    serve.check_payload(npl, (good, L, npl.scale * (1 + 2.0 ** -32)))
    bad = [(good, L - 1, npl.scale),                                # level
           (good, L, npl.scale * (1 + 2.0 ** -20)),                 # scale beyond 2^-30 relative
           (good, L, float("nan")),
           (good[:, :L], L, npl.scale),                             # limbs
           (good.astype(np.int64), L, npl.scale),                   # dtype
           (np.zeros((2, L + 1, N // 2), dtype=np.uint64), L, npl.scale)]
    for b in bad:
        with pytest.raises(ValueError):
            serve.check_payload(npl, b)


@pytest.mark.parametrize("policy,max_wait,size", [("oldest", 1.0, 1), ("largest", 1.0, 3), ("largest", 0.0, 1)])
def test_policy_largest_group_first(net, policy, max_wait, size):
    """One request is a stage ahead of three newer ones.  Oldest-first runs
    its stage alone; largest-first runs the three together, unless the older
    request has waited longer than the cap.  Results bit for bit either way."""
    clock = SimClock()
    pr, o, keys, layers, _ = net
    be = OracleBackend("small", o, keys, layers, clock, per_item=0.0)
    sched = serve.Scheduler({"small": be}, budget_bytes=10 ** 9, window=1, clock=clock.now,
                            policy=policy, max_wait_s=max_wait)
    reqs = requests(net, 4, [0.0] * 4)
    inputs = {r.rid: r.payload.copy() for r in reqs}
    sched.submit(reqs[0])
    sched.step()                        # admitted, its import in flight
    clock.sleep(0.002)
    assert sched.step() == 1 and sched.batches[-1] == ("small", 0, 1)
    for r in reqs[1:]:
        sched.submit(r)
    sched.step()                        # admitted behind the in-flight stage
    clock.sleep(0.01)
    assert sched.step() == 1
    assert sched.batches[-1][2] == size
    serve.run_arrivals(sched, [], clock=clock.now, sleep=clock.sleep, timeout_s=5.0)
    assert sorted(r.rid for r in sched.done) == [0, 1, 2, 3]
    for r in sched.done:
        assert r.error is None
        assert np.array_equal(r.result.data, expected(net, inputs[r.rid]).data)


def test_chained_backend_runs_all_stages_per_dispatch(net):
    """A chained backend runs each group's stages back to back from one
    dispatch: every request is dispatched once (its group at stage 0 runs to
    the end), the batches record every stage, and the results are the
    oracle's bit for bit."""
    clock = SimClock()
    pr, o, keys, layers, _ = net
    be = OracleBackend("small", o, keys, layers, clock)
    be.chain = True
    sched = serve.Scheduler({"small": be}, budget_bytes=10 ** 9, clock=clock.now, policy="largest")
    times = serve.poisson_arrivals(rate=2000.0, count=8, seed=7)
    reqs = requests(net, 8, times)
    inputs = {r.rid: r.payload.copy() for r in reqs}
    started = []
    pick = sched._pick

    def recording_pick():
        d = pick()
        if d is not None:
            started.append((d.stage, len(d.reqs)))
        return d
    sched._pick = recording_pick
    serve.run_arrivals(sched, reqs, clock=clock.now, sleep=clock.sleep)
    assert len(sched.done) == 8 and all(r.error is None for r in sched.done)
    for r in sched.done:
        assert np.array_equal(r.result.data, expected(net, inputs[r.rid]).data)
    nst = len(be.stages)
    assert all(st == nst - 1 for st, _ in started)               # one dispatch per group, to the last stage
    assert sum(n for _, n in started) == 8
    assert len(sched.batches) == nst * len(started)
