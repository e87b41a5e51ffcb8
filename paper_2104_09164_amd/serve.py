"""Continuous-batching request loop for encrypted inference.

Requests for one or more encrypted networks arrive over time (each one an
input ciphertext from a different user; paper, Results: many users send
encrypted skeleton tensors to one cloud that holds the evaluation keys and
the cleartext model).  The loop keeps keys, plaintext diagonals and
in-flight ciphertexts resident on the device and:

  * admits a waiting request when a slot is free and the device-memory
    footprint of all admitted requests stays within the budget;
  * advances requests through the network's stages (dense, rescale, square,
    rescale, ...); each dispatch batches every admitted request of one network
    that waits at the same stage, up to the backend's batch limit, into one
    set of batched launches;
  * keeps at most `window` dispatches in flight on the device, so requests
    that arrive while the device is busy join later batches (continuous
    batching) instead of queueing behind whole inferences;
  * exports each result as soon as its last stage completes and records
    arrival, admission, first-dispatch and finish times.

The scheduler is backend-agnostic: a backend enqueues work and returns
pollable handles.  NetBackend drives the HIP library; tests drive the same
scheduler with a CPU stand-in and a simulated clock.  Batching never changes
a ciphertext: each request's result is bit-identical alone and in any mix.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    net: str
    payload: object                 # backend-specific input (host coefficient-form ciphertext)
    arrival: float
    admit: float | None = None
    start: float | None = None
    finish: float | None = None
    result: object = None
    error: str | None = None
    # scheduler state
    slot: int | None = None
    stage: int = 0
    pending: object = None          # handle of the last enqueued dispatch touching this request


class Backend:
    """Interface of one network's executor (all methods enqueue, none block)."""
    name: str = ""
    stages: list = []               # stage names, executed in order
    max_batch: int = 1
    slot_bytes: int = 0             # device footprint of one admitted request
    weight: float = 1.0             # the "largest" policy's weight of one ready request
    chain: bool = False             # dispatch a group's remaining stages back to back

    def acquire_slot(self) -> int | None: ...
    def release_slot(self, slot: int) -> None: ...
    def load(self, slot: int, payload) -> object: ...                # returns handle
    def run(self, stage: int, slots: list) -> object: ...            # returns handle
    def export(self, slot: int) -> object: ...                       # returns handle
    def done(self, handle) -> bool: ...
    def result(self, handle) -> object: ...


@dataclass
class Dispatch:
    backend: str
    stage: int
    reqs: list
    handle: object


class Scheduler:
    def __init__(self, backends: dict, budget_bytes: int, window: int = 3, clock=time.perf_counter,
                 per_network: bool = False, policy: str = "oldest", max_wait_s: float = 0.02):
        """window: dispatches in flight, over all networks, or per network
        when per_network is set (networks on their own streams then never
        wait for a slot held by another network's batch).  policy "oldest":
        the stage of the oldest ready request goes first; "largest": the
        stage with the most ready requests goes first (larger batches, more
        throughput under load) unless the oldest ready request has waited
        longer than max_wait_s since its arrival; a group counts its requests
        times its backend's `weight` (1 by default), so that a network whose
        requests take longer can be served first.  A backend with `chain` set
        runs a group's remaining stages from one dispatch."""
        self.backends = backends
        self.budget = budget_bytes
        self.window = window
        self.per_network = per_network
        self.policy = policy
        self.max_wait_s = max_wait_s
        self.clock = clock
        self.queue: collections.deque = collections.deque()     # arrived, not admitted
        self.active: dict = {k: [] for k in backends}           # admitted, unfinished
        self.exporting: list = []                               # (req, handle)
        self.inflight: collections.deque = collections.deque()  # Dispatch
        self.used_bytes = 0
        self.done: list = []
        self.batches: list = []                                 # (backend, stage, size) history
        self.dispatch_cpu_s = 0.0                               # host time spent enqueuing dispatches

    # ---------------------------------------------------------------- api
    def submit(self, req: Request) -> None:
        if req.net not in self.backends:
            req.error = f"unknown network {req.net}"
            req.finish = self.clock()
            self.done.append(req)
            return
        self.queue.append(req)

    def idle(self) -> bool:
        return not self.queue and not any(self.active.values()) and not self.exporting and not self.inflight

    def step(self) -> int:
        """One scheduling round; returns the number of dispatches enqueued."""
        self._retire()
        self._admit()
        n = 0
        while self.per_network or len(self.inflight) < self.window:
            d = self._pick()
            if d is None:
                break
            self.inflight.append(d)
            n += 1
        self._retire()
        return n

    # ------------------------------------------------------------ internal
    def _admit(self) -> None:
        keep = collections.deque()
        while self.queue:
            r = self.queue.popleft()
            be = self.backends[r.net]
            if self.used_bytes + be.slot_bytes > self.budget:
                keep.append(r)
                continue
            slot = be.acquire_slot()
            if slot is None:
                keep.append(r)
                continue
            r.slot = slot
            r.admit = self.clock()
            self.used_bytes += be.slot_bytes
            try:
                r.pending = be.load(slot, r.payload)
            except Exception as e:                       # a bad input fails only its own request
                self._fail(r, e)
                continue
            self.active[r.net].append(r)
        self.queue = keep

    def _pick(self) -> Dispatch | None:
        """Oldest-first: the stage of the oldest admitted request not already
        covered by an in-flight dispatch, batched with every request of that
        network waiting at the same stage."""
        best = None
        for name, reqs in self.active.items():
            if self.per_network and sum(d.backend == name for d in self.inflight) >= self.window:
                continue
            for r in reqs:
                if r.stage < len(self.backends[name].stages) and not self._busy(r):
                    if best is None or r.arrival < best.arrival:
                        best = r
                    break
        if best is None:
            return None
        if self.policy == "largest" and self.clock() - best.arrival <= self.max_wait_s:
            # the stage group with the most ready requests (ties: the oldest)
            count = {}
            for name, reqs in self.active.items():
                if self.per_network and sum(d.backend == name for d in self.inflight) >= self.window:
                    continue
                for r in reqs:
                    if r.stage < len(self.backends[name].stages) and not self._busy(r):
                        key = (name, r.stage)
                        n, first = count.get(key, (0, r))
                        count[key] = (n + 1, first)
            def score(v):
                be = self.backends[v[1].net]
                return (min(v[0], be.max_batch) * getattr(be, "weight", 1.0), -v[1].arrival)
            best = max(count.values(), key=score)[1]
        be = self.backends[best.net]
        stage = best.stage
        group = [r for r in self.active[best.net] if r.stage == stage and not self._busy(r)][: be.max_batch]
        now = self.clock()
        c0 = time.perf_counter()
        # a chained backend's group runs all its remaining stages from one
        # dispatch (enqueued in order on the backend's stream; no regrouping
        # between stages, no scheduling wait per stage)
        last = len(be.stages) - 1 if be.chain else stage
        try:
            for st in range(stage, last + 1):
                h = be.run(st, [r.slot for r in group])
                self.batches.append((best.net, st, len(group)))
        except Exception as e:
            for r in group:
                self._fail(r, e)
            return None
        self.dispatch_cpu_s += time.perf_counter() - c0
        for r in group:
            if r.start is None:
                r.start = now
            r.stage = last + 1
            r.pending = h
        return Dispatch(best.net, last, group, h)

    def _busy(self, r: Request) -> bool:
        """A request's next stage is dispatched only once its previous work
        (import or stage) has completed on the device, so requests that arrive
        or finish a stage meanwhile are gathered into the same next batch."""
        return r.pending is not None and not self.backends[r.net].done(r.pending)

    def _retire(self) -> None:
        keep = collections.deque()
        for d in self.inflight:
            be = self.backends[d.backend]
            if not be.done(d.handle):
                keep.append(d)
                continue
            if d.stage != len(be.stages) - 1:
                continue
            for r in d.reqs:                         # the request's last stage has completed
                if r.error is None and r.slot is not None:
                    try:
                        self.exporting.append((r, be.export(r.slot)))
                    except Exception as e:
                        self._fail(r, e)
        self.inflight = keep
        still = []
        for r, h in self.exporting:
            be = self.backends[r.net]
            if be.done(h):
                r.result = be.result(h)
                r.finish = self.clock()
                self._release(r)
                self.done.append(r)
            else:
                still.append((r, h))
        self.exporting = still

    def _release(self, r: Request) -> None:
        be = self.backends[r.net]
        if r in self.active[r.net]:
            self.active[r.net].remove(r)
        if r.slot is not None:
            be.release_slot(r.slot)
            self.used_bytes -= be.slot_bytes
            r.slot = None

    def _fail(self, r: Request, e: Exception) -> None:
        r.error = f"{type(e).__name__}: {e}"
        r.finish = self.clock()
        self._release(r)
        self.done.append(r)

    # ------------------------------------------------------------ metrics
    def metrics(self, t0: float | None = None, t1: float | None = None) -> dict:
        ok = [r for r in self.done if r.error is None]
        lat = np.array([r.finish - r.arrival for r in ok]) if ok else np.zeros(0)
        out = {"completed": len(ok), "failed": len(self.done) - len(ok)}
        if len(lat):
            out.update({"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                        "mean_ms": float(lat.mean() * 1e3)})
            t0 = min(r.arrival for r in ok) if t0 is None else t0
            t1 = max(r.finish for r in ok) if t1 is None else t1
            out["inferences_per_s"] = len(ok) / max(t1 - t0, 1e-9)
        for name in self.backends:
            sizes = [s for n, _, s in self.batches if n == name]
            if sizes:
                out[f"{name}_mean_batch"] = float(np.mean(sizes))
        out["dispatches"] = len(self.batches)
        out["dispatch_host_ms_mean"] = 1e3 * self.dispatch_cpu_s / max(1, len(self.batches))
        return out


def run_arrivals(sched: Scheduler, arrivals: list, clock=time.perf_counter, sleep=time.sleep,
                 timeout_s: float = 600.0) -> None:
    """Feed requests at their arrival times (seconds relative to the start)
    and run the loop until every request finished.  `arrivals` is sorted by
    Request.arrival (relative); arrival times are rebased to the clock."""
    t0 = clock()
    i = 0
    pending = list(arrivals)
    for r in pending:
        r.arrival += t0
    while i < len(pending) or not sched.idle():
        now = clock()
        if now - t0 > timeout_s:
            raise TimeoutError("serving loop did not drain")
        while i < len(pending) and pending[i].arrival <= now:
            sched.submit(pending[i])
            i += 1
        n = sched.step()
        if n == 0 and (i < len(pending) or not sched.idle()):
            nxt = pending[i].arrival - clock() if i < len(pending) else 0.0
            sleep(min(max(nxt, 0.0), 2e-4))


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given total rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, count))


# ------------------------------------------------------------------- GPU
SCALE_RTOL_LOG2 = -30      # the library's rule: operand scales agree within a relative 2^-30


def check_payload(plan, payload) -> None:
    """Rejects a request input that would fail a whole batched launch: the
    batched entry points check level and scale over every item of a call
    (HE_ELEVEL / HE_ESCALE for all of them), so an input at another level or
    scale must be refused when it is admitted, where it fails only its own
    request.  payload = (coefficient-form residues [2][L+1][N] uint64, level,
    scale); raises ValueError."""
    coeff, level, scale = payload
    N = 1 << plan.log_n
    if level != plan.L:
        raise ValueError(f"input at level {level}, the network starts at level {plan.L}")
    a = np.asarray(coeff)
    if a.dtype != np.uint64 or a.shape != (2, plan.L + 1, N):
        raise ValueError(f"input array {a.dtype} {a.shape}, expected uint64 {(2, plan.L + 1, N)}")
    if not (np.isfinite(scale) and abs(scale - plan.scale) <= np.ldexp(abs(plan.scale), SCALE_RTOL_LOG2)):
        raise ValueError(f"input scale {scale!r}, the network expects {plan.scale!r}")


def bucket_sizes(max_batch: int) -> list[int]:
    """Batch sizes that have a captured graph per stage: 1, 2, 3, 4, 6, 8, 12,
    16, 24, 32, ... up to max_batch (a dispatch of g requests replays the
    smallest one >= g; the padding items are computed and discarded)."""
    out, b = [], 1
    while b < max_batch:
        out.append(b)
        if b >= 2 and b + b // 2 < max_batch:
            out.append(b + b // 2)
        b *= 2
    out.append(max_batch)
    return sorted(set(out))


class NetBackend(Backend):
    """One encrypted network on the HIP library: slot pool of device
    ciphertext buffers for every stage, batched launches, async import/export.

    graphs=True: every (stage, bucket size) is captured once as a HIP graph
    over per-stage staging ciphertexts; a dispatch copies its requests' stage
    inputs into the staging inputs (device to device), replays the graph of
    the smallest bucket that holds them, and copies the staging outputs into
    the requests' slots.  The arithmetic is the batched calls' (bit for bit);
    one graph launch replaces the stage's dozens of kernel launches."""

    def __init__(self, name: str, ctx, plan, layers: list, max_batch: int, slots: int, own_stream: bool = False,
                 graphs: bool = True):
        import torch
        from . import he
        self.torch, self.he = torch, he
        self.name, self.ctx, self.plan, self.layers = name, ctx, plan, layers
        # Each network may get its own stream (default priority) so that two
        # networks' batches overlap on the device.
        self.stream = torch.cuda.Stream(device=ctx.device) if own_stream else torch.cuda.current_stream(ctx.device)
        with torch.cuda.stream(self.stream):
            ctx.use_current_stream()
        self.max_batch = max_batch
        self.stages = []
        for li in range(len(plan.layers)):
            self.stages += [("dense", li), ("rescale", li)]
            if li + 1 < len(plan.layers):
                self.stages += [("square", li), ("rescale", li)]
        L, N = plan.L, 1 << plan.log_n
        self.N = N
        self.free = list(range(slots))[::-1]
        # per slot: input ct, one output ct per stage, coefficient staging buffers
        self.bufs = []
        lv = L
        levels = []
        for kind, _ in self.stages:
            if kind == "rescale":
                lv -= 1
            levels.append(lv)
        self.out_level = levels[-1]
        for _ in range(slots):
            s = {"in": ctx.new_ct(L, plan.scale), "stage": [ctx.new_ct(l) for l in levels],
                 "coef_in": torch.empty(2 * (L + 1) * N, dtype=torch.int64, device=ctx.device),
                 "coef_out": torch.empty(2 * (self.out_level + 1) * N, dtype=torch.int64, device=ctx.device),
                 # pinned host staging, allocated once per slot (a slot's buffers are
                 # reused only after its request has finished)
                 "host_in": torch.empty(2 * (L + 1) * N, dtype=torch.int64, pin_memory=True),
                 "host_out": torch.empty(2 * (self.out_level + 1) * N, dtype=torch.int64, pin_memory=True)}
            self.bufs.append(s)
        self.slot_bytes = sum(ctx.ct_bytes(l) for l in levels) + ctx.ct_bytes(L) + \
            8 * 2 * (L + 1) * N + 8 * 2 * (self.out_level + 1) * N
        self.levels = levels
        self.graphs = None
        if graphs:
            self._capture(L)

    def _stage_call(self, stage, ins, outs):
        kind, li = self.stages[stage]
        if kind == "dense":
            self.ctx.eval_dense_batch(ins, self.layers[li], outs)
        elif kind == "rescale":
            self.ctx.rescale_batch(ins, outs)
        else:
            self.ctx.square_batch(ins, outs)

    def _capture(self, L):
        """Staging ciphertexts per stage and one graph per (stage, bucket)."""
        torch, ctx = self.torch, self.ctx
        in_levels = [L] + self.levels[:-1]
        self.buckets = bucket_sizes(self.max_batch)
        self.stage_in = [[ctx.new_ct(lv, self.plan.scale) for _ in range(self.max_batch)] for lv in in_levels]
        self.stage_out = [[ctx.new_ct(lv) for _ in range(self.max_batch)] for lv in self.levels]
        for c in [c for row in self.stage_in for c in row]:
            c.buf.zero_()                    # valid residues until the first dispatch overwrites them
        # staging inputs carry the levels and scales the stages expect
        scale = self.plan.scale
        for st, (kind, li) in enumerate(self.stages):
            for c in self.stage_in[st]:
                c.scale = scale
            self._stage_call(st, self.stage_in[st][:1], self.stage_out[st][:1])
            scale = self.stage_out[st][0].scale
        torch.cuda.synchronize(ctx.device)
        self.graphs = {}
        side = torch.cuda.Stream(device=ctx.device)
        side.wait_stream(torch.cuda.current_stream(ctx.device))
        with torch.cuda.stream(side):
            for st in range(len(self.stages)):
                for c in self.stage_in[st]:
                    c.level, c.scale = in_levels[st], self.stage_in[st][0].scale
                for b in self.buckets:
                    ctx.use_current_stream()
                    self._stage_call(st, self.stage_in[st][:b], self.stage_out[st][:b])   # warm-up
                    side.synchronize()
                    g = ctx.capture(lambda: self._stage_call(st, self.stage_in[st][:b], self.stage_out[st][:b]))
                    self.graphs[(st, b)] = g
        torch.cuda.current_stream(ctx.device).wait_stream(side)
        with torch.cuda.stream(self.stream):
            ctx.use_current_stream()

    def _event(self):
        e = self.torch.cuda.Event()
        e.record(self.stream)
        return e

    def acquire_slot(self):
        return self.free.pop() if self.free else None

    def release_slot(self, slot):
        self.free.append(slot)

    def load(self, slot, payload):
        with self.torch.cuda.stream(self.stream):
            return self._load(slot, payload)

    def run(self, stage, slots):
        with self.torch.cuda.stream(self.stream):
            return self._run(stage, slots)

    def export(self, slot):
        with self.torch.cuda.stream(self.stream):
            return self._export(slot)

    def _load(self, slot, payload):
        check_payload(self.plan, payload)
        coeff, level, scale = payload
        b = self.bufs[slot]
        b["host_in"].numpy()[:] = np.ascontiguousarray(coeff).view(np.int64).reshape(-1)
        b["coef_in"].copy_(b["host_in"], non_blocking=True)
        ct = b["in"]
        c = ct._c()
        rc = self.he.lib().he_ct_from_coeff_dev(self.ctx.h, self.he.C.c_void_p(b["coef_in"].data_ptr()), level,
                                                scale, self.he.C.byref(c))
        if rc:
            self.stream.synchronize()            # the slot's staging copy has landed before the slot is reused
            raise self.he.HeError(rc, "he_ct_from_coeff_dev")
        ct.level, ct.scale = level, scale
        return self._event()

    def _src(self, slot, stage):
        return self.bufs[slot]["in"] if stage == 0 else self.bufs[slot]["stage"][stage - 1]

    def _run(self, stage, slots):
        ins = [self._src(s, stage) for s in slots]
        outs = [self.bufs[s]["stage"][stage] for s in slots]
        if self.graphs is None:
            self._stage_call(stage, ins, outs)
            return self._event()
        b = next(x for x in self.buckets if x >= len(slots))
        for c, st in zip(ins, self.stage_in[stage]):
            st.buf.copy_(c.buf, non_blocking=True)
        self.graphs[(stage, b)].replay()
        for c, st in zip(outs, self.stage_out[stage]):
            c.buf.copy_(st.buf, non_blocking=True)
            c.level, c.scale = st.level, st.scale
        return self._event()

    def _export(self, slot):
        b = self.bufs[slot]
        ct = b["stage"][-1]
        c = ct._c()
        rc = self.he.lib().he_ct_to_coeff_dev(self.ctx.h, self.he.C.byref(c),
                                              self.he.C.c_void_p(b["coef_out"].data_ptr()))
        if rc:
            raise self.he.HeError(rc, "he_ct_to_coeff_dev")
        host = b["host_out"]
        host.copy_(b["coef_out"], non_blocking=True)
        return (self._event(), host, ct.level, ct.scale)

    def done(self, handle):
        ev = handle[0] if isinstance(handle, tuple) else handle
        return ev.query()

    def result(self, handle):
        _, host, level, scale = handle
        return (host.numpy().view(np.uint64).reshape(2, level + 1, self.N).copy(), level, scale)
