"""Autotuner of execution choices, cached as JSON per device and workload.

Two kinds of choices:

* Bit-preserving knobs (``he_ctx_set_knob``): launch shapes and scheduling of
  the same arithmetic -- NTT tile width (sub-transforms per workgroup) and
  NTT phase chunking.  Any setting gives identical ciphertexts.
* Plan choices that the oracle replays: the baby-step count n1 of each dense
  layer (the paper notes that the baby-step/giant-step trade-off depends on
  the ciphertext counts; Methods, "Algorithmic and cryptographic
  optimizations"), whether the layer runs in the lazy-ModDown form (one
  ModDown per inner sum instead of one per baby step) and the rotate-and-sum
  form (sequential, or hoisted groups of rs_bits bits) change which key
  switches run or where they round, hence the output bits, so all three are
  recorded in the plan; and the batch size (requests per launch), chosen for
  throughput under a latency cap.

Every measurement times the real batched entry points on the device with
HIP events, on synthetic residues of the workload's shape.

python -m paper_2104_09164_amd.tune cfg3 [--batch 16] [--out DIR]
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_DIR = os.path.join(HERE, "tuning")

KNOB_SPACE = {"ntt_cols": [16, 32], "ntt_cols_b": [8, 16, 32], "ntt_chunk_mb": [0, 32, 64, 128, 256]}
# The lazy-ModDown form is chosen only when it is at least this much faster.
LAZY_MARGIN = 1.02


def n1_candidates(m: int, max_n1: int = 64) -> list[int]:
    """Powers of two dividing m (every valid baby-step count), up to max_n1."""
    return [1 << k for k in range(0, 16) if (1 << k) <= min(m, max_n1) and m % (1 << k) == 0]


def pick_min(table: dict) -> object:
    """Key with the smallest time (ties: first in insertion order)."""
    return min(table, key=lambda k: (table[k], list(table).index(k)))


def pick_batch(rates: dict, lat_ms: dict, cap_ms: float | None) -> int:
    """Largest throughput among batch sizes whose batch latency meets the cap."""
    ok = {b: r for b, r in rates.items() if cap_ms is None or lat_ms[b] <= cap_ms}
    if not ok:
        return min(rates)
    return max(ok, key=lambda b: (ok[b], -b))


def knob_grid(space: dict = KNOB_SPACE) -> list[dict]:
    keys = sorted(space)
    return [dict(zip(keys, vals)) for vals in itertools.product(*(space[k] for k in keys))]


def device_tag() -> str:
    import torch
    name = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return name


def path_for(workload: str, tag: str | None = None) -> str:
    return os.path.join(TUNING_DIR, f"{tag or device_tag()}_{workload}.json")


def load(workload: str, tag: str | None = None) -> dict | None:
    p = path_for(workload, tag)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        return json.load(f)


def apply_knobs(ctx, tuned: dict | None) -> None:
    if tuned:
        for k, v in tuned.get("knobs", {}).items():
            ctx.set_knob(k, int(v))


# ------------------------------------------------------------------ timing
def _time(fn, reps: int = 5, warmup: int = 2) -> float:
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def _residues(primes, n, prefix, seed):
    from . import synth
    return synth.uniform_residues(primes, n, prefix, seed)


def tune_ntt(ctx, items: int, reps: int = 5) -> tuple[dict, dict]:
    """Forward + inverse NTT over `items` ciphertexts' limbs at the top level."""
    import torch
    N, L1 = ctx.N, len(ctx.q)
    q = torch.tensor(ctx.q, dtype=torch.int64, device=ctx.device).view(1, L1, 1)
    g = torch.Generator(device=ctx.device).manual_seed(5)
    bufs = [(torch.randint(0, 2 ** 62, (2, L1, N), device=ctx.device, generator=g, dtype=torch.int64) % q)
            for _ in range(items)]
    halves = [b[h] for b in bufs for h in range(2)]
    groups = [halves[i:i + 64] for i in range(0, len(halves), 64)]

    def run():
        for gr in groups:
            ctx.ntt(gr, 0, L1, inverse=False)
        for gr in groups:
            ctx.ntt(gr, 0, L1, inverse=True)
    table = {}
    for knobs in knob_grid():
        for k, v in knobs.items():
            ctx.set_knob(k, v)
        table[json.dumps(knobs, sort_keys=True)] = _time(run, reps)
        print(f"[tune] ntt {knobs}: {table[json.dumps(knobs, sort_keys=True)]:.3f} ms", file=sys.stderr, flush=True)
    best = json.loads(pick_min(table))
    for k, v in best.items():
        ctx.set_knob(k, v)
    return best, table


def rs_candidates(m: int, n: int) -> list[int]:
    """Rotate-and-sum forms worth timing: sequential (0) and hoisted groups of
    2 .. min(6, log2(n/m)) bits (1 bit is the sequential form)."""
    total = (n // m).bit_length() - 1
    return [0] + list(range(2, min(6, total) + 1))


def build_context(plan, batch: int, n1_sets: list[list[int]], seed: int = 7):
    """Context with synthetic keys for every rotation step any candidate plan needs."""
    from . import he
    ctx = he.Context(plan.log_n, plan.q, plan.p, plan.alpha)
    max_n1 = max(max(s) for s in n1_sets)
    max_n2 = max(lay.m // min(s) for lay, s in zip(plan.layers, n1_sets))
    ctx.bind(batch, max_n1, max_n2)
    steps = set()
    for lay, cands in zip(plan.layers, n1_sets):
        for n1 in cands:
            for rs in rs_candidates(lay.m, lay.n):
                lay2 = type(lay)(lay.m, lay.n, n1, lay.level, lay.in_scale, lay.pt_scale, False, rs)
                steps.update(lay2.steps())
    N = 1 << plan.log_n
    allp = plan.q + plan.p
    rot = {s: _residues(allp, N, (plan.dnum, 2), seed + i) for i, s in enumerate(sorted(steps))}
    ctx.load_keys(_residues(allp, N, (plan.dnum, 2), seed - 1), rot)
    return ctx


def tune_n1(ctx, plan, batch: int, n1_sets: list[list[int]], reps: int = 3, preset_n1=None):
    """Per layer: time he_eval_dense_batch at every candidate (n1, lazy
    ModDown).  Returns the best n1 and flag per layer, the best flag at the
    preset's n1 (when it is a candidate) and the timing tables."""
    N = 1 << plan.log_n
    best_n1, best_qp, preset_qp, tables = [], [], [], []
    for li, (lay, cands) in enumerate(zip(plan.layers, n1_sets)):
        cts = [ctx.import_ct(_residues(plan.q[: lay.level + 1], N, (2,), 900 + b), lay.level, lay.in_scale)
               for b in range(batch)]
        outs = [ctx.new_ct(lay.level) for _ in range(batch)]
        bias = _residues(plan.q[: lay.level + 1], N, (), 400 + li)
        table = {}
        for qp in (False, True):
            primes = plan.q[: lay.level + 1] + (plan.p if qp else [])
            pts = _residues(primes, N, (lay.m,), 300 + li)
            for n1 in cands:
                if qp and n1 == 1:
                    continue                    # same launches as the plain form
                d = ctx.dense_load(lay.level, lay.m, lay.n, n1, pts, bias, lay.pt_scale, lay.bias_scale, qp=qp)
                table[(n1, qp)] = _time(lambda: ctx.eval_dense_batch(cts, d, outs), reps, 1)
                print(f"[tune] layer {li}: n1={n1} lazy_moddown={qp}: {table[(n1, qp)]:.3f} ms", file=sys.stderr,
                      flush=True)
                del d
        tables.append(table)
        n1, qp = pick_min(table)
        if qp and (n1, False) in table and table[(n1, False)] <= LAZY_MARGIN * table[(n1, True)]:
            qp = False                          # keep the ordinary form unless the lazy one clearly wins
        best_n1.append(n1)
        best_qp.append(qp)
        p = preset_n1[li] if preset_n1 else None
        preset_qp.append(p in {c for c, _ in table} and (p, True) in table
                         and table[(p, True)] * LAZY_MARGIN < table[(p, False)])
    return best_n1, best_qp, preset_qp, tables


def tune_rs(ctx, plan, batch: int, n1s: list[int], qps: list[bool], reps: int = 3):
    """Per layer, at its chosen n1 and form: time every rotate-and-sum form."""
    N = 1 << plan.log_n
    best, tables = [], []
    for li, (lay, n1, qp) in enumerate(zip(plan.layers, n1s, qps)):
        cts = [ctx.import_ct(_residues(plan.q[: lay.level + 1], N, (2,), 900 + b), lay.level, lay.in_scale)
               for b in range(batch)]
        outs = [ctx.new_ct(lay.level) for _ in range(batch)]
        bias = _residues(plan.q[: lay.level + 1], N, (), 400 + li)
        pts = _residues(plan.q[: lay.level + 1] + (plan.p if qp else []), N, (lay.m,), 300 + li)
        table = {}
        for rs in rs_candidates(lay.m, lay.n):
            d = ctx.dense_load(lay.level, lay.m, lay.n, n1, pts, bias, lay.pt_scale, lay.bias_scale, qp=qp,
                               rs_bits=rs)
            table[rs] = _time(lambda: ctx.eval_dense_batch(cts, d, outs), reps, 1)
            print(f"[tune] layer {li}: n1={n1} lazy_moddown={qp} rs_bits={rs}: {table[rs]:.3f} ms", file=sys.stderr,
                  flush=True)
            del d
        b = pick_min(table)
        if b and table[0] <= LAZY_MARGIN * table[b]:
            b = 0                               # keep the sequential form unless the hoisted one clearly wins
        best.append(b)
        tables.append(table)
    return best, tables


def tune_batch(ctx, plan, layers, batches: list[int], cap_ms: float | None, reps: int = 3):
    """Whole-network throughput (graph replay) at each batch size."""
    from .batch import NetworkRunner
    runner = NetworkRunner(ctx, plan, layers, max(batches))
    N = 1 << plan.log_n
    for b, ct in enumerate(runner.inputs):
        ct.buf.copy_(ctx.import_ct(_residues(plan.q, N, (2,), 700 + b), plan.L, plan.scale).buf)
    rates, lat = {}, {}
    for b in batches:
        g = runner.capture(b)
        ms = _time(g.replay, reps, 1)
        rates[b], lat[b] = 1000.0 * b / ms, ms
        print(f"[tune] batch {b}: {rates[b]:.1f} inferences/s", file=sys.stderr, flush=True)
    return pick_batch(rates, lat, cap_ms), rates, lat


def tune_kernel_bench(out_dir: str = TUNING_DIR) -> dict:
    """The kernel micro-benchmark's ring (N = 2^16, 24 + 8 limbs of 50 bits,
    64 ciphertexts): NTT launch knobs only (no plan choices)."""
    from . import he
    q, p = he.prime_chain(16, [50] * 24, [50] * 8)
    ctx = he.Context(16, q, p, 8)
    knobs, ntt_table = tune_ntt(ctx, items=64)
    res = {"device": device_tag(), "workload": "cfg2", "knobs": knobs, "measurements": {"ntt_ms": ntt_table}}
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, f"{res['device']}_cfg2.json"), "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
    return res


def tune_workload(name: str, batch: int, cap_ms: float | None = None, out_dir: str = TUNING_DIR,
                  batches=(1, 4, 8, 16, 32)) -> dict:
    from . import netplan
    plan = netplan.preset_plan(name)
    # n1 <= 64 and n2 = m / n1 <= 32 bound the baby and inner-sum workspaces
    n1_sets = [[n for n in n1_candidates(lay.m, 64) if lay.m // n <= 32] for lay in plan.layers]
    ctx = build_context(plan, max(max(batches), batch), n1_sets)
    knobs, ntt_table = tune_ntt(ctx, items=min(batch, 64))
    n1s, qps, qp_preset, n1_tables = tune_n1(ctx, plan, batch, n1_sets,
                                             preset_n1=[l.n1 for l in plan.layers])
    # the rotate-and-sum form, timed at the preset split (it follows the layer's m and n, not n1)
    rs_bits, rs_tables = tune_rs(ctx, plan, batch, [l.n1 for l in plan.layers], qp_preset)
    shapes = [(l.m, l.n, n1, qp, rs) for l, n1, qp, rs in zip(plan.layers, n1s, qps, rs_bits)]
    plan2 = netplan.plan_network(plan.log_n, plan.q, plan.p, plan.alpha, int(np.log2(plan.scale)), shapes)
    N = 1 << plan.log_n
    layers = [ctx.dense_load(l.level, l.m, l.n, l.n1,
                             _residues(plan.q[: l.level + 1] + (plan.p if l.qp else []), N, (l.m,), 300 + i),
                             _residues(plan.q[: l.level + 1], N, (), 400 + i), l.pt_scale, l.bias_scale, qp=l.qp,
                             rs_bits=l.rs_bits)
              for i, l in enumerate(plan2.layers)]
    bbest, rates, lat = tune_batch(ctx, plan2, layers, list(batches), cap_ms)
    res = {"device": device_tag(), "workload": name, "knobs": knobs, "n1": n1s, "qp": qps, "qp_preset": qp_preset,
           "rs_bits": rs_bits, "batch": bbest, "latency_cap_ms": cap_ms,
           "measurements": {"ntt_ms": ntt_table,
                            "dense_ms": [{f"{k[0]}{'q' if k[1] else ''}": v for k, v in t.items()}
                                         for t in n1_tables],
                            "rotate_sum_ms": [{str(k): v for k, v in t.items()} for t in rs_tables],
                            "batch_inferences_per_s": {str(k): v for k, v in rates.items()},
                            "batch_latency_ms": {str(k): v for k, v in lat.items()}}}
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, f"{res['device']}_{name}.json"), "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["cfg1", "cfg2", "cfg3", "cfg4"])
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--cap-ms", type=float, default=None)
    ap.add_argument("--out", default=TUNING_DIR)
    args = ap.parse_args()
    if args.workload == "cfg2":
        res = tune_kernel_bench(args.out)
        print(json.dumps({k: res[k] for k in ("device", "workload", "knobs")}), flush=True)
        return
    res = tune_workload(args.workload, args.batch, args.cap_ms, args.out)
    print(json.dumps({k: res[k] for k in ("device", "workload", "knobs", "n1", "qp", "qp_preset", "rs_bits", "batch")}),
          flush=True)


if __name__ == "__main__":
    main()
