"""Benchmark: encrypted inferences/s of the large dense net, batched vs plain.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B] [--large-batch B]
                [--serve-rates 50,100,200,300,400] [--serve-requests 2000] [--serve-requests-top 10000]
                [--no-small] [--no-serve] [--no-ntt] [--no-ks] [--no-conv] [--no-client] [--no-cpu] ...

One step = one batched encrypted inference of B = 32 requests through the
whole large network (N=2^16, 11 limbs, P = 3 x 60b; dense 4096->256 ->
rescale -> square -> rescale -> dense 256->64 -> rescale -> square -> rescale
-> dense 64->2 -> rescale; every dense layer = hoisted baby-step rotations,
MultPlain inner sums, giant-step and rotate-and-sum key switches, bias, in the
committed tuned plan), replayed from a captured HIP graph, inputs resident in
HBM.  `value` is that leg's inferences/s.  Reported beside it, in the same
JSON line:
  * plain one-request-at-a-time inferences/s and p50/p99 latency of the large
    net (a batch of one replayed from its own graph; eager launches beside it);
  * the small net (N=2^15, 1024->128->2, 16 per launch) batched and plain,
    with its own roofline, and with the autotuner's baby-step counts;
  * the plain RNS-CKKS request (N=2^13, 256->64->2): one request at a time,
    p50/p99;
  * serving: Poisson arrivals at five rates, 70% small / 30% large requests,
    continuous batching, p50/p99 from arrival to exported result;
  * the NTT micro-benchmark (64 ciphertexts x 2 x 24 limbs at N=2^16,
    forward + inverse) in algorithmic HBM GB/s;
  * the key-switch micro-benchmark (the same 64 ciphertexts' shape, dnum = 3,
    32 random rotation steps; hoisted: one ModUp per ciphertext), with the
    whole pass's HBM roofline and its dominant kernel class;
  * the roofline of the headline step's dominant kernel class: the same step
    run eagerly with the library tracer on (HIP events around every launch on
    the library stream, algorithmic bytes per launch), plus the NTT leg's;
  * the CPU oracle, untuned, timed end to end on this host: one large-net
    request (cpu_baseline), and in cpu_protocol the small net (median of 3),
    the plain request at 1 thread and at all threads (median of 3) and the
    oracle's NTT throughput, with the CPU model and thread counts.
Inputs are seeded uniform residues (keys, plaintext diagonals, ciphertexts):
every kernel's work and memory traffic is independent of the residue values,
and the arithmetic of exactly these call sequences is checked bit for bit
against the oracle by the GPU tests.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "encrypted inferences/s + p50/p99 latency (batched vs plain); NTT HBM GB/s"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def residues(primes, n, prefix, seed):
    from paper_2104_09164_amd import synth
    return synth.uniform_residues(primes, n, prefix, seed)


def setup(plan, batch, seed=7):
    from paper_2104_09164_amd import he
    from paper_2104_09164_amd.batch import NetworkRunner
    ctx = he.Context(plan.log_n, plan.q, plan.p, plan.alpha)
    ctx.bind(batch, plan.max_n1(), plan.max_n2())
    allp = plan.q + plan.p
    N = 1 << plan.log_n
    steps = plan.steps()
    log(f"keys: relin + {len(steps)} rotation keys, dnum={plan.dnum}")
    relin = residues(allp, N, (plan.dnum, 2), seed)
    rot = {s: residues(allp, N, (plan.dnum, 2), seed + 1 + i) for i, s in enumerate(steps)}
    ctx.load_keys(relin, rot)
    del relin, rot
    layers = []
    for li, lay in enumerate(plan.layers):
        # lazy-ModDown layers hold their diagonals over Q_l u P
        pts = residues(plan.q[: lay.level + 1] + (plan.p if lay.qp else []), N, (lay.m,), seed + 100 + li)
        bias = residues(plan.q[: lay.level + 1], N, (), seed + 200 + li)
        layers.append(ctx.dense_load(lay.level, lay.m, lay.n, lay.n1, pts, bias, lay.pt_scale, lay.bias_scale,
                                     qp=lay.qp, rs_bits=lay.rs_bits))
    runner = NetworkRunner(ctx, plan, layers, batch)
    for b in range(batch):
        x = residues(plan.q, N, (2,), seed + 1000 + b)
        ct = ctx.import_ct(x, plan.L, plan.scale)
        runner.inputs[b].buf.copy_(ct.buf)
    return ctx, runner


def time_events(fn, reps, stream=None):
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


def ntt_leg(reps=10):
    """64 ciphertexts x 2 polys x 24 limbs of 50-bit primes at N=2^16, forward + inverse."""
    import torch
    from paper_2104_09164_amd import he
    log_n, items, limbs = 16, 64, 24
    q, p = he.prime_chain(log_n, [50] * limbs, [50] * 8)
    ctx = he.Context(log_n, q, p, 8)
    from paper_2104_09164_amd import tune
    tuned = tune.load("cfg2")                  # autotuned NTT launch knobs of this ring, if present
    tune.apply_knobs(ctx, tuned)
    N = 1 << log_n
    qt = torch.tensor(q, dtype=torch.int64, device="cuda").view(1, 1, limbs, 1)
    bufs = []
    g = torch.Generator(device="cuda").manual_seed(11)
    for _ in range(items):
        x = torch.randint(0, 2 ** 62, (1, 2, limbs, N), device="cuda", generator=g, dtype=torch.int64)
        bufs.append((x % qt).contiguous())
    # each item: 2 polys x 24 limbs, primes 0..23 repeated for both polys -> two calls of 24 limbs
    halves = [b.view(2, limbs, N)[h] for b in bufs for h in range(2)]
    groups = [halves[i:i + 64] for i in range(0, len(halves), 64)]

    def fwd():
        for gr in groups:
            ctx.ntt(gr, 0, limbs, inverse=False)

    def inv():
        for gr in groups:
            ctx.ntt(gr, 0, limbs, inverse=True)
    for _ in range(2):
        fwd()
        inv()
    torch.cuda.synchronize()
    tf = time_events(fwd, reps)
    ti = time_events(inv, reps)
    polys = items * 2 * limbs
    alg_bytes = polys * N * 8 * 2              # one read + one write of every word per transform
    f, i = float(np.median(tf)), float(np.median(ti))
    return {"workload": "64 ct x 2 x 24 limbs x 2^16 (50-bit primes)", "knobs": tuned.get("knobs") if tuned else None,
            "fwd_ms": f, "inv_ms": i,
            "fwd_gbs": alg_bytes / f / 1e6, "inv_gbs": alg_bytes / i / 1e6,
            "fwd_inv_gbs": 2 * alg_bytes / (f + i) / 1e6, "alg_bytes_per_transform": alg_bytes}


def fast_conv_leg(ctx, plan, reps):
    """The fast convolution (merge-and-conquer) at Table 1's 1D-CNN-64 conv3
    shape: 8 punctured inputs (pooled maps of 120 at stride 4, slot distance
    512, 16 channels each), load number 4: two merges of 4 ciphertexts, the
    multi-channel convolution of the 2 merged ciphertexts into 16 outputs,
    rotate-and-sum by 2 and 1, rescales; one request, random residues."""
    import torch
    from paper_2104_09164_amd.conv import FastConv
    N = 1 << plan.log_n
    c, f, dist, nP, n_in, n_out = 16, 3, 512, 4, 8, 16
    pre_g = [-p for p in range(nP)]
    baby = [nP * (k - f // 2) for k in range(f)]
    giant = [dist * l for l in range(c)]
    post = [2, 1]
    allp = plan.q + plan.p
    steps = sorted(set(pre_g + baby + giant + post) - {0})
    R = 2
    ctx.bind(R * max(n_in, n_out), 1, c)
    ctx.load_keys(None, {s: residues(allp, N, (plan.dnum, 2), 800 + i) for i, s in enumerate(steps)})
    pre = residues(plan.q, N, (nP, 1, nP, 1), 1900)
    pts = residues(plan.q[:-1], N, (c, n_out, n_in // nP, f), 1901)
    fc = FastConv(ctx, plan.L, nP, pre_g, pre, baby, giant, pts, post, plan.scale)
    del pre, pts
    cts = [ctx.import_ct(residues(plan.q, N, (2,), 1950 + i), plan.L, plan.scale) for i in range(n_in)]
    for _ in range(2):
        fc.run(cts)
    torch.cuda.synchronize()
    t = time_events(lambda: fc.run(cts), reps)
    cts_b = cts + [ctx.import_ct(residues(plan.q, N, (2,), 1970 + i), plan.L, plan.scale) for i in range(n_in)]
    fc.run(cts_b)
    torch.cuda.synchronize()
    tb = float(np.median(time_events(lambda: fc.run(cts_b), reps)))
    return {"batched": {"requests": R, "ms_per_call": tb, "ms_per_request": tb / R},
            "workload": (f"1D-CNN-64 conv3 shape, fast convolution: 8 punctured inputs (map 120 at stride {nP}, "
                         f"slot distance {dist}, {c} channels each), load number {nP}, 2 merged -> {n_out} outputs, "
                         f"kernel width {f}; N=2^{plan.log_n}, one request"),
            "ms_per_layer": float(np.median(t)),
            "paper_context_ms": {"ordinary_conv": 422, "fast_conv_total": 242,
                                 "note": "Table 1, 1D-CNN-64 conv3, 16-thread Xeon with SEAL; context only"}}


def conv_leg(reps=5):
    """The paper's multi-channel homomorphic convolution at the shape of Table
    1's 1D-CNN-64 conv2 (output map 240, 64 -> 128 channels, 16 per ciphertext
    so n_in = 4, n_out = 8, kernel width 3) on the small net's ring (N = 2^15,
    top level), one request: 8 baby rotations (hoisted per input), 4 x 8 x 16
    inner sums of 12 products, 8 x 15 giant rotations.  Random residues as
    keys, plaintexts and ciphertexts (the call sequence is tested bit for bit
    against the oracle at this shape)."""
    import torch
    from paper_2104_09164_amd import he, netplan, tune
    plan = netplan.preset_plan("cfg3")
    N, L1 = 1 << plan.log_n, len(plan.q)
    c, f, L, n_in, n_out = 16, 3, 240, 4, 8
    dist = 1 << (L - 1).bit_length()
    baby = [k - f // 2 for k in range(f)]
    giant = [dist * l for l in range(c)]
    R = 4                                      # requests per batched call
    ctx = he.Context(plan.log_n, plan.q, plan.p, plan.alpha)
    tune.apply_knobs(ctx, tune.load("cfg3"))
    ctx.bind(R * max(n_in, n_out), 1, c)
    allp = plan.q + plan.p
    steps = sorted(set(baby + giant) - {0})
    ctx.load_keys(None, {s: residues(allp, N, (plan.dnum, 2), 700 + i) for i, s in enumerate(steps)})
    pts = residues(plan.q, N, (c, n_out, n_in, f), 900)
    lt = ctx.linear_load(plan.L, baby, giant, pts, plan.scale)
    del pts
    cts = [ctx.import_ct(residues(plan.q, N, (2,), 950 + i), plan.L, plan.scale) for i in range(n_in)]
    outs = [ctx.new_ct(plan.L) for _ in range(n_out)]
    for _ in range(2):
        ctx.eval_linear(cts, lt, outs)
    torch.cuda.synchronize()
    t = time_events(lambda: ctx.eval_linear(cts, lt, outs), reps)
    ctx.trace_read()
    ctx.set_knob("trace", 1)
    ctx.eval_linear(cts, lt, outs)
    tab = ctx.trace_read()
    ctx.set_knob("trace", 0)
    ms = float(np.median(t))
    # R requests in one call: the plaintexts are read once per batch
    cts_b = [ctx.import_ct(residues(plan.q, N, (2,), 960 + i), plan.L, plan.scale) for i in range(R * n_in)]
    outs_b = [ctx.new_ct(plan.L) for _ in range(R * n_out)]
    ctx.eval_linear_batch(cts_b, lt, outs_b)
    torch.cuda.synchronize()
    tb = float(np.median(time_events(lambda: ctx.eval_linear_batch(cts_b, lt, outs_b), reps)))
    del lt, cts, outs, cts_b, outs_b
    torch.cuda.synchronize()
    fast = fast_conv_leg(ctx, plan, reps)
    return {"fast_conv": fast, "batched": {"requests": R, "ms_per_call": tb, "ms_per_request": tb / R},
            "workload": (f"1D-CNN-64 conv2 shape: map {L} (slot distance {dist}), 64 -> 128 channels, {c} per "
                         f"ciphertext (n_in {n_in}, n_out {n_out}), kernel width {f}; N=2^{plan.log_n}, "
                         f"{L1} limbs, one request"),
            "ms_per_layer": ms, "rotations": n_in * (f - 1) + n_out * (c - 1), "multplain": c * n_out * n_in * f,
            "classes": {k: {"launches": v[0], "ms": v[1], "gbs": v[2] / (v[1] * 1e-3) / 1e9 if v[1] > 0 else None}
                        for k, v in sorted(tab.items(), key=lambda kv: -kv[1][1])},
            "paper_context_ms": {"ordinary_conv": 409, "fast_conv_total": 390,
                                 "note": "Table 1, 1D-CNN-64 conv2, 16-thread Xeon with SEAL; context only"}}


def client_leg(reps=10, R=16):
    """Client side on the small net's ring (N = 2^15, 7 limbs): the end users'
    encode + public-key encryption of R request inputs at the top level, and
    the monitoring service's decryption + decode of R network outputs at the
    output level, each one batched call sequence.  Random residues as pk and
    as the ciphertexts, a random ternary sk (the timing does not depend on
    the key values; the calls are tested bit for bit against the oracle)."""
    import torch
    from paper_2104_09164_amd import he, netplan, synth, tune
    plan = netplan.preset_plan("cfg3")
    N = 1 << plan.log_n
    ctx = he.Context(plan.log_n, plan.q, plan.p, plan.alpha)
    tune.apply_knobs(ctx, tune.load("cfg3"))
    ctx.bind(1, 1, 1)
    pk = residues(plan.q, N, (2,), 1200)
    sk = np.random.default_rng(1201).integers(-1, 2, N).astype(np.int64)
    cl = ctx.client(R, pk=pk, sk=sk)
    xs = [synth.request_input(1024, r) for r in range(R)]
    z = torch.zeros((R, N // 2), dtype=torch.complex128)
    for r, x in enumerate(xs):
        z[r, :1024] = torch.from_numpy(x)
    z = z.cuda()
    noise = torch.from_numpy(np.stack([synth.encryption_noise(N, 1300 + r) for r in range(R)])).cuda()
    cts = [ctx.new_ct(plan.L) for _ in range(R)]
    lo = plan.out_level
    outs = [ctx.import_ct(residues(plan.q[: lo + 1], N, (2,), 1400 + r), lo, plan.scale) for r in range(R)]

    def enc():
        cl.encrypt(cl.encode(z, plan.scale, plan.L), noise, plan.L, plan.scale, outs=cts)

    def dec():
        cl.decode(cl.decrypt(outs), lo, plan.scale)

    for f in (enc, dec):
        f()
    torch.cuda.synchronize()
    te = float(np.median(time_events(enc, reps)))
    td = float(np.median(time_events(dec, reps)))
    ctx.trace_read()
    ctx.set_knob("trace", 1)
    enc()
    dec()
    tab = ctx.trace_read()
    ctx.set_knob("trace", 0)
    return {"workload": (f"N=2^{plan.log_n}: encode + encrypt at level {plan.L} ({plan.L + 1} limbs), decrypt + "
                         f"decode at level {lo}; {R} requests per batched call"),
            "requests": R, "encrypt_ms_per_call": te, "encrypt_us_per_request": te * 1e3 / R,
            "decrypt_ms_per_call": td, "decrypt_us_per_request": td * 1e3 / R,
            "classes": {k: {"launches": v[0], "ms": v[1], "gbs": v[2] / (v[1] * 1e-3) / 1e9 if v[1] > 0 else None}
                        for k, v in sorted(tab.items(), key=lambda kv: -kv[1][1])},
            "paper_context_ms": {"encrypt_per_sample": "22-25", "decrypt": 1.6,
                                 "note": "Results, time requirement, steps (iii) and (v); CPU with SEAL; context only"}}


def ks_leg(reps=3, items=64, n_steps=32):
    """Kernel micro-benchmark, key switching: 64 ciphertexts at N=2^16 with 24
    limbs of 50-bit primes, hybrid key switching with dnum = 3 (8 special
    primes), every ciphertext rotated by each of 32 random steps.

    Hoisted (the paper's hoisting, Methods "Algorithmic and cryptographic
    optimizations": the decomposition and base extension of c1 are common to
    every rotation of one ciphertext): one he_rotate_hoisted_batch call per
    pass, one ModUp per ciphertext for all 32 steps, then per step the inner
    product, ModDown and epilogue of all 64 ciphertexts; 2048 output
    ciphertexts (48 GiB) written.  Per step (the second figure): one call per
    step, so every (ciphertext, step) pays its own ModUp.  Rotation keys are
    resident (32 keys x 3 digits x 2 x 32 limbs x 2^16 words, with their
    Shoup companions 6.4 GB).

    Whole-pass HBM roofline of the hoisted pass: the algorithmic bytes of the
    whole pass (read the 64 ciphertexts and the 32 keys once, write the 2048
    rotated ciphertexts) over its time, against 8 TB/s."""
    import torch
    from paper_2104_09164_amd import he, synth
    log_n, limbs, K = 16, 24, 8
    q, p = he.prime_chain(log_n, [50] * limbs, [50] * K)
    ctx = he.Context(log_n, q, p, K)
    from paper_2104_09164_amd import tune
    tune.apply_knobs(ctx, tune.load("cfg2"))
    N = 1 << log_n
    dnum = -(-limbs // K)
    ctx.bind(items, 1, 1)
    steps = synth.rotation_steps_random(n_steps, N // 2)
    log(f"ks leg: {len(steps)} rotation keys, dnum={dnum}, {items} ciphertexts")
    rot = {s: residues(q + p, N, (dnum, 2), 500 + i) for i, s in enumerate(steps)}
    ctx.load_keys(None, rot)
    del rot
    qt = torch.tensor(q, dtype=torch.int64, device="cuda").view(1, limbs, 1)
    g = torch.Generator(device="cuda").manual_seed(13)
    cts = []
    for _ in range(items):
        ct = ctx.new_ct(limbs - 1, 2.0 ** 50)
        ct.buf.view(2, limbs, N).copy_(torch.randint(0, 2 ** 62, (2, limbs, N), device="cuda", generator=g,
                                                     dtype=torch.int64) % qt)
        cts.append(ct)
    outs_all = [ctx.new_ct(limbs - 1) for _ in range(items * n_steps)]

    def hoisted():
        ctx.rotate_hoisted_batch(cts, steps, outs_all)
    outs = outs_all[:items]

    def per_step():
        for st in steps:
            ctx.rotate_hoisted_batch(cts, [st], outs)
    res = {}
    for name, fn in (("hoisted", hoisted), ("per_step", per_step)):
        fn()
        torch.cuda.synchronize()
        ms = float(np.median(time_events(fn, reps)))
        ctx.trace_read()
        ctx.set_knob("trace", 1)
        fn()
        tab = ctx.trace_read()
        ctx.set_knob("trace", 0)
        res[name] = {"key_switches_per_s": items * n_steps / (ms * 1e-3), "ms_per_pass": ms,
                     "modups_per_pass": items if name == "hoisted" else items * n_steps,
                     "dominant_class": step_roofline(tab, 1)}
    ct_bytes = 2 * limbs * N * 8
    key_bytes = n_steps * dnum * 2 * (limbs + K) * N * 8
    alg = items * ct_bytes + key_bytes + items * n_steps * ct_bytes
    ms = res["hoisted"]["ms_per_pass"]
    achieved = alg / (ms * 1e-3) / 1e9
    out = {"workload": (f"{items} ct x N=2^16, 24 x 50-bit limbs, dnum={dnum} (8 x 50-bit special primes), "
                        f"{n_steps} random rotation steps; hoisted: one ModUp per ciphertext for all steps"),
           "key_switches_per_s": res["hoisted"]["key_switches_per_s"], "ms_per_pass": ms,
           "hoisted": res["hoisted"], "per_step": res["per_step"],
           "roofline": {"bound": "hbm", "scope": "whole hoisted pass (every launch of one call)",
                        "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "alg_bytes_per_pass": alg,
                        "alg_bytes_note": "read 64 ciphertexts and 32 keys once, write 2048 rotated ciphertexts"}}
    del ctx, cts, outs, outs_all
    torch.cuda.synchronize()
    return out


def ntt_roofline(nt):
    """Dominant kernel: the forward NTT, one he_ntt call = one phase-A and one
    phase-B launch over 1536 limb-polys of 2^16 words.  Algorithmic bytes =
    one read + one write of every word (16 B per coefficient); `traffic` is
    the rocprofv3 FETCH_SIZE + WRITE_SIZE of those two launches (calibrated by
    a 1 GiB copy), taken from profiles/ and dropped if the NTT source changed."""
    import hashlib
    polys = nt["alg_bytes_per_transform"] // (2 * 8 * 65536) // 2          # per call
    alg = polys * 65536 * 8 * 2
    t_call = nt["fwd_ms"] / 2 * 1e-3
    achieved = alg / t_call / 1e9
    traffic = None
    try:
        prof = json.load(open(os.path.join(ROOT, "profiles", "ntt_traffic.json")))
        src = open(os.path.join(ROOT, "paper_2104_09164_amd", "csrc", "ntt.hip"), "rb").read()
        if prof["kernel_source_sha256"] == hashlib.sha256(src).hexdigest() and prof["polys_per_call"] == polys:
            traffic = prof["fetch_bytes_per_call"] + prof["write_bytes_per_call"]
    except (OSError, KeyError, ValueError):
        traffic = None
    # the same launches against the integer VALU peak: logN / 2 butterflies per coefficient, and
    # the final reduction of every coefficient
    ops = polys * 65536 * (16 // 2 * OPS_BUTTERFLY + OPS_NTT_OUT)
    tops = ops / t_call / 1e12
    return {"bound": "hbm", "kernel": f"forward NTT N=2^16, one call = phase-A + phase-B launch over {polys} limb-polys",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic, "alg_bytes": alg, "ms_per_call": t_call * 1e3,
            "valu_view": {"achieved_tops": tops, "peak": VALU_PEAK_TOPS, "frac": tops / VALU_PEAK_TOPS,
                          "alg_ops_per_call": ops, "ops_per_butterfly": OPS_BUTTERFLY,
                          "ops_per_coefficient_out": OPS_NTT_OUT}}


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_inference_times(plan, threads, runs, seed=3):
    """The oracle (untuned) evaluating one request end to end through `plan`
    (the same layers, baby-step splits, lazy-ModDown flags and rotate-and-sum
    groups the GPU ran): dense -> rescale -> square -> rescale -> ... ->
    dense -> rescale.  Evaluation only: keys, plaintext diagonals, biases and
    the input ciphertext are random residues of their real shapes (the
    oracle's work does not depend on the values).  Returns (seconds per run,
    OpenMP threads used)."""
    from oracle import ckks, params as oparams
    from paper_2104_09164_amd import synth
    L = ckks.lib()
    used = L.orc_threads(threads)
    pr = oparams.Params(plan.log_n, plan.q, plan.p, plan.alpha, int(round(np.log2(plan.scale))))
    o = ckks.Oracle(pr)
    N = 1 << plan.log_n
    key = synth.uniform_residues(plan.q + plan.p, N, (plan.dnum, 2), seed)
    keys = ckks.Keys(None, None, key, {s: key for s in plan.steps()})
    lays = []
    for li, lay in enumerate(plan.layers):
        primes = plan.q[: lay.level + 1] + (plan.p if lay.qp else [])
        one = synth.uniform_residues(primes, N, (), seed + 10 + li)
        pts = np.ascontiguousarray(np.broadcast_to(one, (lay.m,) + one.shape))
        bias = synth.uniform_residues(plan.q[: lay.level + 1], N, (), seed + 20 + li)
        lays.append(ckks.DenseLayer(lay.m, lay.n, lay.n1, lay.level, pts, bias, lay.pt_scale, lay.bias_scale,
                                    lay.qp, lay.rs_bits))
    ct = ckks.Ciphertext(synth.uniform_residues(plan.q, N, (2,), seed + 30), plan.L, plan.scale)
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        o.eval_network(ct, lays, keys, progress=lambda li: log(f"  oracle layer {li} done"))
        ts.append(time.perf_counter() - t0)
    del lays, keys, o
    return ts, used


def oracle_ntt_gbs(threads, reps=3):
    """The oracle's negacyclic transform, forward then inverse, on one
    ciphertext of the key-switch ring (2 x 24 limbs of 50-bit primes at 2^16)
    in algorithmic GB/s (one read and one write of every word per transform)."""
    import ctypes as C
    from oracle import ckks, params as oparams
    from paper_2104_09164_amd import he, synth
    L = ckks.lib()
    used = L.orc_threads(threads)
    q, p = he.prime_chain(16, [50] * 24, [50] * 8)
    o = ckks.Oracle(oparams.Params(16, q, p, 8, 40))
    a = np.ascontiguousarray(synth.uniform_residues(q, 1 << 16, (2,), 17).reshape(48, 1 << 16))
    idx = np.array(list(range(24)) * 2, dtype=np.int32)
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        L.orc_ntt_roundtrip(o._h, 48, idx.ctypes.data_as(C.POINTER(C.c_int)), a.ctypes.data_as(C.POINTER(C.c_uint64)))
        ts.append(time.perf_counter() - t0)
    t = float(np.median(ts))
    alg = 2 * 48 * (1 << 16) * 8 * 2
    return {"workload": "1 ct x 2 x 24 limbs x 2^16 (50-bit primes), forward + inverse", "threads": used,
            "s_per_roundtrip": t, "gbs": alg / t / 1e9, "alg_bytes": alg}


def cpu_protocol(plans, gpu_plans_note):
    """The oracle timed on this host's cores: the large net once at all
    threads (the headline workload), the small net at all threads (median of
    3), the plain-request net at 1 thread and at all threads (median of 3),
    and the oracle's NTT throughput."""
    nproc = os.cpu_count() or 1
    out = {"cpu_model": cpu_model(), "nproc": nproc, "plans": gpu_plans_note}
    for name, runs, threads in (("cfg1", 3, (1, nproc)), ("cfg3", 3, (nproc,)), ("cfg4", 1, (nproc,))):
        r = {}
        for th in threads:
            log(f"cpu baseline: oracle {name}, {th} thread(s), {runs} run(s)")
            ts, used = oracle_inference_times(plans[name], th, runs)
            r[f"threads_{used}"] = {"s_per_inference": float(np.median(ts)), "runs_s": ts,
                                    "inferences_per_s": 1.0 / float(np.median(ts)),
                                    "statistic": "median of 3" if runs == 3 else "single run"}
        out[name] = r
    log("cpu baseline: oracle NTT")
    out["ntt"] = oracle_ntt_gbs(nproc)
    return out


KERNEL_LABEL = {
    "ntt_fwd_phaseA": "forward NTT, phase A (column transforms)",
    "ntt_fwd_phaseB": "forward NTT, phase B (row transforms)",
    "ntt_inv_phaseB": "inverse NTT, phase B (row transforms)",
    "ntt_inv_phaseA": "inverse NTT, phase A (column transforms, N^-1)",
    "ks_final": "key-switch epilogue ((u - conv) P^-1 + sigma(c0) + accumulators)",
    "ks_inner_steps": "key-switch inner product (eval keys x extended digits, automorphism), every step of a batch in one launch",
    "ks_final_steps": "key-switch epilogue, all hoisted steps of a batch in one launch",
    "multplain": "MultPlain inner sums (one baby step)",
    "ks_final_multplain": "baby-step key-switch epilogue folded into the MultPlain inner sums",
    "ks_inner_ext_multplain": "fused extended sums: the key inner products of every hoisted step (lazy-ModDown "
                              "baby steps, hoisted rotate-and-sum groups) summed over Q u P in registers, with "
                              "the plaintext diagonals for the baby steps",
    "ext_multplain": "lazy-ModDown inner sums over Q u P from stored key-switch products",
}


def trace_steps(ctx, runner, batch, steps):
    """Run `steps` batched inferences eagerly with the library tracer on: every
    launch bracketed by HIP events on the library stream, carrying its
    algorithmic byte count.  Same launches as the graph the timed leg replays."""
    import torch
    runner.run(batch)
    torch.cuda.synchronize()
    ctx.trace_read()
    ctx.set_knob("trace", 1)
    tab = {}
    for _ in range(steps):
        runner.run(batch)
        # read after every step: the library keeps at most 8192 traced launches between reads
        for k, (n, ms, by) in ctx.trace_read().items():
            n0, ms0, by0 = tab.get(k, (0, 0.0, 0.0))
            tab[k] = (n0 + n, ms0 + ms, by0 + by)
    ctx.set_knob("trace", 0)
    return tab


def traffic_record(kernel, launches_per_step, workload="cfg4"):
    """rocprofv3 FETCH_SIZE/WRITE_SIZE of one kernel class of one workload's
    step, per launch, from profiles/; dropped unless taken on the current
    sources of the evaluation kernels (every file under csrc/ but the client
    path's client.hip)."""
    import hashlib
    try:
        prof = json.load(open(os.path.join(ROOT, "profiles", "roofline_traffic.json")))
        h = hashlib.sha256()
        for f in sorted(os.listdir(os.path.join(ROOT, "paper_2104_09164_amd", "csrc"))):
            if f != "client.hip":
                h.update(open(os.path.join(ROOT, "paper_2104_09164_amd", "csrc", f), "rb").read())
        rec = prof.get("workloads", {}).get(workload, {})
        k = rec.get("kernels", {}).get(kernel)
        if k and rec["csrc_sha256"] == h.hexdigest() and k["launches_per_step"] == launches_per_step:
            return k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        pass
    return None


# Integer VALU peak of MI355X: 256 CUs x 64 lanes x 2.4 GHz (one 32-bit lane
# operation per lane per clock; v_mad_u64_u32 and v_mul_lo/hi_u32 issue at that
# rate on gfx950).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Minimal VALU lane operations per modular product in the gfx950 code of this
# library (instruction sequences read from its own disassembly): a key product
# folded into a running sum (add_shoup4: 2 v_mul_hi_u32, 3 v_mad_u64_u32,
# 4 v_mul_lo_u32, 2 v_add3_u32) 11; a plaintext product and its 64-bit
# accumulation (shoup_lazy4 + add) 14; the lift of c0 by P (Shoup product) 8.
# Primes below 2^50 in the LDS-shared form (batches of 3 or more) take the
# inner sums as exact 28-bit column sums: a plaintext product is 4
# v_mad_u64_u32 (OPS_COL), a plain sum 2 adds (OPS_COL_PLAIN), and splitting
# each step's value into its two columns 2 (OPS_SPLIT, per value).  The
# LDS-shared form reads the lift P c0 formed once per coefficient (the
# lift_c0 kernel, a class of its own): one 64-bit add per step (OPS_LIFT_ADD).
OPS_KEY, OPS_PT, OPS_LIFT = 11, 14, 8
OPS_COL, OPS_COL_PLAIN, OPS_SPLIT = 4, 2, 2
OPS_LIFT_ADD = 1
# Forward NTT on primes below 2^57 (no per-stage conditional subtraction): a
# butterfly is add_shoup4 (11) plus the difference 2X + 4q - S (one
# v_lshl_add_u64 and a 64-bit subtract, 3); each coefficient's final
# reduction (reduce_lazy, then two conditional subtractions) about 14.
OPS_BUTTERFLY, OPS_NTT_OUT = 14, 14
WIDE_Q = 1 << 50
LDS_MIN_BATCH = 3
# Kernel classes bound by VALU issue rather than HBM (rocprofv3 SQ counters:
# VALU instructions issued in most of the kernel's cycles, HBM traffic a
# fraction of the copy rate): their roofline is the integer VALU peak.
ALU_CLASSES = ("ks_inner_ext_multplain",)


def fused_ops(plan, batch) -> int:
    """Algorithmic VALU lane operations of the fused extended-sum kernels of
    one inference step.  Lazy-ModDown baby steps: per item, baby step and
    coefficient, 2 beta key products and 2 n2 plaintext products on every limb
    of Q_l u P plus the lift of c0 on the Q-limbs; the unrotated term adds 2
    lifts and 2 n2 plaintext products per Q-limb.  Hoisted rotate-and-sum
    groups of b bits: the same with 2^b - 1 steps, n2 = 1 and plain sums.
    Limbs below 2^50 in batches of 3 or more (the LDS-shared form) count the
    column form of the inner sums (OPS_COL per product, OPS_COL_PLAIN per
    plain sum, OPS_SPLIT per summed value); the others a Shoup product per
    term (OPS_PT).  In that form the lift is read (OPS_LIFT_ADD per step, the
    unrotated term's P c0 free)."""
    N, K = 1 << plan.log_n, len(plan.p)
    total = 0
    for lay in plan.layers:
        l1 = lay.level + 1
        beta = -(-l1 // plan.alpha)
        limbs = [(plan.q[t], t < l1) for t in range(l1)] + [(p, False) for p in plan.p]

        def per_item(steps, n2, plain):
            ops = 0
            lds = batch >= LDS_MIN_BATCH
            for q, qlimb in limbs:
                col = lds and q < WIDE_Q
                prod = (OPS_COL_PLAIN if plain else OPS_COL) if col else OPS_PT
                split = 2 * OPS_SPLIT if col else 0
                lift = (OPS_LIFT_ADD if lds else OPS_LIFT) if qlimb else 0
                ops += steps * (2 * beta * OPS_KEY + 2 * n2 * prod + split + lift)
                if qlimb:
                    ops += (1 if lds else 2) * OPS_LIFT + 2 * n2 * prod + split
            return ops
        if lay.qp and lay.n1 > 1 and lay.n2 <= 8:
            total += batch * N * per_item(lay.n1 - 1, lay.n2, False)
        if lay.rs_bits > 0:
            left = (lay.n // lay.m).bit_length() - 1
            while left > 0:
                b = min(lay.rs_bits, left)
                left -= b
                total += batch * N * per_item((1 << b) - 1, 1, True)
    return total


def step_roofline(tab, steps, alu_ops_per_step=0, workload="cfg4"):
    """Roofline of the dominant kernel class of one step (largest summed time):
    achieved = its algorithmic bytes per launch / its mean launch duration
    (HBM), or, for a VALU-bound class, its algorithmic VALU lane operations
    (fused_ops) / its duration."""
    kern = max(tab, key=lambda k: tab[k][1])
    n, ms, by = tab[kern]
    gbs = by / (ms * 1e-3) / 1e9
    per_step = n // steps
    total_ms = sum(v[1] for v in tab.values())
    if kern in ALU_CLASSES and alu_ops_per_step:
        ops = alu_ops_per_step * steps
        achieved = ops / (ms * 1e-3) / 1e12
        head = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                "unit": "TOP/s (32-bit integer VALU lane ops)", "frac": achieved / VALU_PEAK_TOPS,
                "alg_ops_per_launch": ops / n,
                "ops_per_product": {"key": OPS_KEY, "plaintext": OPS_PT, "lift": OPS_LIFT, "column_product": OPS_COL,
                                    "column_plain_sum": OPS_COL_PLAIN, "column_split": OPS_SPLIT,
                                    "lift_read": OPS_LIFT_ADD},
                "hbm_view": {"achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS}}
    else:
        head = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    return {**head, "kernel": KERNEL_LABEL.get(kern, kern), "kernel_class": kern,
            "traffic": traffic_record(kern, per_step, workload), "alg_bytes_per_launch": by / n,
            "us_per_launch": ms * 1e3 / n, "launches_per_step": per_step,
            "share_of_kernel_time": ms / total_ms,
            "classes": {k: {"launches_per_step": v[0] // steps, "ms_per_step": v[1] / steps,
                            "gbs": v[2] / (v[1] * 1e-3) / 1e9 if v[1] > 0 else None}
                        for k, v in sorted(tab.items(), key=lambda kv: -kv[1][1])}}


def pcie_inclusive(ctx, runner, plan, batch, step, steps):
    """The batched step with the host interchange included: every input
    ciphertext copied from pinned host memory in coefficient form and
    converted on the device (he_ct_from_coeff_dev), the step, every output
    converted back (he_ct_to_coeff_dev) and copied to pinned host memory, all
    in order on the context's stream."""
    import ctypes
    import torch
    from paper_2104_09164_amd import he
    lib = he.lib()
    ins, outs = runner.inputs[:batch], runner.outputs(batch)
    host_in = [torch.from_numpy(ctx.export_ct(c).view(np.int64).reshape(-1).copy()).pin_memory() for c in ins]
    dev_in = [torch.empty_like(h, device=ctx.device) for h in host_in]
    ow = 2 * (outs[0].level + 1) * (1 << plan.log_n)
    dev_out = [torch.empty(ow, dtype=torch.int64, device=ctx.device) for _ in outs]
    host_out = [torch.empty(ow, dtype=torch.int64, pin_memory=True) for _ in outs]

    def run():
        for h, d, c in zip(host_in, dev_in, ins):
            d.copy_(h, non_blocking=True)
            cs = c._c()
            rc = lib.he_ct_from_coeff_dev(ctx.h, ctypes.c_void_p(d.data_ptr()), c.level, c.scale, ctypes.byref(cs))
            if rc:
                raise he.HeError(rc, "he_ct_from_coeff_dev")
        step()
        for c, d, h in zip(outs, dev_out, host_out):
            rc = lib.he_ct_to_coeff_dev(ctx.h, ctypes.byref(c._c()), ctypes.c_void_p(d.data_ptr()))
            if rc:
                raise he.HeError(rc, "he_ct_to_coeff_dev")
            h.copy_(d, non_blocking=True)

    run()
    torch.cuda.synchronize()
    t = time_events(run, steps)
    ms = float(np.median(t))
    in_mb = sum(h.numel() for h in host_in) * 8 / 1e6
    out_mb = sum(h.numel() for h in host_out) * 8 / 1e6
    return {"inferences_per_s": batch * 1000.0 / ms, "ms_per_step": ms, "host_to_device_mb": in_mb,
            "device_to_host_mb": out_mb}


def network_legs(name, batch, steps, warmup, plain_n, graph=True, use_tuning=True, tuned_n1=True, trace=True):
    """Batched (graph replay) and plain (one request at a time) legs of one preset.
    A committed tuning file (paper_2104_09164_amd/tuning/<gfx>_<name>.json)
    supplies the execution knobs and, with tuned_n1, the per-layer baby-step
    counts (else the preset's)."""
    import torch
    from paper_2104_09164_amd import netplan, tune
    tuned = tune.load(name) if use_tuning else None
    plan = netplan.preset_plan(name, netplan.tuned_shapes(name, tuned, tuned_n1))
    log(f"{name}: N=2^{plan.log_n}, L={plan.L}, K={len(plan.p)}, alpha={plan.alpha}, batch={batch}, "
        f"n1={[l.n1 for l in plan.layers]}, lazy ModDown={[l.qp for l in plan.layers]}, "
        f"rotate-and-sum bits={[l.rs_bits for l in plan.layers]}, "
        f"knobs={tuned.get('knobs') if tuned else None}")
    ctx, runner = setup(plan, batch)
    tune.apply_knobs(ctx, tuned)
    torch.cuda.synchronize()
    step = runner.capture(batch).replay if graph else (lambda: runner.run(batch))
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    log(f"{name}: batched leg")
    per_step = time_events(step, steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"{name}: PCIe-inclusive leg")
    pcie = pcie_inclusive(ctx, runner, plan, batch, step, steps)
    log(f"{name}: plain leg")
    lat_eager = [float("nan")]
    if plain_n > 0:
        # one request at a time: the same network for a batch of one, replayed
        # from its own graph (and, for reference, launched eagerly)
        one = runner.capture(1).replay if graph else (lambda: runner.run(1))
        for _ in range(2):
            one()
            runner.run(1)
        torch.cuda.synchronize()
        lat = time_events(one, plain_n)
        lat_eager = time_events(lambda: runner.run(1), plain_n)
    else:
        lat = [float("nan")]
    c = netplan.PRESETS[name]
    res = {"batch": batch, "inferences_per_s": batch * steps / wall, "ms_per_step": wall * 1e3 / steps,
           "batched_p50_ms": float(np.percentile(per_step, 50)), "batched_p99_ms": float(np.percentile(per_step, 99)),
           "plain_inferences_per_s": 1000.0 / float(np.mean(lat)),
           "plain_p50_ms": float(np.percentile(lat, 50)), "plain_p99_ms": float(np.percentile(lat, 99)),
           "plain_eager_p50_ms": float(np.percentile(lat_eager, 50)),
           "workload": (f"{name}: N=2^{plan.log_n}, q bits {c['q_bits'][0]}+{len(c['q_bits']) - 1}x{c['q_bits'][1]}, "
                        f"P {len(c['p_bits'])}x{c['p_bits'][0]}b, alpha={plan.alpha}, layers "
                        + ", ".join(f"{l.n}->{l.m} (n1={l.n1}{', lazy ModDown' if l.qp else ''}"
                                    f"{f', rotate-and-sum hoisted {l.rs_bits} bits' if l.rs_bits else ''})"
                                    for l in plan.layers) + ", x^2 between"),
           "ops_per_inference": plan.op_counts(),
           "tuning": {"knobs": tuned.get("knobs"), "n1": tuned.get("n1") if tuned_n1 else None,
                      "lazy_moddown": [l.qp for l in plan.layers],
                      "rotate_sum_bits": [l.rs_bits for l in plan.layers]} if tuned else None}
    res["batched_over_plain"] = res["inferences_per_s"] / res["plain_inferences_per_s"]
    res["pcie_inclusive"] = pcie
    if trace:
        log(f"{name}: traced eager pass")
        res["trace"] = trace_steps(ctx, runner, batch, steps)
    return plan, ctx, runner, res


def plain_request_leg(reps=50):
    """The plain RNS-CKKS request (N = 2^13, q0 45b + 3 x 35b, P 45b, alpha =
    1; dense 256->64 with 8 baby steps, x^2, dense 64->2): one request at a
    time, its whole network replayed from a captured graph of a batch of one,
    p50/p99 over `reps` requests; eager launches beside it.  Random residues
    as keys, diagonals and ciphertext (the same call sequence is checked bit
    for bit against the oracle at this ring by the GPU tests)."""
    import torch
    from paper_2104_09164_amd import netplan
    plan = netplan.preset_plan("cfg1")
    ctx, runner = setup(plan, 1)
    one = runner.capture(1).replay
    for _ in range(3):
        one()
        runner.run(1)
    torch.cuda.synchronize()
    lat = time_events(one, reps)
    eager = time_events(lambda: runner.run(1), reps)
    c = netplan.PRESETS["cfg1"]
    res = {"workload": (f"cfg1: N=2^13, q bits {c['q_bits'][0]}+{len(c['q_bits']) - 1}x{c['q_bits'][1]}, P 1x45b, "
                        f"alpha=1, layers " + ", ".join(f"{l.n}->{l.m} (n1={l.n1})" for l in plan.layers)
                        + ", x^2 between; one request at a time, graph replay"),
           "requests": reps, "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "inferences_per_s": 1000.0 / float(np.mean(lat)),
           "eager_p50_ms": float(np.percentile(eager, 50)), "eager_p99_ms": float(np.percentile(eager, 99)),
           "ops_per_inference": plan.op_counts()}
    del ctx, runner
    torch.cuda.synchronize()
    return plan, res


def serving_leg(nets, rates, counts, seed=21, window=4, per_network=False, policy="largest", weights=None,
                chain=()):
    """Poisson arrivals (total rate lambda, the superposition of 256 camera
    streams), 70% small-net / 30% large-net requests, keys and plaintexts
    resident, admission by device-memory footprint, continuous batching
    (largest ready stage group first, oldest first past 20 ms of waiting;
    the networks in `chain` run a group's stages from one dispatch)."""
    import torch
    from paper_2104_09164_amd import serve
    backends = {}
    payloads = {}
    for name, (plan, ctx, max_batch) in nets.items():
        backends[name] = serve.NetBackend(name, ctx, plan, runner_layers[name], max_batch=max_batch,
                                          slots=2 * max_batch + 8, own_stream=True)
        if weights and name in weights:
            backends[name].weight = weights[name]
        backends[name].chain = name in chain
        N = 1 << plan.log_n
        payloads[name] = [(residues(plan.q, N, (2,), seed + 50 + k), plan.L, plan.scale) for k in range(4)]
    budget = int(0.5 * torch.cuda.get_device_properties(0).total_memory)
    out = {}
    for rate, count in zip(rates, counts):
        rng = np.random.default_rng(seed + int(rate))
        times = serve.poisson_arrivals(rate, count, seed + int(rate))
        kinds = np.where(rng.random(count) < 0.7, "small", "large")
        reqs = [serve.Request(i, str(kinds[i]), payloads[str(kinds[i])][i % 4], float(times[i])) for i in range(count)]
        sched = serve.Scheduler(backends, budget_bytes=budget, window=window, per_network=per_network, policy=policy)
        log(f"serving: {count} requests at {rate} req/s")
        serve.run_arrivals(sched, reqs, timeout_s=120)
        torch.cuda.synchronize()
        m = sched.metrics()
        for name in nets:
            lat = [1e3 * (r.finish - r.arrival) for r in sched.done if r.net == name and r.error is None]
            if lat:
                m[f"{name}_p50_ms"] = float(np.percentile(lat, 50))
                m[f"{name}_p99_ms"] = float(np.percentile(lat, 99))
                m[f"{name}_samples"] = len(lat)
        m["requests"] = count
        m["p99_tail_samples"] = max(1, int(round(0.01 * m.get("completed", 0))))
        out[str(rate)] = m
    out["scheduler"] = {"policy": policy, "max_wait_ms": 20.0, "window": window, "per_network": per_network,
                        "weights": weights or {}, "chained": sorted(chain)}
    return out


runner_layers = {}


def calibration_copy():
    """1 GiB read + 1 GiB written by one device copy: scales the HBM counters."""
    import torch
    src = torch.empty(1 << 27, dtype=torch.int64, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=16, help="requests per launch, small net")
    ap.add_argument("--large-batch", type=int, default=32, help="requests per launch, large net (headline)")
    ap.add_argument("--plain", type=int, default=8, help="one-request inferences timed for the plain legs")
    ap.add_argument("--serve-rates", default="50,100,200,300,400")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per rate below the top rate")
    ap.add_argument("--serve-requests-top", type=int, default=10000, help="requests at the top rate")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-tuning", action="store_true", help="ignore committed tuning files")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ntt", action="store_true")
    ap.add_argument("--no-ks", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="skip the small-net legs")
    ap.add_argument("--no-plain-request", action="store_true", help="skip the N=2^13 plain-request leg")
    ap.add_argument("--no-tuned-split", action="store_true", help="skip the small-net leg with tuned baby steps")
    ap.add_argument("--no-conv", action="store_true", help="skip the multi-channel convolution leg")
    ap.add_argument("--no-client", action="store_true", help="skip the client encode/encrypt/decrypt leg")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only a traced pass (profiling runs): 1 GiB calibration copy, setup, one untimed "
                         "step, --steps traced steps of --roofline-net")
    ap.add_argument("--roofline-net", default="cfg4", choices=("cfg4", "cfg3"))
    ap.add_argument("--client-only", action="store_true",
                    help="only the client encode/encrypt/decrypt leg (profiling runs)")
    ap.add_argument("--large-only", action="store_true",
                    help="only the large-net batched and plain legs (profiling runs)")
    ap.add_argument("--ks-only", action="store_true", help="only the key-switch leg (profiling runs)")
    ap.add_argument("--cpu-only", action="store_true", help="only the CPU oracle baseline (no GPU use)")
    ap.add_argument("--ntt-only", action="store_true",
                    help="only the NTT leg (profiling runs), preceded by a 1 GiB device copy whose "
                         "FETCH_SIZE / WRITE_SIZE calibrate the HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one MI355X: the library has no multi-GPU path (requests would shard across "
              "GPUs with no exchange between them). Run with --gpus 1.", file=sys.stderr)
        return 2
    from paper_2104_09164_amd import netplan, tune

    def gpu_plan(name, tuned_n1):
        tuned = tune.load(name, "gfx950") if not args.no_tuning else None
        return netplan.preset_plan(name, netplan.tuned_shapes(name, tuned, tuned_n1))
    if args.cpu_only:
        plans = {"cfg1": netplan.preset_plan("cfg1"), "cfg3": gpu_plan("cfg3", False), "cfg4": gpu_plan("cfg4", True)}
        print(json.dumps({"cpu_protocol": cpu_protocol(plans, "as the GPU legs")}), flush=True)
        return 0
    import torch
    if args.client_only:
        print(json.dumps({"client": client_leg()}), flush=True)
        return 0
    if args.ks_only:
        print(json.dumps({"key_switch": ks_leg()}), flush=True)
        return 0
    if args.large_only:
        _, _, _, large = network_legs("cfg4", args.large_batch, max(3, args.steps // 2), 1, max(3, args.plain // 2),
                                      graph=not args.no_graph, use_tuning=not args.no_tuning, trace=False)
        print(json.dumps({"large_net": large}), flush=True)
        return 0
    if args.ntt_only:
        calibration_copy()
        print(json.dumps({"ntt": ntt_leg()}), flush=True)
        return 0
    if args.roofline_only:
        calibration_copy()
        name = args.roofline_net
        tuned = tune.load(name)
        plan = netplan.preset_plan(name, netplan.tuned_shapes(name, tuned, tuned_n1=(name == "cfg4")))
        batch = args.large_batch if name == "cfg4" else args.batch
        ctx, runner = setup(plan, batch)
        tune.apply_knobs(ctx, tuned)
        tab = trace_steps(ctx, runner, batch, args.steps)
        print(json.dumps({"roofline": step_roofline(tab, args.steps, fused_ops(plan, batch), name)}), flush=True)
        return 0
    # headline: the large net (the largest single-GPU configuration), 32 requests per launch, the
    # committed tuned plan (baby-step splits, lazy ModDown, rotate-and-sum groups) and knobs
    plan4, ctx4, run4, large = network_legs("cfg4", args.large_batch, args.steps, args.warmup, max(3, args.plain // 2),
                                            graph=not args.no_graph, use_tuning=not args.no_tuning)
    runner_layers["large"] = run4.layers
    out = {"metric": METRIC, "value": large["inferences_per_s"], "unit": "inferences/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": large["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
           "config": {"workload": ("large-net batched encrypted inference, " + large["workload"]
                                   + f", {args.large_batch} requests per launch, HIP graph replay"),
                      "batch": args.large_batch, "ops_per_inference": large["ops_per_inference"],
                      "tuning": large["tuning"]},
           "latency_ms": {"batched_p50": large["batched_p50_ms"], "batched_p99": large["batched_p99_ms"],
                          "plain_p50": large["plain_p50_ms"], "plain_p99": large["plain_p99_ms"],
                          "plain_eager_p50": large["plain_eager_p50_ms"]},
           "roofline": step_roofline(large.pop("trace"), args.steps, fused_ops(plan4, args.large_batch), "cfg4"),
           "plain_inferences_per_s": large["plain_inferences_per_s"],
           "pcie_inclusive": large["pcie_inclusive"],
           "batched_over_plain": large["batched_over_plain"]}
    nets = {"large": (plan4, ctx4, args.large_batch)}
    plan3 = None
    if not args.no_small:
        # the small net with the preset split (32 baby steps in the first layer) and the lazy-ModDown /
        # rotate-and-sum forms the tuner chose for it
        plan3, ctx3, run3, small = network_legs("cfg3", args.batch, args.steps, args.warmup, args.plain,
                                                graph=not args.no_graph, use_tuning=not args.no_tuning,
                                                tuned_n1=False)
        runner_layers["small"] = run3.layers
        small["roofline"] = step_roofline(small.pop("trace"), args.steps, fused_ops(plan3, args.batch), "cfg3")
        out["small_net"] = small
        nets["small"] = (plan3, ctx3, args.batch)
        if not args.no_tuning and not args.no_tuned_split:
            _, ctx3t, _, small_t = network_legs("cfg3", args.batch, args.steps, 1, 0, graph=not args.no_graph,
                                                tuned_n1=True, trace=False)
            out["small_net_tuned_split"] = {k: small_t[k] for k in ("inferences_per_s", "ms_per_step",
                                                                    "batched_p50_ms", "batched_p99_ms", "workload",
                                                                    "tuning")}
            del ctx3t, small_t
    if not args.no_plain_request:
        log("plain-request leg (N=2^13)")
        plan1, out["plain_request"] = plain_request_leg()
    if not args.no_serve and not args.no_small:
        rates = [float(r) for r in args.serve_rates.split(",") if r]
        counts = [args.serve_requests_top if r == max(rates) else args.serve_requests for r in rates]
        out["serving"] = serving_leg(nets, rates, counts, window=2, chain=("large",))
    del nets
    torch.cuda.synchronize()
    if not args.no_ntt:
        log("ntt leg")
        nt = ntt_leg()
        out["ntt"] = nt
        out["ntt_roofline"] = ntt_roofline(nt)
    if not args.no_ks:
        log("key-switch leg")
        out["key_switch"] = ks_leg()
    if not args.no_conv:
        log("convolution leg")
        out["conv"] = conv_leg()
    if not args.no_client:
        log("client leg")
        out["client"] = client_leg()
    if not args.no_cpu:
        plans = {"cfg1": netplan.preset_plan("cfg1"), "cfg3": plan3 or gpu_plan("cfg3", False), "cfg4": plan4}
        proto = cpu_protocol(plans, "the plans of the GPU legs (cfg4 tuned, cfg3 preset split, cfg1 preset)")
        c4 = proto["cfg4"]
        key = next(iter(c4))
        out["cpu_baseline"] = {
            "value": c4[key]["inferences_per_s"], "unit": "inferences/s", "cores": int(key.split("_")[1]),
            "kind": "oracle",
            "sample": (f"one large-net request (the headline workload, same plan as the GPU) evaluated end to end "
                       f"by the oracle, evaluation only, single run: {c4[key]['s_per_inference']:.1f} s; "
                       f"{proto['cpu_model']}, nproc {proto['nproc']}; more runs in cpu_protocol")}
        out["cpu_protocol"] = proto
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
