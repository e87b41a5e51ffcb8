"""Full-size parity in the benchmark's launch configurations.

cfg4 (N = 2^16, 11 limbs, three 60-bit special primes; the benchmark's
`value` workload): two requests through the whole large network with the
committed tuned plan (64 / 32 / 2 baby steps, lazy ModDown in the first two
layers, hoisted rotate-and-sum groups of 2 / 2 / 3 bits), in one batched graph
replay, bit for bit against the oracle, plus the FP64 tolerance; once more
with the inputs encoded and encrypted, and the outputs decrypted and decoded,
by the device client path.
cfg3 (N = 2^15): whole network by graph replay, bit for bit against the oracle
plus FP64 tolerance, with the preset BSGS split and with the autotuner's split,
and with per-feature trained quadratic activations folded into the dense
layers (bit for bit, and against the FP64 quadratic network).
cfg2 (N = 2^16, 24 x 50-bit limbs, dnum = 3: the key-switch micro-benchmark):
one batch of 64 ciphertexts rotated by all 32 random steps in one hoisted call
(one ModUp per ciphertext), as timed; every step of the encrypted ciphertext at
batch position 0 and four steps of the one at position 37 compared bit for bit
with the oracle's rotations, and their decryptions against the rotated
messages.

The oracle's evaluations of different requests (or steps) are independent and
run in a small thread pool (the C++ core releases the interpreter lock), so
the CPU side of these tests fits the suite's time budget.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import ckks, params, plainnet, plan
from paper_2104_09164_amd import netplan, synth, tune

pytestmark = pytest.mark.gpu


def run_network(name, requests, check_bits, tuned_split=True, quadratic=False, client=False):
    import torch
    from paper_2104_09164_amd import he
    from paper_2104_09164_amd.batch import NetworkRunner
    c = netplan.PRESETS[name]
    tuned = tune.load(name, "gfx950")
    shapes = netplan.tuned_shapes(name, tuned, tuned_split)     # (m, n, n1, lazy ModDown)
    pr = params.preset(name)
    o = ckks.Oracle(pr)
    rs = [s[4] if len(s) > 4 else 0 for s in shapes]
    steps = ckks.network_steps([s[:3] for s in shapes], rs)
    print(f"[fullsize] {name}: keygen for {len(steps)} rotation keys, plan {shapes}", flush=True)
    keys = o.keygen(synth.SEED_KEYS, steps)
    Ws, bs = synth.network_weights([s[:3] for s in shapes], c["sigma"])
    acts = None
    Wr, br = Ws, bs                    # the FP64 reference network
    if quadratic:
        # trained quadratic activations folded into the dense layers (squares only)
        acts = synth.activation_coeffs([s[:3] for s in shapes])
        Ws, bs = netplan.fold_quadratic_activations(Ws, bs, acts)
    lays = o.prepare_network(Ws, bs, [s[2] for s in shapes], qps=[len(s) > 3 and s[3] for s in shapes], rs_bits=rs)
    npl = netplan.plan_network(pr.log_n, pr.q, pr.p, pr.alpha, c["scale_bits"], shapes)
    ctx = he.Context(pr.log_n, pr.q, pr.p, pr.alpha)
    tune.apply_knobs(ctx, tuned)
    B = len(requests)
    ctx.bind(B, npl.max_n1(), npl.max_n2())
    ctx.load_keys(keys.rlk, keys.rot)
    dls = [ctx.dense_load(l.level, l.m, l.n, l.n1, l.pts, l.bias, l.pt_scale, l.bias_scale, qp=l.qp, rs_bits=l.rs_bits)
           for l in lays]
    runner = NetworkRunner(ctx, npl, dls, B)
    cts, xs = [], []
    for i, r in enumerate(requests):
        x = synth.request_input(shapes[0][1], r)
        xs.append(x)
        if not client:
            ct = o.encrypt(plan.input_slots(x, pr.slots), keys.pk, synth.request_seed(r))
            runner.inputs[i].buf.copy_(ctx.import_ct(ct.data, ct.level, ct.scale).buf)
            cts.append(ct)
    cl = None
    if client:
        # the end users' side on the device: encode and encrypt every request in one batch
        cl = ctx.client(B, pk=keys.pk, sk=keys.sk)
        z = torch.from_numpy(np.stack([plan.input_slots(x, pr.slots) for x in xs]).astype(np.complex128))
        noise = torch.from_numpy(np.stack([synth.encryption_noise(pr.n, synth.request_seed(r)) for r in requests]))
        cl.encrypt(cl.encode(z, pr.scale, pr.L), noise.cuda(), pr.L, pr.scale, outs=runner.inputs[:B])
    g = runner.capture(B)
    g.replay()
    torch.cuda.synchronize()
    outs = runner.outputs(B)
    wants = None
    if check_bits:
        print(f"[fullsize] {name}: oracle network for requests {requests}", flush=True)
        def one(i):
            done = lambda li: print(f"[fullsize] {name}: oracle request {requests[i]} layer {li} done", flush=True)
            return o.eval_network(cts[i], lays, keys, progress=done)
        with ThreadPoolExecutor(max_workers=min(B, 2)) as ex:
            wants = list(ex.map(one, range(B)))
    for i in range(B):
        got = ctx.export_ct(outs[i])
        assert outs[i].level == npl.out_level and outs[i].scale == npl.out_scale
        if check_bits:
            want = wants[i]
            assert want.scale == outs[i].scale
            assert np.array_equal(got, want.data), f"{name} request {requests[i]} differs from the oracle"
        y = o.decrypt_decode(ckks.Ciphertext(got, outs[i].level, outs[i].scale), keys.sk).real[:2]
        if cl is not None:
            # the monitoring service's side on the device: decrypt and decode
            yd = cl.decode(cl.decrypt([outs[i]]), outs[i].level, outs[i].scale).cpu().numpy()[0].real[:2]
            assert np.max(np.abs(yd - y)) <= 2.0 ** -30
        yr = plainnet.forward(xs[i], Wr, br, acts)
        assert np.max(np.abs(y - yr)) <= 2.0 ** -12
        if abs(yr[0] - yr[1]) >= 2.0 ** -11:
            assert plainnet.predict(y) == plainnet.predict(yr)


def test_cfg3_network_full_size_bit_exact():
    run_network("cfg3", [0, 1], check_bits=True, tuned_split=False)


def test_cfg3_network_tuned_split_bit_exact():
    run_network("cfg3", [2], check_bits=True, tuned_split=True)


def test_cfg3_network_quadratic_activation_bit_exact():
    run_network("cfg3", [3], check_bits=True, tuned_split=False, quadratic=True)


def test_cfg4_network_full_size_bit_exact():
    run_network("cfg4", [0, 1], check_bits=True)


def test_cfg4_network_device_client_round_trip():
    """The large net's ring (N = 2^16, 11 limbs) end to end on the device:
    inputs encoded and encrypted by he_encode / he_encrypt, the network from
    its graph, outputs decrypted and decoded by he_decrypt / he_decode (equal
    to the oracle's decryption within 2^-30), logits within 2^-12 of FP64."""
    run_network("cfg4", [2, 3], check_bits=False, client=True)


def test_cfg2_key_switch_batch_full_size():
    import torch
    from paper_2104_09164_amd import he
    pr = params.preset("cfg2")
    o = ckks.Oracle(pr)
    steps = synth.rotation_steps_random(32, pr.slots)
    print(f"[fullsize] cfg2: keygen for {len(steps)} steps", flush=True)
    keys = o.keygen(synth.SEED_KEYS, steps, relin=False)
    enc_pos = {0: 0, 37: 1}                       # batch position -> request
    xs = {p: synth.request_input(pr.slots, r) for p, r in enc_pos.items()}
    encs = {p: o.encrypt(xs[p], keys.pk, synth.request_seed(r)) for p, r in enc_pos.items()}
    ctx = he.Context(pr.log_n, pr.q, pr.p, pr.alpha)
    B = 64
    ctx.bind(B, 1, 1)
    ctx.load_keys(None, keys.rot)
    L1, N = len(pr.q), pr.n
    qt = torch.tensor(pr.q, dtype=torch.int64, device="cuda").view(1, L1, 1)
    g = torch.Generator(device="cuda").manual_seed(13)
    cts = []
    for b in range(B):
        if b in encs:
            cts.append(ctx.import_ct(encs[b].data, encs[b].level, encs[b].scale))
            continue
        c = ctx.new_ct(pr.L, encs[0].scale)
        c.buf.view(2, L1, N).copy_(torch.randint(0, 2 ** 62, (2, L1, N), device="cuda", generator=g,
                                                 dtype=torch.int64) % qt)
        cts.append(c)
    # every ciphertext by every step: one ModUp per ciphertext, 2048 outputs (48 GiB)
    outs = [ctx.new_ct(pr.L) for _ in range(B * len(steps))]
    print("[fullsize] cfg2: rotate_hoisted_batch, 64 ciphertexts x 32 steps", flush=True)
    ctx.rotate_hoisted_batch(cts, steps, outs)
    torch.cuda.synchronize()
    cases = [(0, s) for s in steps] + [(37, s) for s in steps[:4]]
    got = {(p, s): ctx.export_ct(outs[p * len(steps) + steps.index(s)]) for p, s in cases}
    del outs
    torch.cuda.empty_cache()
    print(f"[fullsize] cfg2: {len(cases)} oracle rotations", flush=True)
    def one(c):
        w = o.rotate(encs[c[0]], c[1], keys)
        print(f"[fullsize] cfg2: oracle rotation of position {c[0]} by {c[1]} done", flush=True)
        return w
    with ThreadPoolExecutor(max_workers=2) as ex:
        wants = list(ex.map(one, cases))
    for (p, s), want in zip(cases, wants):
        assert np.array_equal(got[(p, s)], want.data), f"position {p}: rotation by {s} differs from the oracle"
    for p in enc_pos:
        s = steps[0]
        y = o.decrypt_decode(wants[cases.index((p, s))], keys.sk)
        assert np.max(np.abs(y - np.roll(xs[p], -s))) < 2.0 ** -20
