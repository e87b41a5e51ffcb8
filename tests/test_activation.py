"""Trained quadratic activations a x^2 + b x + c per feature (paper, "Network
architecture" and "Non-convolutional layers").

The library folds them into the adjacent dense layers (netplan.
fold_quadratic_activations) so that the encrypted network still only
squares.  Checked here against the oracle's direct FP64 evaluation of the
quadratic network (CPU), through the CPU oracle's RNS-CKKS evaluation of the
folded network, and on the GPU bit for bit against that oracle.
"""
import numpy as np
import pytest

from oracle import ckks, params, plainnet, plan
from paper_2104_09164_amd import netplan, synth


@pytest.mark.parametrize("name", ["cfg1", "cfg3", "cfg4"])
def test_fold_equals_direct_quadratic_fp64(name):
    layers = params.preset(name).layers
    Ws, bs = synth.network_weights(layers, 0.05)
    acts = synth.activation_coeffs(layers)
    Wf, bf = netplan.fold_quadratic_activations(Ws, bs, acts)
    assert [W.shape for W in Wf] == [W.shape for W in Ws]
    for r in range(3):
        x = synth.request_input(layers[0][1], r)
        want = plainnet.forward(x, Ws, bs, acts)
        got = plainnet.forward(x, Wf, bf)                 # squares only
        assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))


def test_fold_identity_and_rejection():
    layers = [(4, 8, 2), (2, 4, 2)]
    Ws, bs = synth.network_weights(layers, 0.1)
    ones, zeros = np.ones(4), np.zeros(4)
    Wf, bf = netplan.fold_quadratic_activations(Ws, bs, [(ones, zeros, zeros)])   # x^2 itself
    assert all(np.array_equal(a, b) for a, b in zip(Wf + bf, Ws + bs))
    with pytest.raises(ValueError):
        netplan.fold_quadratic_activations(Ws, bs, [(np.array([1.0, 0.0, 1.0, 1.0]), ones, zeros)])


def test_fold_bounds_small_a():
    """A small |a| against its b is refused (shift b / 2a or cancelled constant
    b^2 / 4a beyond the bounds), also for a negative a; the largest allowed
    shift folds and still equals the direct FP64 network."""
    layers = [(4, 8, 2), (2, 4, 2)]
    Ws, bs = synth.network_weights(layers, 0.1)
    ones, zeros = np.ones(4), np.zeros(4)
    for a in (1e-3, -1e-3, 0.02):
        with pytest.raises(ValueError):
            netplan.fold_quadratic_activations(Ws, bs, [(np.full(4, a), np.full(4, 0.5), zeros)])
    a, b = 0.05, 0.79                      # shift 7.9, cancelled constant 3.12: inside the bounds
    acts = [(np.full(4, a), np.full(4, b), np.full(4, 0.1))]
    Wf, bf = netplan.fold_quadratic_activations(Ws, bs, acts)
    x = synth.request_input(8, 0)
    want = plainnet.forward(x, Ws, bs, acts)
    assert np.max(np.abs(plainnet.forward(x, Wf, bf) - want)) <= 1e-12


def test_network_cfg1_quadratic_oracle_at_fold_bound(oracle_lib):
    """The cfg1 network with every activation at the largest allowed shift
    (a = 0.05, b = 0.79: shift 7.9): the CPU oracle's RNS-CKKS evaluation of
    the folded network is within 2^-12 of the FP64 quadratic network."""
    pr = params.preset("cfg1")
    o = ckks.Oracle(pr)
    Ws, bs = synth.network_weights(pr.layers, pr.sigma_w)
    m1 = pr.layers[0][0]
    acts = [(np.full(m1, 0.05), np.full(m1, 0.79), np.full(m1, 0.1))]
    Wf, bf = netplan.fold_quadratic_activations(Ws, bs, acts)
    keys = o.keygen(synth.SEED_KEYS, ckks.network_steps(pr.layers))
    lays = o.prepare_network(Wf, bf, [l[2] for l in pr.layers])
    x = synth.request_input(pr.layers[0][1], 0)
    ct = o.encrypt(plan.input_slots(x, pr.slots), keys.pk, synth.request_seed(0))
    y = o.decrypt_decode(o.eval_network(ct, lays, keys), keys.sk).real[:2]
    assert np.max(np.abs(y - plainnet.forward(x, Ws, bs, acts))) <= 2.0 ** -12


def test_network_cfg1_quadratic_oracle(oracle_lib):
    """RNS-CKKS evaluation (CPU oracle) of the folded network: logits within
    2^-12 of the FP64 network with the quadratic activation, same class."""
    pr = params.preset("cfg1")
    o = ckks.Oracle(pr)
    Ws, bs = synth.network_weights(pr.layers, pr.sigma_w)
    acts = synth.activation_coeffs(pr.layers)
    Wf, bf = netplan.fold_quadratic_activations(Ws, bs, acts)
    keys = o.keygen(synth.SEED_KEYS, ckks.network_steps(pr.layers))
    lays = o.prepare_network(Wf, bf, [l[2] for l in pr.layers])
    for r in range(2):
        x = synth.request_input(pr.layers[0][1], r)
        ct = o.encrypt(plan.input_slots(x, pr.slots), keys.pk, synth.request_seed(r))
        y = o.decrypt_decode(o.eval_network(ct, lays, keys), keys.sk).real[:2]
        yr = plainnet.forward(x, Ws, bs, acts)
        assert np.max(np.abs(y - yr)) <= 2.0 ** -12
        if abs(yr[0] - yr[1]) >= 2.0 ** -11:
            assert plainnet.predict(y) == plainnet.predict(yr)


@pytest.mark.gpu
def test_network_cfg1_quadratic_gpu():
    """The folded cfg1 network on the GPU: bit-exact against the oracle,
    logits within 2^-12 of the FP64 quadratic network."""
    from paper_2104_09164_amd import he
    pr = params.preset("cfg1")
    o = ckks.Oracle(pr)
    Ws, bs = synth.network_weights(pr.layers, pr.sigma_w)
    acts = synth.activation_coeffs(pr.layers)
    Wf, bf = netplan.fold_quadratic_activations(Ws, bs, acts)
    keys = o.keygen(synth.SEED_KEYS, ckks.network_steps(pr.layers))
    lays = o.prepare_network(Wf, bf, [l[2] for l in pr.layers])
    ctx = he.Context(pr.log_n, pr.q, pr.p, pr.alpha)
    ctx.bind(1, 8, 8)
    ctx.load_keys(keys.rlk, keys.rot)
    dls = [ctx.dense_load(l.level, l.m, l.n, l.n1, l.pts, l.bias, l.pt_scale, l.bias_scale) for l in lays]
    x = synth.request_input(pr.layers[0][1], 4)
    ct = o.encrypt(plan.input_slots(x, pr.slots), keys.pk, synth.request_seed(4))
    g = ctx.import_ct(ct.data, ct.level, ct.scale)
    for li, d in enumerate(dls):
        g = ctx.rescale(ctx.eval_dense(g, d))
        if li + 1 < len(dls):
            g = ctx.rescale(ctx.square(g))
    want = o.eval_network(ct, lays, keys)
    got = ctx.export_ct(g)
    assert g.scale == want.scale and np.array_equal(got, want.data)
    y = o.decrypt_decode(ckks.Ciphertext(got, g.level, g.scale), keys.sk).real[:2]
    assert np.max(np.abs(y - plainnet.forward(x, Ws, bs, acts))) <= 2.0 ** -12
