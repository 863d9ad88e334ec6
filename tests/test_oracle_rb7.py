"""Pins of the oracle's residual-block layers (RB7, Sec. 2.3 and the model
table) against facts outside the oracle: PyTorch's float64 convolutions,
the plain network they reduce to when a block's branch is zero, hand-worked
selector blocks, and the multiply-add count the table gives.  CPU only."""
import numpy as np
import pytest
import torch

import synth
from tests.test_oracle_pins import _bf16

D, L = 50, 111


def torch_rb_forward(layers, ws, bs, x, bf16=False):
    """PyTorch float64 reference: conv1d (kernel 2, stride 2), conv1d
    (kernel 1) for the pointwise layers, the block input added back by the
    residual half, linear on the channel-major flatten.  bf16: the form's
    roundings (inputs, weights, every hidden output; biases and sums exact)."""
    q = _bf16 if bf16 else (lambda t: t)
    h = q(torch.from_numpy(np.asarray(x, np.float64)).transpose(1, 2))  # [B][D][L]
    block_in = None
    last = len(layers) - 1
    for i, (ly, w, b) in enumerate(zip(layers, ws, bs)):
        w = q(torch.from_numpy(np.asarray(w, np.float64)))
        b = torch.from_numpy(np.asarray(b, np.float64))
        if ly.kind == synth.CONV:
            h = torch.nn.functional.conv1d(h, w, b, stride=2)
        elif ly.kind == synth.PW:
            block_in = h
            h = torch.nn.functional.conv1d(h, w, b)
        elif ly.kind == synth.PWRES:
            h = torch.nn.functional.conv1d(h, w, b) + block_in
        else:
            h = torch.nn.functional.linear(h.reshape(h.shape[0], -1), w, b)
        if ly.relu:
            h = torch.relu(h)
        if i != last:
            h = q(h)
    return h.numpy()


def small_rb(n_blocks=2, expand=24):
    """A narrow residual network on the 111 x 50 window: C3-like convs of 8,
    8, 16 channels, n_blocks blocks, FC 208 -> 12 -> 3."""
    layers = [synth.Layer(synth.CONV, D, 8, 1), synth.Layer(synth.CONV, 8, 8, 1),
              synth.Layer(synth.CONV, 8, 16, 1)]
    for _ in range(n_blocks):
        layers += [synth.Layer(synth.PW, 16, expand, 1), synth.Layer(synth.PWRES, expand, 16, 1)]
    return layers + [synth.Layer(synth.FC, 16 * 13, 12, 1), synth.Layer(synth.FC, 12, 3, 0)]


def rand_windows(n, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, L, D)) * rng.choice([1.0, 20.0], size=(n, L, D))


def test_rb7_layer_list_and_multiply_adds():
    """The table of models gives RB7 93 million multiplications per
    inference; the reading's layer list has 92,818,176 multiply-adds."""
    layers = synth.net_rb7()
    assert sum(ly.kind in (synth.PW, synth.PWRES) for ly in layers) == 2 * 7
    ch, ln, mac = D, L, 0
    for ly in layers:
        if ly.kind == synth.CONV:
            ln //= 2
            mac += ln * ly.c_out * ly.c_in * 2
        elif ly.kind in (synth.PW, synth.PWRES):
            mac += ln * ly.c_out * ly.c_in
        else:
            assert ly.c_in == ch * ln
            mac += ly.c_out * ly.c_in
            ln = 1
        ch = ly.c_out
    assert mac == 92_818_176 and round(mac / 1e6) == 93
    assert ch == 22


@pytest.mark.parametrize("bf16", [False, True])
def test_small_rb_matches_torch_float64(oracle_lib, bf16):
    layers = small_rb()
    ws, bs = synth.init_weights(3, layers, out_bias=(1.0, 2.0, 3.0))
    x = rand_windows(4, 1)
    got = oracle_lib.Model(layers, ws, bs, D, L, prec=1 if bf16 else 0).forward(x)
    ref = torch_rb_forward(layers, ws, bs, x, bf16=bf16)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_rb7_matches_torch_float64(oracle_lib):
    layers = synth.net_rb7()
    ws, bs = synth.init_weights(2, layers, out_bias=synth.HYB_BIAS)
    x = rand_windows(2, 2)
    got = oracle_lib.Model(layers, ws, bs, D, L).forward(x)
    ref = torch_rb_forward(layers, ws, bs, x)
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


def test_zero_branches_reduce_to_the_plain_network(oracle_lib):
    """With every block's weights and biases zero, a block returns ReLU of
    its (non-negative) input unchanged, so the network is the plain one
    without blocks, exactly."""
    layers = small_rb(n_blocks=3)
    ws, bs = synth.init_weights(5, layers, out_bias=(0.5, 1.0, -2.0))
    for i, ly in enumerate(layers):
        if ly.kind in (synth.PW, synth.PWRES):
            ws[i][:] = 0.0
            bs[i][:] = 0.0
    plain = [ly for ly in layers if ly.kind in (synth.CONV, synth.FC)]
    keep = [i for i, ly in enumerate(layers) if ly.kind in (synth.CONV, synth.FC)]
    x = rand_windows(3, 3)
    for prec in (0, 1):
        a = oracle_lib.Model(layers, ws, bs, D, L, prec=prec).forward(x)
        b = oracle_lib.Model(plain, [ws[i] for i in keep], [bs[i] for i in keep], D, L,
                             prec=prec).forward(x)
        np.testing.assert_array_equal(a, b)


def test_selector_block_by_hand(oracle_lib):
    """One block on a 2-slot, 2-feature window with identity-like convs:
    the expansion copies channel 0 and the negated channel 1, the
    projection sends them to channels 1 and 0, so the block output is
    (x0 + relu(-x1), x1 + relu(x0)) with the skip; worked by hand."""
    layers = [synth.Layer(synth.CONV, 2, 2, 0), synth.Layer(synth.PW, 2, 2, 1),
              synth.Layer(synth.PWRES, 2, 2, 0), synth.Layer(synth.FC, 2, 2, 0)]
    wc = np.zeros((2, 2, 2), np.float32)
    wc[0, 0, 0] = 1.0   # channel 0 <- slot 0 feature 0
    wc[1, 1, 1] = 1.0   # channel 1 <- slot 1 feature 1
    we = np.array([[1.0, 0.0], [0.0, -1.0]], np.float32).reshape(2, 2, 1)
    wp = np.array([[0.0, 1.0], [1.0, 0.0]], np.float32).reshape(2, 2, 1)
    wf = np.eye(2, dtype=np.float32)
    ws = [wc, we, wp, wf]
    bs = [np.zeros(2, np.float32)] * 4
    m = oracle_lib.Model(layers, ws, bs, 2, 2)
    for x0, x1 in [(3.0, 5.0), (-2.0, 4.0), (7.0, -6.0), (-1.0, -1.0)]:
        x = np.array([[[x0, 0.0], [0.0, x1]]])
        got = m.forward(x)[0]
        assert got[0] == x0 + max(-x1, 0.0) and got[1] == x1 + max(x0, 0.0), (x0, x1, got)


def test_residual_layers_rejected_where_undefined(oracle_lib):
    ok = small_rb(n_blocks=1)
    ws, bs = synth.init_weights(1, ok, out_bias=(0.0, 0.0, 0.0))
    # a residual half that does not follow a pointwise layer
    bad = ok[:3] + [ok[4]]
    with pytest.raises(ValueError):
        oracle_lib.Model(bad + ok[5:], ws[:3] + [ws[4]] + ws[5:], bs[:3] + [bs[4]] + bs[5:], D, L)
    # no FP8 form of a network with residual blocks
    with pytest.raises(ValueError):
        oracle_lib.Model(ok, ws, bs, D, L, prec=2, scales=np.ones(1000, np.float32))
