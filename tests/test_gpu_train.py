"""Training form of the predictor on the GPU (Sec. 2.3's hybrid head, Sec. 4's
training set-up): forward with saved activations, hybrid loss, hand-written
backward, Adam, through the C ABI.

Bars.  The forward is held to the inference bar, |y32 - y64| <= 1e-5 *
max(s, 1) with s = |b| + sum |w a| of the head (BF16 form: 2^-8 * max(s, 1)
against the oracle's BF16 form).  Gradients are FP32 sums of up to B*52 or
3,328 products through five layers; each parameter tensor, dlogits and dx
are held to a normwise relative error of max(5e-5, 4 u sqrt(52 B)) against
the oracle's FP64 gradient (unit roundoff u = 6e-8 times the square root of
the longest sum, conv1's weight gradient over B * 52 positions, times a
depth margin: 5e-5 up to B = 40, 1.1e-4 at B = 4,096), and elementwise to
twice that of the tensor's largest entry.  The finite-difference check uses
the GPU's own FP32 loss along each layer's gradient direction, where the
derivative is the gradient's norm, on a 64-window batch.

The batch the training benchmark times (4,096 windows) is checked in both
forms: there the GEMMs dispatch differently from the small batches (no
split-K on the input-gradient products, which take the vector epilogue in
the BF16 form, and a deeper split on the weight gradients)."""
import numpy as np
import pytest

import synth
from tests.common import realistic_windows, rel_err

pytestmark = pytest.mark.gpu

D, L = 50, 111
COLS = synth.dynamic_columns(D)
CFG = (D, L, 2, 8, COLS[0], COLS[1], COLS[2])


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def sn():
    import paper_2105_05821_amd as m
    m.lib()
    return m


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def inputs(B, seed, with_rows=False):
    layers = synth.net_c3_hybrid()
    ws, bs = synth.init_weights(seed, layers, out_bias=None, out_gain=1.0)
    feat = synth.trace_features(1, 4000, D)
    x = realistic_windows(CFG, feat, B, seed=seed)
    rng = np.random.default_rng(seed)
    lat = rng.integers(0, 420, size=(B, 2)).astype(np.int32)  # includes the overflow class
    return layers, ws, bs, x, lat


def layer_slices(layers):
    out, off = [], 0
    for (ws, bs) in synth.layer_param_shapes(layers):
        n = int(np.prod(ws))
        out.append(("w", off, off + n))
        off += n
        out.append(("b", off, off + bs[0]))
        off += bs[0]
    return out


def normwise(got, ref):
    ref = np.asarray(ref, np.float64)
    return np.linalg.norm(np.asarray(got, np.float64) - ref) / max(np.linalg.norm(ref), 1e-300)


def f32_bar(B):
    return max(5e-5, 4 * 6e-8 * np.sqrt(52.0 * B))


def check_grad(name, got, ref, nw=5e-5, ew=1e-4):
    e = normwise(got, ref)
    m = np.abs(np.asarray(got, np.float64) - ref).max() / max(np.abs(ref).max(), 1e-300)
    assert e <= nw and m <= ew, (name, e, m)
    return e


@pytest.mark.parametrize("B", [1, 37])
def test_train_forward_parity_f32(torch, sn, oracle_lib, B):
    layers, ws, bs, x, _ = inputs(B, 11 + B)
    pred = sn.Predictor(layers, sn.SIM_FP32)
    pred.load_weights(layers, sn.flat_params(ws, bs))
    z, _ = pred.forward(dev(torch, x))
    ref, scale = oracle_lib.Model(layers, ws, bs, D, L).forward(x, want_scale=True)
    assert rel_err(z.cpu().numpy(), ref, scale).max() <= 1e-5
    pred.close()


def test_train_forward_parity_bf16(torch, sn, oracle_lib):
    B = 37
    layers, ws, bs, x, _ = inputs(B, 5)
    pred = sn.Predictor(layers, sn.SIM_BF16)
    pred.load_weights(layers, sn.flat_params(ws, bs))
    z, _ = pred.forward(dev(torch, x))
    ref, scale = oracle_lib.Model(layers, ws, bs, D, L, prec=1).forward(x, want_scale=True)
    err = rel_err(z.cpu().numpy(), ref, scale)
    assert err.max() <= 2.0 ** -8 and np.median(err) <= 1e-4, (err.max(), np.median(err))
    pred.close()


def gpu_grads(torch, sn, pred, x, lat, want_dx=True):
    dx_ = dev(torch, x)
    z, save = pred.forward(dx_)
    loss, dz = pred.loss(z, dev(torch, lat))
    dparams = torch.empty(2_204_642, dtype=torch.float32, device="cuda")
    dx = pred.backward(dx_, save, dz, dparams, want_dx=want_dx)
    torch.cuda.synchronize()
    return (float(loss.item()), dz.cpu().numpy(), dparams.cpu().numpy(),
            None if dx is None else dx.cpu().numpy())


@pytest.mark.parametrize("B", [1, 37])
def test_train_gradients_match_oracle_f32(torch, sn, oracle_lib, B):
    layers, ws, bs, x, lat = inputs(B, 21 + B)
    pred = sn.Predictor(layers, sn.SIM_FP32)
    pred.load_weights(layers, sn.flat_params(ws, bs))
    loss, dz, dp, dx = gpu_grads(torch, sn, pred, x, lat)
    ref = oracle_lib.train_step(oracle_lib.Model(layers, ws, bs, D, L), x, lat,
                                want_dlogits=True, want_dx=True)
    assert abs(loss - ref["loss"]) <= 1e-5 * abs(ref["loss"])
    bar = f32_bar(B)
    check_grad("dlogits", dz, ref["dlogits"], bar, 2 * bar)
    for (kind, lo, hi), li in zip(layer_slices(layers), np.repeat(np.arange(len(layers)), 2)):
        check_grad(f"layer {li} {kind}", dp[lo:hi], ref["dparams"][lo:hi], bar, 2 * bar)
    check_grad("dx", dx, ref["dx"], bar, 2 * bar)
    # slots past the 104 that feed conv1 get no gradient
    assert not np.any(dx[:, 104:, :])
    pred.close()


def test_train_gradients_bf16_form_match_oracle(torch, sn, oracle_lib):
    """BF16 form against the oracle's FP64 evaluation of the same form (the
    same values rounded to bfloat16 at the same points).  The GPU sums in
    FP32, so a value whose FP32 sum lands on the other side of a bfloat16
    rounding boundary moves by one bfloat16 unit (2^-8 relative) and carries
    that into what it feeds; such values are a small fraction, so each
    tensor's normwise relative error stays well under one unit: bar 2^-8.
    The loss is held to 1e-4 relative."""
    B = 40
    layers, ws, bs, x, lat = inputs(B, 51)
    pred = sn.Predictor(layers, sn.SIM_BF16)
    pred.load_weights(layers, sn.flat_params(ws, bs))
    loss, dz, dp, dx = gpu_grads(torch, sn, pred, x, lat)
    ref = oracle_lib.train_step(oracle_lib.Model(layers, ws, bs, D, L, prec=1), x, lat,
                                want_dlogits=True, want_dx=True)
    assert abs(loss - ref["loss"]) <= 1e-4 * abs(ref["loss"]), (loss, ref["loss"])
    errs = {"dlogits": normwise(dz, ref["dlogits"]), "dx": normwise(dx, ref["dx"])}
    for (kind, lo, hi), li in zip(layer_slices(layers), np.repeat(np.arange(len(layers)), 2)):
        errs[f"{li}{kind}"] = normwise(dp[lo:hi], ref["dparams"][lo:hi])
    print("bf16 form gradient normwise errors", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) <= 2.0 ** -8, errs
    pred.close()


def full_batch_grads(torch, sn, oracle_lib, layers, ws, bs, x, lat, prec):
    pred = sn.Predictor(layers, sn.SIM_FP32 if prec == 0 else sn.SIM_BF16)
    pred.load_weights(layers, sn.flat_params(ws, bs))
    loss, dz, dp, dx = gpu_grads(torch, sn, pred, x, lat)
    pred.close()
    ref = oracle_lib.train_step(oracle_lib.Model(layers, ws, bs, D, L, prec=prec), x, lat,
                                want_dlogits=True, want_dx=True)
    return loss, dz, dp, dx, ref


def test_train_gradients_full_batch_f32(torch, sn, oracle_lib):
    """4,096 windows, the training benchmark's batch, FP32 against the
    oracle's FP64 gradient.

    At this size a few windows have a pre-activation within FP32 rounding
    of zero, so their ReLU mask differs from FP64's and their gradient
    differs by O(1) (PyTorch's own FP32 autograd on this batch: 3 of 4,096
    windows, per-window dx errors up to 2.7 %, the other windows' median
    5e-7).  A window's input gradient depends on its own forward only, so
    the check has two passes: (1) the whole batch: loss, dlogits, and the
    input gradient window by window, where at most 0.5 % of the windows may
    exceed the bar (each then a ReLU-boundary window); (2) the batch without
    those windows (the same GEMM paths), where the loss and every tensor are
    held to the bar."""
    B = 4096
    layers, ws, bs, x, lat = inputs(B, 61)
    loss, dz, dp, dx, ref = full_batch_grads(torch, sn, oracle_lib, layers, ws, bs, x, lat, 0)
    bar = f32_bar(B)
    assert abs(loss - ref["loss"]) <= 1e-5 * abs(ref["loss"]), (loss, ref["loss"])
    check_grad("dlogits", dz, ref["dlogits"], bar, 2 * bar)
    rx = ref["dx"].reshape(B, -1)
    pw = (np.linalg.norm(dx.reshape(B, -1) - rx, axis=1)
          / np.maximum(np.linalg.norm(rx, axis=1), 1e-300))
    kink = pw > bar
    print(f"f32 B={B}: {int(kink.sum())} windows past the bar, per-window dx error median "
          f"{np.median(pw):.2e} max {pw.max():.2e}")
    assert kink.mean() <= 0.005, int(kink.sum())
    assert not np.any(dx[:, 104:, :])

    keep = ~kink
    B2 = int(keep.sum())
    loss, dz, dp, dx, ref = full_batch_grads(torch, sn, oracle_lib, layers, ws, bs,
                                             np.ascontiguousarray(x[keep]),
                                             np.ascontiguousarray(lat[keep]), 0)
    bar = f32_bar(B2)
    assert abs(loss - ref["loss"]) <= 1e-5 * abs(ref["loss"]), (loss, ref["loss"])
    errs = {"dlogits": check_grad("dlogits", dz, ref["dlogits"], bar, 2 * bar),
            "dx": check_grad("dx", dx, ref["dx"], bar, 2 * bar)}
    for (kind, lo, hi), li in zip(layer_slices(layers), np.repeat(np.arange(len(layers)), 2)):
        errs[f"{li}{kind}"] = check_grad(f"layer {li} {kind}", dp[lo:hi], ref["dparams"][lo:hi],
                                         bar, 2 * bar)
    print(f"f32 B={B2} gradient normwise errors", {k: f"{v:.2e}" for k, v in errs.items()})


def test_train_gradients_full_batch_bf16_form(torch, sn, oracle_lib):
    """4,096 windows in the BF16 form against the oracle's FP64 evaluation of
    the same form: every tensor within 2^-8 normwise, as at B = 40 (the few
    ReLU-boundary windows move the sums by well under one bfloat16 unit)."""
    B = 4096
    layers, ws, bs, x, lat = inputs(B, 62)
    loss, dz, dp, dx, ref = full_batch_grads(torch, sn, oracle_lib, layers, ws, bs, x, lat, 1)
    assert abs(loss - ref["loss"]) <= 1e-4 * abs(ref["loss"]), (loss, ref["loss"])
    errs = {"dlogits": normwise(dz, ref["dlogits"]), "dx": normwise(dx, ref["dx"])}
    for (kind, lo, hi), li in zip(layer_slices(layers), np.repeat(np.arange(len(layers)), 2)):
        errs[f"{li}{kind}"] = normwise(dp[lo:hi], ref["dparams"][lo:hi])
    print(f"bf16 form B={B} gradient normwise errors", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) <= 2.0 ** -8, errs
    assert not np.any(dx[:, 104:, :])


def test_train_finite_differences_f32(torch, sn):
    """(L(p + h u) - L(p - h u)) / 2h along u = g_l / |g_l| for each layer's
    weight tensor, and along dx / |dx| for the windows; the GPU loss at the
    perturbed parameters is the FP32 forward + loss."""
    B = 24
    layers, ws, bs, x, lat = inputs(B, 31)
    p0 = sn.flat_params(ws, bs).astype(np.float64)
    pred = sn.Predictor(layers, sn.SIM_FP32)
    pred.load_weights(layers, p0.astype(np.float32))
    _, _, g, gx = gpu_grads(torch, sn, pred, x, lat)
    dlat = dev(torch, lat)

    def loss_at(p, xx):
        pred.load_weights(layers, np.asarray(p, np.float32))
        z, _ = pred.forward(dev(torch, np.asarray(xx, np.float32)))
        loss, _ = pred.loss(z, dlat)
        return float(loss.item())

    for kind, lo, hi in layer_slices(layers):
        if kind != "w":
            continue
        gl = g[lo:hi].astype(np.float64)
        n = np.linalg.norm(gl)
        u = np.zeros_like(p0)
        u[lo:hi] = gl / n
        h = 1e-2 * np.linalg.norm(p0[lo:hi]) / np.sqrt(hi - lo)
        fd = (loss_at(p0 + h * u, x) - loss_at(p0 - h * u, x)) / (2 * h)
        assert abs(fd - n) <= 2e-2 * n, (lo, fd, n)
    n = np.linalg.norm(gx)
    h = 1e-2
    fd = (loss_at(p0, x + h * gx / n) - loss_at(p0, x - h * gx / n)) / (2 * h)
    assert abs(fd - n) <= 2e-2 * n, ("dx", fd, n)
    pred.close()


def test_train_accumulate_and_autograd(torch, sn):
    """accumulate=1 adds to dparams; the torch.autograd.Function returns the
    same gradients as predictor_bwd for the same upstream gradient."""
    B = 20
    layers, ws, bs, x, lat = inputs(B, 41)
    flat = sn.flat_params(ws, bs)
    pred = sn.Predictor(layers, sn.SIM_FP32)
    pred.load_weights(layers, flat)
    xd = dev(torch, x)
    z, save = pred.forward(xd)
    gen = torch.Generator(device="cpu").manual_seed(0)
    up = torch.randn(z.shape, generator=gen).cuda()
    g1 = torch.empty(flat.size, dtype=torch.float32, device="cuda")
    dx = pred.backward(xd, save, up, g1, want_dx=True)
    g2 = g1.clone()
    pred.backward(xd, save, up, g2, accumulate=True)
    torch.cuda.synchronize()
    np.testing.assert_allclose(g2.cpu().numpy(), 2 * g1.cpu().numpy(), rtol=1e-6,
                               atol=1e-6 * float(g1.abs().max()))
    params = dev(torch, flat).requires_grad_(True)
    xa = xd.clone().requires_grad_(True)
    za = sn.predictor_apply(xa, params, pred)
    (za * up).sum().backward()
    np.testing.assert_array_equal(za.detach().cpu().numpy(), z.cpu().numpy())
    np.testing.assert_array_equal(params.grad.cpu().numpy(), g1.cpu().numpy())
    np.testing.assert_array_equal(xa.grad.cpu().numpy(), dx.cpu().numpy())
    pred.close()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_adam_load_equals_adam_then_load_weights(torch, sn, prec):
    """sim_adam_load (the update and the re-layout in one pass) leaves the
    same parameters and moments as sim_adam and the same kernel weights as
    a following sim_load_weights: bit-identical parameters, forward outputs
    and gradients over three steps; a wrong parameter count is refused."""
    B = 40
    layers, ws, bs, x, lat = inputs(B, 43)
    flat = sn.flat_params(ws, bs)
    form = sn.SIM_FP32 if prec == "f32" else sn.SIM_BF16
    p1, p2 = sn.Predictor(layers, form), sn.Predictor(layers, form)
    w1, w2 = dev(torch, flat), dev(torch, flat)
    p1.load_weights(layers, w1)
    p2.load_weights(layers, w2)
    m1, v1 = torch.zeros_like(w1), torch.zeros_like(w1)
    m2, v2 = torch.zeros_like(w1), torch.zeros_like(w1)
    xd = dev(torch, x)
    gen = torch.Generator(device="cpu").manual_seed(5)
    for t in range(1, 4):
        g = (torch.randn(flat.size, generator=gen) * 0.1).cuda()
        p1.adam(w1, g, m1, v1, t, lr=1e-2)
        p1.load_weights(layers, w1)
        p2.adam_load(w2, g, m2, v2, t, lr=1e-2)
        torch.cuda.synchronize()
        for a, b in ((w1, w2), (m1, m2), (v1, v2)):
            np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
        z1, s1 = p1.forward(xd)
        z2, s2 = p2.forward(xd)
        np.testing.assert_array_equal(z1.cpu().numpy(), z2.cpu().numpy())
        up = torch.randn(z1.shape, generator=gen).cuda()
        g1 = torch.empty_like(w1)
        g2 = torch.empty_like(w1)
        d1 = p1.backward(xd, s1, up, g1, want_dx=True)
        d2 = p2.backward(xd, s2, up, g2, want_dx=True)
        np.testing.assert_array_equal(g1.cpu().numpy(), g2.cpu().numpy())
        np.testing.assert_array_equal(d1.cpu().numpy(), d2.cpu().numpy())
    with pytest.raises(sn.SimError) as e:
        p2.adam_load(w2[:-1], g[:-1], m2[:-1], v2[:-1], 4)
    assert e.value.code == sn.SIM_EINVAL
    p1.close()
    p2.close()


def analytic_batch(B, seed):
    """Windows ending at trace row i with the analytic model's latencies of
    row i as labels."""
    fields = synth.trace_fields(1, 0, 4000)
    feat = synth.trace_features(1, 4000, D)
    lab = synth.analytic_latencies(fields)
    rng = np.random.default_rng(seed)
    rows = rng.integers(L, 4000, size=B)
    x = np.zeros((B, L, D), np.float32)
    for b, i in enumerate(rows):
        occ = int(rng.integers(0, L))
        x[b, 0] = feat[i]
        x[b, 0, COLS[0]] = 0
        x[b, 0, COLS[1]] = 0
        for k in range(1, occ + 1):
            x[b, k] = feat[i - k]
            x[b, k, COLS[0]] = k
            x[b, k, COLS[1]] = lab[i - k, 1]
    return x, lab[rows].astype(np.int32)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_trainer_reduces_loss(torch, sn, prec):
    layers = synth.net_c3_hybrid()
    ws, bs = synth.init_weights(3, layers, out_bias=None, out_gain=1.0)
    x, lat = analytic_batch(64, 3)
    tr = sn.Trainer(layers, sn.flat_params(ws, bs),
                    prec=sn.SIM_FP32 if prec == "f32" else sn.SIM_BF16, lr=1e-3)
    xd, ld = dev(torch, x), dev(torch, lat)
    losses = [float(tr.step(xd, ld).item()) for _ in range(30)]
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0], losses
    tr.close()
