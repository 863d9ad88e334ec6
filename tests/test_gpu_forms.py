"""Reduced-precision forms of the predictor inside the step loop (BF16, FP8).

Each form is checked against the oracle's FP64 evaluation of the same form
(the same roundings at the same points, exact sums).  The GPU accumulates in
FP32, so a hidden activation can land on the other side of a rounding
boundary; the bar is one unit in the last place of the form at the output's
magnitude: |y_gpu - y_form| <= u * max(s, 1), u = 2^-8 for BF16 and 2^-4 for
FP8 (half of e4m3's 2^-3 spacing), s being the form's |b| + sum |w a| of the
output layer.  Cycle results are bit-exact given the same latencies.  FP8
scales come from each side's own calibration on identical windows and must
be equal."""
import numpy as np
import pytest

import synth
from tests.common import near_half, realistic_windows, rel_err

pytestmark = pytest.mark.gpu

FORMS = {"bf16": (1, 2.0 ** -8), "fp8": (2, 2.0 ** -4)}
CAL_STEPS = 64


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


def setup(torch, sn, oracle, net, N, K, warm, prec):
    if net == "small":
        layers, D, L = synth.net_small(), 32, 16
    else:
        layers, D, L = synth.net_c3(), 50, 111
    cols = synth.dynamic_columns(D)
    ws, bs = synth.init_weights(2, layers)
    feat = synth.trace_features(1, N, D)
    start, length, warm_ = sn.partition(N, K, warm)
    dfeat = dev(torch, feat)
    sim = sn.Simulator(dfeat, L, cols, start, length, warm_, prec=prec)
    sim.load_weights(layers, sn.flat_params(ws, bs))
    cfg = oracle.sim_cfg(D, L, 2, 8, cols)
    exact = oracle.Model(layers, ws, bs, D, L)
    scales = None
    if prec == 2:
        # both sides calibrate on the same windows: latencies injected
        n_pred = int(length.sum() + warm_.sum())
        table = synth.latency_table(77, n_pred, 2)
        sim.calibrate(CAL_STEPS, sn.SIM_LAT_INJECT, dev(torch, table))
        amax = oracle.calibrate(cfg, feat, start, length, warm_, exact, CAL_STEPS, lat_table=table)
        scales = oracle.fp8_scales(amax)
        np.testing.assert_array_equal(sim.act_scales()[:scales.size], scales)
    form = oracle.Model(layers, ws, bs, D, L, prec=prec, scales=scales)
    return dict(sim=sim, feat=feat, dfeat=dfeat, cfg=cfg, form=form, exact=exact, start=start,
                scales=scales,
                len=length, warm=warm_, n_pred=int(length.sum() + warm_.sum()), layers=layers,
                ws=ws, bs=bs)


@pytest.mark.parametrize("form", sorted(FORMS))
@pytest.mark.parametrize("net", ["small", "c3"])
@pytest.mark.parametrize("B", [1, 37, 100])
def test_forward_form_parity(torch, sn, oracle_lib, form, net, B):
    prec, tol = FORMS[form]
    S = setup(torch, sn, oracle_lib, net, 3000, 1, 0, prec)
    x = realistic_windows(S["cfg"], S["feat"], B, seed=B + 1)
    got = S["sim"].forward(dev(torch, x)).cpu().numpy()
    ref, scale = S["form"].forward(x.astype(np.float64), want_scale=True)
    err = rel_err(got, ref, scale)
    assert err.max() <= tol, err.max()
    assert np.median(err) <= 1e-4, np.median(err)


@pytest.mark.parametrize("form", sorted(FORMS))
@pytest.mark.parametrize("net,N,K,warm", [("small", 4000, 9, 64), ("c3", 8000, 20, 256)])
def test_form_free_run_replayed_by_oracle(torch, sn, oracle_lib, form, net, N, K, warm):
    """A free run of the form, replayed by the oracle's evaluation of the same
    form from the GPU's own rounded latencies."""
    prec, tol = FORMS[form]
    S = setup(torch, sn, oracle_lib, net, N, K, warm, prec)
    logits = torch.zeros((S["n_pred"], 2), dtype=torch.float32, device="cuda")
    S["sim"].record_logits(logits)
    g = S["sim"].run()
    gl = logits.cpu().numpy().astype(np.float64)
    lat = np.clip(np.rint(gl), 0, 65535).astype(np.int32)
    rep = oracle_lib.simulate(S["cfg"], S["feat"], S["start"], S["len"], S["warm"],
                              model=S["form"], mode=oracle_lib.INJECT, lat_table=lat,
                              want_logits=True, want_scale=True)
    for key in ("fetch", "drain", "final", "warm_tick"):
        np.testing.assert_array_equal(g[key], rep[key], err_msg=key)
    err = rel_err(gl, rep["logits"], rep["scale"])
    assert err.max() <= tol, err.max()
    lat_o = np.clip(np.rint(rep["logits"]), 0, 65535).astype(np.int32)
    assert not np.any((lat_o != lat) & ~near_half(rep["logits"], rep["scale"], tol))


@pytest.mark.parametrize("net", ["small", "c3"])
def test_fp8_needs_calibration(torch, sn, oracle_lib, net):
    D, L, layers = (32, 16, synth.net_small()) if net == "small" else (50, 111, synth.net_c3())
    feat = dev(torch, synth.trace_features(1, 500, D))
    start, length, warm = sn.partition(500, 3, 0)
    sim = sn.Simulator(feat, L, synth.dynamic_columns(D), start, length, warm, prec=sn.SIM_FP8E4M3)
    ws, bs = synth.init_weights(2, layers)
    sim.load_weights(layers, sn.flat_params(ws, bs))
    with pytest.raises(sn.SimError) as e:
        sim.run()
    assert e.value.code == sn.SIM_ESTATE
    sim.calibrate(8)
    sim.run()
