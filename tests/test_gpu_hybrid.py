"""The hybrid inference head inside the step (Sec. 2.3, from output to
latency): per latency type 10 class scores and one direct output; the most
probable class is the latency unless it is the "larger than 8" class, whose
latency is the rounded direct output.

Bars: outputs as the regression head's (FP32 1e-5 * max(s, 1); BF16 form
2^-8 * max(s, 1) against the oracle's BF16 form).  Decisions: the kernel
decides in FP32 from its own outputs; the oracle, replaying the GPU's
latencies, must reproduce its cycles exactly, and its own FP64 decisions
must agree wherever they are not within the output bar of a tie (two top
class scores, or a direct output within the bar of a .5 boundary)."""
import numpy as np
import pytest

import synth
from tests.common import realistic_windows, rel_err

pytestmark = pytest.mark.gpu

D, L = 50, 111
COLS = synth.dynamic_columns(D)
CFG = (D, L, 2, 8, COLS[0], COLS[1], COLS[2])
TOL = {0: 1e-5, 1: 2.0 ** -8}


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


def hybrid_weights(seed=2):
    layers = synth.net_c3_hybrid_infer()
    ws, bs = synth.init_weights(seed, layers, out_bias=synth.HYB_BIAS)
    return layers, ws, bs


def select_all(oracle_lib, z):
    """Latencies [n][2] from [n][22] outputs by the oracle's rule."""
    out = np.zeros((z.shape[0], 2), np.int32)
    for i in range(z.shape[0]):
        for t in range(2):
            out[i, t] = oracle_lib.hybrid_select(z[i, t * 11:(t + 1) * 11])[0]
    return out


def ambiguous(z, scale, tol):
    """Per (prediction, type): the decision may legitimately differ between
    an FP32 and an FP64 evaluation of the same outputs."""
    amb = np.zeros((z.shape[0], 2), bool)
    for t in range(2):
        cls = z[:, t * 11:t * 11 + 10]
        band = tol * np.maximum(scale[:, t * 11:t * 11 + 10].max(axis=1), 1.0)
        top2 = np.sort(cls, axis=1)[:, -2:]
        near_tie = top2[:, 1] - top2[:, 0] <= 2 * band
        reg = z[:, t * 11 + 10]
        rband = tol * np.maximum(scale[:, t * 11 + 10], 1.0)
        near_half = np.abs(reg - np.floor(reg) - 0.5) <= rband
        larger = np.argmax(cls, axis=1) == 9
        amb[:, t] = near_tie | (larger & near_half)
    return amb


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("B", [1, 37])
def test_hybrid_forward_parity(torch, sn, oracle_lib, prec, B):
    layers, ws, bs = hybrid_weights()
    feat = synth.trace_features(1, 3000, D)
    x = realistic_windows(CFG, feat, B, seed=B)
    sim = sn.Simulator(torch.from_numpy(feat).cuda(), L, COLS, *sn.partition(3000, 1, 0),
                       prec=prec)
    sim.load_weights(layers, sn.flat_params(ws, bs))
    got = sim.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    assert got.shape == (B, 22)
    ref, scale = oracle_lib.Model(layers, ws, bs, D, L, prec=prec).forward(x, want_scale=True)
    err = rel_err(got, ref, scale)
    assert err.max() <= TOL[prec], err.max()
    sim.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_hybrid_free_run_replayed_by_oracle(torch, sn, oracle_lib, prec):
    layers, ws, bs = hybrid_weights()
    N, K = 4000, 24
    feat = synth.trace_features(1, N, D)
    start, length, warm = sn.partition(N, K, 64)
    sim = sn.Simulator(torch.from_numpy(feat).cuda(), L, COLS, start, length, warm, prec=prec)
    sim.load_weights(layers, sn.flat_params(ws, bs))
    lg = torch.zeros((sim.n_pred, 22), dtype=torch.float32, device="cuda")
    sim.record_logits(lg)
    g = sim.run()
    z32 = lg.cpu().numpy().astype(np.float64)
    lat = select_all(oracle_lib, z32)
    # both regimes occur: classes and the direct output
    assert (lat[:, 1] > 8).any() and (lat[:, 0] <= 8).any()
    cfg = oracle_lib.sim_cfg(D, L, 2, 8, COLS, head=1)
    form = oracle_lib.Model(layers, ws, bs, D, L, prec=prec)
    o = oracle_lib.simulate(cfg, feat, start, length, warm, model=form, mode=oracle_lib.INJECT,
                            lat_table=lat, want_logits=True, want_scale=True, want_lat=True)
    for k in ("fetch", "drain", "final", "warm_tick"):
        np.testing.assert_array_equal(g[k], o[k], err_msg=k)
    err = rel_err(z32, o["logits"], o["scale"])
    assert err.max() <= TOL[prec], err.max()
    own = select_all(oracle_lib, o["logits"])
    diff = own != lat
    amb = ambiguous(o["logits"], o["scale"], TOL[prec])
    assert not np.any(diff & ~amb), int(np.sum(diff & ~amb))
    # the same latencies injected in shadow mode: every decision reproduced
    sim.reset()
    s = sim.run(sn.SIM_LAT_SHADOW, torch.from_numpy(lat).cuda())
    assert s["n_shadow_mismatch"] == 0 and s["total"] == g["total"]
    sim.close()


def test_hybrid_graph_replay_and_fp8_rejected(torch, sn):
    layers, ws, bs = hybrid_weights()
    N, K = 2000, 16
    feat = synth.trace_features(1, N, D)
    start, length, warm = sn.partition(N, K, 0)
    dfeat = torch.from_numpy(feat).cuda()
    sim = sn.Simulator(dfeat, L, COLS, start, length, warm, prec=1)
    sim.load_weights(layers, sn.flat_params(ws, bs))
    ref = sim.run()
    sim.use_graph(True)
    for _ in range(3):
        sim.reset()
        torch.cuda.synchronize()
        r = sim.run()
        assert r["total"] == ref["total"]
        np.testing.assert_array_equal(r["final"], ref["final"])
    sim.close()
    sim8 = sn.Simulator(dfeat, L, COLS, start, length, warm, prec=2)
    with pytest.raises(sn.SimError) as ei:
        sim8.load_weights(layers, sn.flat_params(ws, bs))
    assert ei.value.code == sn.SIM_EUNSUPPORTED
    sim8.close()
