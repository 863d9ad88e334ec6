"""RB7 on the GPU (Sec. 2.3, residual blocks; the model table's deepest CNN
with the hybrid head): the C3 convolutions inside the gather, seven
residual blocks over every window's 13 positions, FC 512 and the hybrid
head, then the update, as separate kernels per step.

Bars: outputs FP32 1e-5 * max(s, 1), BF16 form 2^-8 * max(s, 1) against the
oracle's BF16 form; cycles bit-exact against the oracle replaying the GPU's
latencies; the oracle's own decisions agree outside the tie band (as for
the C3 hybrid head)."""
import numpy as np
import pytest

import synth
from tests.common import realistic_windows, rel_err
from tests.test_gpu_hybrid import ambiguous, select_all

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


@pytest.fixture(scope="module")
def rb7():
    layers = synth.net_rb7()
    ws, bs = synth.init_weights(2, layers, out_bias=synth.HYB_BIAS)
    return layers, ws, bs


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("B", [1, 37])
def test_rb7_forward_parity(torch, sn, oracle_lib, rb7, prec, B):
    """predictor_fwd: a ragged last tile of windows and of block rows."""
    layers, ws, bs = rb7
    feat = synth.trace_features(1, 3000, D)
    x = realistic_windows(CFG, feat, B, seed=B + 5)
    sim = sn.Simulator(torch.from_numpy(feat).cuda(), L, COLS, *sn.partition(3000, 1, 0),
                       prec=prec)
    sim.load_weights(layers, sn.flat_params(ws, bs))
    got = sim.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    assert got.shape == (B, 22)
    ref, scale = oracle_lib.Model(layers, ws, bs, D, L, prec=prec).forward(x, want_scale=True)
    err = rel_err(got, ref, scale)
    assert err.max() <= TOL[prec], err.max()
    sim.close()


def test_rb7_blocks_matter(torch, sn, rb7):
    """The residual blocks change the outputs (zeroing them gives the C3
    hybrid network's outputs on the same trunk, FC and head weights)."""
    layers, ws, bs = rb7
    feat = synth.trace_features(1, 3000, D)
    x = torch.from_numpy(realistic_windows(CFG, feat, 20, seed=9)).cuda()
    sim = sn.Simulator(torch.from_numpy(feat).cuda(), L, COLS, *sn.partition(3000, 1, 0))
    sim.load_weights(layers, sn.flat_params(ws, bs))
    full = sim.forward(x).cpu().numpy()
    ws0 = [w.copy() for w in ws]
    bs0 = [b.copy() for b in bs]
    for i, ly in enumerate(layers):
        if ly.kind in (synth.PW, synth.PWRES):
            ws0[i][:] = 0.0
            bs0[i][:] = 0.0
    sim.load_weights(layers, sn.flat_params(ws0, bs0))
    zeroed = sim.forward(x).cpu().numpy()
    plain = synth.net_c3_hybrid_infer()
    keep = [i for i, ly in enumerate(layers) if ly.kind in (synth.CONV, synth.FC)]
    sim.load_weights(plain, sn.flat_params([ws[i] for i in keep], [bs[i] for i in keep]))
    c3 = sim.forward(x).cpu().numpy()
    np.testing.assert_allclose(zeroed, c3, rtol=1e-6, atol=1e-5)
    assert np.abs(full - c3).max() > 1e-2
    sim.close()


def uneven(K, seed, lo=2, hi=40):
    rng = np.random.default_rng(seed)
    length = rng.integers(lo, hi, size=K).astype(np.int64)
    start = np.concatenate([[0], np.cumsum(length)[:-1]]).astype(np.int64)
    warm = np.minimum(start, rng.integers(0, 6, size=K)).astype(np.int32)
    return start, length, warm, int(length.sum())


@pytest.mark.parametrize("prec", [0, 1])
def test_rb7_free_run_replayed_by_oracle(torch, sn, oracle_lib, rb7, prec):
    """Uneven sub-traces over three workgroups (the last partly empty, slots
    finishing at different steps): the GPU's latencies replayed by the
    oracle give the same cycles; outputs within the bar; the oracle's own
    decisions agree outside the tie band; shadow mode reproduces every
    decision."""
    layers, ws, bs = rb7
    start, length, warm, N = uneven(40, 3 + prec)
    feat = synth.trace_features(1, N, D)
    sim = sn.Simulator(torch.from_numpy(feat).cuda(), L, COLS, start, length, warm, prec=prec)
    sim.load_weights(layers, sn.flat_params(ws, bs))
    lg = torch.zeros((sim.n_pred, 22), dtype=torch.float32, device="cuda")
    sim.record_logits(lg)
    g = sim.run()
    z32 = lg.cpu().numpy().astype(np.float64)
    lat = select_all(oracle_lib, z32)
    cfg = oracle_lib.sim_cfg(D, L, 2, 8, COLS, head=1)
    form = oracle_lib.Model(layers, ws, bs, D, L, prec=prec)
    o = oracle_lib.simulate(cfg, feat, start, length, warm, model=form, mode=oracle_lib.INJECT,
                            lat_table=lat, want_logits=True, want_scale=True)
    for k in ("fetch", "drain", "final", "warm_tick"):
        np.testing.assert_array_equal(g[k], o[k], err_msg=k)
    err = rel_err(z32, o["logits"], o["scale"])
    assert err.max() <= TOL[prec], err.max()
    own = select_all(oracle_lib, o["logits"])
    diff = own != lat
    assert not np.any(diff & ~ambiguous(o["logits"], o["scale"], TOL[prec]))
    sim.reset()
    s = sim.run(sn.SIM_LAT_SHADOW, torch.from_numpy(lat).cuda())
    assert s["n_shadow_mismatch"] == 0 and s["total"] == g["total"]
    sim.close()


def test_rb7_inject_and_steps(torch, sn, oracle_lib, rb7):
    """Injected latencies need no predictor and are bit-exact; sim_step in
    pieces then a run to the end equals one run; a graph request is served
    eagerly with the same result; FP8 is refused."""
    layers, ws, bs = rb7
    start, length, warm, N = uneven(24, 7)
    feat = synth.trace_features(1, N, D)
    dfeat = torch.from_numpy(feat).cuda()
    n_pred = int(length.sum() + warm.sum())
    rng = np.random.default_rng(1)
    table = np.stack([rng.integers(0, 3, n_pred), rng.integers(0, 30, n_pred)], 1).astype(np.int32)
    sim = sn.Simulator(dfeat, L, COLS, start, length, warm, prec=1)
    sim.load_weights(layers, sn.flat_params(ws, bs))
    g = sim.run(sn.SIM_LAT_INJECT, torch.from_numpy(table).cuda())
    o = oracle_lib.simulate(oracle_lib.sim_cfg(D, L, 2, 8, COLS), feat, start, length, warm,
                            mode=oracle_lib.INJECT, lat_table=table)
    for k in ("fetch", "drain", "final", "warm_tick"):
        np.testing.assert_array_equal(g[k], o[k], err_msg=k)
    sim.reset()
    ref = sim.run()
    sim.reset()
    sim.step(5)
    sim.step(3)
    part = sim.run()
    assert part["total"] == ref["total"]
    np.testing.assert_array_equal(part["final"], ref["final"])
    sim.use_graph(True)
    sim.reset()
    gr = sim.run()
    assert gr["total"] == ref["total"]
    sim.close()
    sim8 = sn.Simulator(dfeat, L, COLS, start, length, warm, prec=2)
    with pytest.raises(sn.SimError) as ei:
        sim8.load_weights(layers, sn.flat_params(ws, bs))
    assert ei.value.code == sn.SIM_EUNSUPPORTED
    sim8.close()
