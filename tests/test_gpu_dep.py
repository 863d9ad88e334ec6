"""Memory dependency flags built in the gather (Sec. 2.1): five flags per
context instruction (same instruction cache line, instruction page, data
address, data cache line, data page as the current instruction), from the
trace's program counters and data addresses.  Window contents read back
through a selector network must equal the oracle's exactly; free runs are
replayed by the oracle (FP32 bar 1e-5 * max(s, 1))."""
import numpy as np
import pytest

import synth
from tests.common import near_half, rel_err

pytestmark = pytest.mark.gpu

D, L = 50, 111
COLS = synth.dynamic_columns(D)
DC = synth.DEP_COLS


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


def selector(slot, col):
    """C3 weights whose fetch output is x[slot][col] (>= 0, so every ReLU
    passes it) and whose execution output is 0."""
    layers = synth.net_c3()
    shapes = synth.layer_param_shapes(layers)
    ws = [np.zeros(w, np.float32) for w, _ in shapes]
    bs = [np.zeros(b, np.float32) for _, b in shapes]
    ws[0][0, col, slot % 2] = 1.0
    ws[1][0, 0, (slot // 2) % 2] = 1.0
    ws[2][0, 0, (slot // 4) % 2] = 1.0
    ws[3][0, slot // 8] = 1.0
    ws[4][0, 0] = 1.0
    return layers, ws, bs


@pytest.mark.parametrize("codes", [False, True])
@pytest.mark.parametrize("slot,f", [(0, 0), (1, 0), (1, 3), (2, 1), (5, 2), (9, 4), (30, 3),
                                    (64, 1), (103, 0)])
def test_dependency_flags_window(torch, sn, oracle_lib, slot, f, codes):
    N, K = 8000, 32
    feat = synth.trace_features(1, N, D)
    mem = synth.trace_mem(1, N)
    start, length, warm = sn.partition(N, K, 16)
    n_pred = int(length.sum() + warm.sum())
    rng = np.random.default_rng(slot * 5 + f)
    F = rng.integers(0, 2, size=n_pred)
    F[rng.random(n_pred) < 0.6] = 0
    table = np.stack([F, rng.integers(0, 80, size=n_pred)], 1).astype(np.int32)
    layers, ws, bs = selector(slot, DC + f)
    t = dev(torch, synth.trace_codes(1, N).view(np.int32)) if codes else dev(torch, feat)
    dmem = dev(torch, mem.view(np.int32))
    sim = sn.Simulator(t, L, COLS, start, length, warm, n_feat=D if codes else None, mem=dmem,
                       col_dep=DC)
    sim.load_weights(layers, sn.flat_params(ws, bs))
    lg = torch.zeros((n_pred, 2), dtype=torch.float32, device="cuda")
    sim.record_logits(lg)
    sim.run(sn.SIM_LAT_SHADOW, dev(torch, table))
    cfg = oracle_lib.sim_cfg(D, L, 2, 8, COLS, dep_col=DC)
    o = oracle_lib.simulate(cfg, feat, start, length, warm,
                            model=oracle_lib.Model(layers, ws, bs, D, L), mode=oracle_lib.INJECT,
                            lat_table=table, want_logits=True, mem=mem)
    got = lg.cpu().numpy()[:, 0].astype(np.float64)
    np.testing.assert_array_equal(got, o["logits"][:, 0])
    if slot == 0:
        assert not np.any(got)
    else:
        assert 0 < np.count_nonzero(got)
    sim.close()


def test_dependency_flags_free_run(torch, sn, oracle_lib):
    wl = synth.workload("c3dep_1m")
    ws, bs = synth.init_weights(2, wl.layers)
    N, K = 6000, 24
    feat = synth.trace_features(1, N, D)
    mem = synth.trace_mem(1, N)
    start, length, warm = sn.partition(N, K, 64)
    sim = sn.Simulator(dev(torch, feat), L, COLS, start, length, warm,
                       mem=dev(torch, mem.view(np.int32)), col_dep=DC)
    sim.load_weights(wl.layers, sn.flat_params(ws, bs))
    lg = torch.zeros((sim.n_pred, 2), dtype=torch.float32, device="cuda")
    sim.record_logits(lg)
    g = sim.run()
    z = lg.cpu().numpy().astype(np.float64)
    lat = np.clip(np.rint(z), 0, 65535).astype(np.int32)
    cfg = oracle_lib.sim_cfg(D, L, 2, 8, COLS, dep_col=DC)
    m = oracle_lib.Model(wl.layers, ws, bs, D, L)
    o = oracle_lib.simulate(cfg, feat, start, length, warm, model=m, mode=oracle_lib.INJECT,
                            lat_table=lat, want_logits=True, want_scale=True, mem=mem)
    for k in ("fetch", "drain", "final", "warm_tick"):
        np.testing.assert_array_equal(g[k], o[k], err_msg=k)
    assert rel_err(z, o["logits"], o["scale"]).max() <= 1e-5
    own = np.clip(np.rint(o["logits"]), 0, 65535).astype(np.int32)
    assert not np.any((own != lat) & ~near_half(o["logits"], o["scale"], 1e-5))
    # the flags change the predictions: without them the run differs
    o0 = oracle_lib.simulate(oracle_lib.sim_cfg(D, L, 2, 8, COLS), feat, start, length, warm,
                             model=m, want_logits=True)
    assert not np.array_equal(o0["logits"], o["logits"])
    sim.close()
