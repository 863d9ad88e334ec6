"""Store latency and the memory write queue on the GPU (Sec. 3.2, context
management): three latencies per instruction; a store enters the memory
write queue when it leaves the processor queue and leaves it, in order, when
its residence exceeds its store latency; the context shows the processor
queue newest first, then the memory write queue newest first.

Integer results are bit-exact against the oracle's cycle-by-cycle two-queue
model given the same latencies; the window contents are read back through a
selector network (exact small integers); free runs are replayed by the
oracle as for the two-latency path (FP32 bar 1e-5 * max(s, 1))."""
import numpy as np
import pytest

import synth
from tests.common import near_half, realistic_windows, rel_err

pytestmark = pytest.mark.gpu

D, L = 50, 111
COLS = synth.dynamic_columns(D)   # residence 47, execution 48, store 49
SC = synth.STORE_COL


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


def ocfg(oracle_lib, W=8):
    return oracle_lib.sim_cfg(D, L, 3, W, COLS, store_col=SC)


def assert_same(g, o):
    for k in ("fetch", "drain", "final", "warm_tick"):
        np.testing.assert_array_equal(g[k], o[k], err_msg=k)
    assert g["total"] == o["total"]


def store_table(seed, n, f_hi=3, e_hi=40, s_hi=120, zero_f=0.0):
    rng = np.random.default_rng(seed)
    F = rng.integers(0, f_hi, size=n)
    F[rng.random(n) < zero_f] = 0
    return np.stack([F, rng.integers(0, e_hi, size=n), rng.integers(0, s_hi, size=n)],
                    1).astype(np.int32)


@pytest.mark.parametrize("case", ["mixed", "queues_overflow", "codes"])
def test_mwq_inject_bit_exact(torch, sn, oracle_lib, case):
    N, K, warm = 20000, 96, 40
    feat = synth.trace_features(1, N, D)
    start, length, wm = sn.partition(N, K, warm)
    n_pred = int(length.sum() + wm.sum())
    if case == "queues_overflow":
        # long fetch-free runs fill the processor queue past C; long store
        # latencies keep the memory write queue full
        table = store_table(5, n_pred, f_hi=2, e_hi=300, s_hi=2000, zero_f=0.7)
    else:
        table = store_table(4, n_pred)
    if case == "codes":
        codes = synth.trace_codes(1, N)
        t = dev(torch, codes.view(np.int32))
        feat = synth.expand_codes(codes, D)
    else:
        t = dev(torch, feat)
    sim = sn.Simulator(t, L, COLS, start, length, wm, n_out=3, store_col=SC,
                       n_feat=D if case == "codes" else None)
    g = sim.run(sn.SIM_LAT_INJECT, dev(torch, table))
    o = oracle_lib.simulate(ocfg(oracle_lib), feat, start, length, wm, mode=oracle_lib.INJECT,
                            lat_table=table)
    assert_same(g, o)
    # the memory write queue mattered: without stores the cycles differ
    o2 = oracle_lib.simulate(oracle_lib.sim_cfg(D, L, 2, 8, COLS), feat, start, length, wm,
                             mode=oracle_lib.INJECT, lat_table=np.ascontiguousarray(table[:, :2]))
    assert o2["total"] != o["total"]
    sim.close()


def selector_c3(slot, col):
    """C3 store-network weights whose first output is x[slot][col] (a value
    >= 0 passes every ReLU unchanged) and whose others are 0."""
    layers = synth.net_c3_store()
    shapes = synth.layer_param_shapes(layers)
    ws = [np.zeros(w, np.float32) for w, _ in shapes]
    bs = [np.zeros(b, np.float32) for _, b in shapes]
    t1, t2, t3, p = slot % 2, (slot // 2) % 2, (slot // 4) % 2, slot // 8
    ws[0][0, col, t1] = 1.0
    ws[1][0, 0, t2] = 1.0
    ws[2][0, 0, t3] = 1.0
    ws[3][0, 0 * 13 + p] = 1.0
    ws[4][0, 0] = 1.0
    return layers, ws, bs


@pytest.mark.parametrize("slot,col", [(1, 48), (2, 47), (3, 49), (9, 47), (17, 49), (40, 48),
                                      (77, 47), (103, 49), (5, 0), (60, 2)])
def test_mwq_window_contents(torch, sn, oracle_lib, slot, col):
    """The windows the kernel builds, read back through a selector network
    in inject mode, equal the oracle's (processor queue, then memory write
    queue, residence / execution / store columns)."""
    N, K = 6000, 16
    feat = synth.trace_features(1, N, D)
    start, length, wm = sn.partition(N, K, 0)
    n_pred = int(length.sum())
    table = store_table(slot * 7 + col, n_pred, f_hi=2, e_hi=60, s_hi=400, zero_f=0.5)
    layers, ws, bs = selector_c3(slot, col)
    sim = sn.Simulator(dev(torch, feat), L, COLS, start, length, wm, n_out=3, store_col=SC)
    sim.load_weights(layers, sn.flat_params(ws, bs))
    lg = torch.zeros((n_pred, 3), dtype=torch.float32, device="cuda")
    sim.record_logits(lg)
    sim.run(sn.SIM_LAT_SHADOW, dev(torch, table))
    m = oracle_lib.Model(layers, ws, bs, D, L)
    o = oracle_lib.simulate(ocfg(oracle_lib), feat, start, length, wm, model=m,
                            mode=oracle_lib.INJECT, lat_table=table, want_logits=True)
    got = lg.cpu().numpy()[:, 0].astype(np.float64)
    np.testing.assert_array_equal(got, o["logits"][:, 0])
    # the slot is populated (slot 1's residence would be 0: fetched this tick)
    assert np.count_nonzero(got) > n_pred // 20
    sim.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_mwq_forward_parity(torch, sn, oracle_lib, prec):
    layers = synth.net_c3_store()
    ws, bs = synth.init_weights(2, layers, out_bias=synth.OUT_BIAS_STORE)
    feat = synth.trace_features(1, 3000, D)
    x = realistic_windows((D, L, 3, 8) + tuple(COLS), feat, 37, seed=3)
    x[:, 1:, COLS[2]] = np.where(x[:, 1:, COLS[0]] > 0, 17.0, 0.0)  # some store latencies
    sim = sn.Simulator(dev(torch, feat), L, COLS, *sn.partition(3000, 1, 0), prec=prec, n_out=3,
                       store_col=SC)
    sim.load_weights(layers, sn.flat_params(ws, bs))
    got = sim.forward(dev(torch, x)).cpu().numpy()
    ref, scale = oracle_lib.Model(layers, ws, bs, D, L, prec=prec).forward(x, want_scale=True)
    assert rel_err(got, ref, scale).max() <= (1e-5 if prec == 0 else 2.0 ** -8)
    sim.close()


def test_mwq_free_run_replayed_by_oracle(torch, sn, oracle_lib):
    layers = synth.net_c3_store()
    ws, bs = synth.init_weights(2, layers, out_bias=synth.OUT_BIAS_STORE)
    N, K, warm = 8000, 32, 64
    feat = synth.trace_features(1, N, D)
    start, length, wm = sn.partition(N, K, warm)
    sim = sn.Simulator(dev(torch, feat), L, COLS, start, length, wm, n_out=3, store_col=SC)
    sim.load_weights(layers, sn.flat_params(ws, bs))
    lg = torch.zeros((sim.n_pred, 3), dtype=torch.float32, device="cuda")
    sim.record_logits(lg)
    g = sim.run()
    z = lg.cpu().numpy().astype(np.float64)
    lat = np.clip(np.rint(z), 0, 65535).astype(np.int32)
    assert (lat[:, 2] > 0).mean() > 0.5  # store latencies are not degenerate
    m = oracle_lib.Model(layers, ws, bs, D, L)
    o = oracle_lib.simulate(ocfg(oracle_lib), feat, start, length, wm, model=m,
                            mode=oracle_lib.INJECT, lat_table=lat, want_logits=True,
                            want_scale=True)
    assert_same(g, o)
    assert rel_err(z, o["logits"], o["scale"]).max() <= 1e-5
    own = np.clip(np.rint(o["logits"]), 0, 65535).astype(np.int32)
    diff = own != lat
    assert not np.any(diff & ~near_half(o["logits"], o["scale"], 1e-5))
    sim.close()
