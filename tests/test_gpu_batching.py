"""Uneven sub-traces through the persistent work queue (more sub-traces than
slots, finished ones replaced by unstarted ones, longest first) and the
packed 32-bit trace encoding."""
import numpy as np
import pytest

import synth
from tests.common import near_half, rel_err

pytestmark = pytest.mark.gpu


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


def independent_streams(n_sub, lo, hi, seed=3):
    length = synth.loguniform_lengths(seed, n_sub, lo, hi)
    start = np.concatenate([[0], np.cumsum(length)[:-1]]).astype(np.int64)
    return start, length.astype(np.int64), np.zeros(n_sub, np.int32), int(length.sum())


def assert_same(a, b, keys=("fetch", "drain", "final", "warm_tick")):
    for k in keys:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    assert a["total"] == b["total"]


def test_codes_equal_dense_rows(torch, sn):
    layers = synth.net_c3()
    ws, bs = synth.init_weights(2, layers)
    N = 6000
    codes = synth.trace_codes(1, N)
    feat = synth.expand_codes(codes, 50)
    start, length, warm = sn.partition(N, 24, 256)
    cols = synth.dynamic_columns(50)
    out = []
    for prec in (sn.SIM_FP32, sn.SIM_BF16):
        for src in ("rows", "codes"):
            t = (torch.from_numpy(feat).cuda() if src == "rows"
                 else torch.from_numpy(codes.view(np.int32)).cuda())
            sim = sn.Simulator(t, 111, cols, start, length, warm, prec=prec, n_feat=50)
            sim.load_weights(layers, sn.flat_params(ws, bs))
            lg = torch.zeros((sim.n_pred, 2), dtype=torch.float32, device="cuda")
            sim.record_logits(lg)
            res = sim.run()
            out.append((res, lg.cpu().numpy()))
        assert_same(out[-2][0], out[-1][0])
        np.testing.assert_array_equal(out[-2][1], out[-1][1])


def test_more_subtraces_than_slots_inject(torch, sn, oracle_lib):
    """5,000 uneven streams on the C3 window: more than the slots one GPU
    holds, so slots are refilled; bit-exact against the oracle."""
    start, length, warm, N = independent_streams(5000, 1, 60)
    feat = synth.trace_features(1, N, 50)
    n_pred = int(length.sum())
    table = synth.latency_table(21, n_pred, 2, heavy=0.05)
    sim = sn.Simulator(torch.from_numpy(feat).cuda(), 111, synth.dynamic_columns(50),
                       start, length, warm)
    g = sim.run(sn.SIM_LAT_INJECT, torch.from_numpy(table).cuda())
    cfg = oracle_lib.sim_cfg(50, 111, 2, 8, synth.dynamic_columns(50))
    o = oracle_lib.simulate(cfg, None, start, length, warm, mode=oracle_lib.INJECT,
                            lat_table=table, n_instr=N)
    assert_same(g, o)


def test_more_subtraces_than_slots_predict(torch, sn, oracle_lib):
    """Free run with refills, replayed by the oracle from the GPU's own
    rounded latencies."""
    start, length, warm, N = independent_streams(4500, 1, 25, seed=5)
    codes = synth.trace_codes(7, N)
    feat = synth.expand_codes(codes, 50)
    layers = synth.net_c3()
    ws, bs = synth.init_weights(2, layers)
    sim = sn.Simulator(torch.from_numpy(codes.view(np.int32)).cuda(), 111,
                       synth.dynamic_columns(50), start, length, warm, n_feat=50)
    sim.load_weights(layers, sn.flat_params(ws, bs))
    lg = torch.zeros((sim.n_pred, 2), dtype=torch.float32, device="cuda")
    sim.record_logits(lg)
    g = sim.run()
    gl = lg.cpu().numpy().astype(np.float64)
    lat = np.clip(np.rint(gl), 0, 65535).astype(np.int32)
    cfg = oracle_lib.sim_cfg(50, 111, 2, 8, synth.dynamic_columns(50))
    model = oracle_lib.Model(layers, ws, bs, 50, 111)
    rep = oracle_lib.simulate(cfg, feat, start, length, warm, model=model, mode=oracle_lib.INJECT,
                              lat_table=lat, want_logits=True, want_scale=True)
    assert_same(g, rep)
    assert rel_err(gl, rep["logits"], rep["scale"]).max() <= 1e-5
    lat_o = np.clip(np.rint(rep["logits"]), 0, 65535).astype(np.int32)
    assert not np.any((lat_o != lat) & ~near_half(rep["logits"], rep["scale"], 1e-4))


def test_chunked_steps_with_refills_equal_one_run(torch, sn):
    start, length, warm, N = independent_streams(5000, 1, 40, seed=9)
    feat = synth.trace_features(2, N, 50)
    n_pred = int(length.sum())
    table = torch.from_numpy(synth.latency_table(5, n_pred, 2)).cuda()
    sim = sn.Simulator(torch.from_numpy(feat).cuda(), 111, synth.dynamic_columns(50),
                       start, length, warm)
    a = sim.run(sn.SIM_LAT_INJECT, table)
    sim.reset()
    for _ in range(30):
        sim.step(3, sn.SIM_LAT_INJECT, table)
    b = sim.run(sn.SIM_LAT_INJECT, table)
    assert_same(a, b)
    sim.reset()
    c = sim.run(sn.SIM_LAT_INJECT, table)
    assert_same(a, c)


def test_uneven_bf16_sample_replayed(torch, sn, oracle_lib):
    """A scaled-down uneven workload (300 streams, 100..2,000 instructions,
    BF16): a sample of sub-traces replayed by the oracle's BF16 form."""
    start, length, warm, N = independent_streams(300, 100, 2000, seed=3)
    codes = synth.trace_codes(1, N)
    layers = synth.net_c3()
    ws, bs = synth.init_weights(2, layers)
    sim = sn.Simulator(torch.from_numpy(codes.view(np.int32)).cuda(), 111,
                       synth.dynamic_columns(50), start, length, warm, prec=sn.SIM_BF16,
                       n_feat=50)
    sim.load_weights(layers, sn.flat_params(ws, bs))
    lg = torch.zeros((sim.n_pred, 2), dtype=torch.float32, device="cuda")
    sim.record_logits(lg)
    g = sim.run()
    gl = lg.cpu().numpy().astype(np.float64)
    off = np.concatenate([[0], np.cumsum(length)]).astype(np.int64)
    ks = np.array([0, 1, 57, 150, 299, int(np.argmax(length)), int(np.argmin(length))])
    lat = np.concatenate([np.clip(np.rint(gl[off[k]:off[k + 1]]), 0, 65535) for k in ks]).astype(np.int32)
    feat = synth.expand_codes(codes, 50)
    cfg = oracle_lib.sim_cfg(50, 111, 2, 8, synth.dynamic_columns(50))
    form = oracle_lib.Model(layers, ws, bs, 50, 111, prec=1)
    rep = oracle_lib.simulate(cfg, feat, start[ks], length[ks], warm[ks], model=form,
                              mode=oracle_lib.INJECT, lat_table=lat, want_logits=True,
                              want_scale=True)
    for key in ("fetch", "drain", "final", "warm_tick"):
        np.testing.assert_array_equal(rep[key], g[key][ks], err_msg=key)
    glk = np.concatenate([gl[off[k]:off[k + 1]] for k in ks])
    assert rel_err(glk, rep["logits"], rep["scale"]).max() <= 2.0 ** -8


def test_graph_replay_equals_direct_run(torch, sn):
    start, length, warm, N = independent_streams(5000, 1, 40, seed=12)
    codes = synth.trace_codes(3, N)
    layers = synth.net_c3()
    ws, bs = synth.init_weights(2, layers)
    sim = sn.Simulator(torch.from_numpy(codes.view(np.int32)).cuda(), 111,
                       synth.dynamic_columns(50), start, length, warm, prec=sn.SIM_BF16, n_feat=50)
    sim.load_weights(layers, sn.flat_params(ws, bs))
    a = sim.run()
    sim.use_graph(True)
    for _ in range(3):  # replays, with eager work and synchronisation between them
        sim.reset()
        b = sim.run()
        assert_same(a, b)
        torch.cuda.synchronize()
    table = torch.from_numpy(synth.latency_table(4, sim.n_pred, 2)).cuda()
    sim.use_graph(False)
    sim.reset()
    c = sim.run(sn.SIM_LAT_INJECT, table)
    sim.use_graph(True)
    sim.reset()
    d = sim.run(sn.SIM_LAT_INJECT, table)
    assert_same(c, d)


def test_autotune_choice_does_not_change_results(torch, sn, tmp_path):
    """sim_autotune tries every kernel variant that needs no scratch memory
    (every variant when all need some) and slot count; the chosen shape,
    every variant including those left out, and the cached choice all give
    the same cycles."""
    layers = synth.net_c3()
    ws, bs = synth.init_weights(2, layers)
    start, length, warm, N = independent_streams(600, 20, 900)
    codes = synth.trace_codes(1, N)
    sim = sn.Simulator(torch.from_numpy(codes.view(np.int32)).cuda(), 111,
                       synth.dynamic_columns(50), start, length, warm, prec=sn.SIM_BF16, n_feat=50)
    sim.load_weights(layers, sn.flat_params(ws, bs))
    ref = sim.run()
    cache = str(tmp_path / "tune.json")
    t = sim.autotune(50, cache=cache)
    assert not t["cached"] and len(t["trials"]) >= 3
    assert (t["variant"], t["n_wg"]) in [(v, n) for v, n, _ in t["trials"]]
    scratch = [sim.variant_scratch(v) for v in range(4)]
    free = {v for v in range(4) if scratch[v] == 0}
    assert {v for v, _, _ in t["trials"]} == (free or set(range(4))), scratch
    assert_same(sim.run(), ref)
    for v, n, _ in t["trials"]:
        sim.set_tuning(v, n)
        assert_same(sim.run(), ref)
    for v in range(4):
        sim.set_tuning(v, t["n_wg"])
        assert_same(sim.run(), ref)
    t2 = sim.autotune(50, cache=cache)
    assert t2["cached"] and (t2["variant"], t2["n_wg"]) == (t["variant"], t["n_wg"])
    assert_same(sim.run(), ref)
    with pytest.raises(sn.SimError):
        sim.set_tuning(4, 1)
    sim.close()


def test_c3_uneven_full_run_sampled_replay(torch, sn, oracle_lib):
    """The uneven-streams workload at its full size (20,000 streams of
    log-uniform length in [1e3, 2e5], packed codes, BF16), run as one graph
    in the autotuned launch shape, as the benchmark runs it.  The 32 shortest
    streams and 4 seeded-random ones (among those of at most 4,000
    instructions, so that the FP64 oracle finishes in seconds) are replayed
    by the oracle's BF16 form from the GPU's own latencies: identical cycles,
    outputs within one BF16 unit at the output's magnitude, and the oracle's
    own rounding decisions equal outside that tie band."""
    wl = synth.workload("c3_uneven")
    length = synth.loguniform_lengths(wl.length_seed, wl.n_sub, *wl.len_range)
    start = np.concatenate([[0], np.cumsum(length)[:-1]]).astype(np.int64)
    warm = np.zeros(wl.n_sub, np.int32)
    n_instr = int(length.sum())
    dcodes = torch.empty(n_instr, dtype=torch.int32, device="cuda")
    for lo in range(0, n_instr, 1 << 26):
        hi = min(n_instr, lo + (1 << 26))
        dcodes[lo:hi] = synth.trace_codes_torch(wl.trace_seed, lo, hi, device="cuda")
    ws, bs = synth.init_weights(wl.weight_seed, wl.layers,
                                out_bias=wl.extra.get("out_bias", synth.OUT_BIAS))
    sim = sn.Simulator(dcodes, wl.n_slot, wl.cols, start, length, warm, prec=sn.SIM_BF16,
                       n_feat=wl.n_feat)
    sim.load_weights(wl.layers, sn.flat_params(ws, bs))
    sim.autotune(300)
    logits = torch.zeros((n_instr, 2), dtype=torch.float32, device="cuda")
    sim.record_logits(logits)
    sim.use_graph(True)
    g = sim.run()
    assert g["measured"] == n_instr and g["n_nonfinite"] == 0
    assert g["total"] == int((g["final"] - g["warm_tick"]).sum())
    assert np.array_equal(g["final"], g["warm_tick"] + g["fetch"] + g["drain"])
    assert np.all(g["fetch"] >= 0) and np.all(g["drain"] >= 0)

    rng = np.random.default_rng(17)
    short = np.argsort(length, kind="stable")[:32]
    pool = np.setdiff1d(np.flatnonzero(length <= 4000), short)
    ks = np.sort(np.concatenate([short, rng.choice(pool, 4, replace=False)]))
    gl = np.concatenate([logits[start[k]:start[k] + length[k]].cpu().numpy() for k in ks])
    sim.close()
    del logits
    gl = gl.astype(np.float64)
    lat = np.clip(np.rint(gl), 0, 65535).astype(np.int32)
    feat = np.concatenate([synth.expand_codes(synth.trace_codes(wl.trace_seed, n_instr,
                                                                int(start[k]),
                                                                int(start[k] + length[k])),
                                              wl.n_feat) for k in ks])
    s_len = length[ks].astype(np.int64)
    s_start = np.concatenate([[0], np.cumsum(s_len)[:-1]]).astype(np.int64)
    cfg = oracle_lib.sim_cfg(wl.n_feat, wl.n_slot, 2, wl.retire_width, wl.cols)
    form = oracle_lib.Model(wl.layers, ws, bs, wl.n_feat, wl.n_slot, prec=1)
    rep = oracle_lib.simulate(cfg, feat, s_start, s_len, np.zeros(len(ks), np.int32), model=form,
                              mode=oracle_lib.INJECT, lat_table=lat, want_logits=True,
                              want_scale=True)
    for key in ("fetch", "drain", "final", "warm_tick"):
        np.testing.assert_array_equal(rep[key], g[key][ks], err_msg=key)
    tol = 2.0 ** -8
    assert rel_err(gl, rep["logits"], rep["scale"]).max() <= tol
    lat_o = np.clip(np.rint(rep["logits"]), 0, 65535).astype(np.int32)
    assert not np.any((lat_o != lat) & ~near_half(rep["logits"], rep["scale"], tol))
