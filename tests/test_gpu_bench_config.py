"""The benchmark's headline configuration: the 1,000,000-instruction C3
workload (4,096 sub-traces, 256-instruction warm-up) in the BF16 form, in
the launch shapes the autotuner chooses from (the four kernel variants with
all 256 workgroups, and 3/4 and 1/2 of the workgroups).

Every shape gives the same cycles and the same outputs (same products in
the same order).  The oracle's BF16 form replays a sample of sub-traces
from the GPU's own latencies with identical cycles; outputs lie within one
BF16 unit at the output's magnitude, |y_gpu - y_form| <= 2^-8 * max(s, 1);
the oracle's own rounded decisions agree outside that tie band."""
import numpy as np
import pytest

import synth
from tests.common import near_half, rel_err

pytestmark = pytest.mark.gpu

TOL = 2.0 ** -8


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


def test_c3_1m_bf16_every_launch_shape(torch, sn, oracle_lib):
    wl = synth.workload("c3_1m")
    feat = synth.trace_features(wl.trace_seed, wl.n_instr, wl.n_feat)
    ws, bs = synth.init_weights(wl.weight_seed, wl.layers)
    start, length, warm = sn.partition(wl.n_instr, wl.n_sub, wl.warmup)
    n_pred = int(length.sum() + warm.sum())
    assert n_pred == 2_048_309
    sim = sn.Simulator(torch.from_numpy(feat).cuda(), wl.n_slot, wl.cols, start, length, warm,
                       prec=sn.SIM_BF16)
    sim.load_weights(wl.layers, sn.flat_params(ws, bs))
    logits = torch.zeros((n_pred, 2), dtype=torch.float32, device="cuda")
    sim.record_logits(logits)
    sim.set_tuning(1, 256)
    ref = sim.run()
    ref_logits = logits.clone()
    assert ref["measured"] == 1_000_000 and ref["n_nonfinite"] == 0
    for variant, n_wg in [(0, 256), (2, 256), (3, 256), (1, 192), (3, 192), (0, 128)]:
        sim.reset()
        logits.zero_()
        sim.set_tuning(variant, n_wg)
        g = sim.run()
        for key in ("fetch", "drain", "final", "warm_tick"):
            np.testing.assert_array_equal(g[key], ref[key], err_msg=f"{key} {variant} {n_wg}")
        assert g["total"] == ref["total"]
        assert torch.equal(logits, ref_logits), (variant, n_wg)
    sim.close()

    gl = ref_logits.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(length + warm)]).astype(np.int64)
    rng = np.random.default_rng(5)
    ks = np.array(sorted(set([0, 1, 2047, 4095] + list(rng.integers(0, wl.n_sub, 4)))))
    lat = np.concatenate([np.clip(np.rint(gl[off[k]:off[k + 1]].astype(np.float64)), 0, 65535)
                          for k in ks]).astype(np.int32)
    cfg = oracle_lib.sim_cfg(wl.n_feat, wl.n_slot, 2, wl.retire_width, wl.cols)
    form = oracle_lib.Model(wl.layers, ws, bs, wl.n_feat, wl.n_slot, prec=1)
    rep = oracle_lib.simulate(cfg, feat, start[ks], length[ks], warm[ks], model=form,
                              mode=oracle_lib.INJECT, lat_table=lat, want_logits=True,
                              want_scale=True)
    for key in ("fetch", "drain", "final", "warm_tick"):
        np.testing.assert_array_equal(rep[key], ref[key][ks], err_msg=key)
    glk = np.concatenate([gl[off[k]:off[k + 1]] for k in ks]).astype(np.float64)
    err = rel_err(glk, rep["logits"], rep["scale"])
    assert err.max() <= TOL, err.max()
    lat_o = np.clip(np.rint(rep["logits"]), 0, 65535).astype(np.int32)
    assert not np.any((lat_o != lat) & ~near_half(rep["logits"], rep["scale"], TOL))
