"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: cycle and queue results bit-exact given identical latencies; FP32
predictor outputs within |y32 - y64| <= 1e-5 * max(s, 1) (and 1e-6, which
the kernel's FP32 sums also meet), s being the FP64
magnitude |b| + sum |w a| of the output layer (relative error of a computed
sum, measured against the magnitude of its terms); free-running
simulations exact wherever no prediction sits within the FP32/FP64 rounding
ambiguity of a .5 boundary, and otherwise exactly reproducible by the oracle
from the GPU's own latency decisions."""
import math

import numpy as np
import pytest

import synth
from tests.common import near_half, realistic_windows, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-5
# the kernel's FP32 sums are far inside TOL (about 1e-7 of s): held to a
# tenth of it as well, so that a lost digit shows
TIGHT = 1e-6
TIE_TOL = 1e-4


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


class Setup:
    def __init__(self, torch, sn, oracle, net, N, K, warm, trace_seed=1, weight_seed=2, W=8,
                 lengths=None):
        self.net = net
        if net == "small":
            self.layers, self.D, self.L = synth.net_small(), 32, 16
        else:
            self.layers, self.D, self.L = synth.net_c3(), 50, 111
        self.cols = synth.dynamic_columns(self.D)
        self.ws, self.bs = synth.init_weights(weight_seed, self.layers)
        self.feat = synth.trace_features(trace_seed, N, self.D)
        if lengths is None:
            self.start, self.len, self.warm = sn.partition(N, K, warm)
        else:
            self.start, self.len, self.warm = lengths
        self.N, self.W = N, W
        self.cfg = oracle.sim_cfg(self.D, self.L, 2, W, self.cols)
        self.model = oracle.Model(self.layers, self.ws, self.bs, self.D, self.L)
        self.n_pred = int(np.sum(self.len) + np.sum(self.warm))
        self.dfeat = dev(torch, self.feat)
        self.sim = sn.Simulator(self.dfeat, self.L, self.cols, self.start, self.len, self.warm,
                                retire_width=W)
        self.sim.load_weights(self.layers, sn.flat_params(self.ws, self.bs))

    def oracle(self, oracle, **kw):
        return oracle.simulate(self.cfg, self.feat, self.start, self.len, self.warm,
                               model=self.model, **kw)


def assert_same_results(g, o, K):
    for key in ("fetch", "drain", "final", "warm_tick"):
        np.testing.assert_array_equal(g[key], o[key], err_msg=key)
    assert g["total"] == o["total"]


# ---------------------------------------------------------------- forward ---

@pytest.mark.parametrize("net", ["small", "c3"])
@pytest.mark.parametrize("B", [1, 16, 37, 100])
def test_forward_parity(torch, sn, oracle_lib, net, B):
    S = Setup(torch, sn, oracle_lib, net, 4000, 1, 0)
    x = realistic_windows(S.cfg, S.feat, B, seed=B)
    if B > 3:
        x[:3] = np.random.default_rng(B).normal(size=(3, S.L, S.D)) * 5
    got = S.sim.forward(dev(torch, x)).cpu().numpy()
    ref, scale = S.model.forward(x.astype(np.float64), want_scale=True)
    err = rel_err(got, ref, scale)
    assert err.max() <= TOL, (err.max(), np.unravel_index(err.argmax(), err.shape))
    assert err.max() <= TIGHT, err.max()


def test_forward_empty_batch(torch, sn, oracle_lib):
    S = Setup(torch, sn, oracle_lib, "small", 100, 1, 0)
    x = torch.zeros((0, 16, 32), dtype=torch.float32, device="cuda")
    out = torch.zeros((0, 2), dtype=torch.float32, device="cuda")
    S.sim.forward(x, out)


# ------------------------------------------------------ injected latencies ---

INJECT_CASES = [
    # net, N, K, warm, W, heavy
    ("small", 3000, 1, 0, 8, 0.0),
    ("small", 3000, 17, 50, 8, 0.0),
    ("small", 2000, 5, 10, 1, 0.05),
    ("small", 2000, 33, 0, 16, 0.3),
    ("c3", 20000, 37, 256, 8, 0.0),
    ("c3", 6000, 16, 256, 3, 0.2),
]


@pytest.mark.parametrize("net,N,K,warm,W,heavy", INJECT_CASES)
def test_inject_bit_exact(torch, sn, oracle_lib, net, N, K, warm, W, heavy):
    S = Setup(torch, sn, oracle_lib, net, N, K, warm, W=W)
    table = synth.latency_table(17 + K, S.n_pred, 2, heavy=heavy)
    g = S.sim.run(sn.SIM_LAT_INJECT, dev(torch, table))
    o = S.oracle(oracle_lib, mode=oracle_lib.INJECT, lat_table=table)
    assert_same_results(g, o, K)
    assert g["measured"] == N and g["predicted"] == S.n_pred


def test_window_overflow_keeps_newest(torch, sn, oracle_lib):
    """Long execution latencies with zero fetch latency: more instructions in
    flight than window slots; the shadow-mode logits expose the window."""
    S = Setup(torch, sn, oracle_lib, "small", 600, 3, 0)
    table = np.zeros((S.n_pred, 2), np.int32)
    table[:, 1] = 300
    table[::50, 0] = 1
    logits = torch.zeros((S.n_pred, 2), dtype=torch.float32, device="cuda")
    S.sim.record_logits(logits)
    g = S.sim.run(sn.SIM_LAT_SHADOW, dev(torch, table))
    o = S.oracle(oracle_lib, mode=oracle_lib.INJECT, lat_table=table, want_logits=True,
                 want_scale=True)
    assert_same_results(g, o, 3)
    err = rel_err(logits.cpu().numpy(), o["logits"], o["scale"])
    assert err.max() <= TOL
    assert err.max() <= TIGHT, err.max()


@pytest.mark.parametrize("net,N,K,warm", [("small", 4000, 7, 100), ("c3", 8000, 20, 256)])
def test_shadow_logits_on_identical_windows(torch, sn, oracle_lib, net, N, K, warm):
    """Shadow mode: the state advances with injected latencies, so both sides
    see identical windows; every recorded prediction must match."""
    S = Setup(torch, sn, oracle_lib, net, N, K, warm)
    o_free = S.oracle(oracle_lib, want_lat=True)
    table = o_free["lat"]  # the oracle's own latencies: mismatches are the precision effect
    logits = torch.zeros((S.n_pred, 2), dtype=torch.float32, device="cuda")
    S.sim.record_logits(logits)
    g = S.sim.run(sn.SIM_LAT_SHADOW, dev(torch, table))
    o = S.oracle(oracle_lib, mode=oracle_lib.INJECT, lat_table=table, want_logits=True,
                 want_scale=True)
    assert_same_results(g, o, K)
    gl = logits.cpu().numpy()
    err = rel_err(gl, o["logits"], o["scale"])
    assert err.max() <= TOL, err.max()
    assert err.max() <= TIGHT, err.max()
    ties = int(near_half(o["logits"], o["scale"], TIE_TOL).sum())
    assert g["n_shadow_mismatch"] <= ties


# ------------------------------------------------------------- free runs ---

def check_free_run(torch, sn, oracle_lib, S, g, gl):
    """The GPU's free run, replayed by the oracle from the GPU's own rounded
    latencies: identical cycles, logits within TOL, identical rounding away
    from near-ties.  Returns the oracle's own free run for exact comparison."""
    lat_gpu = np.clip(np.rint(gl.astype(np.float64)), 0, 65535).astype(np.int32)
    rep = S.oracle(oracle_lib, mode=oracle_lib.INJECT, lat_table=lat_gpu, want_logits=True,
                   want_scale=True)
    assert_same_results(g, rep, S.sim.n_sub)
    err = rel_err(gl, rep["logits"], rep["scale"])
    assert err.max() <= TOL, err.max()
    assert err.max() <= TIGHT, err.max()
    lat_o = np.clip(np.rint(rep["logits"]), 0, 65535).astype(np.int32)
    diff = lat_o != lat_gpu
    assert not np.any(diff & ~near_half(rep["logits"], rep["scale"], TIE_TOL))
    return rep


def test_free_run_tiny_workload(torch, sn, oracle_lib):
    """10,000 instructions, one sub-trace, 16 x 32 windows (per-step latency
    bound, B = 1)."""
    wl = synth.workload("tiny")
    S = Setup(torch, sn, oracle_lib, "small", wl.n_instr, 1, 0)
    logits = torch.zeros((S.n_pred, 2), dtype=torch.float32, device="cuda")
    S.sim.record_logits(logits)
    g = S.sim.run()
    gl = logits.cpu().numpy()
    check_free_run(torch, sn, oracle_lib, S, g, gl)
    o = S.oracle(oracle_lib, want_logits=True, want_scale=True)
    if not near_half(o["logits"], o["scale"], TIE_TOL).any():
        assert_same_results(g, o, 1)
        assert g["n_clamped"] == o["n_clamped"] and g["n_nonfinite"] == 0


@pytest.mark.parametrize("net,N,K,warm", [("small", 5000, 40, 64), ("c3", 12000, 48, 256)])
def test_free_run_many_subtraces(torch, sn, oracle_lib, net, N, K, warm):
    S = Setup(torch, sn, oracle_lib, net, N, K, warm)
    logits = torch.zeros((S.n_pred, 2), dtype=torch.float32, device="cuda")
    S.sim.record_logits(logits)
    g = S.sim.run()
    check_free_run(torch, sn, oracle_lib, S, g, logits.cpu().numpy())
    o = S.oracle(oracle_lib, want_logits=True, want_scale=True)
    if not near_half(o["logits"], o["scale"], TIE_TOL).any():
        assert_same_results(g, o, K)


def test_recording_does_not_change_results(torch, sn, oracle_lib):
    S = Setup(torch, sn, oracle_lib, "c3", 6000, 24, 256)
    a = S.sim.run()
    S.sim.reset()
    logits = torch.zeros((S.n_pred, 2), dtype=torch.float32, device="cuda")
    S.sim.record_logits(logits)
    b = S.sim.run()
    assert_same_results(a, b, 24)


def test_steps_in_chunks_equal_one_run(torch, sn, oracle_lib):
    S = Setup(torch, sn, oracle_lib, "c3", 6000, 24, 256)
    a = S.sim.run()
    S.sim.reset()
    for _ in range(20):
        S.sim.step(13)
    b = S.sim.run()
    assert_same_results(a, b, 24)
    table = synth.latency_table(3, S.n_pred, 2)
    S.sim.reset()
    c = S.sim.run(sn.SIM_LAT_INJECT, dev(torch, table))
    S.sim.reset()
    S.sim.step(1, sn.SIM_LAT_INJECT, dev(torch, table))
    S.sim.step(250, sn.SIM_LAT_INJECT, dev(torch, table))
    d = S.sim.run(sn.SIM_LAT_INJECT, dev(torch, table))
    assert_same_results(c, d, 24)


def test_short_and_uneven_subtraces(torch, sn, oracle_lib):
    """Sub-traces of length 1 and of very different lengths in one tile."""
    N = 3000
    lengths = np.array([1, 1, 2, 700, 5, 1000, 3, 1, 17, 270], np.int64)
    start = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)
    warm = np.minimum(start, 9).astype(np.int32)
    S = Setup(torch, sn, oracle_lib, "small", N, 0, 0, lengths=(start, lengths, warm))
    table = synth.latency_table(8, S.n_pred, 2)
    g = S.sim.run(sn.SIM_LAT_INJECT, dev(torch, table))
    o = S.oracle(oracle_lib, mode=oracle_lib.INJECT, lat_table=table)
    assert_same_results(g, o, len(lengths))
    S.sim.reset()
    logits = torch.zeros((S.n_pred, 2), dtype=torch.float32, device="cuda")
    S.sim.record_logits(logits)
    g = S.sim.run()
    check_free_run(torch, sn, oracle_lib, S, g, logits.cpu().numpy())


def test_constant_model_closed_form(torch, sn, oracle_lib):
    """Zero weights, output bias (1, 5): every sub-trace gives len*1 + 5 + 1."""
    S = Setup(torch, sn, oracle_lib, "c3", 5000, 20, 256)
    ws = [np.zeros_like(w) for w in S.ws]
    bs = [np.zeros_like(b) for b in S.bs]
    bs[-1] = np.array([1.0, 5.0], np.float32)
    S.sim.load_weights(S.layers, sn.flat_params(ws, bs))
    g = S.sim.run()
    assert g["total"] == 5000 + 20 * 6
    np.testing.assert_array_equal(g["fetch"], S.len)


# ----------------------------------------------------------- full size ---

def test_full_c3_workload_sampled(torch, sn, oracle_lib):
    """1,000,000 instructions in 4,096 sub-traces with 256 warm-up, in the
    launch configuration the benchmark times.  The oracle replays a sample of
    sub-traces from the GPU's own latencies; invariants hold for all."""
    wl = synth.workload("c3_1m")
    S = Setup(torch, sn, oracle_lib, "c3", wl.n_instr, wl.n_sub, wl.warmup)
    plain = S.sim.run()
    S.sim.reset()
    logits = torch.zeros((S.n_pred, 2), dtype=torch.float32, device="cuda")
    S.sim.record_logits(logits)
    g = S.sim.run()
    assert_same_results(plain, g, wl.n_sub)
    assert g["predicted"] == 2_048_309 and g["measured"] == 1_000_000
    assert g["n_nonfinite"] == 0
    np.testing.assert_array_equal(g["final"] - g["warm_tick"], g["fetch"] + g["drain"])
    assert (g["drain"] >= 1).all()
    assert g["total"] == int(np.sum(g["final"] - g["warm_tick"]))
    gl = logits.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(S.len + S.warm)]).astype(np.int64)
    rng = np.random.default_rng(0)
    sample = sorted(set([0, 1, 2, 2047, 4095] + list(rng.integers(0, wl.n_sub, 5))))
    ks = np.array(sample)
    lat_gpu = np.concatenate([np.clip(np.rint(gl[off[k]:off[k + 1]].astype(np.float64)), 0, 65535)
                              for k in ks]).astype(np.int32)
    rep = oracle_lib.simulate(S.cfg, S.feat, S.start[ks], S.len[ks], S.warm[ks], model=S.model,
                              mode=oracle_lib.INJECT, lat_table=lat_gpu, want_logits=True,
                              want_scale=True)
    for key in ("fetch", "drain", "final", "warm_tick"):
        np.testing.assert_array_equal(rep[key], g[key][ks], err_msg=key)
    glk = np.concatenate([gl[off[k]:off[k + 1]] for k in ks])
    assert rel_err(glk, rep["logits"], rep["scale"]).max() <= TOL
    assert rel_err(glk, rep["logits"], rep["scale"]).max() <= TIGHT
    lat_o = np.clip(np.rint(rep["logits"]), 0, 65535).astype(np.int32)
    assert not np.any((lat_o != lat_gpu) & ~near_half(rep["logits"], rep["scale"], TIE_TOL))


# ------------------------------------------------------------ error paths ---

def test_error_paths(torch, sn, oracle_lib):
    S = Setup(torch, sn, oracle_lib, "small", 500, 2, 0)
    with pytest.raises(sn.SimError) as e:
        S.sim.step(1, sn.SIM_LAT_INJECT, None)
    assert e.value.code == sn.SIM_EINVAL
    bad = [np.array(w) for w in S.ws]
    bad[1][0, 0, 0] = np.nan
    with pytest.raises(sn.SimError) as e:
        S.sim.load_weights(S.layers, sn.flat_params(bad, S.bs))
    assert e.value.code == sn.SIM_ENONFINITE
    wrong = list(S.layers)
    wrong[1] = synth.Layer(synth.CONV, 32, 48, 1)
    with pytest.raises(sn.SimError) as e:
        S.sim.load_weights(wrong, sn.flat_params(S.ws, S.bs))
    assert e.value.code == sn.SIM_EUNSUPPORTED
    a = S.sim.run()
    with pytest.raises(sn.SimError) as e:
        S.sim.run()
    assert e.value.code == sn.SIM_ESTATE
    S.sim.reset()
    b = S.sim.run()
    assert_same_results(a, b, 2)


@pytest.mark.parametrize("variant,n_wg", [(0, None), (1, None), (1, 1), (2, None), (2, 1)])
def test_small_network_step_forms(torch, sn, oracle_lib, variant, n_wg):
    """The small network's FP32 step as a workgroup per 16 slots (variant 0),
    as one wavefront per slot (variant 1) and as four wavefronts per slot,
    one per block of the conv tree (variant 2), the latter two also with 16
    slots for 40 sub-traces (slots refilled from the work queue): injected
    latencies bit-exact; free runs replayed by the oracle from the GPU's own
    latencies; shadow mode on the oracle's own latencies reproduces its
    rounded outputs away from ties."""
    S = Setup(torch, sn, oracle_lib, "small", 5000, 40, 64)
    S.sim.set_tuning(variant, n_wg or (40 + 15) // 16)  # (all slots: 16 per workgroup)
    table = synth.latency_table(29, S.n_pred, 2, heavy=0.1)
    g = S.sim.run(sn.SIM_LAT_INJECT, dev(torch, table))
    assert_same_results(g, S.oracle(oracle_lib, mode=oracle_lib.INJECT, lat_table=table), 40)
    S.sim.reset()
    logits = torch.zeros((S.n_pred, 2), dtype=torch.float32, device="cuda")
    S.sim.record_logits(logits)
    g = S.sim.run()
    check_free_run(torch, sn, oracle_lib, S, g, logits.cpu().numpy())
    o = S.oracle(oracle_lib, want_lat=True, want_logits=True, want_scale=True)
    S.sim.reset()
    logits.zero_()
    sh = S.sim.run(sn.SIM_LAT_SHADOW, dev(torch, o["lat"]))
    assert_same_results(sh, o, 40)
    gl = logits.cpu().numpy()
    assert rel_err(gl, o["logits"], o["scale"]).max() <= TIGHT
    ties = near_half(o["logits"], o["scale"], TIE_TOL)
    own = np.clip(np.rint(gl.astype(np.float64)), 0, 65535).astype(np.int32)
    assert not np.any((own != o["lat"]) & ~ties)
    assert sh["n_shadow_mismatch"] == int(((own != o["lat"])).sum())


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_small_network_steps_in_pieces(torch, sn, oracle_lib, variant):
    """A run in pieces of 7 steps (each launch writes the sub-traces' state,
    queue ring included, back to memory and the next reads it) equals one
    run, in each of the small network's step forms."""
    S = Setup(torch, sn, oracle_lib, "small", 3000, 9, 64)
    table = synth.latency_table(31, S.n_pred, 2, heavy=0.1)
    S.sim.set_tuning(variant, 1)
    a = S.sim.run(sn.SIM_LAT_INJECT, dev(torch, table))
    S.sim.reset()
    for _ in range(40):
        S.sim.step(7, sn.SIM_LAT_INJECT, dev(torch, table))
    b = S.sim.run(sn.SIM_LAT_INJECT, dev(torch, table))
    assert_same_results(a, b, 9)
    S.sim.reset()
    logits = torch.zeros((S.n_pred, 2), dtype=torch.float32, device="cuda")
    S.sim.record_logits(logits)
    c = S.sim.run()
    d_logits = logits.clone()
    S.sim.reset()
    logits.zero_()
    for _ in range(40):
        S.sim.step(7)
    d = S.sim.run()
    assert_same_results(c, d, 9)
    assert torch.equal(logits, d_logits)
