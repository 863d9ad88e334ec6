"""Seeded input generators: determinism, chunk independence, category rates."""
import numpy as np

import synth


def test_trace_is_counter_based():
    a = synth.trace_codes(1, 50_000)
    b = np.concatenate([synth.trace_codes(1, 50_000, 0, 12_345),
                        synth.trace_codes(1, 50_000, 12_345, 50_000)])
    np.testing.assert_array_equal(a, b)
    assert not np.array_equal(a, synth.trace_codes(2, 50_000))


def test_category_frequencies():
    f = synth.trace_fields(1, 0, 400_000)
    op = np.bincount(f["op"], minlength=5) / 400_000
    np.testing.assert_allclose(op, synth.OP_PROBS, atol=0.003)
    lv = np.bincount(f["level"], minlength=3) / 400_000
    np.testing.assert_allclose(lv, synth.LEVEL_PROBS, atol=0.002)
    br = f["op"] == synth.OP_BRANCH
    assert abs(f["mispredict"][br].mean() - synth.MISPREDICT_RATE) < 0.004
    assert f["mispredict"][~br].sum() == 0
    assert f["regs"].min() == 0 and f["regs"].max() == 31


def test_feature_rows_layout():
    for D in (32, 50):
        x = synth.trace_features(1, 1000, D)
        assert x.shape == (1000, D) and x.dtype == np.float32
        np.testing.assert_array_equal(x[:, 0:5].sum(1), 1)
        for r in range(3):
            np.testing.assert_array_equal(x[:, 5 + 7 * r:12 + 7 * r].sum(1), 1)
        np.testing.assert_array_equal(x[:, 26:29].sum(1), 1)
        res, exe, sto = synth.dynamic_columns(D)
        assert not x[:, res].any() and not x[:, exe].any()
        if D == 50:
            assert not x[:, 30:].any()


def test_weights_deterministic_and_shaped():
    layers = synth.net_c3()
    w1, b1 = synth.init_weights(2, layers)
    w2, b2 = synth.init_weights(2, layers)
    for a, b in zip(w1 + b1, w2 + b2):
        np.testing.assert_array_equal(a, b)
    assert w1[0].shape == (64, 50, 2) and w1[3].shape == (512, 3328)
    assert sum(w.size + b.size for w, b in zip(w1, b1)) == 1_794_242
    np.testing.assert_array_equal(b1[-1], np.float32(synth.OUT_BIAS))


def test_loguniform_lengths_range():
    n = synth.loguniform_lengths(3, 20_000, 1e3, 2e5)
    assert n.min() >= 1000 and n.max() <= 200_000
    assert abs(n.mean() / ((2e5 - 1e3) / np.log(200)) - 1) < 0.03


def test_torch_code_generator_matches_numpy():
    a = synth.trace_codes(1, 300_000, 12_345, 300_000)
    b = synth.trace_codes_torch(1, 12_345, 300_000).numpy().view(np.uint32)
    np.testing.assert_array_equal(a, b)


def test_analytic_labeller_hand_worked():
    """Tiny traces worked by hand (builder-defined pipeline model)."""
    def fields(ops, regs, levels, mis):
        return {"op": np.array(ops), "regs": np.array(regs), "level": np.array(levels),
                "mispredict": np.array(mis)}
    # int, int (depends on the first), load L2, FP
    f = fields([0, 0, 1, 4], [[1, 0, 0], [2, 1, 0], [3, 0, 0], [4, 3, 2]],
               [0, 0, 1, 0], [0, 0, 0, 0])
    lat = synth.analytic_latencies(f)
    # fetch: groups of 3 -> 1, 0, 0, 1 ; times 1, 1, 1, 2
    np.testing.assert_array_equal(lat[:, 0], [1, 0, 0, 1])
    # i0: start 1, end 2, E 1; i1 waits for r1 (2): end 3, E 2; i2 load L2: 1+29 = 30, end 31,
    # E 30; i3 FP waits r3 (31) and r2 (3): end 35, E 33
    np.testing.assert_array_equal(lat[:, 1], [1, 2, 30, 33])
    # a mispredicted branch adds its execution latency to the next fetch
    g = fields([3, 0], [[0, 0, 0], [0, 0, 0]], [0, 0], [1, 0])
    lat = synth.analytic_latencies(g)
    np.testing.assert_array_equal(lat, [[1, 1], [1, 1]])
    h = synth.analytic_latencies(synth.trace_fields(1, 0, 5000))
    assert h.min() >= 0 and h.max() <= 400 and h[:, 1].mean() > 1
