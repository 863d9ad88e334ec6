"""Shared set-up for the parity tests: seeded inputs from ``synth`` fed to
both the oracle and the HIP library.  No expected value is computed here."""
from __future__ import annotations

import numpy as np

import synth


def small_net_inputs(seed_w=2):
    layers = synth.net_small()
    ws, bs = synth.init_weights(seed_w, layers)
    return layers, ws, bs


def c3_net_inputs(seed_w=2):
    layers = synth.net_c3()
    ws, bs = synth.init_weights(seed_w, layers)
    return layers, ws, bs


def rel_err(got, ref, scale):
    """|y32 - y64| / max(s, 1) elementwise, where s = |b| + sum |w a| of the
    output layer in FP64 (the magnitude rounding errors are proportional to;
    s >= |y64|, so this is never looser than relative to max(|y|, 1) by more
    than the cancellation in the last layer)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.abs(got - ref) / np.maximum(np.asarray(scale, np.float64), 1.0)


def near_half(logits, scale, band):
    """Predictions whose rounding may legitimately differ between an FP32 and
    an FP64 evaluation: within band * max(s, 1) of a .5 boundary."""
    frac = np.abs(logits - np.floor(logits) - 0.5)
    return frac <= band * np.maximum(scale, 1.0)


def realistic_windows(cfg, feat, n_windows, seed=0):
    """Windows shaped like the simulator's: slot 0 a trace row with zero
    dynamic columns, slots 1..occ the preceding rows with residence and
    execution latencies of realistic size, the rest zero."""
    rng = np.random.default_rng(seed)
    n_slot, n_feat = int(cfg[1]), int(cfg[0])
    cres, cexe = int(cfg[4]), int(cfg[5])
    x = np.zeros((n_windows, n_slot, n_feat), np.float32)
    N = feat.shape[0]
    for b in range(n_windows):
        i = int(rng.integers(n_slot, N))
        occ = int(rng.integers(0, n_slot))
        x[b, 0] = feat[i]
        x[b, 0, cres] = 0
        x[b, 0, cexe] = 0
        res = np.sort(rng.integers(0, 200, size=occ))
        for k in range(1, occ + 1):
            x[b, k] = feat[i - k]
            x[b, k, cres] = res[k - 1]
            x[b, k, cexe] = rng.integers(0, 60)
    return x
