"""Python access to the FP64 SimNet oracle (``simnet_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  It shares
no code with the HIP library; both only consume inputs made by ``synth``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "simnet_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

PREDICT, INJECT = 0, 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, IEEE double, no contraction)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, SRC,
                               "-lpthread", "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        L.ol_model_new.restype = P
        L.ol_model_new.argtypes = [C.c_int, i32p, f32p, C.c_int, C.c_int]
        L.ol_model_new_prec.restype = P
        L.ol_model_new_prec.argtypes = [C.c_int, i32p, f32p, C.c_int, C.c_int, C.c_int]
        L.ol_model_free.argtypes = [P]
        L.ol_model_nout.restype = C.c_int
        L.ol_model_nout.argtypes = [P]
        L.ol_forward.restype = C.c_int
        L.ol_forward.argtypes = [P, C.c_int64, f64p, f64p, P]
        L.ol_round.restype = C.c_int32
        L.ol_round.argtypes = [C.c_double, C.c_int32, C.POINTER(C.c_int32)]
        L.ol_hybrid_select.restype = C.c_int32
        L.ol_hybrid_select.argtypes = [f64p, C.c_int32, C.POINTER(C.c_int32)]
        L.ol_partition.restype = C.c_int
        L.ol_partition.argtypes = [C.c_int64, C.c_int32, C.c_int32, i64p, i64p, i32p]
        L.ol_simulate.restype = C.c_int
        L.ol_simulate.argtypes = [P, i32p, P, P, C.c_int64, C.c_int32, i64p, i64p, i32p,
                                  C.c_int32, P, i64p, i64p, i64p, i64p, P, P, P, i64p, C.c_int32,
                                  C.c_int64, P]
        L.ol_model_new_fp8.restype = P
        L.ol_model_new_fp8.argtypes = [C.c_int, i32p, f32p, C.c_int, C.c_int, f32p]
        L.ol_scales_from_amax.argtypes = [f64p, C.c_int32, f32p]
        L.ol_scales_from_amax.restype = None
        L.ol_round_e4m3.argtypes = [C.c_double]
        L.ol_round_e4m3.restype = C.c_double
        L.ol_round_bf16.argtypes = [C.c_double]
        L.ol_round_bf16.restype = C.c_double
        L.ol_train.restype = C.c_int
        L.ol_train.argtypes = [P, C.c_int64, f64p, i32p, C.c_int32, P, f64p, P, P, C.c_int32]
        L.ol_hybrid_loss.restype = C.c_double
        L.ol_hybrid_loss.argtypes = [f64p, i32p, C.c_int64, C.c_int32]
        _lib = L
    return _lib


def flat_params(ws: Sequence[np.ndarray], bs: Sequence[np.ndarray]) -> np.ndarray:
    parts = []
    for w, b in zip(ws, bs):
        parts.append(np.asarray(w, np.float32).ravel())
        parts.append(np.asarray(b, np.float32).ravel())
    return np.ascontiguousarray(np.concatenate(parts), dtype=np.float32)


class Model:
    """The predictor with its parameters held in double precision.  prec=1
    evaluates the BF16 form (inputs, weights and hidden activations rounded
    to bfloat16, exact sums)."""

    def __init__(self, layers, ws, bs, n_feat: int, n_slot: int, prec: int = 0,
                 scales: Optional[np.ndarray] = None):
        """prec 2 is the FP8 form and needs ``scales`` (one per input channel
        of every layer, the window's features first)."""
        desc = np.array([[ly.kind, ly.c_in, ly.c_out, ly.relu] for ly in layers],
                        dtype=np.int32).ravel()
        self._params = flat_params(ws, bs)
        self.n_feat, self.n_slot = n_feat, n_slot
        if prec == 2:
            self._scales = np.ascontiguousarray(scales, np.float32)
            self.ptr = lib().ol_model_new_fp8(len(layers), desc, self._params, n_feat, n_slot,
                                              self._scales)
        else:
            self.ptr = lib().ol_model_new_prec(len(layers), desc, self._params, n_feat, n_slot,
                                               prec)
        if not self.ptr:
            raise ValueError("layer list does not fit the window shape")
        self.n_out = lib().ol_model_nout(self.ptr)
        self.hidden_widths = [ly.c_out for ly in layers[:-1]]

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.ol_model_free(self.ptr)
            self.ptr = None

    def forward(self, x: np.ndarray, want_scale: bool = False):
        """Outputs [B][n_out]; with want_scale also the last layer's
        |b| + sum |w a| per output (the magnitude rounding errors scale with)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.shape[1:] == (self.n_slot, self.n_feat)
        out = np.zeros((x.shape[0], self.n_out), dtype=np.float64)
        scale = np.zeros_like(out) if want_scale else None
        lib().ol_forward(self.ptr, x.shape[0], x, out,
                         scale.ctypes.data if want_scale else None)
        return (out, scale) if want_scale else out


def round_latency(v: float, lat_max: int = 65535):
    fl = C.c_int32(0)
    r = lib().ol_round(float(v), int(lat_max), C.byref(fl))
    return int(r), int(fl.value)


def partition(n_instr: int, n_sub: int, warm_max: int = 0):
    start = np.zeros(n_sub, np.int64)
    length = np.zeros(n_sub, np.int64)
    warm = np.zeros(n_sub, np.int32)
    if lib().ol_partition(n_instr, n_sub, warm_max, start, length, warm) != 0:
        raise ValueError("cannot partition")
    return start, length, warm


def default_threads() -> int:
    """CPU threads for the oracle: the cores this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


HYB_CLASSES = 10
HYB_PER_TYPE = HYB_CLASSES + 1


def sim_cfg(n_feat, n_slot, n_out=2, retire_width=8, cols=(-1, -1, -1), lat_max=65535,
            head=0, store_col=-1, dep_col=-1):
    """head 0: regression head (n_out outputs); 1: hybrid head (Sec. 2.3),
    HYB_PER_TYPE outputs per latency type.  n_out = 3 adds store latencies
    and the memory write queue; store_col is then the trace column whose
    nonzero value marks a store.  dep_col >= 0: the 5 memory-dependency flag
    columns start there (needs the trace's addresses, `mem`)."""
    return np.array([n_feat, n_slot, n_out, retire_width, cols[0], cols[1], cols[2], lat_max,
                     head, store_col, dep_col], dtype=np.int32)


def n_logits(cfg) -> int:
    return int(cfg[2]) * (HYB_PER_TYPE if int(cfg[8]) == 1 else 1)


def hybrid_select(z, lat_max: int = 65535):
    """Latency of one type from its HYB_PER_TYPE hybrid-head outputs."""
    z = np.ascontiguousarray(z, np.float64)
    fl = C.c_int32(0)
    r = lib().ol_hybrid_select(z, int(lat_max), C.byref(fl))
    return int(r), int(fl.value)


def simulate(cfg: np.ndarray, feat: Optional[np.ndarray], start, length, warm,
             model: Optional[Model] = None, mode: int = PREDICT,
             lat_table: Optional[np.ndarray] = None, want_logits: bool = False,
             want_lat: bool = False, n_instr: Optional[int] = None, threads: int = 0,
             want_scale: bool = False, max_pos: int = 0, want_amax: bool = False,
             mem: Optional[np.ndarray] = None) -> dict:
    """Run the oracle over every sub-trace; returns per-sub-trace int64 arrays
    and optionally the per-prediction logits (float64) and latencies.  mem:
    uint32 [n_instr][2] program counters and data addresses (needed with
    dependency flags)."""
    if mem is not None:
        mem = np.ascontiguousarray(mem, np.uint32)
    start = np.ascontiguousarray(start, np.int64)
    length = np.ascontiguousarray(length, np.int64)
    warm = np.ascontiguousarray(warm, np.int32)
    K = start.shape[0]
    n_out = int(cfg[2])
    n_pred = int(np.sum(warm.astype(np.int64) + length))
    if feat is not None:
        feat = np.ascontiguousarray(feat, np.float32)
        n_instr = feat.shape[0]
    elif n_instr is None:
        n_instr = int(np.max(start + length))
    res = {k: np.zeros(K, np.int64) for k in ("fetch", "drain", "final", "warm_tick")}
    n_log = n_logits(cfg)
    logits = np.zeros((n_pred, n_log), np.float64) if want_logits else None
    lat = np.zeros((n_pred, n_out), np.int32) if want_lat else None
    scale = np.zeros((n_pred, n_log), np.float64) if want_scale else None
    if lat_table is not None:
        lat_table = np.ascontiguousarray(lat_table, np.int32)
        assert lat_table.size >= n_pred * n_out
    counters = np.zeros(2, np.int64)
    amax = None
    if want_amax:
        n_amax = model.n_feat + sum(ly_out for ly_out in model.hidden_widths)
        amax = np.zeros(n_amax, np.float64)
    if threads <= 0:
        threads = default_threads()
    rc = lib().ol_simulate(model.ptr if model else None, cfg,
                           feat.ctypes.data if feat is not None else None,
                           mem.ctypes.data if mem is not None else None, n_instr, K,
                           start, length, warm, mode,
                           lat_table.ctypes.data if lat_table is not None else None,
                           res["fetch"], res["drain"], res["final"], res["warm_tick"],
                           logits.ctypes.data if logits is not None else None,
                           scale.ctypes.data if scale is not None else None,
                           lat.ctypes.data if lat is not None else None,
                           counters, threads, max_pos,
                           amax.ctypes.data if amax is not None else None)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    res["total"] = int(np.sum(res["final"] - res["warm_tick"]))
    res["n_clamped"], res["n_nonfinite"] = int(counters[0]), int(counters[1])
    res["logits"], res["lat"], res["scale"], res["amax"] = logits, lat, scale, amax
    return res


def fp8_scales(amax: np.ndarray) -> np.ndarray:
    """Per-channel FP8 scales from calibration maxima (the oracle's rule)."""
    amax = np.ascontiguousarray(amax, np.float64)
    out = np.zeros(amax.size, np.float32)
    lib().ol_scales_from_amax(amax, amax.size, out)
    return out


def calibrate(cfg, feat, start, length, warm, model: Model, n_steps: int,
              lat_table: Optional[np.ndarray] = None, threads: int = 0) -> np.ndarray:
    """Largest |input| per channel of every layer over the first n_steps
    positions of every sub-trace (inject mode when a table is given)."""
    res = simulate(cfg, feat, start, length, warm, model=model,
                   mode=INJECT if lat_table is not None else PREDICT, lat_table=lat_table,
                   threads=threads, max_pos=n_steps, want_amax=True)
    return res["amax"]


N_BINS = 400


def train_step(model: Model, x: np.ndarray, lat: np.ndarray, want_dlogits: bool = False,
               want_dx: bool = False, threads: int = 0):
    """FP64 hybrid loss, its gradient w.r.t. the flat PyTorch-order
    parameters, and optionally w.r.t. the head outputs and the input."""
    x = np.ascontiguousarray(x, np.float64)
    lat = np.ascontiguousarray(lat, np.int32)
    B = x.shape[0]
    n_params = model._params.size
    dparams = np.zeros(n_params, np.float64)
    loss = C.c_double(0.0)
    dlogits = np.zeros((B, model.n_out), np.float64) if want_dlogits else None
    dx = np.zeros_like(x) if want_dx else None
    rc = lib().ol_train(model.ptr, B, x, lat, N_BINS, C.byref(loss), dparams,
                        dlogits.ctypes.data if dlogits is not None else None,
                        dx.ctypes.data if dx is not None else None,
                        threads if threads > 0 else default_threads())
    if rc != 0:
        raise ValueError("oracle rejected the training arguments")
    return {"loss": loss.value, "dparams": dparams, "dlogits": dlogits, "dx": dx}


def hybrid_loss(z: np.ndarray, lat: np.ndarray) -> float:
    z = np.ascontiguousarray(z, np.float64)
    lat = np.ascontiguousarray(lat, np.int32)
    return lib().ol_hybrid_loss(z, lat, z.shape[0], N_BINS)
