"""Thin Python binding of libsimnet.so (C ABI in include/simnet.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of the library.  PyTorch supplies device memory and streams.  There
is no fallback: if the built library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsimnet.so")

SIM_OK, SIM_EINVAL, SIM_ENOMEM, SIM_EDEVICE, SIM_ESTATE, SIM_ENONFINITE, SIM_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
SIM_FP32, SIM_BF16, SIM_FP8E4M3 = 0, 1, 2
SIM_LAT_PREDICT, SIM_LAT_INJECT, SIM_LAT_SHADOW = 0, 1, 2
SIM_FEAT_F32, SIM_FEAT_CODE32 = 0, 1
CONV, FC = 0, 1
NOALLOC_MAX_B = 65536  # SIM_NOALLOC_MAX_B: largest batch of sim_loss_noalloc

STATUS_NAMES = {0: "SIM_OK", -1: "SIM_EINVAL", -2: "SIM_ENOMEM", -3: "SIM_EDEVICE",
                -4: "SIM_ESTATE", -5: "SIM_ENONFINITE", -6: "SIM_EUNSUPPORTED"}

EXPORTED = ("sim_validate_config", "sim_partition", "sim_init", "sim_load_weights", "sim_step",
            "sim_run",
            "sim_reset", "sim_record_logits", "sim_calibrate", "sim_act_scales", "sim_set_graph",
            "sim_autotune", "sim_set_tuning", "sim_variant_scratch",
            "predictor_fwd", "predictor_save_bytes", "sim_loss", "sim_loss_noalloc",
            "predictor_bwd", "sim_adam", "sim_adam_load",
            "sim_destroy", "sim_last_error")


class sim_layer(C.Structure):
    _fields_ = [("kind", C.c_int32), ("c_in", C.c_int32), ("c_out", C.c_int32),
                ("relu", C.c_int32)]


class sim_config(C.Structure):
    _fields_ = [("n_feat", C.c_int32), ("n_slot", C.c_int32), ("n_out", C.c_int32),
                ("retire_width", C.c_int32), ("col_res", C.c_int32), ("col_exe", C.c_int32),
                ("col_sto", C.c_int32), ("lat_max", C.c_int32), ("prec", C.c_int32),
                ("store_col", C.c_int32), ("col_dep", C.c_int32), ("stream", C.c_void_p)]


class sim_trace(C.Structure):
    _fields_ = [("feat", C.c_void_p), ("feat_dtype", C.c_int32), ("n_sub", C.c_int32),
                ("n_instr", C.c_int64), ("start", C.POINTER(C.c_int64)),
                ("len", C.POINTER(C.c_int64)), ("warm", C.POINTER(C.c_int32)),
                ("mem", C.c_void_p)]


class sim_tuning(C.Structure):
    _fields_ = [("variant", C.c_int32), ("n_wg", C.c_int32), ("ms", C.c_float),
                ("n_tried", C.c_int32), ("tried_variant", C.c_int32 * 16),
                ("tried_n_wg", C.c_int32 * 16), ("tried_ms", C.c_float * 16)]


class sim_result(C.Structure):
    _fields_ = [("total_cycles", C.c_int64), ("measured_instr", C.c_int64),
                ("predicted_instr", C.c_int64), ("n_clamped", C.c_int64),
                ("n_nonfinite", C.c_int64), ("n_shadow_mismatch", C.c_int64),
                ("fetch_cycles", C.POINTER(C.c_int64)), ("drain_cycles", C.POINTER(C.c_int64)),
                ("final_tick", C.POINTER(C.c_int64)), ("warm_tick", C.POINTER(C.c_int64))]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2105_05821_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.sim_validate_config.argtypes = [C.POINTER(sim_config), C.POINTER(sim_trace)]
        L.sim_partition.argtypes = [C.c_int64, C.c_int32, C.c_int32, P, P, P]
        L.sim_init.argtypes = [C.POINTER(sim_config), C.POINTER(sim_trace), C.POINTER(P)]
        L.sim_load_weights.argtypes = [P, C.POINTER(sim_layer), C.c_int32, P, C.c_int32]
        L.sim_step.argtypes = [P, C.c_int32, C.c_int32, P]
        L.sim_run.argtypes = [P, C.c_int32, P, C.POINTER(sim_result)]
        L.sim_reset.argtypes = [P]
        L.sim_record_logits.argtypes = [P, P]
        L.predictor_fwd.argtypes = [P, P, C.c_int64, P, P]
        L.sim_calibrate.argtypes = [P, C.c_int32, C.c_int32, P]
        L.sim_act_scales.argtypes = [P, P, C.c_int32]
        L.sim_set_graph.argtypes = [P, C.c_int32]
        L.predictor_save_bytes.argtypes = [P, C.c_int64]
        L.sim_autotune.argtypes = [P, C.c_int32, C.c_int32, P, C.POINTER(sim_tuning)]
        L.sim_set_tuning.argtypes = [P, C.c_int32, C.c_int32]
        L.sim_variant_scratch.argtypes = [P, C.c_int32, C.POINTER(C.c_int64)]
        L.sim_loss.argtypes = [P, P, P, C.c_int64, P, P]
        L.sim_loss_noalloc.argtypes = [P, P, P, C.c_int64, P, P]
        L.predictor_bwd.argtypes = [P, P, P, P, C.c_int64, P, P, C.c_int32]
        L.sim_adam.argtypes = [P, P, P, P, P, C.c_int64, C.c_float, C.c_float, C.c_float,
                               C.c_float, C.c_int32]
        L.sim_adam_load.argtypes = [P, P, P, P, P, C.c_int64, C.c_float, C.c_float,
                                    C.c_float, C.c_float, C.c_int32]
        L.sim_destroy.argtypes = [P]
        L.sim_destroy.restype = None
        L.sim_last_error.argtypes = [P]
        L.sim_last_error.restype = C.c_char_p
        for n in EXPORTED[:-2]:
            getattr(L, n).restype = C.c_int
        L.predictor_save_bytes.restype = C.c_int64
        _lib = L
    return _lib


class SimError(RuntimeError):
    def __init__(self, call: str, code: int, msg: str = ""):
        super().__init__(f"{call} -> {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def make_config(n_feat: int, n_slot: int, cols: Sequence[int], retire_width: int = 8,
                lat_max: int = 65535, prec: int = SIM_FP32, n_out: int = 2,
                stream=None, store_col: int = 0, col_dep: int = -1) -> sim_config:
    return sim_config(n_feat, n_slot, n_out, retire_width, cols[0], cols[1], cols[2], lat_max,
                      prec, store_col, col_dep, stream)


def make_trace(feat_ptr: Optional[int], n_instr: int, start, length, warm,
               feat_dtype: int = SIM_FEAT_F32, mem_ptr: Optional[int] = None):
    start = np.ascontiguousarray(start, np.int64)
    length = np.ascontiguousarray(length, np.int64)
    warm = np.ascontiguousarray(warm, np.int32)
    tr = sim_trace(feat_ptr, feat_dtype, start.shape[0], n_instr,
                   start.ctypes.data_as(C.POINTER(C.c_int64)),
                   length.ctypes.data_as(C.POINTER(C.c_int64)),
                   warm.ctypes.data_as(C.POINTER(C.c_int32)), mem_ptr)
    tr._keep = (start, length, warm)
    return tr


def sim_validate_config(cfg: sim_config, trace: sim_trace) -> int:
    return lib().sim_validate_config(C.byref(cfg), C.byref(trace))


def partition(n_instr: int, n_sub: int, warm_max: int = 0):
    """(start, len, warm) of the library's partition (sim_partition)."""
    start = np.zeros(max(n_sub, 0), np.int64)
    length = np.zeros(max(n_sub, 0), np.int64)
    warm = np.zeros(max(n_sub, 0), np.int32)
    rc = lib().sim_partition(n_instr, n_sub, warm_max, start.ctypes.data, length.ctypes.data,
                             warm.ctypes.data)
    if rc != SIM_OK:
        raise ValueError(f"sim_partition({n_instr}, {n_sub}, {warm_max}) -> "
                         f"{STATUS_NAMES.get(rc, rc)}")
    return start, length, warm


class Simulator:
    """One sim_ctx.  ``feat`` is a device tensor that must outlive the
    simulator: float32 [n_instr][n_feat] rows, or int32 [n_instr] packed
    instruction codes (then ``n_feat`` gives the expanded width)."""

    def __init__(self, feat, n_slot: int, cols: Sequence[int], start, length, warm,
                 retire_width: int = 8, lat_max: int = 65535, prec: int = SIM_FP32,
                 stream=None, n_feat: Optional[int] = None, n_out: int = 2,
                 store_col: int = 0, mem=None, col_dep: int = -1):
        import torch
        if not feat.is_cuda or not feat.is_contiguous():
            raise ValueError("feat must be a contiguous device tensor")
        if feat.dtype == torch.float32 and feat.dim() == 2:
            kind, width = SIM_FEAT_F32, feat.shape[1]
        elif feat.dtype == torch.int32 and feat.dim() == 1 and n_feat:
            kind, width = SIM_FEAT_CODE32, n_feat
        else:
            raise ValueError("feat must be float32 [n][D] rows or int32 [n] codes with n_feat")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.feat = feat
        self.cfg = make_config(width, n_slot, cols, retire_width, lat_max, prec, n_out=n_out,
                               stream=self.stream.cuda_stream, store_col=store_col,
                               col_dep=col_dep)
        if mem is not None and (not mem.is_cuda or not mem.is_contiguous() or mem.dim() != 2
                                or mem.shape[1] != 2 or mem.element_size() != 4):
            raise ValueError("mem must be a contiguous 32-bit device tensor [n_instr][2]")
        self.mem = mem
        self.n_out = n_out
        self.trace = make_trace(feat.data_ptr(), feat.shape[0], start, length, warm, kind,
                                mem.data_ptr() if mem is not None else None)
        self.n_sub = int(self.trace.n_sub)
        self.n_pred = int(np.sum(self.trace._keep[1]) + np.sum(self.trace._keep[2]))
        h = C.c_void_p()
        rc = lib().sim_init(C.byref(self.cfg), C.byref(self.trace), C.byref(h))
        if rc != SIM_OK:
            raise SimError("sim_init", rc)
        self.ctx = h

    def _check(self, call: str, rc: int):
        if rc != SIM_OK:
            raise SimError(call, rc, lib().sim_last_error(self.ctx).decode())

    def load_weights(self, layers, params) -> None:
        """params: flat float32 (numpy host array or device tensor), PyTorch
        order: w0, b0, w1, b1, ..."""
        arr = (sim_layer * len(layers))(*[sim_layer(l.kind, l.c_in, l.c_out, l.relu)
                                          for l in layers])
        self.n_outputs = int(layers[-1].c_out)
        if isinstance(params, np.ndarray):
            params = np.ascontiguousarray(params, np.float32)
            self._check("sim_load_weights",
                        lib().sim_load_weights(self.ctx, arr, len(layers), params.ctypes.data, 0))
        else:
            self._check("sim_load_weights",
                        lib().sim_load_weights(self.ctx, arr, len(layers), params.data_ptr(), 1))

    RUN_TO_END = 2 ** 31 - 1

    def step(self, n_steps: int, lat_mode: int = SIM_LAT_PREDICT, lat_table=None) -> None:
        self._check("sim_step", lib().sim_step(self.ctx, n_steps, lat_mode, _ptr(lat_table)))

    def run(self, lat_mode: int = SIM_LAT_PREDICT, lat_table=None, per_sub: bool = True) -> dict:
        K = self.n_sub
        arrs = {k: np.zeros(K, np.int64) for k in ("fetch", "drain", "final", "warm_tick")}
        P64 = C.POINTER(C.c_int64)
        res = sim_result()
        if per_sub:
            res.fetch_cycles = arrs["fetch"].ctypes.data_as(P64)
            res.drain_cycles = arrs["drain"].ctypes.data_as(P64)
            res.final_tick = arrs["final"].ctypes.data_as(P64)
            res.warm_tick = arrs["warm_tick"].ctypes.data_as(P64)
        self._check("sim_run", lib().sim_run(self.ctx, lat_mode, _ptr(lat_table), C.byref(res)))
        out = {"total": res.total_cycles, "measured": res.measured_instr,
               "predicted": res.predicted_instr, "n_clamped": res.n_clamped,
               "n_nonfinite": res.n_nonfinite, "n_shadow_mismatch": res.n_shadow_mismatch}
        if per_sub:
            out.update(arrs)
        return out

    def reset(self) -> None:
        self._check("sim_reset", lib().sim_reset(self.ctx))

    def autotune(self, n_steps: int = 200, lat_mode: int = SIM_LAT_PREDICT, lat_table=None,
                 cache: Optional[str] = None) -> dict:
        """Choose the step kernel's launch shape (sim_autotune).  With a cache
        file (JSON), a choice recorded for the same device, window, network,
        precision and sub-trace count is applied instead of timing again."""
        import json
        import torch
        key = "|".join(str(v) for v in (torch.cuda.get_device_name(), self.cfg.n_feat,
                                         self.cfg.n_slot, getattr(self, "n_outputs", 0),
                                         self.cfg.prec, self.n_sub, self.trace.feat_dtype,
                                         lat_mode))
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                table = json.load(fh)
        if key in table:
            t = table[key]
            self._check("sim_set_tuning", lib().sim_set_tuning(self.ctx, t["variant"], t["n_wg"]))
            return dict(t, cached=True)
        out = sim_tuning()
        self._check("sim_autotune", lib().sim_autotune(self.ctx, n_steps, lat_mode,
                                                       _ptr(lat_table), C.byref(out)))
        t = {"variant": out.variant, "n_wg": out.n_wg, "ms": out.ms,
             "trials": [(out.tried_variant[i], out.tried_n_wg[i], out.tried_ms[i])
                        for i in range(out.n_tried)]}
        if cache:
            table[key] = t
            with open(cache, "w") as fh:
                json.dump(table, fh, indent=1)
        return dict(t, cached=False)

    def set_tuning(self, variant: int, n_wg: int) -> None:
        self._check("sim_set_tuning", lib().sim_set_tuning(self.ctx, variant, n_wg))

    def variant_scratch(self, variant: int) -> int:
        """Scratch bytes per lane of the C3 step kernel of `variant` in this
        form (nonzero: register spills)."""
        b = C.c_int64(0)
        self._check("sim_variant_scratch", lib().sim_variant_scratch(self.ctx, variant, C.byref(b)))
        return int(b.value)

    def calibrate(self, n_steps: int = 64, lat_mode: int = SIM_LAT_PREDICT, lat_table=None):
        self._check("sim_calibrate",
                    lib().sim_calibrate(self.ctx, n_steps, lat_mode, _ptr(lat_table)))

    def act_scales(self) -> np.ndarray:
        out = np.zeros(4096, np.float32)
        self._check("sim_act_scales", lib().sim_act_scales(self.ctx, out.ctypes.data, out.size))
        return out

    def use_graph(self, enable: bool = True) -> None:
        self._check("sim_set_graph", lib().sim_set_graph(self.ctx, int(enable)))

    def record_logits(self, buf) -> None:
        self._check("sim_record_logits", lib().sim_record_logits(self.ctx, _ptr(buf)))

    def forward(self, x, logits=None):
        import torch
        if not x.is_cuda or x.dtype != torch.float32 or not x.is_contiguous():
            raise ValueError("x must be a contiguous float32 device tensor")
        B = x.shape[0]
        if logits is None:
            logits = torch.empty((B, getattr(self, "n_outputs", 2)), dtype=torch.float32,
                                 device=x.device)
        self._check("predictor_fwd",
                    lib().predictor_fwd(self.ctx, x.data_ptr(), B, logits.data_ptr(), None))
        return logits

    def close(self) -> None:
        if getattr(self, "ctx", None):
            lib().sim_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def flat_params(ws, bs) -> np.ndarray:
    parts = []
    for w, b in zip(ws, bs):
        parts.append(np.asarray(w, np.float32).ravel())
        parts.append(np.asarray(b, np.float32).ravel())
    return np.ascontiguousarray(np.concatenate(parts), np.float32)


# ----------------------------------------------------------------- training ---

N_BINS = 400
TRAIN_OUT = 2 * (N_BINS + 1)


class Predictor:
    """A predictor-only context for the training head (C3 trunk + FC 512 ->
    802): forward with saved activations, hybrid loss, backward and Adam, all
    in the library's kernels.  Windows are float32 [B][111][50] device
    tensors; labels int32 [B][2]."""

    def __init__(self, layers, prec: int = SIM_FP32, stream=None, n_feat: int = 50,
                 n_slot: int = 111):
        import torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.cfg = make_config(n_feat, n_slot, (-1, -1, -1), prec=prec,
                               stream=self.stream.cuda_stream)
        z64 = np.zeros(0, np.int64)
        self.trace = make_trace(None, 0, z64, z64, np.zeros(0, np.int32))
        h = C.c_void_p()
        rc = lib().sim_init(C.byref(self.cfg), C.byref(self.trace), C.byref(h))
        if rc != SIM_OK:
            raise SimError("sim_init", rc)
        self.ctx = h
        self.layers = list(layers)
        self.n_slot, self.n_feat = n_slot, n_feat

    _check = Simulator._check
    load_weights = Simulator.load_weights
    close = Simulator.close
    __del__ = Simulator.__del__

    def save_bytes(self, B: int) -> int:
        n = lib().predictor_save_bytes(self.ctx, B)
        if n < 0:
            raise SimError("predictor_save_bytes", SIM_ESTATE, "weights of the training head "
                           "not loaded")
        return int(n)

    def forward(self, x):
        """Logits [B][802] and the save buffer for backward."""
        import torch
        _check_windows(x, self.n_slot, self.n_feat)
        B = x.shape[0]
        logits = torch.empty((B, TRAIN_OUT), dtype=torch.float32, device=x.device)
        save = torch.empty(max(1, self.save_bytes(B)), dtype=torch.uint8, device=x.device)
        self._check("predictor_fwd", lib().predictor_fwd(self.ctx, x.data_ptr(), B,
                                                         logits.data_ptr(), save.data_ptr()))
        return logits, save

    def loss(self, logits, labels, out=None, noalloc: bool = False):
        """Mean hybrid loss (device scalar) and its gradient w.r.t. logits.
        out = (loss, dlogits) device tensors to write into; noalloc selects
        sim_loss_noalloc (the library's static scratch, no allocation)."""
        import torch
        if labels.dtype != torch.int32 or not labels.is_contiguous():
            raise ValueError("labels must be contiguous int32 [B][2]")
        B = logits.shape[0]
        if out is None:
            out = (torch.empty((), dtype=torch.float32, device=logits.device),
                   torch.empty_like(logits))
        loss, dz = out
        name = "sim_loss_noalloc" if noalloc else "sim_loss"
        self._check(name, getattr(lib(), name)(self.ctx, logits.data_ptr(), labels.data_ptr(), B,
                                               loss.data_ptr(), dz.data_ptr()))
        return loss, dz

    def backward(self, x, save, dlogits, dparams, want_dx: bool = False,
                 accumulate: bool = False):
        import torch
        dlogits = dlogits.contiguous().float()
        B = x.shape[0]
        dx = torch.empty_like(x) if want_dx else None
        self._check("predictor_bwd",
                    lib().predictor_bwd(self.ctx, x.data_ptr(), save.data_ptr(),
                                        dlogits.data_ptr(), B, _ptr(dx), dparams.data_ptr(),
                                        int(accumulate)))
        return dx

    def adam(self, params, grads, m, v, step: int, lr: float = 1e-3, betas=(0.9, 0.999),
             eps: float = 1e-8):
        self._check("sim_adam", lib().sim_adam(self.ctx, params.data_ptr(), grads.data_ptr(),
                                               m.data_ptr(), v.data_ptr(), params.numel(), lr,
                                               betas[0], betas[1], eps, step))

    def adam_load(self, params, grads, m, v, step: int, lr: float = 1e-3, betas=(0.9, 0.999),
                  eps: float = 1e-8):
        """adam(), then the predictor's weights are the updated parameters
        (as load_weights would make them), in one launch."""
        self._check("sim_adam_load",
                    lib().sim_adam_load(self.ctx, params.data_ptr(), grads.data_ptr(),
                                        m.data_ptr(), v.data_ptr(), params.numel(), lr, betas[0],
                                        betas[1], eps, step))


def _check_windows(x, n_slot, n_feat):
    import torch
    if (not x.is_cuda or x.dtype != torch.float32 or not x.is_contiguous() or x.dim() != 3
            or x.shape[1] != n_slot or x.shape[2] != n_feat):
        raise ValueError(f"x must be a contiguous float32 device tensor [B][{n_slot}][{n_feat}]")


def _autograd():
    import torch

    class PredictorFunction(torch.autograd.Function):
        """logits = predictor(x; params) through the library's forward and
        backward kernels.  params is the flat PyTorch-order float32 device
        vector; it is (re)loaded into the context on every forward."""

        @staticmethod
        def forward(ctx, x, params, pred):
            x = x.contiguous()
            pred.load_weights(pred.layers, params.detach().contiguous())
            logits, save = pred.forward(x)
            ctx.pred = pred
            ctx.save_for_backward(x, save)
            return logits

        @staticmethod
        def backward(ctx, dlogits):
            x, save = ctx.saved_tensors
            dparams = torch.empty(ctx.pred.n_params, dtype=torch.float32, device=x.device)
            dx = ctx.pred.backward(x, save, dlogits, dparams, want_dx=ctx.needs_input_grad[0])
            return dx, dparams, None

    return PredictorFunction


_fn = None


def predictor_apply(x, params, pred: Predictor):
    """Differentiable predictor forward (torch.autograd)."""
    global _fn
    if _fn is None:
        _fn = _autograd()
    pred.n_params = params.numel()
    return _fn.apply(x, params, pred)


class Trainer:
    """Training loop of the predictor on windows and labelled latencies:
    forward, hybrid loss, backward and Adam, every step in the library's
    kernels, parameters resident on the device."""

    def __init__(self, layers, params, prec: int = SIM_FP32, lr: float = 1e-3,
                 betas=(0.9, 0.999), eps: float = 1e-8):
        import torch
        self.pred = Predictor(layers, prec)
        p = torch.as_tensor(np.ascontiguousarray(params, np.float32))
        self.params = p.cuda().contiguous()
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.lr, self.betas, self.eps = lr, betas, eps
        self.pred.load_weights(layers, self.params)

    def step(self, x, labels):
        """One optimisation step on a batch; returns the loss (device scalar)
        measured before the update."""
        logits, save = self.pred.forward(x)
        loss, dz = self.pred.loss(logits, labels)
        self.pred.backward(x, save, dz, self.grads)
        self.t += 1
        self.pred.adam_load(self.params, self.grads, self.m, self.v, self.t, self.lr, self.betas,
                            self.eps)
        return loss

    def close(self):
        self.pred.close()
