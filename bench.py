"""Benchmark: simulated MIPS of the SimNet step loop on one MI355X.

One benchmark step = one complete simulation of the workload (every
sub-trace from its first instruction, warm-up included, to its drain) with
the trace and weights resident in HBM: sim_reset + the persistent step
kernel + the device reduction, through the C ABI.

Workloads (--workload):
  c3_1m (default)  1,000,000-instruction synthetic trace, 50 features per
                   instruction, 4,096 equal sub-traces with 256-instruction
                   warm-up, 111-slot windows, CNN conv 64/128/256 (kernel 2,
                   stride 2) + FC 512 + FC 2, random-init weights.  Every
                   precision form is run (FP32, BF16, FP8 e4m3), and each is
                   compared with the FP64 oracle on a fixed sample of
                   sub-traces (every 16th: shadow-mode mismatch fraction,
                   per-sub-trace and total-cycle error of a free run); the
                   headline value is the fastest form whose total-cycle error
                   on the sample is at most 1 %, the others are reported
                   beside it.
  tiny             10,000 instructions, one sub-trace, 16 x 32 windows, conv
                   32/64 + FC 2, FP32: bound by per-step latency (B = 1).
  c3dep_1m         c3_1m with the 5 memory-dependency flags per context slot,
                   from synthetic PCs and data addresses, FP32 and BF16.
  c3st_1m          c3_1m with store latencies (FC 512 -> 3) and the memory
                   write queue that stores pass through, FP32 and BF16.
  c3hyb_1m         c3_1m with the paper's hybrid inference head (FC 512 -> 22:
                   per latency type 10 class scores + 1 direct output), FP32
                   and BF16.
  c3_uneven        20,000 independent streams with log-uniform lengths in
                   [1e3, 2e5] (7.5e8 instructions), packed instruction codes,
                   BF16, slots refilled longest-first, run as one graph.
  c3_train         predictor training: one step = forward with saved
                   activations, hybrid loss (400-bin CE + L1 on log1p), backward
                   and Adam on 4,096 labelled 111x50 contexts, C3 trunk + FC
                   512 -> 802 head, BF16 (FP32 master weights); contexts/s.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "simulated MIPS on 1 MI355X, FP32 vs BF16/FP8 at ≤1% total-cycle error"
# FLOP per prediction from the layer lists (multiply-adds x 2); the kernels
# skip window slots and conv positions no output depends on, so they execute
# slightly fewer (6,631,424 for the C3 network).
FLOP_PER_PRED = {"c3": 6_702_592, "small": 66_560, "c3hyb": 6_723_072, "c3st": 6_703_616,
                 "rb7": 185_636_352}
# Training step per context: forward 3,760,896 MAC (trunk + FC 512 -> 802),
# backward twice that less conv1's input gradient (352,000 MAC), x 2 FLOP.
FLOP_PER_TRAIN_CTX = 21_861_376
PEAK = {"f32": 157.3, "bf16": 2500.0, "fp8": 5000.0}  # published dense MFMA, TFLOP/s
PREC = {"f32": 0, "bf16": 1, "fp8": 2}
# HBM bytes of one step-kernel launch (one full c3_1m simulation) from two
# rocprofv3 passes (FETCH_SIZE, WRITE_SIZE) scaled by the same counters over a
# 1 GiB copy.  They hold for the kernel source they were measured on only:
# reported while csrc/kernels.hip hashes to KERNEL_SHA, else null.
KERNEL_SHA = "44addb45ea113718"
TRAFFIC = {"c3_1m": {"bf16": 22_771_582_666, "fp8": 43_861_012_163}}


def measured_traffic(workload, form):
    import hashlib
    path = os.path.join(ROOT, "paper_2105_05821_amd", "csrc", "kernels.hip")
    with open(path, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    if sha != KERNEL_SHA:
        return None
    return TRAFFIC.get(workload, {}).get(form)


def measure_peaks():
    """Project-written probes on this GPU: MFMA issue rate of the three
    matrix instructions the kernels use, HBM read and copy bandwidth."""
    import ctypes as C
    import torch
    lib = C.CDLL(os.path.join(ROOT, "paper_2105_05821_amd", "libsimnet_peaks.so"))
    stream = torch.cuda.current_stream().cuda_stream
    seed = torch.randint(1, 2 ** 30, (64,), dtype=torch.int32, device="cuda")
    blocks = 2048  # 8 workgroups of 4 waves per CU
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    res = {}
    for prec, name, n_iter, flop in [(0, "f32", 10000, 2048), (1, "bf16", 20000, 16384),
                                     (3, "bf16_32x32", 20000, 16384), (2, "fp8", 20000, 16384)]:
        best = None
        for _ in range(4):  # the first launch warms up
            ms = C.c_float(0.0)
            rc = lib.peaks_mfma(prec, blocks, n_iter, C.c_void_p(seed.data_ptr()),
                                C.c_void_p(out.data_ptr()), C.c_void_p(stream), C.byref(ms))
            if rc != 0:
                raise RuntimeError(f"peaks_mfma rc {rc}")
            best = ms.value if best is None else min(best, ms.value)
        tflops = blocks * 4 * n_iter * 8 * flop / (best / 1e3) / 1e12
        pub = PEAK[name.split("_")[0]]
        res[f"mfma_{name}"] = {"tflops": round(tflops, 1), "published": pub,
                               "ratio": round(tflops / pub, 3)}
    nbytes = 1 << 31
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for mode, name, moved in [(0, "read", nbytes), (1, "copy", 2 * nbytes)]:
        best = None
        for _ in range(4):
            ms = C.c_float(0.0)
            rc = lib.peaks_hbm(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                               C.c_int64(nbytes), mode, 256 * 16, 1, C.c_void_p(stream),
                               C.byref(ms))
            if rc != 0:
                raise RuntimeError(f"peaks_hbm rc {rc}")
            best = ms.value if best is None else min(best, ms.value)
        gbs = moved / (best / 1e3) / 1e9
        res[f"hbm_{name}"] = {"gb_s": round(gbs, 1), "published": 8000.0,
                              "ratio": round(gbs / 8000.0, 3)}
    # L2 -> CU: every workgroup (one per CU, and four per CU) re-reads the
    # same 1 MiB
    for per_cu in (1, 4):
        blocks, reps, region = 256 * per_cu, 64, 1 << 20
        best = None
        for _ in range(4):
            ms = C.c_float(0.0)
            rc = lib.peaks_hbm(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                               C.c_int64(region), 2, blocks, reps, C.c_void_p(stream),
                               C.byref(ms))
            if rc != 0:
                raise RuntimeError(f"peaks_hbm rc {rc}")
            best = ms.value if best is None else min(best, ms.value)
        gbs = blocks * reps * region / (best / 1e3) / 1e9
        res[f"l2_read_{per_cu}wg_per_cu"] = {"gb_s": round(gbs, 1),
                                             "per_cu_bytes_per_clk_at_2.4GHz":
                                                 round(gbs / 256 / 2.4, 1)}
    return res


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(wl, feat, start, length, warm, ws, bs, budget_s=15.0, mem=None):
    """The FP64 oracle on the host cores over a bounded sample of the
    workload's sub-traces (every step-th), scaled to MIPS."""
    import oracle
    oracle.build(force=not os.path.exists(oracle.LIB))
    model = oracle.Model(wl.layers, ws, bs, wl.n_feat, wl.n_slot)
    cfg = oracle.sim_cfg(wl.n_feat, wl.n_slot, wl.n_out, wl.retire_width, wl.cols,
                         head=wl.extra.get("head", 0), store_col=wl.extra.get("store_col", -1),
                         dep_col=wl.extra.get("dep_col", -1))
    threads = oracle.default_threads()
    K = len(start)
    if wl.name == "rb7_1m":
        # one RB7 prediction costs the FP64 oracle ~0.1 s: one sub-trace per
        # thread, each cut to its first 48 instructions (no warm-up)
        ks = np.arange(0, K, K // threads)[:threads]
        cut = np.minimum(length[ks], 48)
        t0 = time.perf_counter()
        oracle.simulate(cfg, feat, start[ks], cut, np.zeros(len(ks), np.int32), model=model,
                        threads=threads, mem=mem)
        dt = time.perf_counter() - t0
        meas = int(cut.sum())
        return {"value": round(meas / dt / 1e6, 9), "unit": "MIPS", "cores": threads,
                "kind": "oracle",
                "sample": f"{len(ks)} of {K} sub-traces (every {K // threads}th), the first "
                          f"{int(cut.max())} instructions of each, no warm-up, FP64, {dt:.1f} s"}
    if K == 1:
        ks = np.array([0])
        step = 1
    else:
        probe = np.arange(0, K, max(1, K // 8))
        t0 = time.perf_counter()
        oracle.simulate(cfg, feat, start[probe], length[probe], warm[probe], model=model,
                        threads=threads, mem=mem)
        dt = time.perf_counter() - t0
        per_sub = dt / len(probe) * min(threads, len(probe))
        n = int(max(threads, min(K // 8, budget_s / max(per_sub, 1e-6) * threads)))
        step = max(1, K // n)
        ks = np.arange(0, K, step)
    t0 = time.perf_counter()
    oracle.simulate(cfg, feat, start[ks], length[ks], warm[ks], model=model, threads=threads,
                    mem=mem)
    dt = time.perf_counter() - t0
    meas = int(length[ks].sum())
    return {"value": round(meas / dt / 1e6, 6), "unit": "MIPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{len(ks)} of {K} sub-traces (every {step}th), {meas} measured + "
                      f"{int(warm[ks].sum())} warm-up instructions, FP64, {dt:.1f} s"}


ACC_EVERY = 16  # accuracy sample: every 16th sub-trace (256 of c3_1m's 4,096)


def fp64_reference(wl, feat, start, length, warm, ws, bs):
    """The FP64 oracle's own simulation of a fixed sample of sub-traces: its
    rounded latencies (the shadow-mode table) and per-sub-trace cycles, timed
    on the host cores (this run is also the CPU baseline)."""
    import oracle
    oracle.build(force=not os.path.exists(oracle.LIB))
    model = oracle.Model(wl.layers, ws, bs, wl.n_feat, wl.n_slot)
    cfg = oracle.sim_cfg(wl.n_feat, wl.n_slot, wl.n_out, wl.retire_width, wl.cols)
    threads = oracle.default_threads()
    ks = np.arange(0, len(start), ACC_EVERY)
    t0 = time.perf_counter()
    ref = oracle.simulate(cfg, feat, start[ks], length[ks], warm[ks], model=model,
                          threads=threads, want_lat=True)
    dt = time.perf_counter() - t0
    meas = int(length[ks].sum())
    base = {"value": round(meas / dt / 1e6, 6), "unit": "MIPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{len(ks)} of {len(start)} sub-traces (every {ACC_EVERY}th), {meas} "
                      f"measured + {int(warm[ks].sum())} warm-up instructions, FP64, {dt:.1f} s"}
    return {"ks": ks, "lat": ref["lat"], "cycles": (ref["final"] - ref["warm_tick"]),
            "cpu_baseline": base}


def form_accuracy(sn, torch, sim, ref, length, warm):
    """Accuracy of a form against the FP64 oracle on the reference sample, on
    the simulator the form was timed with (same weights, same FP8 scales):
      mismatch_fraction: shadow mode (the oracle's latencies advance every
        sample sub-trace, so the windows are the oracle's), rounded outputs
        of the form that differ from the oracle's;
      per-sub-trace and total-cycle error: a free run, |C - C64| / C64."""
    ks = ref["ks"]
    n = (length + warm).astype(np.int64)
    off = np.concatenate([[0], np.cumsum(n)])
    n_pred = int(off[-1])
    rows = np.concatenate([np.arange(off[k], off[k + 1]) for k in ks])
    table = np.zeros((n_pred, 2), np.int32)
    table[rows] = ref["lat"]
    dtable = torch.from_numpy(table).cuda()
    logits = torch.zeros((n_pred, 2), dtype=torch.float32, device="cuda")
    sim.reset()
    sim.record_logits(logits)
    sim.run(sn.SIM_LAT_SHADOW, dtable)
    sim.record_logits(None)
    z = logits.cpu().numpy()[rows].astype(np.float64)
    own = np.clip(np.rint(np.nan_to_num(z, nan=0.0, posinf=0.0, neginf=0.0)), 0, 65535)
    mism = int((own.astype(np.int32) != ref["lat"]).sum())
    sim.reset()
    free = sim.run()
    c = (free["final"] - free["warm_tick"])[ks].astype(np.float64)
    c64 = ref["cycles"].astype(np.float64)
    err = np.abs(c - c64) / c64
    return {"mismatch_fraction": round(mism / ref["lat"].size, 6),
            "total_cycle_error": round(abs(c.sum() - c64.sum()) / c64.sum(), 6),
            "per_subtrace_error_mean": round(float(err.mean()), 6),
            "per_subtrace_error_max": round(float(err.max()), 6),
            "sample_total_cycles": int(c.sum()), "fp64_sample_total_cycles": int(c64.sum())}


def time_form(sn, torch, dfeat, wl, start, length, warm, ws, bs, prec, steps, warmup,
              n_feat=None, graph=False, dmem=None, tune=False, ref=None):
    """Run the workload `steps` times after `warmup` runs; returns the time of
    the whole runs (host clock) and of the step kernel (HIP events on the
    stream the library launches on)."""
    sim = sn.Simulator(dfeat, wl.n_slot, wl.cols, start, length, warm, prec=PREC[prec],
                       n_feat=n_feat, n_out=wl.n_out, store_col=wl.extra.get("store_col", 0),
                       mem=dmem, col_dep=wl.extra.get("dep_col", -1))
    sim.load_weights(wl.layers, sn.flat_params(ws, bs))
    if prec == "fp8":
        sim.calibrate(64)  # per-channel scales from the first 64 FP32 steps (set-up, untimed)
    tuning = None
    if graph or tune:
        # launch shape chosen on the first 300 steps (set-up, untimed)
        tuning = sim.autotune(300)
        log(f"[bench] autotune: variant {tuning['variant']}, {tuning['n_wg']} workgroups; "
            f"trials {tuning['trials']}")
    if graph:
        sim.use_graph(True)
    stream = sim.stream

    def one_run(ev=None):
        sim.reset()
        if ev is not None:
            ev[0].record(stream)
        if graph:
            res = sim.run()  # one graph: step kernel until every slot is empty + total
        else:
            sim.step(sim.RUN_TO_END)  # the persistent step kernel: the whole simulation
        if ev is not None:
            ev[1].record(stream)
        return res if graph else sim.run()

    res = None
    for i in range(warmup):
        res = one_run()
        log(f"[bench] {prec} warmup {i}: total cycles {res['total']}")
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        res = one_run(events[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    k_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    acc = form_accuracy(sn, torch, sim, ref, length, warm) if ref is not None else None
    sim.close()
    return {"elapsed": elapsed, "kernel_ms": k_ms, "res": res, "tuning": tuning, "acc": acc}


def train_bench(sn, torch, wl, steps, warmup, prec):
    """Training steps on one fixed synthetic batch resident in HBM; HIP events
    on the library's stream around each step."""
    import synth
    B = wl.extra["batch"]
    x, lat = synth.training_batch(wl.trace_seed, wl.n_instr, wl.n_feat, wl.n_slot, B, 5)
    ws, bs = synth.init_weights(wl.weight_seed, wl.layers, out_bias=None, out_gain=1.0)
    tr = sn.Trainer(wl.layers, sn.flat_params(ws, bs), prec=PREC[prec], lr=1e-4)
    xd = torch.from_numpy(x).cuda()
    ld = torch.from_numpy(lat).cuda()
    stream = tr.pred.stream
    losses = []
    for i in range(warmup):
        losses.append(float(tr.step(xd, ld).item()))
        log(f"[bench] train warmup {i}: loss {losses[-1]:.4f}")
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
    loss_dev = []
    t0 = time.perf_counter()
    for i in range(steps):
        events[i][0].record(stream)
        loss_dev.append(tr.step(xd, ld))
        events[i][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    k_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    losses += [float(l.item()) for l in loss_dev]
    tr.close()
    return {"elapsed": elapsed, "kernel_ms": k_ms, "B": B, "losses": losses}


WORKLOAD_TEXT = {
    "c3_1m": "c3_1m: 1,000,000-instruction synthetic trace, 4,096 sub-traces (244/245 instr) "
             "+ 256 warm-up, 111x50 windows, conv 64/128/256 k2s2 + FC 512 + FC 2, "
             "random-init weights",
    "tiny": "tiny: 10,000-instruction synthetic trace, one sub-trace, 16x32 windows, "
            "conv 32/64 k2s2 + FC 2, random-init weights",
    "c3dep_1m": "c3dep_1m: the c3_1m trace and partition with the 5 memory-dependency flags "
                "of every context slot (synthetic PCs and data addresses), C3 network",
    "c3st_1m": "c3st_1m: the c3_1m trace and partition with store latencies (FC 512 -> 3: "
               "fetch, execution, store) and the memory write queue, random-init weights",
    "c3hyb_1m": "c3hyb_1m: the c3_1m trace and partition with the hybrid inference head "
                "(per latency type 10 class scores + 1 direct output, FC 512 -> 22), "
                "random-init weights",
    "c3_uneven": "c3_uneven: 20,000 streams, log-uniform lengths 1e3..2e5, packed codes, "
                 "111x50 windows, C3 network, slots refilled longest-first",
    "rb7_1m": "rb7_1m: the c3_1m trace and partition with RB7 (conv 64/128/256 k2s2, seven "
              "residual blocks 256 -> 1920 -> 256 at 13 positions, FC 512, hybrid head FC "
              "512 -> 22), random-init weights",
    "c3_train": "c3_train: training step on 4,096 labelled 111x50 contexts (analytic "
                "latencies 0..400), conv 64/128/256 k2s2 + FC 512 + FC 802 hybrid head, "
                "400-bin CE + L1 log1p loss, Adam, FP32 master weights",
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="c3_1m", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--prec", default=None, choices=sorted(PREC),
                    help="run one form only (c3_1m default: all three)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--peaks", action="store_true",
                    help="only measure this GPU's MFMA and HBM peaks with the project's probes")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES, 3 times (the "
                         "reference kernel that scales HBM byte counters)")
    args = ap.parse_args()
    if args.peaks:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"peaks": measure_peaks()}), flush=True)
        return
    if args.copy_probe:
        import torch
        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the sub-traces "
              "are independent, a multi-GPU run would shard them with no communication, and "
              "that path is not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2105_05821_amd as sn
    import synth

    torch.cuda.set_device(0)
    wl = synth.workload(args.workload)
    if args.workload == "c3_train":
        steps = args.steps if args.steps is not None else 20
        warmup = args.warmup if args.warmup is not None else 3
        prec = args.prec or "bf16"
        if prec == "fp8":
            print("no FP8 training form", file=sys.stderr)
            sys.exit(2)
        r = train_bench(sn, torch, wl, steps, warmup, prec)
        tflops = FLOP_PER_TRAIN_CTX * r["B"] / (r["kernel_ms"] / 1e3) / 1e12
        out = {
            "metric": "training contexts/s on 1 MI355X (forward + hybrid loss + backward + "
                      "Adam)",
            "value": round(r["B"] * steps / r["elapsed"], 1), "unit": "contexts/s",
            "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": round(r["elapsed"] / steps * 1e3, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
            "config": {"workload": WORKLOAD_TEXT["c3_train"], "batch": r["B"],
                       "loss_first": round(r["losses"][0], 5),
                       "loss_last": round(r["losses"][-1], 5)},
            "roofline": {"bound": "mfma", "achieved": round(tflops, 3),
                         "peak": PEAK[prec], "unit": "TFLOP/s",
                         "frac": round(tflops / PEAK[prec], 4), "traffic": None,
                         "kernel": "whole training step (forward kernel, GEMMs, loss, "
                                   "column sums, Adam, re-layout)",
                         "kernel_ms": round(r["kernel_ms"], 3)},
        }
        print(json.dumps(out), flush=True)
        return
    ws, bs = synth.init_weights(wl.weight_seed, wl.layers,
                                out_bias=wl.extra.get("out_bias", synth.OUT_BIAS))
    net = {"tiny": "small", "c3hyb_1m": "c3hyb", "c3st_1m": "c3st",
           "rb7_1m": "rb7"}.get(args.workload, "c3")
    n_feat = None
    feat = None
    mem = dmem = None
    if args.workload == "c3_uneven":
        steps = args.steps if args.steps is not None else 1
        warmup = args.warmup if args.warmup is not None else 0
        length = synth.loguniform_lengths(wl.length_seed, wl.n_sub, *wl.len_range)
        start = np.concatenate([[0], np.cumsum(length)[:-1]]).astype(np.int64)
        warm = np.zeros(wl.n_sub, np.int32)
        n_instr = int(length.sum())
        log(f"[bench] {wl.name}: {wl.n_sub} streams, {n_instr} instructions (codes on the GPU)")
        dfeat = torch.empty(n_instr, dtype=torch.int32, device="cuda")
        chunk = 1 << 26
        for lo in range(0, n_instr, chunk):
            hi = min(n_instr, lo + chunk)
            dfeat[lo:hi] = synth.trace_codes_torch(wl.trace_seed, lo, hi, device="cuda")
        n_feat = wl.n_feat
        forms = [args.prec or "bf16"]
    else:
        steps = args.steps if args.steps is not None else 5
        warmup = args.warmup if args.warmup is not None else 1
        n_instr = wl.n_instr
        log(f"[bench] generating {wl.name}: {n_instr} instructions, {wl.n_sub} sub-traces")
        feat = synth.trace_features(wl.trace_seed, n_instr, wl.n_feat)
        start, length, warm = sn.partition(n_instr, wl.n_sub, wl.warmup)
        dfeat = torch.from_numpy(feat).cuda()
        if "dep_col" in wl.extra:
            mem = synth.trace_mem(wl.trace_seed, n_instr)
            dmem = torch.from_numpy(mem.view(np.int32)).cuda()
        if args.workload == "tiny":
            forms = [args.prec or "f32"]
        elif args.workload in ("c3hyb_1m", "c3st_1m", "c3dep_1m", "rb7_1m"):
            forms = [args.prec] if args.prec else ["f32", "bf16"]
        else:
            forms = [args.prec] if args.prec else ["f32", "bf16", "fp8"]
    n_pred = int(length.sum() + warm.sum())
    measured = int(length.sum())
    ref = None
    if args.workload == "c3_1m" and not args.no_cpu_baseline:
        log(f"[bench] FP64 oracle on every {ACC_EVERY}th sub-trace (accuracy reference and "
            "CPU baseline)")
        ref = fp64_reference(wl, feat, start, length, warm, ws, bs)
        log(f"[bench] oracle: {ref['cpu_baseline']}")

    results = {}
    for f in forms:
        r = time_form(sn, torch, dfeat, wl, start, length, warm, ws, bs, f, steps, warmup,
                      n_feat=n_feat, graph=args.workload == "c3_uneven", dmem=dmem,
                      tune=args.workload == "c3_1m", ref=ref)
        r["mips"] = measured * steps / r["elapsed"] / 1e6
        r["tflops"] = FLOP_PER_PRED[net] * n_pred / (r["kernel_ms"] / 1e3) / 1e12
        results[f] = r
        log(f"[bench] {f}: {steps} runs in {r['elapsed']:.3f} s; step kernel "
            f"{r['kernel_ms']:.3f} ms; {r['mips']:.3f} MIPS; {r['tflops']:.2f} TFLOP/s; "
            f"total cycles {r['res']['total']}")

        if r["acc"]:
            log(f"[bench] {f} vs FP64 oracle: {r['acc']}")

    ref_total = results["f32"]["res"]["total"] if "f32" in results else None
    if ref is not None:
        # the metric's gate: total-cycle error against the FP64 oracle on the
        # sample within 1 %
        gate = "total-cycle error <= 1 % against the FP64 oracle on the accuracy sample"
        ok = [f for f in results if results[f]["acc"]["total_cycle_error"] <= 0.01]
    else:
        gate = "full-run total cycles within 1 % of the FP32 form's (no FP64 reference run)"
        ok = [f for f in results
              if ref_total is None or abs(results[f]["res"]["total"] - ref_total) <= 0.01 * ref_total]
    best = max(ok, key=lambda f: results[f]["mips"])
    b = results[best]
    out = {
        "metric": METRIC, "value": round(b["mips"], 4), "unit": "MIPS", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": round(b["elapsed"] / steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": best, "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "predictions_per_step": n_pred, "measured_instr_per_step": measured,
                   "total_cycles": int(b["res"]["total"])},
        "roofline": {"bound": "mfma", "achieved": round(b["tflops"], 3), "peak": PEAK[best],
                     "unit": "TFLOP/s", "frac": round(b["tflops"] / PEAK[best], 4),
                     "traffic": measured_traffic(args.workload, best),
                     "kernel": ("RB7 step: gather + convolutions, residual blocks, FC 512 + "
                                "head, update (four launches per step, all timed)"
                                if net == "rb7" else
                                "step_kernel (persistent: gather + CNN + round + queue update)"),
                     "kernel_ms": round(b["kernel_ms"], 3)},
    }
    if len(results) > 1:
        out["config"]["headline_gate"] = gate
        out["forms"] = {f: {"mips": round(r["mips"], 4), "kernel_ms": round(r["kernel_ms"], 3),
                            "tflops": round(r["tflops"], 3),
                            "frac": round(r["tflops"] / PEAK[f], 4),
                            "total_cycles": int(r["res"]["total"]),
                            "vs_fp64_oracle": r["acc"],
                            "meets_gate": f in ok}
                        for f, r in results.items()}
        if ref is not None:
            out["config"]["accuracy_sample"] = ref["cpu_baseline"]["sample"]
    if args.workload == "tiny":
        out["steps_per_s"] = round(n_pred * steps / b["elapsed"], 1)
    if b.get("tuning"):
        out["config"]["launch_shape"] = {k: b["tuning"][k] for k in ("variant", "n_wg")}
    if len(results) > 1 and any(r.get("tuning") for r in results.values()):
        for f, r in results.items():
            if r.get("tuning"):
                out["forms"][f]["launch_shape"] = {k: r["tuning"][k] for k in ("variant", "n_wg")}
    if ref is not None:
        out["cpu_baseline"] = ref["cpu_baseline"]
    elif not args.no_cpu_baseline and feat is not None:
        log("[bench] timing the FP64 oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(wl, feat, start, length, warm, ws, bs, mem=mem)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
