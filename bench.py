"""Benchmark: simulated MIPS of the SimNet step loop on one MI355X.

One benchmark step = one complete simulation of the workload (every
sub-trace from its first warm-up instruction to its drain), inputs resident
in HBM: sim_reset + sim_run through the C ABI.

Workload (the one-GPU configuration the headline metric is quoted on):
1,000,000-instruction synthetic trace, 50 features per instruction, cut into
4,096 equal sub-traces with 256-instruction warm-up; 111-slot windows; CNN
conv 64/128/256 (kernel 2, stride 2) + FC 512 + FC 2; random-init weights.
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
FLOP_PER_PRED = 6_702_592     # C3 network, layer-list definition (see the design notes)
PEAK = {"f32": 157.3, "bf16": 2500.0, "fp8": 5000.0}  # published dense MFMA, TFLOP/s
PREC = {"f32": 0, "bf16": 1, "fp8": 2}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(wl, feat, start, length, warm, layers, ws, bs, budget_s=15.0):
    """The FP64 oracle on the host cores over a bounded sample of sub-traces
    of the same workload (every 64th sub-trace, scaled to MIPS)."""
    import oracle
    oracle.build(force=not os.path.exists(oracle.LIB))
    model = oracle.Model(layers, ws, bs, wl.n_feat, wl.n_slot)
    cfg = oracle.sim_cfg(wl.n_feat, wl.n_slot, 2, wl.retire_width, wl.cols)
    threads = oracle.default_threads()
    # size the sample from a short probe so the leg takes about budget_s
    probe = np.arange(0, wl.n_sub, 512)
    t0 = time.perf_counter()
    oracle.simulate(cfg, feat, start[probe], length[probe], warm[probe], model=model,
                    threads=threads)
    dt = time.perf_counter() - t0
    per_sub = dt / len(probe) * min(threads, len(probe))
    n = int(max(threads, min(wl.n_sub // 8, budget_s / max(per_sub, 1e-6) * threads)))
    step = max(1, wl.n_sub // n)
    ks = np.arange(0, wl.n_sub, step)
    t0 = time.perf_counter()
    oracle.simulate(cfg, feat, start[ks], length[ks], warm[ks], model=model, threads=threads)
    dt = time.perf_counter() - t0
    meas = int(length[ks].sum())
    return {"value": round(meas / dt / 1e6, 6), "unit": "MIPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{len(ks)} of {wl.n_sub} sub-traces (every {step}th), {meas} measured + "
                      f"{int(warm[ks].sum())} warm-up instructions, FP64, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="f32", choices=sorted(PREC))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the sub-traces "
              "are independent, a multi-GPU run would shard them with no communication, and "
              "that path is not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2105_05821_amd as sn
    import synth

    wl = synth.workload("c3_1m")
    log(f"[bench] generating {wl.name}: {wl.n_instr} instructions, {wl.n_sub} sub-traces")
    feat = synth.trace_features(wl.trace_seed, wl.n_instr, wl.n_feat)
    ws, bs = synth.init_weights(wl.weight_seed, wl.layers)
    start, length, warm = sn.partition(wl.n_instr, wl.n_sub, wl.warmup)
    n_pred = int(length.sum() + warm.sum())

    torch.cuda.set_device(0)
    dfeat = torch.from_numpy(feat).cuda()
    sim = sn.Simulator(dfeat, wl.n_slot, wl.cols, start, length, warm, prec=PREC[args.prec])
    sim.load_weights(wl.layers, sn.flat_params(ws, bs))
    if args.prec == "fp8":
        sim.calibrate(64)  # per-channel scales from the first 64 FP32 steps (set-up, untimed)
    stream = sim.stream

    def one_run(ev=None):
        sim.reset()
        if ev is not None:
            ev[0].record(stream)
        sim.step(sim.RUN_TO_END)  # the persistent step kernel: the whole simulation
        if ev is not None:
            ev[1].record(stream)
        return sim.run()

    for i in range(args.warmup):
        res = one_run()
        log(f"[bench] warmup {i}: total cycles {res['total']}")
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = one_run(events[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    k_ms = [a.elapsed_time(b) for a, b in events]
    kern_s = float(np.mean(k_ms)) / 1e3
    ms_per_step = elapsed / args.steps * 1e3
    mips = wl.n_instr * args.steps / elapsed / 1e6
    achieved = FLOP_PER_PRED * n_pred / kern_s / 1e12
    log(f"[bench] {args.steps} runs in {elapsed:.3f} s; step kernel {np.mean(k_ms):.3f} ms avg; "
        f"{mips:.3f} MIPS; {achieved:.2f} TFLOP/s; total cycles {res['total']}")

    out = {
        "metric": METRIC, "value": round(mips, 4), "unit": "MIPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.prec, "data": "synthetic",
        "config": {"workload": "c3_1m: 1,000,000-instruction synthetic trace, 4,096 sub-traces "
                               "(244/245 instr) + 256 warm-up, 111x50 windows, conv 64/128/256 "
                               "k2s2 + FC 512 + FC 2, random-init weights",
                   "predictions_per_step": n_pred, "measured_instr_per_step": wl.n_instr,
                   "total_cycles": int(res["total"])},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK[args.prec],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK[args.prec], 4),
                     "traffic": None,
                     "kernel": "step_kernel (persistent: gather + CNN + round + queue update)",
                     "kernel_ms": round(float(np.mean(k_ms)), 3)},
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(wl, feat, start, length, warm, wl.layers, ws, bs)
    print(json.dumps(out), flush=True)
    sim.close()


if __name__ == "__main__":
    main()
