"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds input generation only: instruction-trace feature rows,
random-init predictor weights, sub-trace length streams and injected latency
tables.  None of the simulator's or the predictor's arithmetic lives here.

Every draw comes from a counter-based SplitMix64 stream (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): the
value for (seed, stream, counter) is the SplitMix64 output mixer applied to
``key(seed, stream) + (counter + 1) * GOLDEN``.  A trace row therefore depends
only on its instruction index, never on how the trace is later partitioned
or on how many threads generate it.

Feature layout (the paper lists static-property, instruction-context and
history-context features in its feature table, Sec. 2.2; its per-instruction
counts do not add up, so a synthetic layout with the same roles is used):

  D = 32:  [0,5)   op class one-hot (int-ALU, load, store, branch, FP)
           [5,26)  3 register ids, each one-hot into 7 buckets, bucket = id*7//32
           [26,29) data access level one-hot (L1, L2, DRAM)
           [29]    branch-mispredict flag (drawn for branches only)
           [30]    residence latency   (dynamic, written by the simulator)
           [31]    execution latency   (dynamic, written by the simulator)
  D = 50:  [0,30)  as above, [30,47) reserved zeros,
           [47] residence, [48] execution, [49] store latency (dynamic)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

OP_PROBS = (0.40, 0.25, 0.10, 0.15, 0.10)  # int-ALU, load, store, branch, FP
OP_INT, OP_LOAD, OP_STORE, OP_BRANCH, OP_FP = range(5)
LEVEL_PROBS = (0.90, 0.07, 0.03)  # L1, L2, DRAM
MISPREDICT_RATE = 0.05  # of branch instructions
N_REG_IDS = 32
N_REG_BUCKETS = 7


def _mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> np.uint64:
    base = np.array([(seed * 0x632BE59BD9B4E019 + stream * 0x85EBCA77C2B2AE63)
                     & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    return _mix(base)[0]


def u64(seed: int, stream: int, counter) -> np.ndarray:
    """Raw 64-bit SplitMix64 outputs for an array of counters."""
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = stream_key(seed, stream) + (c + np.uint64(1)) * GOLDEN
    return _mix(z)


def uniform(seed: int, stream: int, counter) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits."""
    return (u64(seed, stream, counter) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _categorical(u: np.ndarray, probs: Sequence[float]) -> np.ndarray:
    edges = np.cumsum(np.asarray(probs, dtype=np.float64))
    edges[-1] = 1.0 + 1e-12
    return np.searchsorted(edges, u, side="right").astype(np.int64)


# ---------------------------------------------------------------- traces ---

TRACE_STREAM = 11
N_FIELDS = 6  # op, reg0, reg1, reg2, level, mispredict


def trace_fields(seed: int, lo: int, hi: int) -> dict:
    """Categorical fields of instructions [lo, hi) of the trace."""
    n = np.arange(lo, hi, dtype=np.uint64)
    base = n * np.uint64(N_FIELDS)
    op = _categorical(uniform(seed, TRACE_STREAM, base + np.uint64(0)), OP_PROBS)
    regs = np.stack([(u64(seed, TRACE_STREAM, base + np.uint64(1 + r)) >> np.uint64(59)).astype(np.int64)
                     for r in range(3)], axis=1)
    level = _categorical(uniform(seed, TRACE_STREAM, base + np.uint64(4)), LEVEL_PROBS)
    mis = (uniform(seed, TRACE_STREAM, base + np.uint64(5)) < MISPREDICT_RATE) & (op == OP_BRANCH)
    return {"op": op, "regs": regs, "level": level, "mispredict": mis.astype(np.int64)}


def pack_codes(fields: dict) -> np.ndarray:
    """One uint32 per instruction: op | r0<<3 | r1<<8 | r2<<13 | level<<18 | mis<<20."""
    r = fields["regs"]
    code = (fields["op"] | (r[:, 0] << 3) | (r[:, 1] << 8) | (r[:, 2] << 13)
            | (fields["level"] << 18) | (fields["mispredict"] << 20))
    return code.astype(np.uint32)


def expand_codes(codes: np.ndarray, n_feat: int) -> np.ndarray:
    """Feature rows (float32, dynamic columns zero) from packed codes."""
    if n_feat not in (32, 50):
        raise ValueError("feature layouts exist for D=32 and D=50")
    c = np.asarray(codes, dtype=np.int64)
    n = c.shape[0]
    x = np.zeros((n, n_feat), dtype=np.float32)
    rows = np.arange(n)
    x[rows, c & 7] = 1.0
    for r in range(3):
        rid = (c >> (3 + 5 * r)) & 31
        x[rows, 5 + 7 * r + (rid * N_REG_BUCKETS) // N_REG_IDS] = 1.0
    x[rows, 26 + ((c >> 18) & 3)] = 1.0
    x[:, 29] = ((c >> 20) & 1).astype(np.float32)
    return x


def trace_codes(seed: int, n_instr: int, lo: int = 0, hi: Optional[int] = None,
                chunk: int = 1 << 22) -> np.ndarray:
    hi = n_instr if hi is None else hi
    out = np.empty(hi - lo, dtype=np.uint32)
    for a in range(lo, hi, chunk):
        b = min(hi, a + chunk)
        out[a - lo:b - lo] = pack_codes(trace_fields(seed, a, b))
    return out


def _t_shr(x, k: int):
    """Logical right shift of int64 tensors holding uint64 bit patterns."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def _t_mix(z):
    z = (z ^ _t_shr(z, 30)) * _signed(0xBF58476D1CE4E5B9)
    z = (z ^ _t_shr(z, 27)) * _signed(0x94D049BB133111EB)
    return z ^ _t_shr(z, 31)


def _signed(u: int) -> int:
    return u - (1 << 64) if u >= 1 << 63 else u


def trace_codes_torch(seed: int, lo: int, hi: int, device="cpu"):
    """The same packed codes as trace_codes, computed with torch int64
    (wrapping) arithmetic on any device; returns an int32 tensor whose bits
    are the uint32 codes."""
    import torch
    n = torch.arange(lo, hi, dtype=torch.int64, device=device)
    key = _signed(int(stream_key(seed, TRACE_STREAM)))
    gold = _signed(int(GOLDEN))
    base = n * N_FIELDS

    def raw(f):
        return _t_mix(key + (base + (f + 1)) * gold)

    def unif(f):
        return _t_shr(raw(f), 11).to(torch.float64) * (2.0 ** -53)

    def cat(u, probs):
        edges = torch.tensor(np.cumsum(np.asarray(probs, np.float64)), dtype=torch.float64,
                             device=device)
        edges[-1] = 1.0 + 1e-12
        return torch.searchsorted(edges, u, right=True)

    op = cat(unif(0), OP_PROBS)
    code = op.clone()
    for r in range(3):
        code |= _t_shr(raw(1 + r), 59) << (3 + 5 * r)
    code |= cat(unif(4), LEVEL_PROBS) << 18
    mis = (unif(5) < MISPREDICT_RATE) & (op == OP_BRANCH)
    code |= mis.to(torch.int64) << 20
    return code.to(torch.int32)


def trace_features(seed: int, n_instr: int, n_feat: int, lo: int = 0,
                   hi: Optional[int] = None) -> np.ndarray:
    return expand_codes(trace_codes(seed, n_instr, lo, hi), n_feat)


# ------------------------------------------------- instruction/data addresses ---

MEM_STREAM = 501
CODE_BASE, CODE_SPAN = 0x400000, 1 << 16      # 64 KB of code
HEAP_BASE, HEAP_SPAN = 0x10000000, 1 << 20    # 1 MB of data
TAKEN_RATE, DATA_JUMP_RATE = 0.5, 0.4
DEP_COLS = 42                                  # first of the 5 dependency-flag columns (D = 50)


def trace_mem(seed: int, n_instr: int) -> np.ndarray:
    """Program counter and data address of every instruction, uint32 [n][2]
    (data address 0 for instructions without a data access).

    PCs advance by 4 and jump to a uniform 4-aligned target in a 64 KB code
    region after a taken branch (half of the branches).  Loads and stores
    walk the 1 MB heap in 8-byte steps and jump on 40 % of accesses: half of
    the jumps go back to where the previous run started (reuse), the others
    to a uniform 8-aligned address."""
    op = trace_fields(seed, 0, n_instr)["op"]
    ctr = np.arange(n_instr, dtype=np.uint64) * np.uint64(4)
    u_take = uniform(seed, MEM_STREAM, ctr)
    u_tgt = u64(seed, MEM_STREAM, ctr + np.uint64(1))
    u_jump = uniform(seed, MEM_STREAM, ctr + np.uint64(2))
    u_addr = u64(seed, MEM_STREAM, ctr + np.uint64(3))
    idx = np.arange(n_instr, dtype=np.int64)
    # PC: segments start at 0 and after every taken branch
    taken = (op == OP_BRANCH) & (u_take < TAKEN_RATE)
    seg_start = np.zeros(n_instr, np.int64)
    seg_start[1:] = np.where(taken[:-1], idx[1:], 0)
    seg_start = np.maximum.accumulate(seg_start)
    target = CODE_BASE + ((u_tgt >> np.uint64(40)).astype(np.int64) % (CODE_SPAN // 4)) * 4
    target[0] = CODE_BASE
    pc = target[seg_start] + 4 * (idx - seg_start)
    pc = CODE_BASE + (pc - CODE_BASE) % CODE_SPAN
    # data addresses: over memory instructions only, runs of 8-byte steps
    mem = (op == OP_LOAD) | (op == OP_STORE)
    m_idx = np.nonzero(mem)[0]
    addr = np.zeros(n_instr, np.int64)
    if m_idx.size:
        k = np.arange(m_idx.size, dtype=np.int64)
        jump = u_jump[m_idx] < DATA_JUMP_RATE
        jump[0] = True
        run_start = np.maximum.accumulate(np.where(jump, k, 0))
        fresh = HEAP_BASE + ((u_addr[m_idx] >> np.uint64(40)).astype(np.int64) % (HEAP_SPAN // 8)) * 8
        # runs in order; a reusing run starts where the previous run started
        starts = np.nonzero(jump)[0]
        reuse = (u_addr[m_idx][starts] & np.uint64(1)).astype(bool)
        reuse[0] = False
        r = np.arange(starts.size)
        src = np.maximum.accumulate(np.where(reuse, 0, r))
        run_base = np.zeros(m_idx.size, np.int64)
        run_base[starts] = fresh[starts[src]]
        a = run_base[run_start] + 8 * (k - run_start)
        addr[m_idx] = HEAP_BASE + (a - HEAP_BASE) % HEAP_SPAN
    return np.stack([pc, addr], axis=1).astype(np.uint32)


def dynamic_columns(n_feat: int) -> Tuple[int, int, int]:
    """(residence, execution, store) column of each layout; -1 = absent."""
    return (30, 31, -1) if n_feat == 32 else (47, 48, 49)


# --------------------------------------------------------------- weights ---

@dataclass(frozen=True)
class Layer:
    kind: int      # 0 = conv (kernel 2, stride 2), 1 = fully connected,
    c_in: int      # 2 = pointwise conv (kernel 1), 3 = pointwise conv plus the
    c_out: int     #     input of the preceding pointwise layer (residual)
    relu: int


CONV, FC, PW, PWRES = 0, 1, 2, 3


def layer_param_shapes(layers: Sequence[Layer]) -> List[Tuple[Tuple[int, ...], Tuple[int]]]:
    """PyTorch parameter shapes: conv weight [co][ci][2], pointwise conv
    weight [co][ci][1], fc weight [out][in]."""
    out = []
    for ly in layers:
        if ly.kind == CONV:
            out.append(((ly.c_out, ly.c_in, 2), (ly.c_out,)))
        elif ly.kind in (PW, PWRES):
            out.append(((ly.c_out, ly.c_in, 1), (ly.c_out,)))
        else:
            out.append(((ly.c_out, ly.c_in), (ly.c_out,)))
    return out


WEIGHT_STREAM = 101
OUT_GAIN = 8.0
OUT_BIAS = (-6.0, 8.0)
RES_GAIN = 0.25  # residual branches start small, so seven blocks keep the scale


def init_weights(seed: int, layers: Sequence[Layer], out_bias: Optional[Sequence[float]] = OUT_BIAS,
                 out_gain: float = OUT_GAIN):
    """Random-init parameters, one SplitMix64 stream per tensor.

    Hidden layers: weights U(+-sqrt(6/fan_in)) (He et al. 2015 uniform, which
    keeps activation scale through ReLU), biases U(+-1/sqrt(fan_in)).
    The second half of a residual block (PWRES) scales its weight bound
    by RES_GAIN.  Output layer: weights U(+-out_gain/sqrt(fan_in)) and bias
    ``out_bias``
    (fetch, execution), chosen so that rounded latencies are spread out
    (fetch mostly 0-3, execution ~4-40 cycles) instead of all rounding to the
    bias.  Returns lists of float32 arrays in PyTorch layouts."""
    ws, bs = [], []
    last = len(layers) - 1
    for li, (ly, (wshape, bshape)) in enumerate(zip(layers, layer_param_shapes(layers))):
        fan_in = ly.c_in * (2 if ly.kind == CONV else 1)
        gain = out_gain if li == last else math.sqrt(6.0) * (RES_GAIN if ly.kind == PWRES else 1.0)
        wbound = gain / math.sqrt(fan_in)
        bbound = 1.0 / math.sqrt(fan_in)
        nw = int(np.prod(wshape))
        w = (2.0 * uniform(seed, WEIGHT_STREAM + 2 * li, np.arange(nw)) - 1.0) * wbound
        b = (2.0 * uniform(seed, WEIGHT_STREAM + 2 * li + 1, np.arange(bshape[0])) - 1.0) * bbound
        ws.append(w.astype(np.float32).reshape(wshape))
        bs.append(b.astype(np.float32))
    if out_bias is not None:
        bs[-1] = np.asarray(out_bias, dtype=np.float32).copy()
    return ws, bs


# ------------------------------------------------------ latency injection ---

LAT_STREAM = 201


def latency_table(seed: int, n_pred: int, n_out: int, f_max: int = 12, e_max: int = 48,
                  heavy: float = 0.0) -> np.ndarray:
    """Injected integer latencies [n_pred][n_out] (int32): fetch mostly 0-2,
    execution skewed towards small values; ``heavy`` is the probability of a
    long-latency outlier (drawn up to 8*e_max)."""
    idx = np.arange(n_pred * n_out, dtype=np.uint64)
    u = uniform(seed, LAT_STREAM, idx).reshape(n_pred, n_out)
    v = uniform(seed, LAT_STREAM + 1, idx).reshape(n_pred, n_out)
    t = np.zeros((n_pred, n_out), dtype=np.int64)
    f = _categorical(u[:, 0], (0.35, 0.45, 0.10, 0.10))
    f = np.where(f == 3, 3 + np.floor(v[:, 0] * (f_max - 2)).astype(np.int64), f)
    t[:, 0] = f
    for o in range(1, n_out):
        e = np.floor((u[:, o] ** 2) * (e_max + 1)).astype(np.int64)
        if heavy > 0:
            e = np.where(v[:, o] < heavy, np.floor(u[:, o] * 8 * e_max).astype(np.int64), e)
        t[:, o] = e
    return t.astype(np.int32)


# ------------------------------------------------------- training labels ---

# A small analytic pipeline model labels synthetic traces with fetch and
# execution latencies for the training form (the paper's labels come from a
# modified gem5, Sec. 2.4, which is not available).  It is a label source
# for training data, not part of the simulator.  Latencies by op class
# (int-ALU, load, store, branch, FP) and memory level (L1 5 and L2 29 cycles
# from the default O3CPU configuration table; DRAM 200 assumed).
EXEC_BASE = (1, 1, 1, 1, 4)
MEM_LATENCY = (5, 29, 200)
FETCH_WIDTH = 3
LABEL_MAX = 400


def analytic_latencies(fields: dict) -> np.ndarray:
    """(fetch, execution) latency per instruction, int32 [n][2], in [0, 400].

    Fetch: one cycle per group of FETCH_WIDTH instructions (the first of each
    group pays it), plus the execution latency of a mispredicted branch just
    before.  Execution: the instruction starts when its source registers
    (reg1, reg2) are ready and ends EXEC_BASE[op] (+ MEM_LATENCY[level] for
    loads and stores) cycles later; it is measured from its fetch; every
    instruction other than stores and branches writes reg0."""
    op = fields["op"]
    regs = fields["regs"]
    level = fields["level"]
    mis = fields["mispredict"]
    n = op.shape[0]
    out = np.zeros((n, 2), np.int32)
    done = np.zeros(32, np.int64)
    t_fetch = 0
    prev_mis_e = 0
    for i in range(n):
        f = (1 if i % FETCH_WIDTH == 0 else 0) + prev_mis_e
        f = min(f, LABEL_MAX)
        t_fetch += f
        o = int(op[i])
        start = max(t_fetch, int(done[regs[i, 1]]), int(done[regs[i, 2]]))
        lat = EXEC_BASE[o] + (MEM_LATENCY[int(level[i])] if o in (OP_LOAD, OP_STORE) else 0)
        end = start + lat
        e = min(end - t_fetch, LABEL_MAX)
        if o not in (OP_STORE, OP_BRANCH):
            done[regs[i, 0]] = end
        out[i, 0] = f
        out[i, 1] = e
        prev_mis_e = e if (o == OP_BRANCH and mis[i]) else 0
    return out


# -------------------------------------------------------- training batches ---

TRAIN_STREAM = 401


def training_batch(trace_seed: int, n_instr: int, n_feat: int, n_slot: int, B: int,
                   batch_seed: int):
    """Synthetic training contexts labelled by ``analytic_latencies``.

    Context b ends at trace row i_b (uniform in [n_slot, n_instr)) and holds
    occ_b (uniform in [0, n_slot)) older rows: slot 0 is row i_b with the
    dynamic columns zero, slot k the row i_b - k with residence = the fetch
    cycles from its fetch to i_b's and execution = its analytic execution
    latency; slots past occ_b are zero.  Labels are row i_b's (fetch,
    execution) latencies.  Returns x float32 [B][n_slot][n_feat] and labels
    int32 [B][2]."""
    fields = trace_fields(trace_seed, 0, n_instr)
    lab = analytic_latencies(fields)
    feat = trace_features(trace_seed, n_instr, n_feat)
    cres, cexe, _ = dynamic_columns(n_feat)
    ctr = np.arange(B, dtype=np.uint64) * np.uint64(2)
    rows = n_slot + (uniform(batch_seed, TRAIN_STREAM, ctr) * (n_instr - n_slot)).astype(np.int64)
    occ = (uniform(batch_seed, TRAIN_STREAM, ctr + np.uint64(1)) * n_slot).astype(np.int64)
    k = np.arange(n_slot)
    src = rows[:, None] - k[None, :]                       # [B][n_slot]
    live = k[None, :] <= occ[:, None]
    x = np.where(live[:, :, None], feat[np.maximum(src, 0)], 0.0).astype(np.float32)
    cum = np.concatenate([[0], np.cumsum(lab[:, 0].astype(np.int64))])
    res = cum[rows + 1][:, None] - cum[np.maximum(src, 0) + 1]
    x[:, :, cres] = np.where(live, res, 0)
    x[:, :, cexe] = np.where(live, lab[np.maximum(src, 0), 1], 0)
    x[:, 0, cres] = 0
    x[:, 0, cexe] = 0
    return x, lab[rows].astype(np.int32)


# ------------------------------------------------------------ sub-traces ---

LEN_STREAM = 301


def loguniform_lengths(seed: int, n_sub: int, lo: float, hi: float) -> np.ndarray:
    """round(exp(U(ln lo, ln hi))) per sub-trace (int64)."""
    u = uniform(seed, LEN_STREAM, np.arange(n_sub))
    return np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)


# --------------------------------------------------------------- configs ---

@dataclass
class Workload:
    name: str
    n_instr: int
    n_feat: int
    n_slot: int
    layers: List[Layer]
    n_sub: int = 1
    warmup: int = 0
    retire_width: int = 8
    lat_max: int = 65535
    n_out: int = 2
    trace_seed: int = 1
    weight_seed: int = 2
    length_seed: int = 3
    lengths: Optional[str] = None   # None = one trace split equally
    len_range: Tuple[float, float] = (1e3, 2e5)
    extra: dict = field(default_factory=dict)

    @property
    def cols(self) -> Tuple[int, int, int]:
        return dynamic_columns(self.n_feat)


def net_small() -> List[Layer]:
    """32 -> conv 32 -> conv 64 -> FC 2 over 16 slots."""
    return [Layer(CONV, 32, 32, 1), Layer(CONV, 32, 64, 1), Layer(FC, 256, 2, 0)]


def net_c3() -> List[Layer]:
    """50 -> conv 64 -> conv 128 -> conv 256 -> FC 512 -> FC 2 over 111 slots."""
    return [Layer(CONV, 50, 64, 1), Layer(CONV, 64, 128, 1), Layer(CONV, 128, 256, 1),
            Layer(FC, 256 * 13, 512, 1), Layer(FC, 512, 2, 0)]


HYB_CLASSES = 10  # hybrid inference head: classes for latencies 0..8 and "larger"


def net_c3_hybrid_infer() -> List[Layer]:
    """The C3 trunk with the paper's hybrid inference head: per latency type
    (fetch, execution) 10 class scores and one regression output, FC 512 ->
    22."""
    return net_c3()[:-1] + [Layer(FC, 512, 2 * (HYB_CLASSES + 1), 0)]


# Output bias of the hybrid inference head under random init: fetch leans to
# latencies 0 and 1, execution to the "larger" class whose regression output
# sits near 12 cycles.
HYB_BIAS = tuple([2.0, 1.0] + [0.0] * 8 + [2.0]) + tuple([0.0] * 9 + [2.0] + [12.0])


RB7_BLOCKS, RB7_EXPAND = 7, 1920


def net_rb7() -> List[Layer]:
    """RB7 with the hybrid head: the C3 convolutions (50 -> 64 -> 128 -> 256
    over 111 -> 55 -> 27 -> 13 positions), seven residual blocks at the 13
    positions (pointwise 256 -> 1920 with ReLU, pointwise 1920 -> 256, plus
    the block input, ReLU), FC 3328 -> 512 -> 2 x 11.  92,818,176
    multiply-adds per prediction."""
    blocks = []
    for _ in range(RB7_BLOCKS):
        blocks += [Layer(PW, 256, RB7_EXPAND, 1), Layer(PWRES, RB7_EXPAND, 256, 1)]
    return net_c3()[:3] + blocks + net_c3_hybrid_infer()[3:]


def net_c3_store() -> List[Layer]:
    """The C3 network with three outputs: fetch, execution and store latency."""
    return net_c3()[:-1] + [Layer(FC, 512, 3, 0)]


OUT_BIAS_STORE = (-6.0, 8.0, 20.0)  # fetch, execution, store
STORE_COL = 2                       # the store op class column of the feature layout


def net_c3_hybrid() -> List[Layer]:
    """The C3 trunk with the training head: per latency type 400 class
    logits and one regression output, FC 512 -> 2 x 401."""
    return net_c3()[:-1] + [Layer(FC, 512, 2 * 401, 0)]


def workload(name: str) -> Workload:
    if name == "tiny":        # 10k instructions, one sub-trace, 16 slots x 32 features
        return Workload("tiny", 10_000, 32, 16, net_small())
    if name == "c3_1m":       # 1M instructions, 4,096 sub-traces, 256 warm-up, 111 x 50
        return Workload("c3_1m", 1_000_000, 50, 111, net_c3(), n_sub=4096, warmup=256)
    if name == "c3dep_1m":    # c3_1m with the 5 memory-dependency flags in the window
        return Workload("c3dep_1m", 1_000_000, 50, 111, net_c3(), n_sub=4096, warmup=256,
                        extra={"dep_col": DEP_COLS})
    if name == "c3st_1m":     # c3_1m with store latencies and the memory write queue
        return Workload("c3st_1m", 1_000_000, 50, 111, net_c3_store(), n_sub=4096, warmup=256,
                        n_out=3, extra={"out_bias": OUT_BIAS_STORE, "store_col": STORE_COL})
    if name == "c3hyb_1m":    # c3_1m with the hybrid inference head
        return Workload("c3hyb_1m", 1_000_000, 50, 111, net_c3_hybrid_infer(), n_sub=4096,
                        warmup=256, extra={"out_bias": HYB_BIAS, "head": 1})
    if name == "rb7_1m":      # c3_1m with the RB7 network (seven residual blocks, hybrid head)
        return Workload("rb7_1m", 1_000_000, 50, 111, net_rb7(), n_sub=4096, warmup=256,
                        extra={"out_bias": HYB_BIAS, "head": 1})
    if name == "c3_train":    # 4,096 labelled contexts per step, hybrid head, BF16
        return Workload("c3_train", 200_000, 50, 111, net_c3_hybrid(), extra={"batch": 4096})
    if name == "c3_uneven":   # 20k independent streams, log-uniform lengths 1e3..2e5
        return Workload("c3_uneven", 0, 50, 111, net_c3(), n_sub=20_000, lengths="loguniform")
    raise KeyError(name)
