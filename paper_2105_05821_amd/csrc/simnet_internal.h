// Internal declarations shared by the HIP kernels and the C-ABI host code of
// libsimnet.so.  Not part of the public interface (include/simnet.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace simnet {

constexpr int MT = 16;       // sub-traces (windows) per workgroup tile: one MFMA row block
constexpr int WMAX = 16;     // largest supported retire width
constexpr int NCOUNTERS = 4; // clamped, non-finite, shadow mismatches, positions advanced

// Compile-time shape of a supported predictor.  A kernel-2 stride-2 stack is
// a tree: output position p of conv level l depends on input slots
// [p*2^(l+1), (p+1)*2^(l+1)) only, so the window is processed in independent
// blocks of BS = 2^NCONV slots, each producing one position of the last conv.
// Slots past NB*BS feed no output (floor lengths) and are never read.
struct NetSmall {  // [16 slots x 32 feat] -> conv 32 -> conv 64 -> FC 2
  static constexpr int D = 32, L = 16, C = 15;
  static constexpr int NCONV = 2, BS = 4, NB = 4;
  static constexpr int CH1 = 32, CH2 = 64, CH3 = 0;
  static constexpr int HID = 0, NOUT = 2;
  static constexpr int NLAT = 2, HEAD = 0;   // latencies per instruction; regression head
  static constexpr bool MWQ = false;         // store latency and memory write queue
  static constexpr int FC1_FRAGS = 8;
  static constexpr int FC1_DEPTH = 2;
  static constexpr int WAVES = 4;
  static constexpr bool LATE_COMMIT = false; // (no hidden FC)
  static constexpr int CHL = CH2;            // channels of the last conv
  static constexpr int NRES = 0, EXPAND = 0; // residual blocks after the convs
};
struct NetC3 {     // [111 slots x 50 feat] -> conv 64 -> conv 128 -> conv 256 -> FC 512 -> FC 2
  static constexpr int D = 50, L = 111, C = 110;
  static constexpr int NCONV = 3, BS = 8, NB = 13;
  static constexpr int CH1 = 64, CH2 = 128, CH3 = 256;
  static constexpr int HID = 512, NOUT = 2;
  static constexpr int NLAT = 2, HEAD = 0;
  static constexpr bool MWQ = false;
  static constexpr int FC1_FRAGS = 8;        // hidden-FC weight fragments per prefetch chunk
  static constexpr int FC1_DEPTH = 2;        // chunks in registers (DEPTH - 1 requested ahead)
  static constexpr int WAVES = 8;
  // the next group's window rows written after the hidden FC, their latency
  // passing under its weight stream (else before it, leaving the stream the
  // registers)
  static constexpr bool LATE_COMMIT = true;
  static constexpr int CHL = CH3;
  static constexpr int NRES = 0, EXPAND = 0;
};
// Hybrid inference head (Sec. 2.3): per latency type HYB_CLASSES class scores
// (latencies 0 .. HYB_CLASSES-2 and "larger") and one direct output.
constexpr int HYB_CLASSES = 10, HYB_PER_TYPE = HYB_CLASSES + 1;
struct NetC3Hyb : NetC3 {  // C3 trunk -> FC 512 -> 2 x 11
  static constexpr int NOUT = 2 * HYB_PER_TYPE, HEAD = 1;
};
// Tuning variants of the C3 step kernel (chosen by sim_autotune): a deeper
// or a shallower hidden-FC weight prefetch (chunks of 16 or 4 fragments, or
// 8-fragment chunks requested two ahead).  The products and their summation
// order are the same in every variant, so results are identical.
struct NetC3V1 : NetC3 {
  static constexpr int FC1_FRAGS = 16;
  static constexpr bool LATE_COMMIT = false;
};
struct NetC3V2 : NetC3 { static constexpr int FC1_FRAGS = 4; };
struct NetC3V3 : NetC3 {
  static constexpr int FC1_DEPTH = 3;
  static constexpr bool LATE_COMMIT = false;
};
constexpr int N_VARIANTS = 4;
// The small network's FP32 step as one wavefront per sub-trace slot
// (wave_step_kernel): the launch variant for runs of few sub-traces.
constexpr int WAVE_VARIANT = 1;
// ... or as four wavefronts per slot, one per block of its conv tree
// (quad_step_kernel).
constexpr int QUAD_VARIANT = 2;
// Store latency (Sec. 3.2): three outputs (fetch, execution, store) and the
// memory write queue that stores enter on leaving the processor queue.
struct NetC3S : NetC3 {  // C3 trunk -> FC 512 -> 3
  static constexpr int NOUT = 3, NLAT = 3;
  static constexpr bool MWQ = true;
};
// RB7 (Sec. 2.3, residual blocks; the model table's deepest CNN): the C3
// convolutions, then NRES residual blocks at the last conv's 13 positions,
// each y = ReLU(x + P ReLU(E x + e) + p) with E: 256 -> EXPAND and P:
// EXPAND -> 256 pointwise, then FC 3328 -> 512 and the hybrid head.  Runs
// as separate kernels per step: the convolutions inside the gather, the
// blocks over all windows' positions at once, FC 512 and the head.
struct NetRB7 : NetC3Hyb {
  static constexpr int NRES = 7, EXPAND = 1920;
};

// Contraction length covered by one 16-byte per-lane MFMA fragment group:
// FP32 16 (four 16x16x4), BF16 32 (one 16x16x32), FP8 64 (two 16x16x32).
constexpr int kgroup(int prec) { return prec == 0 ? 16 : prec == 1 ? 32 : 64; }
// Features per window slot as laid out for the kernels: D rounded up so
// that a slot pair (one conv1 row) is a whole number of fragment groups.
constexpr int padded_feat(int D, int prec) {
  return (D + kgroup(prec) / 2 - 1) / (kgroup(prec) / 2) * (kgroup(prec) / 2);
}

// Features per row of the BF16 copy of an FP32 trace that the BF16 form
// reads: D rounded up to whole 16-byte chunks.
constexpr int staged_feat(int D) { return (D + 7) / 8 * 8; }

// Weights re-laid-out for the kernels (device pointers, owned by the context).
// conv level l: B_l[k][n] with k = t*CH_l + c (t = pair member, c = input
// channel, zero for padded channels), packed per (k-group of KG, n-tile of
// 16) as 64 lanes x 16 bytes: lane holds B[kg*KG + (KG/4)*(lane/16) + e]
// [nt*16 + lane%16], e = 0 .. KG/4-1, in the storage type of the precision.
// Hidden FC (NetC3): one such packed matrix per block j with
// B_j[c][n] = W1[n][c*NB + j].  Final FC (VALU, float): wlast[j][o][c] =
// Wf[o][c*NB + j] when it follows the convs directly, else wlast[o][h] =
// W2[o][h]; values already rounded to the precision (FP8: dequantised, with
// the scale of its input folded in).
// FP8 only: *_ws = per-output-channel weight dequantisation scale, *_ai =
// per-channel reciprocal scale applied before an activation is stored as the
// next layer's FP8 input, x_inv = the same for the window features.
struct DevWeights {
  const void* conv_w[3];
  const float* conv_b[3];
  const float* conv_ws[3];
  const float* conv_ai[3];
  const float* x_inv;
  const void* hid_w;
  const float* hid_b;
  const float* hid_ws;
  const float* hid_ai;
  const float* last_w;
  const float* last_b;
  const void* last_p;  // hybrid head: the final FC packed like a hidden matrix
  // residual blocks (RB7): block i's expansion B[c][e] = E[e][c] (K = CH3,
  // N = EXPAND) then its projection B[e][c] = P[c][e] (K = EXPAND, N = CH3),
  // both packed for the form's residual MFMA tiles (BF16 32x32x16 with k-groups
  // of 16, FP32 16x16), at res_w + i * res_stride bytes; biases
  // res_b + i * (EXPAND + CH3): expansion's, then projection's
  const void* res_w;
  int64_t res_stride;
  const float* res_b;
};

struct DevState {
  // sub-trace table
  const int64_t* first;     // start - warm: trace row of position 0
  const int64_t* n_pos;     // warm + len
  const int32_t* warm;
  const int64_t* pred_off;  // sum_{k'<k}(warm+len)
  // per-sub-trace scalars
  int64_t* cur;
  int64_t* t_w;
  int64_t* r_prev;
  int64_t* pos;
  int32_t* head;
  int32_t* count;
  int64_t* rw;              // [K][WMAX] retire times of the last W pushes
  // processor queue ring [K][C]: the newest C instructions (q_e holds
  // E | S << 16 when store latencies are modelled)
  int32_t* q_idx;
  int32_t* q_e;
  int64_t* q_t;
  int64_t* q_r;
  // stores (store latencies only, else NULL): ring [K][C] of the newest C
  // stores with fetch tick, processor-queue exit r and memory-write-queue
  // exit x; the oldest m_count entries from m_head that have not left; the
  // newest m_inpq of them are still in the processor queue; x_prev = the
  // last store's x
  int32_t* m_idx;
  int32_t* m_es;
  int64_t* m_t;
  int64_t* m_r;
  int64_t* m_x;
  int32_t* m_head;
  int32_t* m_count;
  int32_t* m_inpq;
  int64_t* x_prev;
  // results
  int64_t* fetch;
  int64_t* drain;
  int64_t* final_tick;
  int64_t* warm_tick;
  unsigned long long* counters;
  // work queue
  int32_t* slot_kid;        // [n_wg * MT] sub-trace held by each slot, -1 = none
  const int32_t* order;     // claim order of the sub-traces (longest first)
  unsigned* next;           // claim counter
};

struct StepParams {
  const float* feat;        // dense rows [n_instr][D], or
  const uint16_t* feat16;   // (BF16 form) their BF16 copy [n_instr][staged_feat(D)], or
  const uint32_t* codes;    // packed instruction codes [n_instr] (one of the two)
  int32_t n_wg;             // persistent workgroups (slots = n_wg * MT)
  int32_t n_sub;
  int32_t W;
  int32_t col_res, col_exe, col_sto;
  int32_t store_col;        // store latencies: trace column flagging stores
  int32_t col_dep;          // first dependency-flag column, -1 = none
  const uint2* mem;         // [n_instr] (program counter, data address)
  int32_t lat_max;
  int32_t lat_mode;
  const int32_t* lat_table;
  float* logits_out;
  int32_t n_steps;
  unsigned* cal_out;  // calibration launches: per-channel max |input| (float bits)
  // staged step (RB7): the trunk stage writes each slot's last-conv output
  // [NB][CH3] (storage precision) to trunk_out + slot * NB * CH3 and the
  // slot's activity to active_out[slot]; the update stage reads the slot's
  // raw outputs from ext_logits + slot * NOUT
  void* trunk_out;
  int32_t* active_out;
  const float* ext_logits;
};

// Launchers (kernels.hip).  net: 0 = NetSmall, 1 = NetC3; prec: 0 FP32,
// 1 BF16, 2 FP8 (e4m3).  relu: bit l = ReLU after layer l.
// variant (0 .. N_VARIANTS-1) selects a tuning variant of the C3 network
// (net 1) when the predictor runs, or (net 0, FP32, WAVE_VARIANT) the small
// network's one-wavefront-per-slot step; other networks ignore it.
hipError_t launch_step(int net, int prec, int variant, const DevWeights& w, uint32_t relu,
                       const DevState& s,
                       const StepParams& p, hipStream_t stream);
// Private (scratch) bytes per lane of the C3 step kernel of `variant` with
// the predictor running, the kernels sim_autotune chooses among.
hipError_t c3_step_scratch(int prec, int variant, size_t* bytes);
hipError_t launch_forward(int net, int prec, const DevWeights& w, uint32_t relu, const float* x,
                          int64_t B, float* logits, hipStream_t stream);
// FP32 step launch that also records per-channel max |input| of every layer
// into p.cal_out (calibration_size(net) entries: window features, then each
// hidden layer's outputs in order).
hipError_t launch_calibrate(int net, const DevWeights& w, uint32_t relu, const DevState& s,
                            const StepParams& p, hipStream_t stream);
int calibration_size(int net);
hipError_t launch_reset(const DevState& s, int32_t n_sub, int32_t C, int32_t n_slots,
                        hipStream_t stream);
hipError_t launch_total(const DevState& s, int32_t n_sub, int64_t* total, hipStream_t stream);
// Training form (C3 trunk, hidden layer kept): activations saved by the
// forward for the backward pass, per window, channels-last, in the form's
// storage precision: a1 [52][64], a2 [26][128], a3 [13][256], h [512].
struct SaveBlock {
  void *a1, *a2, *a3, *h;
};
hipError_t launch_forward_save(int prec, const DevWeights& w, uint32_t relu, const float* x,
                               int64_t B, const SaveBlock& sb, hipStream_t stream);

// A GEMM operand: element (r, c) at p[(r / grp) * gs + (r % grp) * rs + c * cs]
// (grp splits the rows into groups with their own stride, e.g. the window
// rows of a batch of 111-slot windows), FP32 or BF16.
constexpr int64_t NO_GROUP = (int64_t)1 << 62;  // GemmOperand.grp of an ungrouped operand
// ext: elements readable along the outer dimension (m of A, n of B) when
// that dimension is the contiguous one (rows of a padded copy), 0 = the
// matrix's own M or N; the pipelined BF16 kernel reads whole 16-element runs
// up to it and keeps what lies past M or N out of the output.
struct GemmOperand {
  const void* p;
  int32_t bf16;
  int64_t rs, cs, grp, gs;
  int64_t ext;
};
// C[M][N] (+)= A(m, k) B(k, n) [+ bias[n]], then zeroed where mask(m, n) <= 0;
// C(m, n) at C + (m / cgrp) * cgs + (m % cgrp) * ldc + col(n), FP32, or
// (c_bf16) rounded to BF16 (nearest even) at the same element offsets of a
// uint16_t array (no accumulation then); col(n) = n, or with ccg > 0
// (n % ccg) * ccm + n / ccg (a weight gradient stored straight into a
// parameter layout whose input columns interleave).
struct GemmArgs {
  GemmOperand A, B, mask;
  float* C;
  int64_t ldc, cgrp, cgs;
  int64_t ccg, ccm;
  int64_t M, N, K;
  const float* bias;
  int32_t beta;
  int32_t c_bf16;
  // optional: the sums of A(m, k) over each k-split's range, rowsum[z][m]
  // (FP32, k in order), written by the pipelined BF16 kernel only
  float* rowsum;
  // set by launch_gemm
  int32_t ksplit, amode, avec, bmode, bvec, evec;
  float* part;
};
// bf16_mma: BF16 MFMA with operands rounded to BF16 (else FP32 MFMA).  part
// (part_cap floats, may be NULL) is scratch for split-K partial products.
// With g.rowsum set, *rowsum_parts receives the number of k-splits whose row
// sums were written there, or 0 if this launch's kernel writes none.
hipError_t launch_gemm(GemmArgs g, int bf16_mma, float* part, int64_t part_cap,
                       hipStream_t stream, int64_t* rowsum_parts = nullptr);
hipError_t launch_loss(const float* z, const int32_t* lat, int64_t B, int32_t n_bins,
                       float* loss_b, float* loss, float* dz, hipStream_t stream);
// at most this many chunk partials per column
constexpr int64_t COLSUM_MAX_CHUNKS = 1024;
constexpr size_t colsum_workspace_floats(int64_t N) { return (size_t)(COLSUM_MAX_CHUNKS * N); }
// Column sums of y [M][ld] (FP32, or BF16 with y_bf16) in two phases, each
// sum in a fixed order: launch_colsum_partial leaves *chunks partial sums
// [*chunks][N] in work (colsum_workspace_floats(N)); launch_sum_partials
// adds several such lists (cnt partials of N outputs at src) into their
// outputs (= or, with beta, +=) in one launch.
hipError_t launch_colsum_partial(const void* y, int y_bf16, int64_t M, int64_t N, int64_t ld,
                                 float* work, int64_t* chunks, hipStream_t stream);
struct SumSeg {
  const float* src;
  int64_t cnt, N;
  float* out;
  int32_t lanes;   // set by launch_sum_partials
  int64_t blocks;  // set by launch_sum_partials
};
struct SumSegs {
  static constexpr int MAX = 8;
  SumSeg seg[MAX];
  int32_t count;
  int32_t beta;
};
hipError_t launch_sum_partials(SumSegs segs, hipStream_t stream);
hipError_t launch_pad_rows(const float* src, int64_t rows, int64_t cols, int64_t ld, void* dst,
                           int32_t dst_bf16, hipStream_t stream);
// dst[i] = src[map[i]] (0 where map[i] < 0) for i < n, in FP32 or rounded
// to BF16, for up to MAX (map, n, dst) segments in one launch.
struct GatherSeg {
  const int32_t* map;
  int64_t n;
  void* dst;
  int32_t bf16;
};
struct GatherSegs {
  static constexpr int MAX = 10;
  GatherSeg seg[MAX];
  int32_t count;
};
hipError_t launch_map_gather_multi(const float* src, const GatherSegs& segs, hipStream_t stream);
hipError_t launch_zero(float* p, int64_t n, hipStream_t stream);
hipError_t launch_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, int32_t t, hipStream_t stream);
// Adam, then master[i] = w[i] and, for inv[i] = (packed byte offset, perm
// byte offset) >= 0, the copies in the form's precision.  With hid_packed
// set, the C3 hidden layer's weights (512 x 256 x 13 from hid_off) go
// through a tiled kernel instead, writing its packed copy at hid_packed and
// its permuted copy at hid_perm in whole runs.
hipError_t launch_adam_relayout(float* w, const float* g, float* m, float* v, int64_t n, float lr,
                                float b1, float b2, float eps, int32_t t, float* master,
                                const int2* inv, void* packed, void* perm, int32_t bf16,
                                int64_t hid_off, void* hid_packed, void* hid_perm,
                                hipStream_t stream);

// RB7, one step in three parts (n_steps = 1 each): stage 1 = gather and
// convolutions into p.trunk_out; then launch_resblocks and launch_rb_head
// on the slots' rows; stage 2 = round and update from p.ext_logits.
hipError_t launch_rb_stage(int prec, int stage, const DevWeights& w, uint32_t relu,
                           const DevState& s, const StepParams& p, hipStream_t stream);
// Residual blocks in place on x [rows][CH3] (storage precision); a tile of
// rows whose windows (row / NB) all have active[window] == 0 is skipped
// (active may be NULL: every row).
hipError_t launch_resblocks(int prec, const DevWeights& w, uint32_t relu, void* x, int64_t rows,
                            const int32_t* active, hipStream_t stream);
// FC 512 and the hybrid head on x [B][NB][CH3] -> logits [B][NOUT].
hipError_t launch_rb_head(int prec, const DevWeights& w, uint32_t relu, const void* x, int64_t B,
                          const int32_t* active, float* logits, hipStream_t stream);
// Convolutions of explicit windows x [B][L][D] (FP32) -> out [B][NB][CH3].
hipError_t launch_rb_trunk(int prec, const DevWeights& w, uint32_t relu, const float* x, int64_t B,
                           void* out, hipStream_t stream);

// BF16 copy of an FP32 trace [n][D] into out [n][staged_feat(D)].
hipError_t launch_stage_bf16(const float* feat, int64_t n, int D, uint16_t* out,
                             hipStream_t stream);

// Graph of the run: step kernel until every slot is empty, then the total.
hipError_t build_run_graph(int net, int prec, int variant, const DevWeights& w, uint32_t relu,
                           const DevState& s, const StepParams& p, int64_t* total,
                           hipGraph_t* out);

}  // namespace simnet
