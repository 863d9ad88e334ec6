/*
 * simnet.h - C ABI of libsimnet.so, an MI355X (gfx950) implementation of the
 * parallel simulation step loop of SimNet (Li et al., "SimNet: Accurate and
 * High-Performance Computer Architecture Simulation using Deep Learning").
 *
 * One step advances every active sub-trace by one instruction:
 *   1. build the instruction's model input from the trace and the sub-trace's
 *      processor queue (Sec. 2.2: the instruction plus its in-flight context
 *      instructions, each with residence and execution latency);
 *   2. run the CNN latency predictor on the whole batch (Sec. 2.3; batched
 *      across sub-traces as in Sec. 3.3);
 *   3. round the predicted latencies to cycles, advance the sub-trace's clock
 *      by the fetch latency, retire ready instructions in order at the retire
 *      width and enqueue the new one (Sec. 3.2, context and clock management).
 * The simulated time of a sub-trace is the sum of its fetch latencies plus
 * the drain after its last fetch (Sec. 3.1, Eq. 1); the total is the sum
 * over sub-traces (Sec. 3.3).
 *
 * Conventions
 *   - Every call returns a sim_status; no exception crosses the ABI.  The
 *     text of the last error of a context is available from sim_last_error.
 *   - Device pointers are HIP device memory of the current device; the
 *     caller owns every buffer it passes and the library never frees it.
 *     Host arrays are read during the call only.
 *   - All work is enqueued on config.stream (a hipStream_t; NULL = the
 *     legacy default stream).  sim_step and predictor_fwd are asynchronous;
 *     sim_run synchronises the stream before it returns.
 *   - A context is not thread-safe; separate contexts are independent.
 *   - Instruction counts and clock ticks are int64.
 */
#ifndef SIMNET_H
#define SIMNET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIMNET_API __attribute__((visibility("default")))

typedef struct sim_ctx sim_ctx; /* opaque, owned by the library */

typedef enum {
  SIM_OK = 0,
  SIM_EINVAL = -1,        /* an argument or a combination of them is invalid */
  SIM_ENOMEM = -2,        /* a device or host allocation failed */
  SIM_EDEVICE = -3,       /* a HIP call failed (message in sim_last_error) */
  SIM_ESTATE = -4,        /* call not valid in the context's current state */
  SIM_ENONFINITE = -5,    /* weights contain NaN or Inf */
  SIM_EUNSUPPORTED = -6   /* valid request with no kernel for it (network shape, precision) */
} sim_status;

typedef enum { SIM_FP32 = 0, SIM_BF16 = 1, SIM_FP8E4M3 = 2 } sim_precision;

/* Where the latencies that advance the clock come from.
 *   PREDICT: the predictor's own rounded outputs (the simulation proper).
 *   INJECT : lat_table; the predictor is not run.
 *   SHADOW : lat_table advances the state; the predictor still runs on the
 *            same windows and every prediction whose rounded value differs
 *            from the table is counted in n_shadow_mismatch. */
typedef enum { SIM_LAT_PREDICT = 0, SIM_LAT_INJECT = 1, SIM_LAT_SHADOW = 2 } sim_lat_mode;

/* Trace encodings.  F32: rows of n_feat float32.  CODE32: one uint32 per
 * instruction, expanded in the kernel into the categorical feature layout
 * op | reg0 << 3 | reg1 << 8 | reg2 << 13 | level << 18 | mispredict << 20
 * -> columns [0,5) op one-hot, [5,26) each register id (0..31) one-hot in
 * 7 buckets (id*7/32), [26,29) data level one-hot, [29] mispredict, the rest
 * zero (needs n_feat >= 30); 4 bytes per instruction instead of 4*n_feat. */
typedef enum { SIM_FEAT_F32 = 0, SIM_FEAT_CODE32 = 1 } sim_feat_dtype;

/* One predictor layer.  kind 0: 1-D convolution over instructions, kernel 2,
 * stride 2, no padding, output length floor(L/2) (Sec. 2.3: non-overlapping
 * kernel-2 convolutions; odd lengths drop the unpaired last slot);
 * kind 1: fully connected on the channel-major flattening (index c*L + p);
 * kind 2: pointwise (kernel 1) convolution, the length unchanged;
 * kind 3: pointwise convolution plus the input of the preceding kind-2
 * layer, added before the ReLU (a residual block, Sec. 2.3, is a kind-2
 * expansion followed by a kind-3 projection back to its input width).
 * relu != 0 applies ReLU after the layer. */
typedef struct {
  int32_t kind, c_in, c_out, relu;
} sim_layer;

typedef struct {
  int32_t n_feat;        /* D: features per instruction (window width) */
  int32_t n_slot;        /* L: window slots = 1 + context capacity C */
  int32_t n_out;         /* predicted latencies per instruction: 2 (fetch, execution),
                            or 3 (and store: stores then pass through the memory
                            write queue, Sec. 3.2; C3 window, FP32/BF16) */
  int32_t retire_width;  /* W: in-order retirements per cycle, 1..16 */
  int32_t col_res;       /* feature column receiving residence latency, -1 = none */
  int32_t col_exe;       /* feature column receiving execution latency, -1 = none */
  int32_t col_sto;       /* feature column receiving store latency (0 when n_out = 2), -1 = none */
  int32_t lat_max;       /* rounded latencies are clamped to [0, lat_max] */
  int32_t prec;          /* sim_precision of the predictor */
  int32_t store_col;     /* n_out = 3: trace feature column whose nonzero value marks
                            a store (packed codes: the expanded column; 2 is the
                            store op class); n_out = 3 also needs lat_max <= 65535.
                            Ignored when n_out = 2. */
  int32_t col_dep;       /* first of 5 consecutive feature columns receiving each
                            context instruction's memory dependency flags (Sec. 2.1):
                            same instruction cache line, same instruction page, same
                            data address, same data cache line, same data page as the
                            current instruction (64-byte lines, 4 KB pages; data flags
                            need both data addresses nonzero); 0 in slot 0 and empty
                            slots.  -1 = none; needs sim_trace.mem. */
  void* stream;          /* hipStream_t borrowed from the caller */
} sim_config;

/* The trace and its partition into sub-traces.  Sub-trace k simulates trace
 * rows [start[k] - warm[k], start[k] + len[k]) in order; the first warm[k]
 * are warm-up (predicted and queued, their fetch cycles not counted). */
typedef struct {
  const void* feat;      /* DEVICE, [n_instr][n_feat] float32 row-major (the
                            dynamic columns are ignored), or [n_instr] uint32
                            codes.  Borrowed: must stay valid and unchanged
                            for the context's lifetime. */
  int32_t feat_dtype;    /* sim_feat_dtype */
  int32_t n_sub;         /* number of sub-traces K >= 1; 0 with feat NULL makes a
                            predictor-only context (predictor_fwd/_bwd, no
                            simulation) */
  int64_t n_instr;       /* rows in feat, < 2^31 */
  const int64_t* start;  /* HOST [n_sub] */
  const int64_t* len;    /* HOST [n_sub], each >= 1 */
  const int32_t* warm;   /* HOST [n_sub], each >= 0 and <= start[k] */
  const void* mem;       /* DEVICE uint32 [n_instr][2]: program counter and data
                            address (0 = no data access) of every instruction, for
                            the dependency flags; NULL when col_dep = -1.
                            Borrowed like feat. */
} sim_trace;

/* Results of sim_run.  Scalars are always written; each per-sub-trace array
 * is a HOST buffer of n_sub int64 owned by the caller, or NULL to skip. */
typedef struct {
  int64_t total_cycles;      /* sum over k of (final_tick[k] - warm_tick[k]) */
  int64_t measured_instr;    /* sum of len */
  int64_t predicted_instr;   /* sum of warm + len */
  int64_t n_clamped;         /* rounded predictions outside [0, lat_max] */
  int64_t n_nonfinite;       /* non-finite predictions (used as 0) */
  int64_t n_shadow_mismatch; /* SHADOW mode: rounded prediction != table */
  int64_t* fetch_cycles;     /* T_last - T_warm: sum of counted fetch latencies */
  int64_t* drain_cycles;     /* final - T_last: Eq. 1's drain */
  int64_t* final_tick;       /* curTick when the queue has emptied */
  int64_t* warm_tick;        /* curTick after the last warm-up instruction (0 if none) */
} sim_result;

/* Pure host check of a configuration and trace description; touches no
 * device memory (feat is only checked for non-NULL).  SIM_OK or SIM_EINVAL. */
SIMNET_API int sim_validate_config(const sim_config* cfg, const sim_trace* trace);

/* Partition of a trace for parallel simulation (Sec. 3.3, parallel
 * simulation: the trace is split into sub-traces simulated independently,
 * each after a warm-up over the instructions that precede it).  Pure host,
 * no device use.  Writes n_sub entries of each HOST array, caller-owned:
 * sub-trace k covers trace rows [start[k], start[k] + len[k]); the rows are
 * cut into equal contiguous pieces, the first n_instr mod n_sub one
 * instruction longer; warm[k] = min(warm_max, start[k]) instructions before
 * start[k] are simulated as warm-up.  SIM_EINVAL unless
 * 1 <= n_sub <= n_instr, warm_max >= 0 and every pointer is non-NULL
 * (nothing is written then). */
SIMNET_API int sim_partition(int64_t n_instr, int32_t n_sub, int32_t warm_max, int64_t* start,
                             int64_t* len, int32_t* warm);

/* Create a context (Sec. 3.3: the partitioned trace and each sub-trace's
 * simulation state, processor queue and clock of Sec. 3.2, stay on the
 * device for the whole run): validates, copies the sub-trace table to the device and
 * allocates the per-sub-trace state (processor queue of n_slot-1 entries,
 * clock, retire history).  *out is NULL on failure. */
SIMNET_API int sim_init(const sim_config* cfg, const sim_trace* trace, sim_ctx** out);

/* Load predictor parameters.  params is the concatenation, layer by layer,
 * of weight then bias in PyTorch layouts (conv [c_out][c_in][2], pointwise
 * conv [c_out][c_in][1], fc [out][in]), float32, on the device if
 * on_device != 0 else on the host.
 * The parameters are copied (and re-laid-out for the kernels), so the
 * caller may free them afterwards.  The layer list must map the window
 * [n_slot][n_feat] to n_out outputs (regression head: each output, rounded,
 * is a latency), or, for the 111x50 C3 network, to 22 outputs: the hybrid
 * head of Sec. 2.3, per latency type 10 class scores (latencies 0..8 and
 * "larger than 8") then one direct output; the latency is the most probable
 * class (the first of equal scores), or the rounded direct output when the
 * "larger" class wins (FP32 and BF16 forms).  RB7 (the model table's
 * residual network, FP32 and BF16 forms): the three C3 convolutions, seven
 * residual blocks (kind 2: 256 -> 1920 with ReLU, kind 3: 1920 -> 256 with
 * ReLU), fc 3328 -> 512 (ReLU), fc 512 -> 22 (the hybrid head); its steps
 * run as four launches each (sim_step stays asynchronous; sim_run checks
 * progress between batches of steps, and with a graph requested still runs
 * them eagerly).  SIM_EUNSUPPORTED if no kernel exists for the shape,
 * SIM_ENONFINITE on NaN/Inf.  Resets the simulation state. */
SIMNET_API int sim_load_weights(sim_ctx* ctx, const sim_layer* layers, int32_t n_layers,
                     const float* params, int32_t on_device);

/* Advance the simulation by up to n_steps steps (asynchronous).  One step
 * is one iteration of the parallel simulation loop of Sec. 3.3 over every
 * sub-trace in a slot: the model input of its next instruction (Sec. 2.2),
 * the predictor (Sec. 2.3), then the clock and queue update of Sec. 3.2
 * (fetch latency advances the clock; in-flight instructions leave in order,
 * at most retire_width per cycle, once their residence exceeds their
 * execution latency).  The
 * library runs a fixed number of sub-trace slots (a multiple of 16, at most
 * a few per compute unit); a slot whose sub-trace finishes takes the next
 * unstarted one, longest first, so with more sub-traces than slots one step
 * advances only the sub-traces currently in slots.  Results do not depend on
 * the slot assignment.  lat_table (DEVICE int32, needed for INJECT and SHADOW) is
 * indexed by the sub-trace's simulated position: row
 * sum_{k'<k}(warm[k']+len[k']) + p, column o (0 fetch, 1 execution). */
SIMNET_API int sim_step(sim_ctx* ctx, int32_t n_steps, int32_t lat_mode, const int32_t* lat_table);

/* Run every sub-trace to completion (one launch that ends when every slot
 * is empty), synchronise, and fill *res: per sub-trace the fetch cycles and
 * the drain after the last fetch (Sec. 3.1, Eq. 1), and their sum over the
 * sub-traces as the simulated time of the whole trace (Sec. 3.3).  A context
 * that has completed must be sim_reset before it runs again. */
SIMNET_API int sim_run(sim_ctx* ctx, int32_t lat_mode, const int32_t* lat_table, sim_result* res);

/* enable != 0: sim_run replays a graph of its kernels (the persistent step
 * kernel run until every slot is empty, then the reduction of the total),
 * instantiated on first use and rebuilt when lat_mode, lat_table, the
 * logits buffer or the weights change.  The graph holds kernel nodes only. */
SIMNET_API int sim_set_graph(sim_ctx* ctx, int32_t enable);

/* Launch shape of the step kernel as chosen by sim_autotune. */
typedef struct {
  int32_t variant;            /* kernel variant: C3 network, the hidden-FC weight
                                 prefetch depth (0, 1, 2: chunks of 8, 16, 4 fragments
                                 requested one chunk ahead; 3: chunks of 8 fragments
                                 requested two ahead); small
                                 network in FP32, 0 = a workgroup per 16 slots, 1 = one
                                 wavefront per slot, 2 = four wavefronts per slot (one
                                 per block of the conv tree) */
  int32_t n_wg;               /* persistent workgroups (16 sub-trace slots each) */
  float ms;                   /* its time per million positions advanced in the trial */
  int32_t n_tried;            /* candidates timed (at most 16 listed) */
  int32_t tried_variant[16], tried_n_wg[16];
  float tried_ms[16];
} sim_tuning;

/* Time n_steps steps (lat_mode/lat_table as in sim_step) from the reset
 * state under each candidate launch shape: every kernel variant (the C3
 * network with the predictor running, or the small network in FP32) x 4/4,
 * 3/4 and 1/2 of the slots sim_init allocated; keep the one with the least
 * time per position advanced and reset the simulation.  The C3 variants
 * differ only in how far ahead weights are fetched, so results do not
 * depend on the choice; the small network's three sum the same products in
 * different orders (all within the FP32 bar of the FP64 oracle).  The small
 * network's FP32 step starts as four wavefronts per slot when the trace has
 * at most 1,024 sub-traces.  C3 variants whose kernel needs scratch memory
 * (register spills, see sim_variant_scratch) are left out when another
 * variant needs none.  Synchronises.  *out receives the choice and the
 * trials. */
SIMNET_API int sim_autotune(sim_ctx* ctx, int32_t n_steps, int32_t lat_mode,
                            const int32_t* lat_table, sim_tuning* out);

/* Private (scratch) memory per lane, in bytes, that the C3 network's step
 * kernel of `variant` (in [0, 4), predictor running) uses in this context's
 * precision form: nonzero means the compiler spilled registers to memory.
 * SIM_EUNSUPPORTED for other networks. */
SIMNET_API int sim_variant_scratch(sim_ctx* ctx, int32_t variant, int64_t* bytes);

/* Apply a launch shape (a cached sim_autotune result): variant in [0, 4),
 * n_wg in [1, slots allocated / 16].  Resets the simulation. */
SIMNET_API int sim_set_tuning(sim_ctx* ctx, int32_t variant, int32_t n_wg);

/* Return every sub-trace to its first instruction (asynchronous). */
SIMNET_API int sim_reset(sim_ctx* ctx);

/* Record every prediction's raw float32 outputs into a DEVICE buffer of
 * [sum(warm+len)][network outputs] float32 (n_out, or 22 for the hybrid
 * head), in prediction order like lat_table (NULL stops recording).  Used
 * for parity checks on identical windows. */
SIMNET_API int sim_record_logits(sim_ctx* ctx, float* logits);

/* Calibrate the FP8 form (also allowed for FP32 contexts, to read the
 * scales): run n_steps steps of every sub-trace with the FP32 predictor
 * (lat_mode/lat_table as in sim_step), take each layer input channel's
 * largest magnitude (window features, then every hidden layer's outputs in
 * order), set that channel's scale to the smallest power of two s with
 * max <= 448 s, and (FP8) build the e4m3 weights: each weight is multiplied
 * by its input channel's scale and then gets a power-of-two scale per output
 * channel on the same rule.  Synchronises; resets the simulation state.
 * FP8 contexts return SIM_ESTATE from sim_step, sim_run and predictor_fwd
 * until calibrated.  SIM_EUNSUPPORTED for BF16 contexts. */
SIMNET_API int sim_calibrate(sim_ctx* ctx, int32_t n_steps, int32_t lat_mode,
                             const int32_t* lat_table);

/* Copy the calibrated per-channel activation scales (HOST out, at least n
 * floats: n_feat + the width of every hidden layer).  SIM_ESTATE before
 * calibration, SIM_EINVAL if n is too small. */
SIMNET_API int sim_act_scales(const sim_ctx* ctx, float* out, int32_t n);

/* Predictor forward on explicit windows (Sec. 2.3): x is DEVICE
 * [B][n_slot][n_feat] float32, logits DEVICE [B][network outputs] float32
 * (n_out = 2 for the regression head, 22 for the hybrid head and RB7).
 * RB7 uses a workspace of B * 13 * 256 elements of the form, kept by the
 * context and grown as needed.  save_or_null must be NULL except for the
 * training head, where it is required.
 *
 * Training head (Sec. 2.3's hybrid output, Sec. 4's training set-up): a
 * 111x50 context loaded with the layer list conv 50->64, conv 64->128,
 * conv 128->256 (ReLU each), fc 3328->512 (ReLU), fc 512->802 (no ReLU).
 * The 802 logits of a window are, per latency o in (fetch, execution), 400
 * class logits at [o*401, o*401+400) and one regression output at o*401+400.
 * FP32 and BF16 forms (BF16: the window, the weights and every hidden
 * activation are rounded to BF16, products accumulate in FP32).  For this
 * head sim_load_weights keeps the parameters on the device and does not
 * check them for NaN/Inf.  save is a
 * DEVICE buffer of predictor_save_bytes(ctx, B) bytes that receives the
 * activations the backward pass needs. */
SIMNET_API int predictor_fwd(sim_ctx* ctx, const void* x, int64_t B, float* logits, void* save_or_null);

/* Bytes of the save buffer predictor_fwd/predictor_bwd need for B windows
 * (training head only; -1 otherwise). */
SIMNET_API int64_t predictor_save_bytes(const sim_ctx* ctx, int64_t B);

/* Hybrid loss of the training head (Sec. 2.3, Sec. 4): for each window b and
 * latency o (fetch, execution) with integer label y = labels[b][o] >= 0
 * (DEVICE int32 [B][2]): cross-entropy over the 400 class logits with target
 * class min(y, 399) (the last class collects every latency >= 399), plus
 * |r - log(1 + y)| on the regression output r.  *loss (DEVICE, one float)
 * receives the mean over windows of the sum of the four terms; dlogits
 * (DEVICE [B][802]) its gradient (sign(0) = 0 for the L1 term). */
SIMNET_API int sim_loss(sim_ctx* ctx, const float* logits, const int32_t* labels, int64_t B,
                        float* loss, float* dlogits);

/* Largest batch of sim_loss_noalloc. */
#define SIM_NOALLOC_MAX_B 65536

/* sim_loss for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving or training loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results, bit for bit, but
 * the per-window losses go to a static device buffer of SIM_NOALLOC_MAX_B
 * floats (256 KB per GPU, held until the process ends) instead of the
 * context's workspace, and nothing is allocated or freed.  Every call on a
 * GPU shares that GPU's buffer: calls that overlap on one GPU (other
 * streams, other contexts, other threads) race and must be ordered by the
 * caller.  Nothing in it needs clearing between calls (each call writes the
 * B entries it reads).  SIM_EINVAL when B > SIM_NOALLOC_MAX_B. */
SIMNET_API int sim_loss_noalloc(sim_ctx* ctx, const float* logits, const int32_t* labels,
                                int64_t B, float* loss, float* dlogits);

/* Backward of predictor_fwd (training head; the predictor of Sec. 2.3 trained
 * on the hybrid loss as Sec. 4 sets up), the chain rule through the
 * head, the hidden layer, the three convolutions and their ReLUs: x and save
 * as passed to the forward, dlogits DEVICE [B][802].  dparams (DEVICE,
 * float32) has the layout of sim_load_weights's params and receives the
 * parameter gradients (accumulate != 0 adds to what it holds).  dx (DEVICE
 * [B][111][50] float32, or NULL) receives the gradient with respect to the
 * window, zero in the slots no output depends on.  Gradients are computed
 * with the current parameters, in FP32 (BF16 form: from the BF16 saved
 * activations). */
SIMNET_API int predictor_bwd(sim_ctx* ctx, const void* x, const void* save, const float* dlogits,
                             int64_t B, float* dx, float* dparams, int32_t accumulate);

/* One Adam step (Sec. 2.4 trains the predictor with Adam, without weight
 * decay; Kingma and Ba's bias-corrected update) on n DEVICE float32
 * parameters, in place, with moments m and v (DEVICE, n floats each, zero
 * before step 1); step counts from 1.  To train a context's predictor: keep
 * the master parameters in a device buffer, update them here, then
 * sim_load_weights(..., on_device = 1) to re-lay them out for the kernels
 * (sim_adam_load does both in one launch, with the same results). */
SIMNET_API int sim_adam(sim_ctx* ctx, float* params, const float* grads, float* m, float* v,
                        int64_t n, float lr, float beta1, float beta2, float eps, int32_t step);

/* sim_adam (Sec. 2.4) on the n = all parameters of a training context's
 * predictor, after which the context's weights are the updated parameters,
 * exactly as
 * after sim_load_weights(..., params, on_device = 1) with the layers it was
 * loaded with, in one launch: each updated weight is also written to the
 * context's master copy and, in the form's precision, to its places in the
 * kernels' re-laid-out copies (no copy, no gather).  Needs weights loaded;
 * n must equal the network's parameter count (SIM_EINVAL otherwise).
 * Asynchronous on the context's stream. */
SIMNET_API int sim_adam_load(sim_ctx* ctx, float* params, const float* grads, float* m,
                             float* v, int64_t n, float lr, float beta1, float beta2, float eps,
                             int32_t step);

SIMNET_API void sim_destroy(sim_ctx* ctx);
SIMNET_API const char* sim_last_error(const sim_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* SIMNET_H */
