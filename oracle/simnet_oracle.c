/*
 * SimNet oracle: a plain, slow, FP64 / exact-int64 CPU reference of the
 * parallel simulation step loop (Li et al., "SimNet: Accurate and
 * High-Performance Computer Architecture Simulation using Deep Learning").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the HIP
 * library.
 *
 * What it follows:
 *   - Sec. 2.2 (model input): each in-flight context instruction contributes
 *     its features plus its residence and execution latency; the instruction
 *     to be predicted carries zeros in those columns.
 *   - Sec. 2.3 (CNN): instructions along one axis, features as channels;
 *     every convolution has kernel 2 and stride 2 with no overlap; ReLU after
 *     each convolution and after the hidden fully connected layer; the last
 *     convolution output is flattened (PyTorch channel-major order) into two
 *     fully connected layers.  Outputs are (fetch, execution) latency.
 *   - Sec. 3.1, Eq. 1: program time = sum of fetch latencies + drain.
 *   - Sec. 3.2 (context and clock management): processor queue is a FIFO;
 *     a fetch latency F > 0 advances curTick by F and ages every queued
 *     instruction; an instruction is ready to retire once its residence
 *     exceeds its execution latency; retirement is in order and limited to
 *     the retire width per cycle; after the last instruction the clock keeps
 *     running until the queue is empty.  This file runs that rule literally,
 *     one cycle at a time.
 *   - Sec. 3.3 (parallel simulation): the trace is cut into equal contiguous
 *     sub-traces that are simulated independently; the total is the sum of
 *     their clocks.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   ready means residence strictly greater than execution latency; the
 *   context snapshot for instruction i is the queue after instruction i-1 was
 *   pushed; at most W retirements per cycle, greedy from the head, none
 *   during a zero fetch latency; slot k >= 1 holds the k-th newest queued
 *   instruction and only the newest n_slot-1 are shown; odd lengths follow
 *   PyTorch Conv1d (floor, the unpaired last slot dropped); rounding is to
 *   nearest, ties to even, clamped to [0, lat_max], non-finite -> 0;
 *   sub-trace k additionally simulates the warm[k] instructions before its
 *   start, whose fetch cycles are excluded from its count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* Layer kinds: kernel-2 stride-2 convolution, fully connected, and the two
 * halves of a residual block (Sec. 2.3 names residual blocks as the
 * alternative to plain convolution layers; RB7 stacks seven): a pointwise
 * (kernel 1) convolution, and a pointwise convolution whose output has the
 * input of the preceding pointwise layer added before its activation. */
enum { OL_CONV = 0, OL_FC = 1, OL_PW = 2, OL_PWRES = 3 };
enum { OL_MAXL = 32 };
enum { OL_PREDICT = 0, OL_INJECT = 1 };

/* cfg[] layout shared with the Python wrapper */
enum { CF_NFEAT = 0, CF_NSLOT, CF_NOUT, CF_W, CF_COLRES, CF_COLEXE, CF_COLSTO, CF_LATMAX, CF_HEAD,
       CF_STCOL, CF_COLDEP, CF_LEN };
/* CF_COLDEP: first of 5 consecutive window columns receiving the memory
 * dependency flags of each context instruction (-1 = none). */
enum { LINE_SHIFT = 6, PAGE_SHIFT = 12 }; /* 64-byte cache lines, 4 KB pages */
/* CF_STCOL: with n_out = 3 (fetch, execution, store latencies), the trace
 * column whose nonzero value marks a store instruction. */
/* CF_HEAD: 0 = regression head (one output per latency type, rounded);
 * 1 = hybrid head (Sec. 2.3): per latency type HYB_CLASSES class scores for
 * latencies 0 .. HYB_CLASSES-2 and "larger", then one regression output. */
enum { HYB_CLASSES = 10, HYB_PER_TYPE = HYB_CLASSES + 1 };

typedef struct {
  int n_layers;
  int32_t desc[OL_MAXL][4]; /* kind, c_in, c_out, relu */
  double* w[OL_MAXL];
  double* b[OL_MAXL];
  int n_feat, n_slot, n_out, max_width;
  int prec;                 /* 0: plain FP64; 1: BF16 form; 2: FP8 form */
  double* in_scale[OL_MAXL + 1];     /* FP8 form: scale of each input channel of layer l */
} ol_model;

/* Nearest bfloat16 value (8 significant bits, ties to even), from the
 * definition: v = m * 2^ex with 0.5 <= |m| < 1, so one unit in the last
 * place is 2^(ex - 8).  Range limits are not reached by the workloads. */
static double round_bf16(double v) {
  if (v == 0.0 || !isfinite(v)) return v;
  int ex;
  frexp(v, &ex);
  const double ulp = ldexp(1.0, ex - 8);
  return nearbyint(v / ulp) * ulp;
}

/* Nearest OCP e4m3 value (1 sign, 4 exponent bits with bias 7, 3 mantissa
 * bits; largest finite 448; subnormal spacing 2^-9), ties to even,
 * saturating: v = m * 2^ex with 0.5 <= |m| < 1 lies in a binade whose
 * spacing is 2^(ex - 4), never below the subnormal spacing 2^-9. */
static double round_e4m3(double v) {
  if (v > 448.0) v = 448.0;
  if (v < -448.0) v = -448.0;
  if (v == 0.0) return v;
  int ex;
  frexp(v, &ex);
  if (ex < -5) ex = -5;
  const double ulp = ldexp(1.0, ex - 4);
  double r = nearbyint(v / ulp) * ulp;
  if (r > 448.0) r = 448.0;
  if (r < -448.0) r = -448.0;
  return r;
}

/* Smallest power of two s with amax <= 448 * s; 1 when amax is 0. */
static double pow2_scale(double amax) {
  if (!(amax > 0.0)) return 1.0;
  int ex;
  const double f = frexp(amax / 448.0, &ex); /* amax/448 = f * 2^ex */
  double s = (f == 0.5) ? ldexp(1.0, ex - 1) : ldexp(1.0, ex);
  while (amax > 448.0 * s) s *= 2.0;        /* guard the division's rounding */
  while (s > 1e-300 && amax <= 448.0 * (s / 2.0)) s /= 2.0;
  return s;
}

/* Rounding of an input value of layer li, channel c, to the form. */
static double qin(const ol_model* m, int li, int c, double v) {
  if (m->prec == 1) return round_bf16(v);
  if (m->prec == 2) {
    const double s = m->in_scale[li][c];
    return round_e4m3(v / s) * s;
  }
  return v;
}

static double qform(const ol_model* m, double v) { return m->prec == 1 ? round_bf16(v) : v; }

/* ------------------------------------------------------------- model --- */

/* params: PyTorch order, concatenated: w0, b0, w1, b1, ...  conv weight is
 * [c_out][c_in][2], fc weight is [out][in]. */
/* prec 1 evaluates the BF16 form of the network: window inputs, weights
 * and every hidden layer's output (after bias and ReLU) are rounded to
 * bfloat16, biases stay as given, products and sums are exact FP64 and the
 * last layer's output is not rounded. */
void* ol_model_new_prec(int n_layers, const int32_t* desc, const float* params,
                        int n_feat, int n_slot, int prec) {
  if (n_layers < 1 || n_layers > OL_MAXL || prec < 0 || prec > 1) return NULL;
  ol_model* m = (ol_model*)calloc(1, sizeof(ol_model));
  m->prec = prec;
  m->n_layers = n_layers;
  m->n_feat = n_feat;
  m->n_slot = n_slot;
  int ch = n_feat, len = n_slot, width = n_feat * n_slot;
  size_t off = 0;
  for (int l = 0; l < n_layers; ++l) {
    for (int j = 0; j < 4; ++j) m->desc[l][j] = desc[4 * l + j];
    int kind = desc[4 * l], ci = desc[4 * l + 1], co = desc[4 * l + 2];
    size_t nw;
    if (kind == OL_CONV) {
      if (ci != ch || len < 2) { free(m); return NULL; }
      nw = (size_t)co * ci * 2;
      len = len / 2;
    } else if (kind == OL_PW || kind == OL_PWRES) {
      /* the residual half adds the preceding pointwise layer's input, so
       * it must follow one and give back that layer's input channels */
      const int ok = ci == ch && (kind == OL_PW || (l > 0 && desc[4 * (l - 1)] == OL_PW &&
                                                    co == desc[4 * (l - 1) + 1]));
      if (!ok) {
        for (int j = 0; j < l; ++j) { free(m->w[j]); free(m->b[j]); }
        free(m);
        return NULL;
      }
      nw = (size_t)co * ci;
    } else {
      if (ci != ch * len) { free(m); return NULL; }
      nw = (size_t)co * ci;
      len = 1;
    }
    ch = co;
    if (ch * len > width) width = ch * len;
    m->w[l] = (double*)malloc(nw * sizeof(double));
    m->b[l] = (double*)malloc((size_t)co * sizeof(double));
    for (size_t i = 0; i < nw; ++i) m->w[l][i] = qform(m, (double)params[off + i]);
    off += nw;
    for (int i = 0; i < co; ++i) m->b[l][i] = (double)params[off + i];
    off += co;
  }
  if (len != 1) { /* the network must end in a fully connected layer */
    for (int l = 0; l < n_layers; ++l) { free(m->w[l]); free(m->b[l]); }
    free(m);
    return NULL;
  }
  m->n_out = ch;
  /* scratch: the layer output, then the residual block's saved input */
  m->max_width = 2 * width;
  return m;
}

void* ol_model_new(int n_layers, const int32_t* desc, const float* params,
                   int n_feat, int n_slot) {
  return ol_model_new_prec(n_layers, desc, params, n_feat, n_slot, 0);
}

/* The FP8 form: scales holds, layer by layer, one power-of-two scale per
 * input channel of that layer (the window's features first).  An input x of
 * channel c is used as e4m3(x / s_c) * s_c.  Each weight is multiplied by its
 * input channel's scale and each output channel n gets the power-of-two
 * scale w_n for its largest such magnitude; the weight used is
 * e4m3(W s_c / w_n) * w_n / s_c.  Biases as given, sums exact. */
void* ol_model_new_fp8(int n_layers, const int32_t* desc, const float* params,
                       int n_feat, int n_slot, const float* scales) {
  for (int l = 0; l < n_layers; ++l)
    if (desc[4 * l] != OL_CONV && desc[4 * l] != OL_FC) return NULL; /* no FP8 residual form */
  ol_model* m = (ol_model*)ol_model_new_prec(n_layers, desc, params, n_feat, n_slot, 0);
  if (!m) return NULL;
  m->prec = 2;
  int ch = n_feat, len = n_slot;
  size_t off = 0;
  for (int l = 0; l < n_layers; ++l) {
    m->in_scale[l] = (double*)malloc(sizeof(double) * (size_t)ch);
    for (int c = 0; c < ch; ++c) m->in_scale[l][c] = (double)scales[off + c];
    off += (size_t)ch;
    const int kind = m->desc[l][0], ci = m->desc[l][1], co = m->desc[l][2];
    const int n_in = kind == OL_CONV ? ci * 2 : ci;
    /* input channel of weight element k of an output's row */
    for (int o = 0; o < co; ++o) {
      double* row = m->w[l] + (size_t)o * n_in;
      double amax = 0.0;
      for (int k = 0; k < n_in; ++k) {
        const int c = kind == OL_CONV ? k / 2 : k / len;
        const double a = fabs(row[k] * m->in_scale[l][c]);
        if (a > amax) amax = a;
      }
      const double ws = pow2_scale(amax);
      for (int k = 0; k < n_in; ++k) {
        const int c = kind == OL_CONV ? k / 2 : k / len;
        const double sc = m->in_scale[l][c];
        row[k] = round_e4m3(row[k] * sc / ws) * ws / sc;
      }
    }
    ch = co;
    len = kind == OL_CONV ? len / 2 : 1;
  }
  return m;
}

void ol_model_free(void* p) {
  ol_model* m = (ol_model*)p;
  if (!m) return;
  for (int l = 0; l < m->n_layers; ++l) { free(m->w[l]); free(m->b[l]); free(m->in_scale[l]); }
  free(m);
}

int ol_model_nout(const void* p) { return ((const ol_model*)p)->n_out; }

/* Forward pass of one window x[n_slot][n_feat] by the layer definitions
 * (Sec. 2.3).  a/t are scratch of at least max_width doubles.
 * Activations are kept channel-major: act[c * len + pos].
 * If scale is not NULL it receives, per output, |b| + sum_j |w_j * a_j| of
 * the last layer: the magnitude against which the rounding error of any
 * finite-precision evaluation of that output is measured. */
static void forward_cal(const ol_model* m, const double* x, double* out, double* a, double* t,
                        double* scale, double* amax);
static void forward_one(const ol_model* m, const double* x, double* out,
                        double* a, double* t, double* scale) {
  forward_cal(m, x, out, a, t, scale, NULL);
}

/* Number of leading positions of conv level li's output that some final
 * output depends on (the rest are the unpaired tails dropped later). */
static int live_len(const ol_model* m, int li, int len_out) {
  int halvings = 0; /* pointwise layers keep the length */
  for (int l = li + 1; l < m->n_layers && m->desc[l][0] != OL_FC; ++l)
    if (m->desc[l][0] == OL_CONV) ++halvings;
  return (len_out >> halvings) << halvings;
}

/* forward_one, optionally recording into amax the largest |input| of every
 * layer per channel over the values some output depends on (window slots
 * and conv positions past the paired prefix are skipped), laid out layer by
 * layer as the FP8 scales are. */
static void forward_cal(const ol_model* m, const double* x, double* out, double* a, double* t,
                        double* scale, double* amax) {
  int ch = m->n_feat, len = m->n_slot;
  if (amax) {
    const int live = live_len(m, -1, len);
    for (int l = 0; l < live; ++l)
      for (int c = 0; c < ch; ++c)
        if (fabs(x[l * ch + c]) > amax[c]) amax[c] = fabs(x[l * ch + c]);
    amax += ch;
  }
  for (int l = 0; l < len; ++l)
    for (int c = 0; c < ch; ++c) a[c * len + l] = qin(m, 0, c, x[l * ch + c]);
  for (int li = 0; li < m->n_layers; ++li) {
    const int32_t* d = m->desc[li];
    const double* w = m->w[li];
    const double* b = m->b[li];
    int co = d[2];
    if (d[0] == OL_CONV) {
      int lout = len / 2;
      for (int o = 0; o < co; ++o)
        for (int p = 0; p < lout; ++p) {
          double s = b[o];
          for (int ci = 0; ci < ch; ++ci)
            for (int k = 0; k < 2; ++k)
              s += w[((size_t)o * ch + ci) * 2 + k] * a[ci * len + 2 * p + k];
          t[o * lout + p] = (d[3] && s < 0.0) ? 0.0 : s;
        }
      len = lout;
    } else if (d[0] == OL_PW || d[0] == OL_PWRES) {
      /* kernel-1 convolution at every position; the residual half adds the
       * block input saved by the preceding pointwise layer (as stored, i.e.
       * rounded to the form), then the activation */
      double* skip = t + m->max_width / 2;
      if (d[0] == OL_PW) memcpy(skip, a, sizeof(double) * (size_t)ch * len);
      for (int o = 0; o < co; ++o)
        for (int p = 0; p < len; ++p) {
          double s = b[o];
          for (int ci = 0; ci < ch; ++ci) s += w[(size_t)o * ch + ci] * a[ci * len + p];
          if (d[0] == OL_PWRES) s += skip[o * len + p];
          t[o * len + p] = (d[3] && s < 0.0) ? 0.0 : s;
        }
    } else {
      int n_in = ch * len; /* flatten: index c*len + p, already the layout of a */
      const int is_last = (li == m->n_layers - 1);
      for (int o = 0; o < co; ++o) {
        double s = b[o];
        double mag = fabs(b[o]);
        for (int j = 0; j < n_in; ++j) {
          s += w[(size_t)o * n_in + j] * a[j];
          if (is_last && scale) mag += fabs(w[(size_t)o * n_in + j] * a[j]);
        }
        t[o] = (d[3] && s < 0.0) ? 0.0 : s;
        if (is_last && scale) scale[o] = mag;
      }
      len = 1;
    }
    ch = co;
    const int last = (li == m->n_layers - 1);
    if (amax && !last) {
      const int live = d[0] != OL_FC ? live_len(m, li, len) : len;
      for (int c = 0; c < ch; ++c)
        for (int p = 0; p < live; ++p)
          if (fabs(t[c * len + p]) > amax[c]) amax[c] = fabs(t[c * len + p]);
      amax += ch;
    }
    for (int i = 0; i < ch * len; ++i) a[i] = last ? t[i] : qin(m, li + 1, i / len, t[i]);
  }
  memcpy(out, a, sizeof(double) * (size_t)m->n_out);
}

/* Batched forward: x [B][n_slot][n_feat] (double) -> out [B][n_out];
 * scale (optional) [B][n_out] as in forward_one. */
int ol_forward(const void* p, int64_t B, const double* x, double* out, double* scale) {
  const ol_model* m = (const ol_model*)p;
  double* a = (double*)malloc(sizeof(double) * m->max_width);
  double* t = (double*)malloc(sizeof(double) * m->max_width);
  size_t win = (size_t)m->n_slot * m->n_feat;
  for (int64_t i = 0; i < B; ++i)
    forward_one(m, x + i * win, out + i * m->n_out, a, t, scale ? scale + i * m->n_out : NULL);
  free(a);
  free(t);
  return 0;
}

/* ------------------------------------------------------------ rounding --- */

/* Round a predicted latency to integer cycles: nearest, ties to even, clamp
 * to [0, lat_max]; a non-finite value becomes 0.  flags: bit0 non-finite,
 * bit1 clamped. */
int32_t ol_round(double v, int32_t lat_max, int32_t* flags) {
  *flags = 0;
  if (!isfinite(v)) { *flags = 1; return 0; }
  double r = nearbyint(v);
  if (r < 0.0) { *flags = 2; return 0; }
  if (r > (double)lat_max) { *flags = 2; return lat_max; }
  return (int32_t)r;
}

/* Hybrid head (Sec. 2.3, "From Output to Latency"): the latency of one type
 * from its HYB_PER_TYPE outputs z.  The class with the largest score wins
 * (the first of equal ones; a NaN score never wins); a class below the last
 * one is its latency, the last class ("larger than HYB_CLASSES-2") takes the
 * regression output z[HYB_CLASSES], rounded as ol_round.  flags as
 * ol_round's (0 when a class decides). */
int32_t ol_hybrid_select(const double* z, int32_t lat_max, int32_t* flags) {
  int best = 0;
  for (int c = 1; c < HYB_CLASSES; ++c)
    if (z[c] > z[best]) best = c;
  *flags = 0;
  if (best < HYB_CLASSES - 1) return best;
  return ol_round(z[HYB_CLASSES], lat_max, flags);
}

/* ----------------------------------------------------------- partition --- */

/* Equal contiguous sub-traces (Sec. 3.3): the first n mod k get one extra
 * instruction; warm[k] = min(warm_max, start[k]). */
int ol_partition(int64_t n_instr, int32_t n_sub, int32_t warm_max,
                 int64_t* start, int64_t* len, int32_t* warm) {
  if (n_sub <= 0 || n_instr < n_sub) return -1;
  int64_t q = n_instr / n_sub, r = n_instr % n_sub, s = 0;
  for (int32_t k = 0; k < n_sub; ++k) {
    start[k] = s;
    len[k] = q + (k < r ? 1 : 0);
    warm[k] = (int32_t)(s < warm_max ? s : warm_max);
    s += len[k];
  }
  return 0;
}

/* ------------------------------------------------- literal queue model --- */

typedef struct { int64_t idx, res; int32_t e, s, store; } qentry;

typedef struct {
  qentry* q;
  int64_t head, tail, cap;
} queue;

static void q_push(queue* Q, qentry e) {
  if (Q->tail == Q->cap) {
    if (Q->head > 0) {
      memmove(Q->q, Q->q + Q->head, sizeof(qentry) * (size_t)(Q->tail - Q->head));
      Q->tail -= Q->head;
      Q->head = 0;
    }
    if (Q->tail == Q->cap) {
      Q->cap = Q->cap ? 2 * Q->cap : 256;
      Q->q = (qentry*)realloc(Q->q, sizeof(qentry) * (size_t)Q->cap);
    }
  }
  Q->q[Q->tail++] = e;
}

/* One clock cycle (Sec. 3.2, clock management): the clock moves by one and
 * every instruction in either queue ages by one; up to W ready instructions
 * (residence > execution latency) leave the processor queue from its head in
 * program order, and a store among them enters the memory write queue (when
 * M is given); then every ready instruction (residence > store latency) at
 * the head of the memory write queue leaves it, in order, any number per
 * cycle. */
static void tick(queue* Q, queue* M, int64_t* cur, int W) {
  *cur += 1;
  for (int64_t j = Q->head; j < Q->tail; ++j) Q->q[j].res += 1;
  if (M)
    for (int64_t j = M->head; j < M->tail; ++j) M->q[j].res += 1;
  int n = 0;
  while (n < W && Q->head < Q->tail && Q->q[Q->head].res > Q->q[Q->head].e) {
    const qentry e = Q->q[Q->head++];
    if (M && e.store) q_push(M, e);
    n++;
  }
  if (M)
    while (M->head < M->tail && M->q[M->head].res > M->q[M->head].s) M->head++;
}

typedef struct {
  const ol_model* m;
  const int32_t* cfg;
  const float* feat;
  const uint32_t* mem; /* [n_instr][2] program counter, data address (0 = none) */
  int32_t n_sub;
  const int64_t* start;
  const int64_t* len;
  const int32_t* warm;
  const int64_t* pred_off;
  int32_t mode;
  const int32_t* lat_table;
  int64_t *fetch, *drain, *final_tick, *warm_tick;
  double* logits_out;
  double* scale_out;
  int32_t* lat_out;
  int64_t counters[2]; /* clamped, non-finite (summed under the lock) */
  int64_t max_pos;     /* > 0: stop each sub-trace after this many positions */
  double* amax;        /* calibration: per layer-input channel max |value| */
  int n_amax;
  int32_t next;
  int32_t err;
  pthread_mutex_t mu;
} sim_job;

static void simulate_one(sim_job* J, int32_t k, double* win, double* a, double* t,
                         queue* Q, queue* MQ, int64_t* cnt, double* amax) {
  const int32_t* cfg = J->cfg;
  const int D = cfg[CF_NFEAT], L = cfg[CF_NSLOT], n_out = cfg[CF_NOUT], W = cfg[CF_W];
  const int cr = cfg[CF_COLRES], ce = cfg[CF_COLEXE], cs = cfg[CF_COLSTO];
  const int cd = cfg[CF_COLDEP];
  const int32_t lat_max = cfg[CF_LATMAX];
  const int C = L - 1;
  const int need_pred = (J->mode == OL_PREDICT) || (J->logits_out != NULL) || (amax != NULL);
  const int hybrid = cfg[CF_HEAD] == 1;
  const int n_logit = hybrid ? HYB_PER_TYPE * n_out : n_out; /* model outputs */
  double out[3 * HYB_PER_TYPE], scl[3 * HYB_PER_TYPE];

  const int stcol = cfg[CF_STCOL];
  queue* M = n_out >= 3 ? MQ : NULL; /* the memory write queue exists with store latencies */
  Q->head = Q->tail = 0;
  MQ->head = MQ->tail = 0;
  int64_t cur = 0, t_w = 0;
  const int64_t w = J->warm[k];
  int64_t n_pos = J->warm[k] + J->len[k];
  if (J->max_pos > 0 && J->max_pos < n_pos) n_pos = J->max_pos;
  const int64_t first = J->start[k] - w;
  for (int64_t p = 0; p < n_pos; ++p) {
    const int64_t i = first + p;
    const int64_t g = J->pred_off[k] + p; /* global prediction index */
    if (need_pred) {
      /* Window (Sec. 2.2, Sec. 3.2): slot 0 = this instruction with zero
       * dynamic columns; then the processor queue newest first, then the
       * memory write queue newest first, C slots in all. */
      memset(win, 0, sizeof(double) * (size_t)L * D);
      for (int c = 0; c < D; ++c) win[c] = J->feat[i * D + c];
      if (cr >= 0) win[cr] = 0.0;
      if (ce >= 0) win[ce] = 0.0;
      if (cs >= 0) win[cs] = 0.0;
      if (cd >= 0)
        for (int f = 0; f < 5; ++f) win[cd + f] = 0.0;
      const int64_t inq = Q->tail - Q->head, inm = M ? M->tail - M->head : 0;
      const int shown = (int)(inq + inm < C ? inq + inm : C);
      for (int j = 1; j <= shown; ++j) {
        const qentry* e = j <= inq ? &Q->q[Q->tail - j] : &M->q[M->tail - (j - inq)];
        double* row = win + (size_t)j * D;
        for (int c = 0; c < D; ++c) row[c] = J->feat[e->idx * D + c];
        if (cr >= 0) row[cr] = (double)e->res;
        if (ce >= 0) row[ce] = (double)e->e;
        if (cs >= 0) row[cs] = (n_out >= 3) ? (double)e->s : 0.0;
        if (cd >= 0) {
          /* memory dependency flags (Sec. 2.1): does the context
           * instruction share this one's instruction cache line, its
           * instruction page, its data address, data cache line, data page */
          const uint32_t pci = J->mem[2 * i], dai = J->mem[2 * i + 1];
          const uint32_t pcj = J->mem[2 * e->idx], daj = J->mem[2 * e->idx + 1];
          const int both = dai != 0 && daj != 0;
          row[cd + 0] = (pci >> LINE_SHIFT) == (pcj >> LINE_SHIFT);
          row[cd + 1] = (pci >> PAGE_SHIFT) == (pcj >> PAGE_SHIFT);
          row[cd + 2] = both && dai == daj;
          row[cd + 3] = both && (dai >> LINE_SHIFT) == (daj >> LINE_SHIFT);
          row[cd + 4] = both && (dai >> PAGE_SHIFT) == (daj >> PAGE_SHIFT);
        }
      }
      forward_cal(J->m, win, out, a, t, J->scale_out ? scl : NULL, amax);
      if (J->logits_out)
        for (int o = 0; o < n_logit; ++o) J->logits_out[g * n_logit + o] = out[o];
      if (J->scale_out)
        for (int o = 0; o < n_logit; ++o) J->scale_out[g * n_logit + o] = scl[o];
    }
    int32_t lat[8];
    for (int o = 0; o < n_out; ++o) {
      if (J->mode == OL_PREDICT) {
        int32_t fl;
        lat[o] = hybrid ? ol_hybrid_select(out + o * HYB_PER_TYPE, lat_max, &fl)
                        : ol_round(out[o], lat_max, &fl);
        if (fl & 2) cnt[0]++;
        if (fl & 1) cnt[1]++;
      } else {
        lat[o] = J->lat_table[g * n_out + o];
      }
      if (J->lat_out) J->lat_out[g * n_out + o] = lat[o];
    }
    /* Clock management (Sec. 3.2): F cycles pass, one at a time. */
    for (int32_t f = 0; f < lat[0]; ++f) tick(Q, M, &cur, W);
    qentry e = {i, 0, lat[1], n_out >= 3 ? lat[2] : 0,
                n_out >= 3 && J->feat[i * D + stcol] != 0.0f};
    q_push(Q, e);
    if (p == w - 1) t_w = cur;
  }
  if (J->max_pos > 0) return; /* partial run (calibration): no results */
  const int64_t t_last = cur;
  while (Q->tail > Q->head || (M && M->tail > M->head)) tick(Q, M, &cur, W); /* drain */
  J->fetch[k] = t_last - t_w;
  J->drain[k] = cur - t_last;
  J->final_tick[k] = cur;
  J->warm_tick[k] = t_w;
}

static void* sim_worker(void* arg) {
  sim_job* J = (sim_job*)arg;
  const int D = J->cfg[CF_NFEAT], L = J->cfg[CF_NSLOT];
  int width = J->m ? J->m->max_width : 1;
  double* win = (double*)malloc(sizeof(double) * (size_t)L * D);
  double* a = (double*)malloc(sizeof(double) * (size_t)width);
  double* t = (double*)malloc(sizeof(double) * (size_t)width);
  queue Q = {NULL, 0, 0, 0}, MQ = {NULL, 0, 0, 0};
  int64_t cnt[2] = {0, 0};
  double* amax = J->amax ? (double*)calloc((size_t)J->n_amax, sizeof(double)) : NULL;
  for (;;) {
    pthread_mutex_lock(&J->mu);
    int32_t k = J->next++;
    pthread_mutex_unlock(&J->mu);
    if (k >= J->n_sub) break;
    simulate_one(J, k, win, a, t, &Q, &MQ, cnt, amax);
  }
  pthread_mutex_lock(&J->mu);
  J->counters[0] += cnt[0];
  J->counters[1] += cnt[1];
  if (amax)
    for (int i = 0; i < J->n_amax; ++i)
      if (amax[i] > J->amax[i]) J->amax[i] = amax[i];
  pthread_mutex_unlock(&J->mu);
  free(amax);
  free(Q.q);
  free(MQ.q);
  free(win);
  free(a);
  free(t);
  return NULL;
}

/* Simulate every sub-trace.  mode OL_PREDICT advances with the model's own
 * rounded predictions; OL_INJECT advances with lat_table[(pred_off[k] + p) *
 * n_out + o] (the model is then only run when logits_out is requested and
 * may be NULL otherwise; scale_out, like logits_out, receives each output's
 * |b| + sum |w a| of the last layer).  max_pos > 0 stops every sub-trace
 * after its first max_pos positions (no per-sub-trace results then); amax,
 * if given, receives per layer-input channel the largest |value| an output
 * depends on (window features, then every hidden layer).  Per-sub-trace results: fetch = T_last - T_w,
 * drain = final - T_last, final tick, T_w.  counters[0] = clamped, [1] =
 * non-finite.  Returns 0, or -1 on invalid arguments. */
int ol_simulate(const void* model, const int32_t* cfg, const float* feat, const uint32_t* mem,
                int64_t n_instr,
                int32_t n_sub, const int64_t* start, const int64_t* len, const int32_t* warm,
                int32_t mode, const int32_t* lat_table,
                int64_t* fetch, int64_t* drain, int64_t* final_tick, int64_t* warm_tick,
                double* logits_out, double* scale_out, int32_t* lat_out, int64_t* counters,
                int32_t n_threads, int64_t max_pos, double* amax) {
  const ol_model* m = (const ol_model*)model;
  if (cfg[CF_NOUT] < 2 || cfg[CF_NOUT] > 3) return -1;
  /* store latencies need the store flags of the trace */
  if (cfg[CF_NOUT] == 3 && (!feat || cfg[CF_STCOL] < 0 || cfg[CF_STCOL] >= cfg[CF_NFEAT]))
    return -1;
  if (cfg[CF_W] < 1 || cfg[CF_NSLOT] < 1) return -1;
  if (cfg[CF_HEAD] < 0 || cfg[CF_HEAD] > 1) return -1;
  if (cfg[CF_COLDEP] >= 0 && (!mem || cfg[CF_COLDEP] + 5 > cfg[CF_NFEAT])) return -1;
  if ((mode == OL_PREDICT || logits_out) && !m) return -1;
  const int n_logit = cfg[CF_HEAD] == 1 ? HYB_PER_TYPE * cfg[CF_NOUT] : cfg[CF_NOUT];
  if (m && (m->n_feat != cfg[CF_NFEAT] || m->n_slot != cfg[CF_NSLOT] || m->n_out != n_logit))
    return -1;
  if (mode == OL_INJECT && !lat_table) return -1;
  int64_t* pred_off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_sub + 1));
  pred_off[0] = 0;
  for (int32_t k = 0; k < n_sub; ++k) {
    if (len[k] < 1 || warm[k] < 0 || start[k] - warm[k] < 0 || start[k] + len[k] > n_instr) {
      free(pred_off);
      return -1;
    }
    pred_off[k + 1] = pred_off[k] + warm[k] + len[k];
  }
  sim_job J;
  memset(&J, 0, sizeof(J));
  J.m = m; J.cfg = cfg; J.feat = feat; J.mem = mem; J.n_sub = n_sub;
  J.start = start; J.len = len; J.warm = warm; J.pred_off = pred_off;
  J.mode = mode; J.lat_table = lat_table;
  J.fetch = fetch; J.drain = drain; J.final_tick = final_tick; J.warm_tick = warm_tick;
  J.logits_out = logits_out; J.scale_out = scale_out; J.lat_out = lat_out;
  J.max_pos = max_pos;
  J.amax = amax;
  if (amax) {
    if (!m) { free(pred_off); return -1; }
    int width = m->n_feat, len = m->n_slot;
    for (int l = 0; l < m->n_layers - 1; ++l) {
      width += m->desc[l][2];
      (void)len;
    }
    J.n_amax = width;
    for (int i = 0; i < width; ++i) amax[i] = 0.0;
  }
  pthread_mutex_init(&J.mu, NULL);
  if (n_threads <= 0) n_threads = (int32_t)sysconf(_SC_NPROCESSORS_ONLN);
  if (n_threads > n_sub) n_threads = n_sub;
  if (n_threads < 1) n_threads = 1;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
  for (int i = 0; i < n_threads; ++i) pthread_create(&th[i], NULL, sim_worker, &J);
  for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
  free(th);
  pthread_mutex_destroy(&J.mu);
  if (counters) { counters[0] = J.counters[0]; counters[1] = J.counters[1]; }
  free(pred_off);
  return 0;
}

/* FP8 scales from calibration maxima: the smallest power of two s with
 * amax <= 448 s, per entry. */
void ol_scales_from_amax(const double* amax, int32_t n, float* scales) {
  for (int32_t i = 0; i < n; ++i) scales[i] = (float)pow2_scale(amax[i]);
}

/* e4m3 rounding of single values (exposed for its pin tests). */
double ol_round_e4m3(double v) { return round_e4m3(v); }
double ol_round_bf16(double v) { return round_bf16(v); }

/* ------------------------------------------------------------ training --- */

/* Hybrid loss of one prediction (training form, read from Sec. 2.3's
 * hybrid scheme and the training of Sec. 2.4): per latency type t the head
 * gives n_bins class logits and one regression output; loss = cross-entropy
 * of the class min(lat, n_bins - 1) + |reg - log1p(lat)|.  Writes d(loss)/d
 * (head outputs) scaled by `scale` into dz (if not NULL); returns the loss. */
static double hybrid_loss(const double* z, const int32_t* lat, int n_types, int n_bins,
                          double scale, double* dz) {
  double loss = 0.0;
  const int per = n_bins + 1;
  for (int t = 0; t < n_types; ++t) {
    const double* zt = z + t * per;
    const int bin = lat[t] < n_bins - 1 ? lat[t] : n_bins - 1;
    double m = zt[0];
    for (int i = 1; i < n_bins; ++i) m = zt[i] > m ? zt[i] : m;
    double se = 0.0;
    for (int i = 0; i < n_bins; ++i) se += exp(zt[i] - m);
    const double lse = m + log(se);
    const double target = log1p((double)lat[t]);
    const double r = zt[n_bins] - target;
    loss += lse - zt[bin] + fabs(r);
    if (dz) {
      for (int i = 0; i < n_bins; ++i)
        dz[t * per + i] = scale * (exp(zt[i] - lse) - (i == bin ? 1.0 : 0.0));
      dz[t * per + n_bins] = scale * (r > 0.0 ? 1.0 : (r < 0.0 ? -1.0 : 0.0));
    }
  }
  return loss;
}

typedef struct {
  const ol_model* m;
  int64_t B;
  const double* x;
  const int32_t* lat;
  int n_bins;
  int64_t next;
  int n_params;
  double* dparams; /* [n_threads][n_params] */
  double* loss;    /* [n_threads] */
  double* dlogits; /* optional [B][n_out] */
  double* dx;      /* optional [B][L][D] */
  pthread_mutex_t mu;
} train_job;

/* Offsets of each layer's weight and bias in the flat PyTorch-order vector. */
static void param_offsets(const ol_model* m, size_t* woff, size_t* boff, size_t* total) {
  int ch = m->n_feat, len = m->n_slot;
  size_t off = 0;
  for (int l = 0; l < m->n_layers; ++l) {
    const int kind = m->desc[l][0], ci = m->desc[l][1], co = m->desc[l][2];
    const size_t nw = kind == OL_CONV ? (size_t)co * ci * 2 : (size_t)co * ci;
    woff[l] = off;
    off += nw;
    boff[l] = off;
    off += co;
    ch = co;
    len = kind == OL_CONV ? len / 2 : 1;
  }
  (void)ch;
  (void)len;
  *total = off;
}

static void* train_worker(void* arg) {
  train_job* J = (train_job*)arg;
  const ol_model* m = J->m;
  const int NL = m->n_layers, L = m->n_slot, D = m->n_feat;
  /* thread index (high bits of the shared counter), assigned under the lock */
  pthread_mutex_lock(&J->mu);
  int tid = (int)(J->next >> 40);
  J->next += (int64_t)1 << 40;
  pthread_mutex_unlock(&J->mu);
  double* dp = J->dparams + (size_t)tid * J->n_params;
  size_t woff[OL_MAXL], boff[OL_MAXL], tot;
  param_offsets(m, woff, boff, &tot);
  /* activations: a[0] = input (channel-major), a[l+1] = output of layer l */
  int ch[OL_MAXL + 1], len[OL_MAXL + 1];
  ch[0] = D;
  len[0] = L;
  for (int l = 0; l < NL; ++l) {
    ch[l + 1] = m->desc[l][2];
    len[l + 1] = m->desc[l][0] == OL_CONV ? len[l] / 2 : 1;
  }
  double* a[OL_MAXL + 1];
  double* g[OL_MAXL + 1];
  for (int l = 0; l <= NL; ++l) {
    a[l] = (double*)calloc((size_t)ch[l] * len[l], sizeof(double));
    g[l] = (double*)calloc((size_t)ch[l] * len[l], sizeof(double));
  }
  for (;;) {
    pthread_mutex_lock(&J->mu);
    const int64_t b = J->next & (((int64_t)1 << 40) - 1);
    if (b < J->B) J->next += 1;
    pthread_mutex_unlock(&J->mu);
    if (b >= J->B) break;
    const double* xb = J->x + (size_t)b * L * D;
    for (int l = 0; l < L; ++l)
      for (int c = 0; c < D; ++c) a[0][c * L + l] = qform(m, xb[l * D + c]);
    /* forward, keeping every layer's output */
    for (int l = 0; l < NL; ++l) {
      const int kind = m->desc[l][0], ci = ch[l], co = ch[l + 1], li = len[l], lo = len[l + 1];
      const double* w = m->w[l];
      const double* bb = m->b[l];
      for (int o = 0; o < co; ++o)
        for (int p = 0; p < lo; ++p) {
          double s = bb[o];
          if (kind == OL_CONV) {
            for (int c = 0; c < ci; ++c)
              for (int t = 0; t < 2; ++t) s += w[((size_t)o * ci + c) * 2 + t] * a[l][c * li + 2 * p + t];
          } else {
            const int n_in = ci * li;
            for (int j = 0; j < n_in; ++j) s += w[(size_t)o * n_in + j] * a[l][j];
          }
          s = (m->desc[l][3] && s < 0.0) ? 0.0 : s;
          a[l + 1][o * lo + p] = l < NL - 1 ? qform(m, s) : s;
        }
    }
    /* loss and its gradient w.r.t. the head outputs */
    const int n_out = ch[NL];
    const double lb = hybrid_loss(a[NL], J->lat + 2 * b, 2, J->n_bins, 1.0 / (double)J->B, g[NL]);
    J->loss[tid] += lb / (double)J->B;
    if (J->dlogits)
      for (int o = 0; o < n_out; ++o) J->dlogits[(size_t)b * n_out + o] = g[NL][o];
    /* backward */
    for (int l = NL - 1; l >= 0; --l) {
      const int kind = m->desc[l][0], ci = ch[l], co = ch[l + 1], li = len[l], lo = len[l + 1];
      const double* w = m->w[l];
      double* gw = dp + woff[l];
      double* gb = dp + boff[l];
      /* through the ReLU: output gradient where the output is positive */
      if (m->desc[l][3])
        for (int i = 0; i < co * lo; ++i)
          if (!(a[l + 1][i] > 0.0)) g[l + 1][i] = 0.0;
      for (int i = 0; i < ci * li; ++i) g[l][i] = 0.0;
      for (int o = 0; o < co; ++o)
        for (int p = 0; p < lo; ++p) {
          /* BF16 form: the output gradient of a hidden layer is kept in
           * bfloat16 (it enters the weight, input and bias gradients
           * rounded); the head's, the loss gradient, enters the weight and
           * input products rounded and its bias gradient unrounded */
          const double dy = qform(m, g[l + 1][o * lo + p]);
          gb[o] += l < NL - 1 ? dy : g[l + 1][o * lo + p];
          if (kind == OL_CONV) {
            for (int c = 0; c < ci; ++c)
              for (int t = 0; t < 2; ++t) {
                gw[((size_t)o * ci + c) * 2 + t] += dy * a[l][c * li + 2 * p + t];
                g[l][c * li + 2 * p + t] += w[((size_t)o * ci + c) * 2 + t] * dy;
              }
          } else {
            const int n_in = ci * li;
            for (int j = 0; j < n_in; ++j) {
              gw[(size_t)o * n_in + j] += dy * a[l][j];
              g[l][j] += w[(size_t)o * n_in + j] * dy;
            }
          }
        }
    }
    if (J->dx)
      for (int l = 0; l < L; ++l)
        for (int c = 0; c < D; ++c) J->dx[((size_t)b * L + l) * D + c] = g[0][c * L + l];
  }
  for (int l = 0; l <= NL; ++l) {
    free(a[l]);
    free(g[l]);
  }
  return NULL;
}

/* Training form in FP64: mean hybrid loss over B windows x [B][L][D] with
 * integer latency labels lat [B][2], its gradient w.r.t. every parameter
 * (flat, PyTorch order) and optionally w.r.t. the head outputs and the
 * input.  The network's last layer must have 2 * (n_bins + 1) outputs.
 * A BF16-form model (prec 1) evaluates the forward as ol_forward's BF16
 * form and, in the backward, rounds each layer's output gradient to
 * bfloat16: a hidden layer's everywhere it is used (weight, input and bias
 * gradients), the head's where it multiplies weights or activations (the
 * head's bias gradient sums it unrounded); sums stay exact FP64. */
int ol_train(const void* p, int64_t B, const double* x, const int32_t* lat, int32_t n_bins,
             double* loss, double* dparams, double* dlogits, double* dx, int32_t n_threads) {
  const ol_model* m = (const ol_model*)p;
  if (!m || m->prec > 1 || m->n_out != 2 * (n_bins + 1) || B < 1) return -1;
  for (int l = 0; l < m->n_layers; ++l)
    if (m->desc[l][0] != OL_CONV && m->desc[l][0] != OL_FC) return -1; /* convs and FCs only */
  size_t woff[OL_MAXL], boff[OL_MAXL], tot;
  param_offsets(m, woff, boff, &tot);
  if (n_threads <= 0) n_threads = 1;
  if (n_threads > B) n_threads = (int32_t)B;
  train_job J;
  memset(&J, 0, sizeof(J));
  J.m = m; J.B = B; J.x = x; J.lat = lat; J.n_bins = n_bins;
  J.n_params = (int)tot;
  J.dparams = (double*)calloc((size_t)n_threads * tot, sizeof(double));
  J.loss = (double*)calloc((size_t)n_threads, sizeof(double));
  J.dlogits = dlogits;
  J.dx = dx;
  pthread_mutex_init(&J.mu, NULL);
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
  for (int i = 0; i < n_threads; ++i) pthread_create(&th[i], NULL, train_worker, &J);
  for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
  free(th);
  pthread_mutex_destroy(&J.mu);
  *loss = 0.0;
  for (size_t i = 0; i < tot; ++i) dparams[i] = 0.0;
  for (int t = 0; t < n_threads; ++t) {
    *loss += J.loss[t];
    for (size_t i = 0; i < tot; ++i) dparams[i] += J.dparams[(size_t)t * tot + i];
  }
  free(J.dparams);
  free(J.loss);
  return 0;
}

/* Mean hybrid loss of given head outputs (for finite differences). */
double ol_hybrid_loss(const double* z, const int32_t* lat, int64_t B, int32_t n_bins) {
  double s = 0.0;
  for (int64_t b = 0; b < B; ++b)
    s += hybrid_loss(z + (size_t)b * 2 * (n_bins + 1), lat + 2 * b, 2, n_bins, 0.0, NULL);
  return s / (double)B;
}
