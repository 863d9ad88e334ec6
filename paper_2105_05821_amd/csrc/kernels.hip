// HIP kernels of libsimnet.so for gfx950 (CDNA4).
//
// One workgroup owns a tile of MT = 16 sub-traces and runs the whole step
// loop for them inside one launch (persistent: sub-traces are independent,
// Sec. 3.3, so no grid-wide synchronisation is needed).  Each step:
//   gather   - builds the tile's windows block by block straight into LDS
//              from the trace rows (FP32, their BF16 copy in the BF16 form, or
//              packed codes) and the sub-trace's processor queue (Sec. 2.2:
//              current instruction with zero dynamic columns, then the
//              in-flight instructions newest first with residence and
//              execution latency; with store latencies, then the memory
//              write queue);
//   predict  - conv levels as MFMA GEMMs on LDS tiles (Sec. 2.3: kernel 2,
//              stride 2, ReLU), the hidden FC accumulated block by block in
//              MFMA accumulators, the final FC on the VALU (the hybrid head
//              as one MFMA tile row);
//   update   - rounding (or the hybrid head's class choice) and the clock /
//              queue update of Sec. 3.2 in its timestamp form: instruction i
//              enters at T_i = T_{i-1} + F_i and leaves at r_i = max(T_i +
//              E_i + 1, r_{i-1}, r_{i-W} + 1); the queue after the advance is
//              the suffix with r > T_i.
// The queue ring and the per-sub-trace scalars stay in LDS for the whole
// launch and are written back to HBM when the launch ends.  RB7, whose
// residual blocks do not fit this loop, runs each step as four launches
// (the step kernel's stages 1 and 2 around resblock_kernel and
// rb_head_kernel).
//
// Precision forms: weights and activations in FP32, BF16 or FP8 (OCP e4m3,
// per-channel power-of-two scales), products accumulated in FP32 in every
// form; biases and the final logits are FP32.
#include <type_traits>

#include "simnet_internal.h"

namespace simnet {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// ------------------------------------------------------ precision forms ---
// Each form stores activations and weights as T and multiplies one 16-byte
// fragment per lane per call of mma(): lane group g = lane/16 holds KG/4
// consecutive k of its row (A) or column (B); A and B use the same
// assignment, so every call adds the full KG-long partial dot products.

// Acc: the accumulator of one MFMA tile; TILE: its side; col4(g, lane):
// the first of the 4 consecutive output columns (weight-first operand
// order: the weights' N) that accumulator elements 4g .. 4g+3 of the lane
// hold, for the activation row lane % TILE.
struct PF32 {
  using T = float;
  using Acc = v4f;
  static constexpr int ID = 0, KG = 16, TILE = 16;
  __device__ static int col4(int, int lane) { return 4 * (lane >> 4); }
  static constexpr bool SCALED = false;
  __device__ static v4f mma(v4f c, uint4 a, uint4 b) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
    return c;
  }
  __device__ static T cvt(float x) { return x; }
  __device__ static float val(T x) { return x; }
};

struct PBF16 {
  using T = uint16_t;  // bfloat16 bits
  using Acc = v4f;
  static constexpr int ID = 1, KG = 32, TILE = 16;
  __device__ static int col4(int, int lane) { return 4 * (lane >> 4); }
  static constexpr bool SCALED = false;
  __device__ static v4f mma(v4f c, uint4 a, uint4 b) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                   __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
  }
  // round to nearest even (inputs are finite)
  __device__ static T cvt(float x) {
    const uint32_t u = __float_as_uint(x);
    return (T)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
  }
  __device__ static float val(T x) { return __uint_as_float((uint32_t)x << 16); }
};

struct PFP8 {
  using T = uint8_t;  // OCP e4m3 (max 448)
  using Acc = v4f;
  static constexpr int ID = 2, KG = 64, TILE = 16;
  __device__ static int col4(int, int lane) { return 4 * (lane >> 4); }
  static constexpr bool SCALED = true;
  __device__ static v4f mma(v4f c, uint4 a, uint4 b) {
    const long a0 = ((long)a.y << 32) | a.x, a1 = ((long)a.w << 32) | a.z;
    const long b0 = ((long)b.y << 32) | b.x, b1 = ((long)b.w << 32) | b.z;
    c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a0, b0, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a1, b1, c, 0, 0, 0);
    return c;
  }
  // round to nearest even, saturating at +-448
  __device__ static T cvt(float x) {
    x = fminf(fmaxf(x, -448.f), 448.f);
    return (T)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.f, 0, false) & 0xff);
  }
  __device__ static float val(T x) { return __builtin_amdgcn_cvt_f32_fp8((int)x, 0); }
};

// BF16 on 32x32x16 tiles: the same storage, twice the FLOP per MFMA
// (32,768).  Lane l holds 8 consecutive k (8 * (l / 32) ..) of row l % 32 of
// either operand; the 16 accumulators of lane l are output columns
// 8 * (i / 4) + 4 * (l / 32) + i % 4 of row l % 32.  On gfx950 this
// instruction issues back to back where the 16x16x32 one leaves gaps.
struct PBF16W : PBF16 {
  using Acc = v16f;
  static constexpr int KG = 16, TILE = 32;
  __device__ static int col4(int g, int lane) { return 8 * g + 4 * (lane >> 5); }
  __device__ static v16f mma(v16f c, uint4 a, uint4 b) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a),
                                                   __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
  }
};

// Blocks per group: the window is processed a group of NG consecutive
// blocks at a time (the conv levels as one GEMM over all the group's
// positions, so each weight fragment serves NG times more rows), as many as
// the form's LDS budget allows beside the queue rings.
template <class Net, class P>
constexpr int group_blocks() {
  // (store latencies: the stores' ring takes LDS, so smaller groups)
  return Net::NCONV == 2 ? Net::NB : Net::MWQ ? (P::ID == 0 ? 1 : 2) : (P::ID == 0 ? 2 : 4);
}

template <class Net, class P>
struct Geo {
  using T = typename P::T;
  static constexpr int NT = Net::WAVES * 64;
  static constexpr int NG = group_blocks<Net, P>();
  static constexpr int PAD = 16 / sizeof(T);                       // 16 bytes of padding
  static constexpr int DP = padded_feat(Net::D, P::ID);            // features per slot
  // A conv reads rows of two consecutive input positions; each such pair is
  // followed by 16 bytes of padding, so the 16 rows of an MFMA tile (16
  // positions) fall in different LDS banks.  R* = elements per pair.
  static constexpr int RX = 2 * DP + PAD;                          // slot pair (conv1 row)
  static constexpr int R1 = 2 * Net::CH1 + PAD;                    // conv1 output pair
  static constexpr int R2 = 2 * Net::CH2 + PAD;                    // conv2 output pair (C3)
  static constexpr int SX = (NG * Net::BS / 2) * RX + PAD;         // a group's window rows, per window
  static constexpr int SA1 = (NG * Net::BS / 4) * R1 + PAD;        // conv1 output
  static constexpr int SA2 = Net::NCONV == 3 ? (NG * Net::BS / 8) * R2 + PAD  // conv2 output
                                             : NG * Net::CH2 + PAD;  // (last conv: flat)
  static constexpr int SA3 = (Net::NCONV == 3 ? NG * Net::CH3 : 0) + PAD;  // conv3 output (flat)
  static constexpr int SAL = Net::NCONV == 3 ? SA3 : SA2;          // last conv output
  // three conv levels: X and conv2's output share memory (X is dead once
  // conv1 has read it), and so do conv1's and conv3's outputs
  static constexpr bool ALIAS = Net::NCONV == 3;
  static constexpr int NXA2 = ALIAS ? (SX > SA2 ? MT * SX : MT * SA2) : MT * SX;
  static constexpr int NA1A3 = ALIAS ? (SA1 > SA3 ? MT * SA1 : MT * SA3) : MT * SA1;
  static constexpr int NA2 = ALIAS ? PAD : MT * SA2;
};

template <class Net, class P>
struct NetSmem {
  using G = Geo<Net, P>;
  // window rows of the group (X), then conv2's output; after the last group
  // also the final FC's cross-wave partial sums
  alignas(16) typename P::T xa2[G::NXA2];
  alignas(16) typename P::T a1a3[G::NA1A3]; // conv1's output, then conv3's output
  alignas(16) typename P::T a2own[G::NA2];  // conv2's output when it does not alias X
  float logit[MT][Net::NOUT];
  float x_inv[Net::D];  // FP8: reciprocal input scale of each window feature
  // The final FC on the VALU after the hidden layer (regression head): its
  // operands copied here once per launch (stage_head), so the end of every
  // prediction reads no global memory.  hb: hidden bias; FP8 hws, hai: the
  // hidden layer's weight and output scales; lw: final weights [NOUT][HID];
  // lb: final bias.
  static constexpr bool HL = Net::HID > 0 && Net::HEAD == 0;
  static constexpr int HLN = HL ? Net::HID : 1, HLS = HL && P::SCALED ? Net::HID : 1;
  float hb[HLN], hws[HLS], hai[HLS], lw[HL ? Net::NOUT * Net::HID : 1], lb[Net::NOUT];
  __device__ void stage_head(const DevWeights& wt, int tid, int nt) {
    if constexpr (HL) {
      // (weights without a final FC, as the training form's trunk has, leave
      // it unstaged: kernels that run the final FC are never given them)
      if (!wt.last_w || !wt.last_b || !wt.hid_b) return;
      for (int i = tid; i < Net::HID; i += nt) {
        hb[i] = wt.hid_b[i];
        if constexpr (P::SCALED) {
          hws[i] = wt.hid_ws[i];
          hai[i] = wt.hid_ai[i];
        }
      }
      for (int i = tid; i < Net::NOUT * Net::HID; i += nt) lw[i] = wt.last_w[i];
      for (int i = tid; i < Net::NOUT; i += nt) lb[i] = wt.last_b[i];
    }
  }
  __device__ typename P::T* x() { return xa2; }
  __device__ typename P::T* a1() { return a1a3; }
  __device__ typename P::T* a2() { return G::ALIAS ? xa2 : a2own; }
  __device__ typename P::T* a3() { return a1a3; }
  // [WAVES][MT][NOUT] partial sums of the final FC (X is dead by then)
  __device__ float* red() { return reinterpret_cast<float*>(xa2); }
  static_assert(Net::HID == 0 || sizeof(xa2) >= sizeof(float) * Net::WAVES * MT * Net::NOUT,
                "final-FC partial sums do not fit X's region");
};

// Epilogue of one accumulator element: bias, (FP8) dequantisation, ReLU.
template <class P>
__device__ __forceinline__ float activation(float acc, int col, const float* bias, const float* ws,
                                            bool relu) {
  float v;
  if constexpr (P::SCALED)
    v = fmaf(acc, ws[col], bias[col]);
  else
    v = acc + bias[col];
  return relu ? fmaxf(v, 0.f) : v;
}
// ... then (FP8) the next layer's input scale and conversion to storage.
template <class P>
__device__ __forceinline__ typename P::T to_storage(float v, int col, const float* ai) {
  if constexpr (P::SCALED) v *= ai[col];
  return P::cvt(v);
}
// The same two with the column's bias b, weight scale s and input scale a
// already in registers.
template <class P>
__device__ __forceinline__ float activation_v(float acc, float b, float s, bool relu) {
  float v;
  if constexpr (P::SCALED)
    v = fmaf(acc, s, b);
  else
    v = acc + b;
  return relu ? fmaxf(v, 0.f) : v;
}
template <class P>
__device__ __forceinline__ typename P::T to_storage_v(float v, float a) {
  if constexpr (P::SCALED) v *= a;
  return P::cvt(v);
}
// Calibration: running per-channel max of |activation| (LDS, as ordered bits).
__device__ __forceinline__ void cal_max(unsigned* cal, int i, float v) {
  atomicMax(cal + i, __float_as_uint(fabsf(v)));
}

// k-groups per chunk when streaming B: a chunk is at most FRAGS fragments
// (4 VGPRs each) and two chunks are in flight; must divide the k-groups.
constexpr int stream_chunk(int kgs, int tpw, int frags = 8) {
  int c = frags / tpw;
  if (c < 1) c = 1;
  if (c > kgs) c = kgs;
  while (kgs % c) --c;
  return c;
}

// One 16-byte weight fragment through a raw buffer load: the resource and
// the fragment's offset are wave-uniform (scalar registers), only the lane's
// 16-byte offset is per lane, so many fragments can be in flight without a
// 64-bit address register each.
__device__ __forceinline__ uint4 load_frag(__amdgpu_buffer_rsrc_t r, int lane_off, int frag_off) {
  return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, lane_off, frag_off, 0));
}

// Workgroup barrier ordering LDS only: global loads in flight (weight
// prefetches) stay in flight across it (__syncthreads waits for them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t frag_rsrc(const uint4* Bp, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint4*>(Bp), (short)0, bytes, 0x00020000);
}

// The first chunk of a weight stream (see mma_stream), requested ahead of
// the stream: before the barrier that precedes it, so that its L2 latency
// passes during the barrier and the previous phase's tail instead of
// stalling every wave at the start of the phase.
template <int CH, int NPW>
struct StreamHead {
  uint4 b[CH][NPW];
};

template <int KGS, int NTILES, int NPW, int FRAGS = 8>
__device__ __forceinline__ StreamHead<stream_chunk(KGS, NPW, FRAGS), NPW> stream_head(
    const uint4* __restrict__ Bp, int nt0, int lane) {
  constexpr int CH = stream_chunk(KGS, NPW, FRAGS);
  const __amdgpu_buffer_rsrc_t rs = frag_rsrc(Bp, KGS * NTILES * 1024);
  const int lo = lane * 16;
  const int wn = __builtin_amdgcn_readfirstlane(nt0) * 1024;
  StreamHead<CH, NPW> h;
#pragma unroll
  for (int kg = 0; kg < CH; ++kg)
#pragma unroll
    for (int j = 0; j < NPW; ++j) h.b[kg][j] = load_frag(rs, lo, wn + (kg * NTILES + j) * 1024);
  return h;
}

// acc[i][j] += W(tile nt0 + j) x A(m-tile i: this lane's row of it), all K.
// The weight fragment is the MFMA's first operand, so lane l ends up
// holding row l % 16 of the activations and output columns 4*(l/16) .. +3
// of the tile: consecutive columns, stored with one vector write.  Each
// weight fragment serves MPW m-tiles.  Weight fragments are requested
// DEPTH - 1 chunks ahead of their use (DEPTH buffers) and the scheduler is
// kept from sinking the requests.  HEAD: the first chunk was requested by
// stream_head (same KGS, NTILES, NPW, FRAGS, Bp and nt0) and is passed in.
template <class P, int KGS, int NTILES, int NPW, int MPW, int FRAGS = 8, bool HEAD = false,
          int DEPTH = 2>
__device__ __forceinline__ void mma_stream(
    typename P::Acc (&acc)[MPW][NPW], const typename P::T* const (&ap)[MPW],
    const uint4* __restrict__ Bp, int nt0, int lane,
    const StreamHead<stream_chunk(KGS, NPW, FRAGS), NPW>* head = nullptr) {
  constexpr int CH = stream_chunk(KGS, NPW, FRAGS), NCH = KGS / CH;
  const __amdgpu_buffer_rsrc_t rs = frag_rsrc(Bp, KGS * NTILES * 1024);
  const int lo = lane * 16;
  const int wn = __builtin_amdgcn_readfirstlane(nt0) * 1024;
  uint4 b[DEPTH][CH][NPW];
  auto request = [&](int c) {
#pragma unroll
    for (int kg = 0; kg < CH; ++kg)
#pragma unroll
      for (int j = 0; j < NPW; ++j)
        b[c % DEPTH][kg][j] = load_frag(rs, lo, wn + ((c * CH + kg) * NTILES + j) * 1024);
  };
  if constexpr (HEAD) {
#pragma unroll
    for (int kg = 0; kg < CH; ++kg)
#pragma unroll
      for (int j = 0; j < NPW; ++j) b[0][kg][j] = head->b[kg][j];
  } else {
    request(0);
  }
#pragma unroll
  for (int c = 1; c < DEPTH - 1 && c < NCH; ++c) request(c);
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    if (c + DEPTH - 1 < NCH) request(c + DEPTH - 1);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kg = 0; kg < CH; ++kg) {
#pragma unroll
      for (int i = 0; i < MPW; ++i) {
        const uint4 a = *reinterpret_cast<const uint4*>(ap[i] + (c * CH + kg) * P::KG);
#pragma unroll
        for (int j = 0; j < NPW; ++j) acc[i][j] = P::mma(acc[i][j], b[c % DEPTH][kg][j], a);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// N consecutive storage elements written with the widest stores the
// destination's alignment (ALIGN bytes) allows.
template <int ALIGN, class T, int N>
__device__ __forceinline__ void store_run(T* dst, const T (&e)[N]) {
  constexpr int BYTES = N * (int)sizeof(T);
  constexpr int W = (ALIGN % 16 == 0 && BYTES % 16 == 0) ? 16
                    : (ALIGN % 8 == 0 && BYTES % 8 == 0) ? 8
                    : (ALIGN % 4 == 0 && BYTES % 4 == 0) ? 4 : (int)sizeof(T);
  uint32_t w[(BYTES + 3) / 4];
  __builtin_memcpy(w, e, BYTES);
  char* d = reinterpret_cast<char*>(dst);
#pragma unroll
  for (int o = 0; o < BYTES; o += W) {
    if constexpr (W == 16)
      *reinterpret_cast<uint4*>(d + o) = uint4{w[o / 4], w[o / 4 + 1], w[o / 4 + 2], w[o / 4 + 3]};
    else if constexpr (W == 8)
      *reinterpret_cast<uint2*>(d + o) = uint2{w[o / 4], w[o / 4 + 1]};
    else if constexpr (W == 4)
      *reinterpret_cast<uint32_t*>(d + o) = w[o / 4];
    else
      *reinterpret_cast<T*>(d + o) = e[o / sizeof(T)];
  }
}

// Waves along N for a conv level: two N tiles per wave where there are
// enough (each A fragment read from LDS then serves two MFMAs, each B
// fragment from L2 serves the wave's M tiles), and never more waves along M
// than there are M tiles.
constexpr int conv_wave_split(int ntiles, int mtiles, int waves) {
  int wn = ntiles / 2 < 1 ? 1 : ntiles / 2 < waves ? ntiles / 2 : waves;
  while (waves / wn > mtiles || waves % wn) wn *= 2;
  return wn;
}

// The tiling of one conv level as a GEMM (see conv_stage): MT windows x POS
// output positions of rows, N output channels, contraction K; the waves'
// split over N and M tiles and the type of the stream's first chunk.
template <class P, int K, int N, int POS, int WAVES>
struct ConvShape {
  static constexpr int ROWS = MT * POS;
  static constexpr int MTILES = ROWS / 16, NTILES = N / 16, KGS = K / P::KG;
  static constexpr int WN = conv_wave_split(NTILES, MTILES, WAVES), WM = WAVES / WN;
  static constexpr int MPW = MTILES / WM, NPW = NTILES / WN;
  static_assert(ROWS % 16 == 0 && N % 16 == 0 && K % P::KG == 0, "tile shape");
  static_assert(WAVES % WN == 0 && MTILES % WM == 0 && NTILES % WN == 0 && MPW >= 1,
                "wave split");
  // weight fragments per chunk: the BF16 form's conv levels run 1.3 %
  // faster with 16 (measured); FP32 and FP8 gain nothing
  static constexpr int FRAGS = P::ID == 1 ? 16 : 8;
  using Head = StreamHead<stream_chunk(KGS, NPW, FRAGS), NPW>;
};

// The first chunk of a conv level's weight stream for this wave (see
// StreamHead), requested ahead of conv_stage<..., HEAD = true>.
template <class P, int K, int N, int POS, int WAVES>
__device__ __forceinline__ typename ConvShape<P, K, N, POS, WAVES>::Head conv_head(
    const void* Bp, int wave, int lane) {
  using S = ConvShape<P, K, N, POS, WAVES>;
  return stream_head<S::KGS, S::NTILES, S::NPW, S::FRAGS>(static_cast<const uint4*>(Bp),
                                                (wave % S::WN) * S::NPW, lane);
}

// One conv level as a GEMM: rows (s, q) = MT windows x POS output positions,
// A row (s, q) is the K = 2*C_in contiguous elements of input positions 2q,
// 2q+1 at A + s*SA + q*IRS; output row (s, q) goes to O + s*SO + q*N, or,
// OPAIR, to O + s*SO + (q/2)*(2N + 16 bytes) + (q%2)*N (the padded pair
// layout the next conv reads).  The
// waves split the N tiles (conv_wave_split), then the M tiles; a wave runs
// MPW x NPW tiles.
// SAVE: also store each output row (s, q) to sv + s*sv_s + q*N (rows with
// s < sv_rows only), the layer's activations kept for the backward pass.
// Rows are numbered position-major, row = q * MT + s: an MFMA tile's 16
// rows are 16 windows at one position, whose window strides spread them
// over the LDS banks (the position stride of a wide level is a multiple of
// the bank count, so window-major tiles would collide).
// HEAD: the weight stream's first chunk was requested by conv_head and is
// passed in (head).
template <class P, int K, int N, int POS, int WAVES, int SA, int IRS, int SO, bool OPAIR,
          bool CAL = false, bool SAVE = false, bool HEAD = false>
__device__ __forceinline__ void conv_stage(
    const typename P::T* __restrict__ A, typename P::T* __restrict__ O,
    const uint4* __restrict__ Bp, const float* __restrict__ bias, const float* __restrict__ ws,
    const float* __restrict__ ai, bool relu, int wave, int lane, unsigned* cal = nullptr,
    const int* row_live = nullptr, typename P::T* sv = nullptr, int64_t sv_s = 0,
    int sv_rows = 0, const typename ConvShape<P, K, N, POS, WAVES>::Head* head = nullptr) {
  using T = typename P::T;
  using S = ConvShape<P, K, N, POS, WAVES>;
  constexpr int MTILES = S::MTILES, NTILES = S::NTILES, KGS = S::KGS;
  constexpr int WN = S::WN, MPW = S::MPW, NPW = S::NPW;
  (void)MTILES;
  const int wm = wave / WN, wn = wave % WN;
  const int nt0 = wn * NPW;
  const T* ap[MPW];
#pragma unroll
  for (int i = 0; i < MPW; ++i) {
    const int row = (wm * MPW + i) * 16 + (lane & 15);
    ap[i] = A + (row % MT) * SA + (row / MT) * IRS + (P::KG / 4) * (lane >> 4);
  }
  v4f acc[MPW][NPW];
#pragma unroll
  for (int i = 0; i < MPW; ++i)
#pragma unroll
    for (int j = 0; j < NPW; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  // the epilogue's operands for this lane's 4 columns of each tile, requested
  // before the products: after them, the wait for these loads would also
  // wait for every weight request in flight behind them
  constexpr int NS = P::SCALED ? NPW : 1;
  v4f eb[NPW], es[NS] = {}, ea[NS] = {};
#pragma unroll
  for (int j = 0; j < NPW; ++j) {
    const int col0 = (nt0 + j) * 16 + 4 * (lane >> 4);
    eb[j] = *reinterpret_cast<const v4f*>(bias + col0);
    if constexpr (P::SCALED) {
      es[j] = *reinterpret_cast<const v4f*>(ws + col0);
      ea[j] = *reinterpret_cast<const v4f*>(ai + col0);
    }
  }
  mma_stream<P, KGS, NTILES, NPW, MPW, S::FRAGS, HEAD>(acc, ap, Bp, nt0, lane, head);
#pragma unroll
  for (int i = 0; i < MPW; ++i) {
    const int row = (wm * MPW + i) * 16 + (lane & 15);
    constexpr int ORS = 2 * N + 16 / (int)sizeof(T);
    const int q = row / MT, s = row % MT;
    T* orow = O + s * SO + (OPAIR ? (q >> 1) * ORS + (q & 1) * N : q * N);
    const bool live = !CAL || row_live[s];
#pragma unroll
    for (int j = 0; j < NPW; ++j) {
      const int col0 = (nt0 + j) * 16 + 4 * (lane >> 4);
      T e[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float v = activation_v<P>(acc[i][j][q], eb[j][q], es[P::SCALED ? j : 0][q], relu);
        if constexpr (CAL)
          if (live) cal_max(cal, col0 + q, v);
        e[q] = to_storage_v<P>(v, ea[P::SCALED ? j : 0][q]);
      }
      store_run<4 * sizeof(T)>(orow + col0, e);
      if constexpr (SAVE)
        if (s < sv_rows) store_run<4 * sizeof(T)>(sv + s * sv_s + q * N + col0, e);
    }
  }
}

// Activations kept for the backward pass (training form, SAVE): per window
// b, channels-last, in storage precision: a1 [NB*BS/2][CH1], a2
// [NB*BS/4][CH2], a3 [NB][CH3], h [HID]; pointers already at the tile's
// first window, rows = windows of the tile that exist.
template <class T>
struct SavePtrs {
  T *a1, *a2, *a3, *h;
  int rows;
};

// Index of the hidden FC in the layer list (after the convs and the
// residual blocks' two pointwise layers each): its ReLU bit.
template <class Net>
constexpr int hidden_layer() {
  return Net::NCONV + 2 * Net::NRES;
}

// The hidden FC's weight stream for a group of NBG blocks (see hidden_fc):
// HT output tiles per wave, KGS k-groups, the packed weights' address.
template <class Net, class P, int NBG>
struct FcShape {
  static constexpr int HT = (Net::HID / 16) / Net::WAVES;
  static constexpr int KGS = NBG * Net::CHL / P::KG;
  using Head = StreamHead<stream_chunk(KGS, HT, Net::FC1_FRAGS), HT>;
  // the packed weights of blocks j0 .. j0 + NBG - 1
  static __device__ __forceinline__ const uint4* weights(const DevWeights& wt, int j0) {
    return static_cast<const uint4*>(wt.hid_w) +
           (size_t)j0 * (Net::CHL / P::KG) * (Net::HID / 16) * 64;
  }
};

// The first chunk of hidden_fc<..., HEAD = true>'s weight stream (see
// StreamHead).
template <class Net, class P, int NBG>
__device__ __forceinline__ typename FcShape<Net, P, NBG>::Head fc_head(const DevWeights& wt,
                                                                      int j0, int wave, int lane) {
  using S = FcShape<Net, P, NBG>;
  return stream_head<S::KGS, Net::HID / 16, S::HT, Net::FC1_FRAGS>(S::weights(wt, j0),
                                                                  wave * S::HT, lane);
}

// Hidden-FC contribution of NBG blocks from block j0: last = the blocks'
// last-conv output in LDS (window s at s * SAL, block-major), hacc += it
// times the per-block packed weights.  A fresh accumulator per group, then
// added, so the FP32 chain is per group.  HEAD: the stream's first chunk
// was requested by fc_head and is passed in (head).
template <class Net, class P, int NBG, bool HEAD = false>
__device__ __forceinline__ void hidden_fc(const DevWeights& wt, const typename P::T* last, int j0,
                                          v4f* hacc, int wave, int lane,
                                          const typename FcShape<Net, P, NBG>::Head* head = nullptr) {
  using G = Geo<Net, P>;
  using T = typename P::T;
  using S = FcShape<Net, P, NBG>;
  constexpr int HT = S::HT;
  const T* const ap[1] = {last + (lane & 15) * G::SAL + (P::KG / 4) * (lane >> 4)};
  v4f bacc[1][HT];
#pragma unroll
  for (int jj = 0; jj < HT; ++jj) bacc[0][jj] = v4f{0.f, 0.f, 0.f, 0.f};
  mma_stream<P, S::KGS, Net::HID / 16, HT, 1, Net::FC1_FRAGS, HEAD, Net::FC1_DEPTH>(
      bacc, ap, S::weights(wt, j0), wave * HT, lane, head);
#pragma unroll
  for (int jj = 0; jj < HT; ++jj) hacc[jj] += bacc[0][jj];
}

// The conv levels and the hidden-FC (or final-FC) contribution of one group
// of NBG blocks starting at block j0, for the tile of MT windows whose
// window rows are in sm.x().  relu_mask bit l = ReLU after layer l.  Ends
// with the group's last-conv output consumed.  issue() requests the next
// group's rows into registers before the last conv level and finish(regs)
// writes them into sm.x() (the region conv2's output used, dead once the
// last level has read it) before the FC.  With three conv levels the first
// weight chunk of conv2, conv3 and the FC is requested before the barrier
// that precedes it (StreamHead) and the barriers order LDS only, so the
// requests stay in flight across them.  (Requesting conv1's across the
// group boundary as well made the hidden-FC stream spill registers.)
// TRUNK: the convolutions only, the last conv's output going to sv.a3 (a1
// and a2 are not written).
template <class Net, class P, int NBG, bool CAL, bool SAVE, bool TRUNK, class Issue, class Finish>
__device__ __forceinline__ void run_group(
    const DevWeights& wt, uint32_t relu_mask, NetSmem<Net, P>& sm, int j0, unsigned* cal,
    const int* row_live, SavePtrs<typename P::T> sv, v4f* hacc, float& fpart, Issue&& issue,
    Finish&& finish) {
  using G = Geo<Net, P>;
  using T = typename P::T;
  constexpr bool XPF = Net::NCONV == 3;  // weight streams requested across the barriers
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  constexpr int P1 = NBG * Net::BS / 2, P2 = NBG * Net::BS / 4;
  constexpr int Q1 = Net::BS / 2, Q2 = Net::BS / 4;  // positions per block
  conv_stage<P, 2 * G::DP, Net::CH1, P1, Net::WAVES, G::SX, G::RX, G::SA1, true, CAL,
             SAVE && !TRUNK>(
      sm.x(), sm.a1(), static_cast<const uint4*>(wt.conv_w[0]), wt.conv_b[0], wt.conv_ws[0],
      wt.conv_ai[0], relu_mask & 1u, wave, lane, cal + Net::D, row_live,
      sv.a1 + (size_t)j0 * Q1 * Net::CH1, (int64_t)Net::NB * Q1 * Net::CH1, sv.rows);
  typename ConvShape<P, 2 * Net::CH1, Net::CH2, P2, Net::WAVES>::Head h2;
  if constexpr (XPF) {
    h2 = conv_head<P, 2 * Net::CH1, Net::CH2, P2, Net::WAVES>(wt.conv_w[1], wave, lane);
    lds_barrier();
  } else {
    __syncthreads();
  }
  conv_stage<P, 2 * Net::CH1, Net::CH2, P2, Net::WAVES, G::SA1, G::R1, G::SA2, Net::NCONV == 3,
             CAL, SAVE && !TRUNK, XPF>(
      sm.a1(), sm.a2(), static_cast<const uint4*>(wt.conv_w[1]), wt.conv_b[1], wt.conv_ws[1],
      wt.conv_ai[1], relu_mask & 2u, wave, lane, cal + Net::D + Net::CH1, row_live,
      sv.a2 + (size_t)j0 * Q2 * Net::CH2, (int64_t)Net::NB * Q2 * Net::CH2, sv.rows, &h2);
  if constexpr (Net::NCONV == 3) {
    auto h3 = conv_head<P, 2 * Net::CH2, Net::CH3, NBG, Net::WAVES>(wt.conv_w[2], wave, lane);
    lds_barrier();
    // the next group's rows are requested now, held through conv3 and
    // written once conv3 has read conv2's output (X's region), so the FC's
    // weight stream has the registers to itself
    auto next_rows = issue();
    conv_stage<P, 2 * Net::CH2, Net::CH3, NBG, Net::WAVES, G::SA2, G::R2, G::SA3, false, CAL,
               SAVE, true>(
        sm.a2(), sm.a3(), static_cast<const uint4*>(wt.conv_w[2]), wt.conv_b[2], wt.conv_ws[2],
        wt.conv_ai[2], relu_mask & 4u, wave, lane, cal + Net::D + Net::CH1 + Net::CH2, row_live,
        sv.a3 + (size_t)j0 * Net::CH3, (int64_t)Net::NB * Net::CH3, sv.rows, &h3);
    if constexpr (!TRUNK && Net::HID > 0) {
      // hidden FC over the group's NBG*CHL inputs per window (block-major,
      // as the packed per-block matrices are consecutive)
      auto hf = fc_head<Net, P, NBG>(wt, j0, wave, lane);
      lds_barrier();
      if constexpr (!Net::LATE_COMMIT) finish(next_rows);
      hidden_fc<Net, P, NBG, true>(wt, sm.a3(), j0, hacc, wave, lane, &hf);
      if constexpr (Net::LATE_COMMIT) finish(next_rows);
      return;
    }
    lds_barrier();
    finish(next_rows);
  } else {
    __syncthreads();
  }
  const T* last = Net::NCONV == 3 ? sm.a3() : sm.a2();
  if constexpr (TRUNK) {
    (void)last;
  } else if constexpr (Net::HID > 0) {
    hidden_fc<Net, P, NBG>(wt, last, j0, hacc, wave, lane);
  } else {
    // final FC on the VALU straight after the convs: (s, o) pairs, LPP lanes
    // each; the next group's rows are requested before it and written after
    constexpr int LPP = G::NT / (MT * Net::NOUT);
    constexpr int CPL = Net::CHL / LPP;
    const int fpair = tid / LPP, fsub = tid % LPP;
    const int fs = fpair / Net::NOUT, fo = fpair % Net::NOUT;
    auto next_rows = issue();
#pragma unroll
    for (int jb = 0; jb < NBG; ++jb) {
      const float* wrow = wt.last_w + ((size_t)(j0 + jb) * Net::NOUT + fo) * Net::CHL + fsub * CPL;
      const T* arow = last + fs * G::SAL + jb * Net::CHL + fsub * CPL;
#pragma unroll
      for (int c = 0; c < CPL; ++c) fpart = fmaf(P::val(arow[c]), wrow[c], fpart);
    }
    finish(next_rows);
  }
}

// Hybrid head (NOUT outputs) after the hidden FC: the hidden layer's
// outputs (bias, ReLU, rounded to the form) go to LDS (X's region, dead
// after the last group), then the final FC runs as one MFMA tile row on the
// first NOUTP/16 waves; raw outputs to sm.logit.
template <class Net, class P, bool CAL>
__device__ __forceinline__ void hybrid_head(const DevWeights& wt, uint32_t relu_mask,
                                            NetSmem<Net, P>& sm, const v4f* hacc, unsigned* cal,
                                            const int* row_live) {
  using G = Geo<Net, P>;
  using T = typename P::T;
  constexpr int HT = (Net::HID / 16) / Net::WAVES;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  (void)tid;
  constexpr int NOUTP = (Net::NOUT + 15) / 16 * 16, NTL = NOUTP / 16;
  constexpr int SH = Net::HID + G::PAD;
  static_assert(sizeof(T) * MT * SH <= sizeof(sm.xa2) && NTL <= Net::WAVES, "hybrid head");
  T* hb = sm.x();
  const bool hrelu = relu_mask & (1u << hidden_layer<Net>());
  const int row = lane & 15;
  const bool live = !CAL || row_live[row];
#pragma unroll
  for (int jj = 0; jj < HT; ++jj) {
    const int col0 = (wave * HT + jj) * 16 + 4 * (lane >> 4);
    T e[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float hv = activation<P>(hacc[jj][i], col0 + i, wt.hid_b, wt.hid_ws, hrelu);
      if constexpr (CAL)
        if (live) cal_max(cal, Net::D + Net::CH1 + Net::CH2 + Net::CH3 + col0 + i, hv);
      e[i] = to_storage<P>(hv, col0 + i, wt.hid_ai);
    }
    store_run<4 * sizeof(T)>(hb + row * SH + col0, e);
  }
  __syncthreads();
  if (wave < NTL) {
    const T* const ap[1] = {hb + row * SH + (P::KG / 4) * (lane >> 4)};
    v4f acc[1][1] = {{v4f{0.f, 0.f, 0.f, 0.f}}};
    mma_stream<P, Net::HID / P::KG, NTL, 1, 1>(acc, ap, static_cast<const uint4*>(wt.last_p),
                                               wave, lane);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int col = wave * 16 + 4 * (lane >> 4) + i;
      if (col < Net::NOUT) sm.logit[row][col] = acc[0][0][i] + wt.last_b[col];
    }
  }
}

// The whole predictor on one tile of MT windows.  The window arrives a group
// of NG blocks (NG*BS slots) at a time: load(j0, nb) requests the rows of
// blocks j0 .. j0+nb-1 into registers, commit(j0, nb, regs, X) writes them,
// in storage precision, to X at window s, slot t of the group, feature c
// (slot pairs padded, see Geo).
// The next group's rows are requested after the current group's conv levels
// and committed before its FC, so their memory latency is hidden.  Both are
// called by all threads; the raw outputs land in sm.logit.  CAL: also record
// per-channel max |input| of every layer into cal (offsets: window D, conv1
// out, conv2 out[, conv3 out, hidden out]), counting only tile rows whose
// row_live[s] is set.  TRUNK: the convolutions only, the last conv's
// output written to sv.a3 (nothing in sm.logit).
template <class Net, class P, bool CAL = false, bool SAVE = false, bool TRUNK = false, class Load,
          class Commit>
__device__ __forceinline__ void predict_tile(const DevWeights& wt, uint32_t relu_mask,
                                             NetSmem<Net, P>& sm, Load&& load, Commit&& commit,
                                             unsigned* cal = nullptr,
                                             const int* row_live = nullptr,
                                             SavePtrs<typename P::T> sv = {}) {
  using G = Geo<Net, P>;
  using T = typename P::T;
  constexpr int NG = G::NG, NFULL = Net::NB / NG, TAIL = Net::NB % NG;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  constexpr int HT = Net::HID > 0 ? (Net::HID / 16) / Net::WAVES : 1;
  v4f hacc[HT];
#pragma unroll
  for (int j = 0; j < HT; ++j) hacc[j] = v4f{0.f, 0.f, 0.f, 0.f};
  float fpart = 0.f;

  {
    auto regs = load(0, NFULL > 0 ? NG : TAIL);
    commit(0, NFULL > 0 ? NG : TAIL, regs, sm.x());
  }
  constexpr bool XPF = Net::NCONV == 3;  // LDS-only barriers (see run_group)
  for (int g = 0; g < NFULL; ++g) {
    if constexpr (XPF)
      lds_barrier();
    else
      __syncthreads();
    const int j0 = g * NG;
    const int nj = j0 + NG, nnb = g + 1 < NFULL ? NG : TAIL;
    run_group<Net, P, NG, CAL, SAVE, TRUNK>(
        wt, relu_mask, sm, j0, cal, row_live, sv, hacc, fpart, [&]() { return load(nj, nnb); },
        [&](const auto& regs) {
          if (nnb > 0) commit(nj, nnb, regs, sm.x());
        });
  }
  if constexpr (TAIL > 0) {
    if constexpr (XPF)
      lds_barrier();
    else
      __syncthreads();
    run_group<Net, P, TAIL, CAL, SAVE, TRUNK>(
        wt, relu_mask, sm, NFULL * NG, cal, row_live, sv, hacc, fpart, []() { return 0; },
        [](int) {});
  }
  if constexpr (TRUNK) {
    __syncthreads();
    return;
  }

  if constexpr (SAVE && Net::HID > 0) {
    // training form: the hidden layer's output is kept, the head runs as a
    // separate GEMM over the whole batch
    const bool hrelu = relu_mask & (1u << hidden_layer<Net>());
    const int row = lane & 15;
#pragma unroll
    for (int jj = 0; jj < HT; ++jj) {
      const int col0 = (wave * HT + jj) * 16 + 4 * (lane >> 4);
      T e[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        e[i] = to_storage<P>(activation<P>(hacc[jj][i], col0 + i, wt.hid_b, wt.hid_ws, hrelu),
                             col0 + i, wt.hid_ai);
      if (row < sv.rows) store_run<4 * sizeof(T)>(sv.h + (size_t)row * Net::HID + col0, e);
    }
  } else if constexpr (Net::HID > 0 && Net::HEAD == 1) {
    hybrid_head<Net, P, CAL>(wt, relu_mask, sm, hacc, cal, row_live);
  } else if constexpr (Net::HID > 0) {
    // bias + ReLU on the hidden layer, rounding to the form's precision, then
    // the final FC: lane l holds row l % 16 and 4 columns of each of its HT
    // tiles; reduce over the 4 lanes sharing the row, then over waves.
    const bool hrelu = relu_mask & (1u << hidden_layer<Net>());
    const int row = lane & 15;
    const bool live = !CAL || row_live[row];
    float p[Net::NOUT];
#pragma unroll
    for (int o = 0; o < Net::NOUT; ++o) p[o] = 0.f;
#pragma unroll
    for (int jj = 0; jj < HT; ++jj) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int col = (wave * HT + jj) * 16 + 4 * (lane >> 4) + i;
        const float hv = activation<P>(hacc[jj][i], col, sm.hb, sm.hws, hrelu);
        if constexpr (CAL)
          if (live) cal_max(cal, Net::D + Net::CH1 + Net::CH2 + Net::CH3 + col, hv);
        const float h = P::val(to_storage<P>(hv, col, sm.hai));
#pragma unroll
        for (int o = 0; o < Net::NOUT; ++o) p[o] = fmaf(h, sm.lw[o * Net::HID + col], p[o]);
      }
    }
#pragma unroll
    for (int o = 0; o < Net::NOUT; ++o) {
      float v = p[o];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (lane < 16) sm.red()[(wave * MT + row) * Net::NOUT + o] = v;
    }
    __syncthreads();
    if (tid < MT * Net::NOUT) {
      const int s = tid / Net::NOUT, o = tid % Net::NOUT;
      float v = 0.f;
#pragma unroll
      for (int w = 0; w < Net::WAVES; ++w) v += sm.red()[(w * MT + s) * Net::NOUT + o];
      v += sm.lb[o];
      if (relu_mask & (1u << (hidden_layer<Net>() + 1))) v = fmaxf(v, 0.f);
      sm.logit[s][o] = v;
    }
  } else {
    constexpr int LPP = G::NT / (MT * Net::NOUT);
    const int fpair = tid / LPP, fsub = tid % LPP;
    const int fs = fpair / Net::NOUT, fo = fpair % Net::NOUT;
#pragma unroll
    for (int m = 1; m < LPP; m <<= 1) fpart += __shfl_xor(fpart, m);
    if (fsub == 0) {
      float v = fpart + wt.last_b[fo];
      if (relu_mask & (1u << Net::NCONV)) v = fmaxf(v, 0.f);
      sm.logit[fs][fo] = v;
    }
  }
  __syncthreads();
}

// One thread's share of a window row: CPT consecutive features from column
// c0.  FP8: the features' input scales are applied (xs: reciprocals by
// feature, in LDS).
template <class P, int CPT, int D>
__device__ __forceinline__ void window_elems(const float (&v)[CPT], const float* xs, int c0,
                                             typename P::T (&e)[CPT]) {
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    float x = v[i];
    if constexpr (P::SCALED) x *= xs[c0 + i < D ? c0 + i : 0];
    e[i] = P::cvt(x);
  }
}

// Registers carrying one thread's share of one window row between load and
// commit: FP32 feature pairs, or (H) BF16 feature pairs in one word each.
template <int CPT, bool H = false>
struct RowRegs {
  typename std::conditional<H, uint32_t, float2>::type v[CPT / 2];
  uint32_t code;
  float res, ex, sto;
  int valid;
  uint2 mem, cur_mem;  // dependency flags: this row's and slot 0's addresses
};

// The five memory dependency flags of a context instruction with addresses
// m against the current instruction's c (Sec. 2.1): same instruction cache
// line, same instruction page, same data address, data cache line, data
// page (64-byte lines, 4 KB pages; data flags need both addresses).
__device__ __forceinline__ float dep_flag(uint2 m, uint2 c, int f) {
  const bool both = m.y != 0u && c.y != 0u;
  switch (f) {
    case 0: return (m.x >> 6) == (c.x >> 6) ? 1.f : 0.f;
    case 1: return (m.x >> 12) == (c.x >> 12) ? 1.f : 0.f;
    case 2: return both && m.y == c.y ? 1.f : 0.f;
    case 3: return both && (m.y >> 6) == (c.y >> 6) ? 1.f : 0.f;
    default: return both && (m.y >> 12) == (c.y >> 12) ? 1.f : 0.f;
  }
}

// Rounded latency in cycles: nearest, ties to even; non-finite -> 0;
// clamped to [0, lat_max].
__device__ __forceinline__ int32_t round_latency(float v, int32_t lat_max, uint32_t& clamped,
                                                 uint32_t& nonfinite) {
  if (!isfinite(v)) {
    ++nonfinite;
    return 0;
  }
  const float r = rintf(v);
  if (r < 0.f) {
    ++clamped;
    return 0;
  }
  if (r > (float)lat_max) {
    ++clamped;
    return lat_max;
  }
  return (int32_t)r;
}

// Execution and store latency (each at most 65535) in one 32-bit word.
__device__ __forceinline__ int32_t pack_es(int32_t e, int32_t s) {
  return (int32_t)((uint32_t)e | ((uint32_t)s << 16));
}

// Hybrid head (Sec. 2.3): the most probable class (the first of equal
// scores; a NaN score never wins) is the latency, unless it is the last
// class ("larger"), which takes the direct output z[HYB_CLASSES], rounded.
__device__ __forceinline__ int32_t hybrid_latency(const float* z, int32_t lat_max,
                                                  uint32_t& clamped, uint32_t& nonfinite) {
  int best = 0;
#pragma unroll
  for (int c = 1; c < HYB_CLASSES; ++c)
    if (z[c] > z[best]) best = c;
  if (best < HYB_CLASSES - 1) return best;
  return round_latency(z[HYB_CLASSES], lat_max, clamped, nonfinite);
}

template <class Net, class P>
struct StepSmem {
  static constexpr int CM = Net::MWQ ? Net::C : 1;
  NetSmem<Net, P> net;
  int32_t q_idx[MT][Net::C];
  int32_t q_e[MT][Net::C];
  int64_t q_t[MT][Net::C];
  int64_t q_r[MT][Net::C];
  int64_t rw[MT][WMAX];
  int64_t cur[MT], t_w[MT], r_prev[MT], pos[MT], first[MT], n_pos[MT], pred_off[MT];
  int32_t head[MT], count[MT], warm[MT], active[MT], kid[MT];
  // stores (store latencies only), as in DevState
  int32_t m_idx[MT][CM];
  int32_t m_es[MT][CM];
  int64_t m_t[MT][CM];
  int64_t m_r[MT][CM];
  int64_t m_x[MT][CM];
  int32_t m_head[MT], m_count[MT], m_inpq[MT];
  int64_t x_prev[MT];
};

// Slot s of the tile takes sub-trace k: its scalars come from the global
// state (the reset state for a sub-trace that has not started).
template <class SM>
__device__ __forceinline__ void load_slot(SM& sm, int s, int k, const DevState& st, int W) {
  sm.kid[s] = k;
  if (k < 0) {
    sm.active[s] = 0;
    return;
  }
  sm.cur[s] = st.cur[k];
  sm.t_w[s] = st.t_w[k];
  sm.r_prev[s] = st.r_prev[k];
  sm.pos[s] = st.pos[k];
  sm.first[s] = st.first[k];
  sm.n_pos[s] = st.n_pos[k];
  sm.pred_off[s] = st.pred_off[k];
  sm.head[s] = st.head[k];
  sm.count[s] = st.count[k];
  sm.warm[s] = st.warm[k];
  if (st.m_head) {
    sm.m_head[s] = st.m_head[k];
    sm.m_count[s] = st.m_count[k];
    sm.m_inpq[s] = st.m_inpq[k];
    sm.x_prev[s] = st.x_prev[k];
  }
  for (int i = 0; i < W; ++i) sm.rw[s][i] = st.rw[(size_t)k * WMAX + i];
  sm.active[s] = sm.pos[s] < sm.n_pos[s];
}

// Next unstarted sub-trace in claim order (longest first), or -1.
__device__ __forceinline__ int claim_subtrace(const DevState& st, int n_sub) {
  const unsigned q = atomicAdd(st.next, 1u);
  return q < (unsigned)n_sub ? st.order[q] : -1;
}

// Feature c of an instruction given as a packed code (trace encoding
// SIM_FEAT_CODE32): op class one-hot [0,5), three register ids one-hot in 7
// buckets each [5,26), data level one-hot [26,29), mispredict flag [29].
__device__ __forceinline__ float code_feature(uint32_t code, int c) {
  if (c < 5) return (int)(code & 7u) == c ? 1.f : 0.f;
  if (c < 26) {
    const int r = (c - 5) / 7, b = (c - 5) % 7;
    const int id = (int)((code >> (3 + 5 * r)) & 31u);
    return (id * 7) >> 5 == b ? 1.f : 0.f;
  }
  if (c < 29) return (int)((code >> 18) & 3u) == c - 26 ? 1.f : 0.f;
  if (c == 29) return (float)((code >> 20) & 1u);
  return 0.f;
}

template <class Net>
constexpr int n_cal() {
  return Net::D + Net::CH1 + Net::CH2 + Net::CH3 + Net::HID;
}

// BF16 copy of an FP32 trace for the BF16 form: row i's D features rounded
// to BF16 (nearest even, as the window conversion does), then zeros to DS.
__global__ void stage_bf16_kernel(const float* __restrict__ feat, int64_t n, int D, int DS,
                                  uint16_t* __restrict__ out) {
  const int64_t total = n * DS;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / DS;
    const int c = (int)(i - r * DS);
    out[i] = c < D ? PBF16::cvt(feat[r * D + c]) : (uint16_t)0;
  }
}

hipError_t launch_stage_bf16(const float* feat, int64_t n, int D, uint16_t* out,
                             hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(stage_bf16_kernel, dim3(2048), dim3(256), 0, stream, feat, n, D,
                     staged_feat(D), out);
  return hipGetLastError();
}

// DEP: the window carries the memory dependency flags (a separate
// instantiation, so that runs without them pay no registers for them).
// STAGE (networks run as separate kernels per step, one step per launch):
// 1 = gather and convolutions only, the last conv's output to p.trunk_out
// and each slot's activity to p.active_out, the state not advanced;
// 2 = the update from the raw outputs in p.ext_logits, no gather.
template <class Net, class P, bool RUN_NET, bool CAL = false, bool DEP = false, int STAGE = 0>
__global__ void __launch_bounds__(Net::WAVES * 64)
    step_kernel(DevWeights wt, uint32_t relu_mask, DevState st, StepParams p) {
  using G = Geo<Net, P>;
  using T = typename P::T;
  constexpr int C = Net::C, NT = G::NT, D = Net::D, DP = G::DP, BS = Net::BS;
  __shared__ StepSmem<Net, P> sm;
  __shared__ unsigned cal[CAL ? n_cal<Net>() : 1];
  const int tid = threadIdx.x;
  const int slot0 = blockIdx.x * MT;
  if constexpr (CAL)
    for (int i = tid; i < n_cal<Net>(); i += NT) cal[i] = 0u;

  // Work queue: a slot keeps its sub-trace across launches; an empty slot
  // claims the next unstarted sub-trace (longest first).  Results are
  // indexed by sub-trace, so they do not depend on which slot runs it.
  if (tid < MT) {
    int k = st.slot_kid[slot0 + tid];
    if (k < 0) k = claim_subtrace(st, p.n_sub);
    load_slot(sm, tid, k, st, p.W);
  }
  if constexpr (RUN_NET) sm.net.stage_head(wt, tid, NT);
  __syncthreads();
  for (int i = tid; i < MT * C; i += NT) {
    const int s = i / C, e = i % C, k = sm.kid[s];
    if (k >= 0) {
      const size_t g = (size_t)k * C + e;
      sm.q_idx[s][e] = st.q_idx[g];
      sm.q_e[s][e] = st.q_e[g];
      sm.q_t[s][e] = st.q_t[g];
      sm.q_r[s][e] = st.q_r[g];
      if constexpr (Net::MWQ) {
        sm.m_idx[s][e] = st.m_idx[g];
        sm.m_es[s][e] = st.m_es[g];
        sm.m_t[s][e] = st.m_t[g];
        sm.m_r[s][e] = st.m_r[g];
        sm.m_x[s][e] = st.m_x[g];
      }
    }
  }
  uint32_t n_clamped = 0, n_nonfinite = 0, n_mismatch = 0, n_pred = 0;

  // Window gather: TPR threads per (sub-trace, slot-of-the-group) row, CPT
  // features each.
  constexpr int GSL = G::NG * BS;
  constexpr int ROWS = MT * GSL, TPR = NT / ROWS, CPT = DP / TPR;
  static_assert(NT % ROWS == 0 && DP % TPR == 0 && CPT % 2 == 0 && D % 2 == 0, "gather split");
  // the BF16 form reads rows of a BF16 copy of the trace (DS features each)
  constexpr bool H16 = P::ID == 1;
  constexpr int DS = staged_feat(D);
  static_assert(!H16 || (CPT % 8 == 0 && DS % 8 == 0), "BF16 rows");
  const int grow = tid / TPR, part = tid % TPR;
  const int gs = grow / GSL, gt = grow % GSL;
  if constexpr (P::SCALED)
    for (int c = tid; c < D; c += NT) sm.net.x_inv[c] = wt.x_inv[c];
  // load(j0, nb): the row's trace index from the queue ring, then the row's
  // features requested (every address in bounds, so all are in flight
  // together); commit: dynamic columns, conversion, one vector store.
  auto load = [&](int j0, int nb) {
    RowRegs<CPT, H16> r;
    const int w = j0 * BS + gt;
    int64_t idx = -1;
    r.res = 0.f;
    r.ex = 0.f;
    r.sto = 0.f;
    if (gt < nb * BS && sm.active[gs]) {
      if (w == 0) {
        idx = sm.first[gs] + sm.pos[gs];
      } else if (w <= sm.count[gs]) {  // processor queue, newest first
        int e = sm.head[gs] + sm.count[gs] - w;
        e = e >= C ? e - C : e;
        idx = sm.q_idx[gs][e];
        r.res = (float)(sm.cur[gs] - sm.q_t[gs][e]);
        const int32_t es = sm.q_e[gs][e];
        r.ex = (float)(Net::MWQ ? es & 0xffff : es);
        if (Net::MWQ) r.sto = (float)((uint32_t)es >> 16);
      } else if (Net::MWQ && w <= sm.count[gs] + sm.m_count[gs] - sm.m_inpq[gs]) {
        // then the memory write queue, newest first: the stores that have
        // left the processor queue and not this one
        int e = sm.m_head[gs] + sm.m_count[gs] - sm.m_inpq[gs] - (w - sm.count[gs]);
        e = e >= C ? e - C : e;
        idx = sm.m_idx[gs][e];
        r.res = (float)(sm.cur[gs] - sm.m_t[gs][e]);
        r.ex = (float)(sm.m_es[gs][e] & 0xffff);
        r.sto = (float)((uint32_t)sm.m_es[gs][e] >> 16);
      }
    }
    r.valid = idx >= 0;
    r.code = 0;
    if constexpr (DEP) {  // addresses of this row and of slot 0 (broadcast)
      r.mem = p.mem[idx < 0 ? 0 : idx];
      r.cur_mem = p.mem[sm.active[gs] ? sm.first[gs] + sm.pos[gs] : 0];
      if (w == 0) r.valid = idx >= 0 ? 2 : 0;  // slot 0: no flags
    }
    if (p.codes) {
      r.code = p.codes[idx < 0 ? 0 : idx];
    } else if constexpr (H16) {
      // BF16 rows of DS features (16-byte aligned): whole 16-byte chunks
      const uint4* src = reinterpret_cast<const uint4*>(p.feat16 + (idx < 0 ? 0 : idx) * DS);
#pragma unroll
      for (int q = 0; q < CPT / 8; ++q) {
        const int c = part * CPT + 8 * q;
        const uint4 w = c < DS ? src[c / 8] : make_uint4(0u, 0u, 0u, 0u);
        r.v[4 * q] = w.x;
        r.v[4 * q + 1] = w.y;
        r.v[4 * q + 2] = w.z;
        r.v[4 * q + 3] = w.w;
      }
    } else {
      const float* src = p.feat + (idx < 0 ? 0 : idx) * D;
#pragma unroll
      for (int cc = 0; cc < CPT; cc += 2) {
        const int c = part * CPT + cc;
        // one thread per row: the padding columns are known at compile time
        if (TPR > 1 || cc < D)
          r.v[cc / 2] = *reinterpret_cast<const float2*>(src + (c < D ? c : D - 2));
        else
          r.v[cc / 2] = make_float2(0.f, 0.f);
      }
    }
    return r;
  };
  auto commit = [&](int j0, int nb, const RowRegs<CPT, H16>& r, T* X) {
    (void)j0;
    if (gt >= nb * BS) return;  // slots past a short group's blocks are never read
    T* dst = X + gs * G::SX + (gt >> 1) * G::RX + (gt & 1) * DP + part * CPT;
    // the row's column c, when this thread's share holds it, set to v
    auto put = [&](int c, float v) {
      if (c >= part * CPT && c < part * CPT + CPT) {
        if constexpr (P::SCALED) v *= sm.net.x_inv[c < D ? c : 0];
        dst[c - part * CPT] = P::cvt(v);
      }
    };
    // the memory dependency flags (after the other columns, as below)
    auto put_dep = [&]() {
      if constexpr (DEP)
#pragma unroll
        for (int f = 0; f < 5; ++f)
          put(p.col_dep + f, r.valid == 1 ? dep_flag(r.mem, r.cur_mem, f) : 0.f);
    };
    if constexpr (!CAL) {
      // The share written whole, then the few columns that are not copied
      // features overwritten one by one: the same values as the per-feature
      // conversion below at a fraction of its VALU work.  The BF16 form's
      // rows are stored as loaded (its BF16 copy of the trace holds exactly
      // the values the conversion would produce).
      if constexpr (H16) {
        if (!p.codes) {
#pragma unroll
          for (int q = 0; q < CPT / 8; ++q) {
            const uint4 w = r.valid ? uint4{r.v[4 * q], r.v[4 * q + 1], r.v[4 * q + 2],
                                            r.v[4 * q + 3]}
                                    : uint4{0u, 0u, 0u, 0u};
            *reinterpret_cast<uint4*>(dst + 8 * q) = w;
          }
          put(p.col_res, r.res);
          put(p.col_exe, r.ex);
          put(p.col_sto, r.sto);
          put_dep();
          return;
        }
      }
      // packed codes: zeros, then the one-hot features of code_feature
      static_assert(D >= 30, "the code's features are columns 0 .. 29");
      if constexpr ((CPT * sizeof(T)) % 16 == 0) {
        if (p.codes) {
#pragma unroll
          for (int q = 0; q < CPT * (int)sizeof(T) / 16; ++q)
            *reinterpret_cast<uint4*>(reinterpret_cast<char*>(dst) + 16 * q) =
                uint4{0u, 0u, 0u, 0u};
          if (r.valid) {
            const uint32_t code = r.code;
            if ((code & 7u) < 5u) put((int)(code & 7u), 1.f);
#pragma unroll
            for (int g = 0; g < 3; ++g)
              put(5 + 7 * g + (((int)((code >> (3 + 5 * g)) & 31u) * 7) >> 5), 1.f);
            if (((code >> 18) & 3u) < 3u) put(26 + (int)((code >> 18) & 3u), 1.f);
            if ((code >> 20) & 1u) put(29, 1.f);
          }
          put(p.col_res, r.res);
          put(p.col_exe, r.ex);
          put(p.col_sto, r.sto);
          put_dep();
          return;
        }
      }
    }
    float v[CPT];
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) {
      const int c = part * CPT + cc;
      float x = 0.f;
      if (r.valid && c < D) {
        if (p.codes)
          x = code_feature(r.code, c);
        else if constexpr (H16)
          x = __uint_as_float(cc & 1 ? r.v[cc / 2] & 0xffff0000u : r.v[cc / 2] << 16);
        else
          x = cc & 1 ? r.v[cc / 2].y : r.v[cc / 2].x;
      }
      if (c == p.col_res) x = r.res;
      if (c == p.col_exe) x = r.ex;
      if (c == p.col_sto) x = r.sto;
      if constexpr (DEP)
        if (c >= p.col_dep && c < p.col_dep + 5)
          x = r.valid == 1 ? dep_flag(r.mem, r.cur_mem, c - p.col_dep) : 0.f;
      if constexpr (CAL)
        if (c < D && r.valid) cal_max(cal, c, x);
      v[cc] = x;
    }
    T e[CPT];
    window_elems<P, CPT, D>(v, sm.net.x_inv, part * CPT, e);
    store_run<(CPT * sizeof(T)) % 16 == 0 ? 16 : 8>(dst, e);
  };

  if constexpr (STAGE == 1)
    if (tid < MT) p.active_out[slot0 + tid] = sm.active[tid];
  int any = __syncthreads_or(tid < MT ? sm.active[tid] : 0);

  for (int it = 0; it < p.n_steps && any; ++it) {
    if constexpr (RUN_NET && STAGE == 1) {
      SavePtrs<T> sv{};
      sv.a3 = static_cast<T*>(p.trunk_out) + (size_t)slot0 * Net::NB * Net::CH3;
      sv.rows = MT;
      predict_tile<Net, P, false, true, true>(wt, relu_mask, sm.net, load, commit, nullptr,
                                              nullptr, sv);
      break;  // the update is a separate launch
    } else if constexpr (RUN_NET && STAGE == 0) {
      predict_tile<Net, P, CAL>(wt, relu_mask, sm.net, load, commit, cal, sm.active);
    }

    if (tid < MT && sm.active[tid]) {
      const int s = tid, k = sm.kid[s];
      const int64_t pos = sm.pos[s];
      const int64_t g = sm.pred_off[s] + pos;
      int32_t lat[Net::NLAT];
      if (RUN_NET) {
        const float* z = STAGE == 2 ? p.ext_logits + (size_t)(slot0 + s) * Net::NOUT
                                    : sm.net.logit[s];
        if (p.logits_out)
          for (int o = 0; o < Net::NOUT; ++o) p.logits_out[g * Net::NOUT + o] = z[o];
#pragma unroll
        for (int o = 0; o < Net::NLAT; ++o) {
          if constexpr (Net::HEAD == 1)
            lat[o] = hybrid_latency(z + o * HYB_PER_TYPE, p.lat_max, n_clamped, n_nonfinite);
          else
            lat[o] = round_latency(z[o], p.lat_max, n_clamped, n_nonfinite);
        }
      }
      ++n_pred;  // positions advanced (the work a launch did)
      if (p.lat_mode != 0) {
#pragma unroll
        for (int o = 0; o < Net::NLAT; ++o) {
          const int32_t inj = p.lat_table[g * Net::NLAT + o];
          if (RUN_NET && inj != lat[o]) ++n_mismatch;
          lat[o] = inj;
        }
      }
      const int64_t Tn = sm.cur[s] + lat[0];
      int head = sm.head[s], count = sm.count[s];
      while (count > 0 && sm.q_r[s][head] <= Tn) {  // retired by Tn: a prefix (r is monotone)
        head = head + 1 == C ? 0 : head + 1;
        --count;
      }
      int64_t r = Tn + lat[1] + 1;
      r = r > sm.r_prev[s] ? r : sm.r_prev[s];
      const int wi = (int)(pos % p.W);
      if (pos >= p.W) {
        const int64_t rb = sm.rw[s][wi] + 1;
        r = r > rb ? r : rb;
      }
      sm.rw[s][wi] = r;
      int slot = head + count;
      slot = slot >= C ? slot - C : slot;
      if (count == C) {
        head = head + 1 == C ? 0 : head + 1;  // only the newest C stay visible
      } else {
        ++count;
      }
      const int64_t ii = sm.first[s] + pos;
      sm.q_idx[s][slot] = (int32_t)ii;
      // store latencies: E and S packed as 16-bit halves (lat_max <= 65535)
      sm.q_e[s][slot] = Net::MWQ ? pack_es(lat[1], lat[Net::NLAT - 1]) : lat[1];
      sm.q_t[s][slot] = Tn;
      sm.q_r[s][slot] = r;
      int64_t final_t = r;
      if constexpr (Net::MWQ) {
        // memory write queue (Sec. 3.2): a store enters it when it leaves
        // the processor queue (r) and leaves, in order, once its residence
        // exceeds its store latency: x = max(T + S + 1, r, previous x)
        int mh = sm.m_head[s], mc = sm.m_count[s];
        while (mc > 0 && sm.m_x[s][mh] <= Tn) {  // gone by Tn: a prefix (x is monotone)
          mh = mh + 1 == C ? 0 : mh + 1;
          --mc;
        }
        const bool is_store = p.codes ? code_feature(p.codes[ii], p.store_col) != 0.f
                                      : p.feat[ii * Net::D + p.store_col] != 0.f;
        if (is_store) {
          int64_t x = Tn + lat[2] + 1;
          x = x > r ? x : r;
          x = x > sm.x_prev[s] ? x : sm.x_prev[s];
          sm.x_prev[s] = x;
          int ms = mh + mc;
          ms = ms >= C ? ms - C : ms;
          if (mc == C) {
            mh = mh + 1 == C ? 0 : mh + 1;  // the newest C stores suffice for the window
          } else {
            ++mc;
          }
          sm.m_idx[s][ms] = (int32_t)ii;
          sm.m_es[s][ms] = pack_es(lat[1], lat[2]);
          sm.m_t[s][ms] = Tn;
          sm.m_r[s][ms] = r;
          sm.m_x[s][ms] = x;
        }
        // the newest stores still in the processor queue at Tn (r > Tn)
        int q = 0;
        while (q < mc) {
          int e = mh + mc - 1 - q;
          e = e >= C ? e - C : e;
          if (sm.m_r[s][e] <= Tn) break;
          ++q;
        }
        sm.m_head[s] = mh;
        sm.m_count[s] = mc;
        sm.m_inpq[s] = q;
        final_t = r > sm.x_prev[s] ? r : sm.x_prev[s];
      }
      sm.head[s] = head;
      sm.count[s] = count;
      sm.r_prev[s] = r;
      sm.cur[s] = Tn;
      sm.pos[s] = pos + 1;
      if (pos + 1 == sm.warm[s]) sm.t_w[s] = Tn;
      if (pos + 1 == sm.n_pos[s]) {  // last instruction: the drain ends (Eq. 1)
        st.fetch[k] = Tn - sm.t_w[s];
        st.drain[k] = final_t - Tn;
        st.final_tick[k] = final_t;
        st.warm_tick[k] = sm.t_w[s];
        st.pos[k] = pos + 1;
        st.cur[k] = Tn;
        // the finished sub-trace leaves the batch; the slot takes the next
        load_slot(sm, s, claim_subtrace(st, p.n_sub), st, p.W);
      }
    }
    any = __syncthreads_or(tid < MT ? sm.active[tid] : 0);
  }

  // (stage 1 leaves the state as it found it, apart from the slots' claims)
  if (tid < MT) {
    const int k = sm.kid[tid];
    st.slot_kid[slot0 + tid] = k;
    if (STAGE != 1 && k >= 0) {
      st.cur[k] = sm.cur[tid];
      st.t_w[k] = sm.t_w[tid];
      st.r_prev[k] = sm.r_prev[tid];
      st.pos[k] = sm.pos[tid];
      st.head[k] = sm.head[tid];
      st.count[k] = sm.count[tid];
      if constexpr (Net::MWQ) {
        st.m_head[k] = sm.m_head[tid];
        st.m_count[k] = sm.m_count[tid];
        st.m_inpq[k] = sm.m_inpq[tid];
        st.x_prev[k] = sm.x_prev[tid];
      }
      for (int i = 0; i < p.W; ++i) st.rw[(size_t)k * WMAX + i] = sm.rw[tid][i];
    }
    if (n_clamped) atomicAdd(&st.counters[0], (unsigned long long)n_clamped);
    if (n_nonfinite) atomicAdd(&st.counters[1], (unsigned long long)n_nonfinite);
    if (n_mismatch) atomicAdd(&st.counters[2], (unsigned long long)n_mismatch);
    if (n_pred) atomicAdd(&st.counters[3], (unsigned long long)n_pred);
  }
  if constexpr (CAL) {
    __syncthreads();
    for (int i = tid; i < n_cal<Net>(); i += NT)
      if (cal[i]) atomicMax(p.cal_out + i, cal[i]);
  }
  for (int i = tid; i < MT * C && STAGE != 1; i += NT) {
    const int s = i / C, e = i % C, k = sm.kid[s];
    if (k >= 0) {
      const size_t g = (size_t)k * C + e;
      st.q_idx[g] = sm.q_idx[s][e];
      st.q_e[g] = sm.q_e[s][e];
      st.q_t[g] = sm.q_t[s][e];
      st.q_r[g] = sm.q_r[s][e];
      if constexpr (Net::MWQ) {
        st.m_idx[g] = sm.m_idx[s][e];
        st.m_es[g] = sm.m_es[s][e];
        st.m_t[g] = sm.m_t[s][e];
        st.m_r[g] = sm.m_r[s][e];
        st.m_x[g] = sm.m_x[s][e];
      }
    }
  }
}

// ------------------------------------------ one wavefront per sub-trace ---
// The small network (16-slot windows of 32 features, conv 32 -> 32 -> 64,
// FC 256 -> 2) when a run has few sub-traces, so that the time of one step,
// not the throughput of many, bounds it: one wavefront (a workgroup of 64
// threads, one sub-trace slot) per sub-trace, no barrier between waves.
// The weights a lane needs stay in its registers for the whole launch; the
// window and the conv1 output pass through 3 KB of LDS; the products are
// VALU FMAs (a prediction is 33 k multiply-adds, ~520 cycles of one SIMD);
// the final FC is a lane reduction, so every lane holds the logits, and the
// clock and queue update runs on wave-uniform values, the retired prefix of
// the queue counted by one ballot over its entries (their retire times are
// non-decreasing along the queue).  The barriers order LDS only, so the next
// instruction's row, requested at the top of a step, stays in flight
// across them.  FP32 form, row or packed-code traces.
// Same state, work queue and results as step_kernel.
constexpr int WV_D = NetSmall::D, WV_C = NetSmall::C, WV_L = NetSmall::L;
constexpr int WV_C1 = NetSmall::CH1, WV_C2 = NetSmall::CH2, WV_NB = NetSmall::NB;

// Element B[k][n] of a weight matrix packed by the FP32 form (k-groups of
// 16, n-tiles of 16, lane = 16 * ((k % 16) / 4) + n % 16, 4 k per lane).
__device__ __forceinline__ float packed_f32(const float* Bp, int N, int k, int n) {
  const int kg = k >> 4, w = k & 15;
  return Bp[((((size_t)kg * (N >> 4) + (n >> 4)) * 64 + ((w >> 2) << 4) + (n & 15)) << 2) +
            (w & 3)];
}

template <bool RUN_NET>
__global__ void __launch_bounds__(64) wave_step_kernel(DevWeights wt, uint32_t relu_mask,
                                                       DevState st, StepParams p) {
  __shared__ __attribute__((aligned(16))) float x[WV_L][WV_D];        // the window
  __shared__ __attribute__((aligned(16))) float a1[WV_L / 2][WV_C1];  // conv1 output
  __shared__ int32_t q_e[WV_C];               // the queue ring
  __shared__ int64_t q_t[WV_C], q_r[WV_C];
  __shared__ int64_t rw[WMAX];                // retire times of the last W instructions
  __shared__ int claimed;
  const int lane = threadIdx.x, slot = blockIdx.x;
  constexpr int D = WV_D, C = WV_C;
  const int W = p.W;

  // weights this lane uses, kept in registers: conv1 output channel lane % 32
  // (its positions: lane / 32, +2, +4, +6), conv2 output channel lane, the
  // final FC's weights of conv2 channel lane at the 4 positions
  float w1[2][D], w2[2][WV_C1], wf[WV_NB][2];
  float b1 = 0.f, b2 = 0.f, bl[2] = {0.f, 0.f};
  const int c1 = lane & (WV_C1 - 1), half = lane >> 5;
  if (RUN_NET) {
    const float* W1 = static_cast<const float*>(wt.conv_w[0]);
    const float* W2 = static_cast<const float*>(wt.conv_w[1]);
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int c = 0; c < D; ++c) w1[t][c] = packed_f32(W1, WV_C1, t * D + c, c1);
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int c = 0; c < WV_C1; ++c) w2[t][c] = packed_f32(W2, WV_C2, t * WV_C1 + c, lane);
#pragma unroll
    for (int j = 0; j < WV_NB; ++j)
#pragma unroll
      for (int o = 0; o < 2; ++o) wf[j][o] = wt.last_w[((size_t)j * 2 + o) * WV_C2 + lane];
    b1 = wt.conv_b[0][c1];
    b2 = wt.conv_b[1][lane];
    bl[0] = wt.last_b[0];
    bl[1] = wt.last_b[1];
  }

  // the slot's sub-trace (a finished or empty slot claims the next one)
  int k = st.slot_kid[slot];
  if (k < 0) {
    if (lane == 0) claimed = claim_subtrace(st, p.n_sub);
    __syncthreads();
    k = claimed;
  }
  int64_t cur = 0, t_w = 0, r_prev = 0, pos = 0, first = 0, n_pos = 0, pred_off = 0;
  int32_t head = 0, count = 0, warm = 0;
  auto load_state = [&]() {
    if (k < 0) return;
    cur = st.cur[k];
    t_w = st.t_w[k];
    r_prev = st.r_prev[k];
    pos = st.pos[k];
    first = st.first[k];
    n_pos = st.n_pos[k];
    pred_off = st.pred_off[k];
    head = st.head[k];
    count = st.count[k];
    warm = st.warm[k];
    if (lane < C) {
      const size_t g = (size_t)k * C + lane;
      q_e[lane] = st.q_e[g];
      q_t[lane] = st.q_t[g];
      q_r[lane] = st.q_r[g];
    }
    if (lane < W) rw[lane] = st.rw[(size_t)k * WMAX + lane];
    lds_barrier();
  };
  // the window's static rows stay in registers: lane (slot w, 8 features)
  // holds trace row i - w; a step shifts them one slot (4 lanes) and takes
  // the next instruction's row, requested a step ahead, into slot 0
  const int ws = lane >> 2, wc = (lane & 3) * 8;
  float rowv[8];
  auto row_of = [&](int64_t row, float (&v)[8]) {
    if (p.codes) {
      const uint32_t code = p.codes[row];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = code_feature(code, wc + e);
    } else {
      const float4* src = reinterpret_cast<const float4*>(p.feat + row * D + wc);
      const float4 lo = src[0], hi = src[1];
      v[0] = lo.x; v[1] = lo.y; v[2] = lo.z; v[3] = lo.w;
      v[4] = hi.x; v[5] = hi.y; v[6] = hi.z; v[7] = hi.w;
    }
  };
  auto load_rows = [&]() {  // rows i - w that belong to the sub-trace
#pragma unroll
    for (int e = 0; e < 8; ++e) rowv[e] = 0.f;
    if (RUN_NET && k >= 0 && pos < n_pos && ws <= pos) row_of(first + pos - ws, rowv);
  };
  load_state();
  load_rows();
  uint32_t n_clamped = 0, n_nonfinite = 0, n_mismatch = 0, n_pred = 0;

  for (int it = 0; it < p.n_steps && k >= 0 && pos < n_pos; ++it) {
    const int64_t i = first + pos, g = pred_off + pos;
    float z[2] = {0.f, 0.f};
    float nxt[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // row i + 1 (slot 0), next step
    if (RUN_NET && ws == 0 && pos + 1 < n_pos) row_of(i + 1, nxt);
    if (RUN_NET) {
      // window: lane = (slot w, 8 features): the current instruction with
      // zero dynamic columns, then the queue newest first (instructions
      // i-1, i-2, ...: the queue holds consecutive ones), zeros past it
      {
        const int w = ws, c0 = wc;
        float res = 0.f, ex = 0.f;
        bool valid = w == 0;
        if (w >= 1 && w <= count) {
          int e = head + count - w;
          e = e >= C ? e - C : e;
          res = (float)(cur - q_t[e]);
          ex = (float)q_e[e];
          valid = true;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int c = c0 + e;
          float v = valid ? rowv[e] : 0.f;
          if (c == p.col_res) v = res;
          if (c == p.col_exe) v = ex;
          if (c == p.col_sto) v = 0.f;
          x[w][c] = v;
        }
      }
      lds_barrier();
      // conv1 (kernel 2, stride 2): channel c1 at positions half, half+2, ...
#pragma unroll
      for (int j = 0; j < WV_L / 4; ++j) {
        const int q = half + 2 * j;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int c = 0; c < D; c += 4) {
            const float4 xv = *reinterpret_cast<const float4*>(&x[2 * q + t][c]);
            acc[0] = fmaf(w1[t][c], xv.x, acc[0]);
            acc[1] = fmaf(w1[t][c + 1], xv.y, acc[1]);
            acc[2] = fmaf(w1[t][c + 2], xv.z, acc[2]);
            acc[3] = fmaf(w1[t][c + 3], xv.w, acc[3]);
          }
        float v = b1 + ((acc[0] + acc[1]) + (acc[2] + acc[3]));
        if (relu_mask & 1u) v = fmaxf(v, 0.f);
        a1[q][c1] = v;
      }
      lds_barrier();
      // conv2: channel lane at positions 0..3, then the final FC's share
      float part[2] = {0.f, 0.f};
#pragma unroll
      for (int q = 0; q < WV_NB; ++q) {
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int c = 0; c < WV_C1; c += 4) {
            const float4 av = *reinterpret_cast<const float4*>(&a1[2 * q + t][c]);
            acc[0] = fmaf(w2[t][c], av.x, acc[0]);
            acc[1] = fmaf(w2[t][c + 1], av.y, acc[1]);
            acc[2] = fmaf(w2[t][c + 2], av.z, acc[2]);
            acc[3] = fmaf(w2[t][c + 3], av.w, acc[3]);
          }
        float v = b2 + ((acc[0] + acc[1]) + (acc[2] + acc[3]));
        if (relu_mask & 2u) v = fmaxf(v, 0.f);
        part[0] = fmaf(wf[q][0], v, part[0]);
        part[1] = fmaf(wf[q][1], v, part[1]);
      }
      // the final FC: sum over the 64 channels (a fixed butterfly)
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        float v = part[o];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
        v += bl[o];
        if (relu_mask & 4u) v = fmaxf(v, 0.f);
        z[o] = v;
      }
    }
    // round, or take the injected latencies
    int32_t lat[2];
    if (RUN_NET) {
      if (p.logits_out && lane == 0)
        for (int o = 0; o < 2; ++o) p.logits_out[g * 2 + o] = z[o];
#pragma unroll
      for (int o = 0; o < 2; ++o) lat[o] = round_latency(z[o], p.lat_max, n_clamped, n_nonfinite);
    }
    ++n_pred;
    if (p.lat_mode != 0) {
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        const int32_t inj = p.lat_table[g * 2 + o];
        if (RUN_NET && inj != lat[o]) ++n_mismatch;
        lat[o] = inj;
      }
    }
    // clock and queue (Sec. 3.2): T = cur + F; the queue's retired prefix
    // (r <= T) leaves; r = max(T + E + 1, r_prev, r_{i-W} + 1); push
    const int64_t Tn = cur + lat[0];
    {
      bool gone = false;
      if (lane < count) {
        int e = head + lane;
        e = e >= C ? e - C : e;
        gone = q_r[e] <= Tn;
      }
      const int n_gone = __popcll(__ballot(gone));
      head += n_gone;
      head = head >= C ? head - C : head;
      count -= n_gone;
    }
    int64_t r = Tn + lat[1] + 1;
    r = r > r_prev ? r : r_prev;
    const int wi = (int)(pos % W);
    if (pos >= W) {
      const int64_t rb = rw[wi] + 1;
      r = r > rb ? r : rb;
    }
    int sl = head + count;
    sl = sl >= C ? sl - C : sl;
    if (count == C) {
      head = head + 1 == C ? 0 : head + 1;  // only the newest C stay visible
    } else {
      ++count;
    }
    lds_barrier();  // every lane has read the ring and rw for this step
    if (lane == 0) {
      rw[wi] = r;
      q_e[sl] = lat[1];
      q_t[sl] = Tn;
      q_r[sl] = r;
    }
    r_prev = r;
    cur = Tn;
    ++pos;
    if (pos == warm) t_w = Tn;
    if (pos == n_pos) {  // the drain ends (Eq. 1); the slot takes the next sub-trace
      if (lane == 0) {
        st.fetch[k] = Tn - t_w;
        st.drain[k] = r - Tn;
        st.final_tick[k] = r;
        st.warm_tick[k] = t_w;
        st.pos[k] = pos;
        st.cur[k] = Tn;
        claimed = claim_subtrace(st, p.n_sub);
      }
      lds_barrier();
      k = claimed;
      load_state();
      load_rows();
    } else {
      if (RUN_NET) {
        // slot w takes slot w-1's row; slot 0 the prefetched one
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float up = __shfl(rowv[e], lane >= 4 ? lane - 4 : lane);
          rowv[e] = ws == 0 ? nxt[e] : up;
        }
      }
      lds_barrier();
    }
  }

  // the slot's state back to memory
  if (lane == 0) {
    st.slot_kid[slot] = k;
    if (k >= 0) {
      st.cur[k] = cur;
      st.t_w[k] = t_w;
      st.r_prev[k] = r_prev;
      st.pos[k] = pos;
      st.head[k] = head;
      st.count[k] = count;
    }
    if (n_clamped) atomicAdd(&st.counters[0], (unsigned long long)n_clamped);
    if (n_nonfinite) atomicAdd(&st.counters[1], (unsigned long long)n_nonfinite);
    if (n_mismatch) atomicAdd(&st.counters[2], (unsigned long long)n_mismatch);
    if (n_pred) atomicAdd(&st.counters[3], (unsigned long long)n_pred);
  }
  if (k >= 0) {
    if (lane < C) {
      const size_t gq = (size_t)k * C + lane;
      st.q_idx[gq] = 0;
      st.q_e[gq] = q_e[lane];
      st.q_t[gq] = q_t[lane];
      st.q_r[gq] = q_r[lane];
    }
    if (lane < W) st.rw[(size_t)k * WMAX + lane] = rw[lane];
  }
}

// ------------------------------------------ four wavefronts per sub-trace ---
// The small network's FP32 step split over the four blocks of its kernel-2
// stride-2 tree: conv2's position j depends on window slots 4j .. 4j+3 only,
// so wave j builds those four slots, runs conv1 at positions 2j and 2j+1 and
// conv2 at position j (each wave reading only what it wrote), and multiplies
// its share of the final FC; the four partial sums meet in LDS, and every
// wave runs the same clock and queue update on the same values (wave 0
// alone writes the ring, the results and the state).  Per lane that is
// 64 + 64 multiply-adds per prediction instead of the single wave's 768.
// The ring has QR = 16 entries for the C = 15 visible ones, so a push never
// lands on an entry read in the same step and two barriers per step
// suffice: one after the partial sums, one after the push.  Each wave keeps
// the retire times of the last W instructions in a register spread over its
// lanes (lane l: the instruction with pos % W == l).  Same state, work queue
// and results as step_kernel (the ring is written back with head 0).
constexpr int QW = 4, QR = 16;
static_assert(WV_NB == QW && WV_L == 16 && WV_C < QR, "four blocks of four slots");

// LDS written by this wave and read by other lanes of it: the wave's LDS
// requests complete in order, so a compiler fence and a wait suffice
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

template <bool RUN_NET>
__global__ void __launch_bounds__(QW * 64) quad_step_kernel(DevWeights wt, uint32_t relu_mask,
                                                           DevState st, StepParams p) {
  constexpr int D = WV_D, C = WV_C;
  __shared__ __attribute__((aligned(16))) float x[QW][4][D];   // each wave's four slots
  __shared__ __attribute__((aligned(16))) float a1[QW][2][WV_C1];  // its conv1 output
  __shared__ float red[QW][2];                                   // partial sums of the final FC
  __shared__ int32_t q_e[QR];
  __shared__ int64_t q_t[QR], q_r[QR];
  __shared__ int claimed;
  const int tid = threadIdx.x, v = tid >> 6, lane = tid & 63, slot = blockIdx.x;
  const int W = p.W;

  // this lane's weights: conv1 channel lane % 32 (position 2v + lane / 32),
  // conv2 channel lane (position v), the final FC's weights of that channel
  // at position v
  const int c1 = lane & (WV_C1 - 1), pl = lane >> 5;
  float w1[2][D], w2[2][WV_C1], wf[2];
  float b1 = 0.f, b2 = 0.f, bl[2] = {0.f, 0.f};
  if (RUN_NET) {
    const float* W1 = static_cast<const float*>(wt.conv_w[0]);
    const float* W2 = static_cast<const float*>(wt.conv_w[1]);
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int c = 0; c < D; ++c) w1[t][c] = packed_f32(W1, WV_C1, t * D + c, c1);
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int c = 0; c < WV_C1; ++c) w2[t][c] = packed_f32(W2, WV_C2, t * WV_C1 + c, lane);
#pragma unroll
    for (int o = 0; o < 2; ++o) wf[o] = wt.last_w[((size_t)v * 2 + o) * WV_C2 + lane];
    b1 = wt.conv_b[0][c1];
    b2 = wt.conv_b[1][lane];
    bl[0] = wt.last_b[0];
    bl[1] = wt.last_b[1];
  }

  int k = st.slot_kid[slot];
  if (k < 0) {
    if (tid == 0) claimed = claim_subtrace(st, p.n_sub);
    __syncthreads();
    k = claimed;
  }
  int64_t cur = 0, t_w = 0, r_prev = 0, pos = 0, first = 0, n_pos = 0, pred_off = 0;
  int32_t head = 0, count = 0, warm = 0;
  int64_t rwv = 0;  // lane l < W: retire time of the last instruction with pos % W == l
  // the sub-trace's state; the ring into LDS from entry 0 (head 0)
  auto load_state = [&]() {
    if (k >= 0) {
      cur = st.cur[k];
      t_w = st.t_w[k];
      r_prev = st.r_prev[k];
      pos = st.pos[k];
      first = st.first[k];
      n_pos = st.n_pos[k];
      pred_off = st.pred_off[k];
      const int h = st.head[k];
      count = st.count[k];
      warm = st.warm[k];
      head = 0;
      if (v == 0 && lane < count) {
        int e = h + lane;
        e = e >= C ? e - C : e;
        const size_t g = (size_t)k * C + e;
        q_e[lane] = st.q_e[g];
        q_t[lane] = st.q_t[g];
        q_r[lane] = st.q_r[g];
      }
      rwv = lane < W ? st.rw[(size_t)k * WMAX + lane] : 0;
    }
    __syncthreads();
  };
  // this lane's window element pair: slot w = 4v + lane / 16, features
  // f0, f0 + 1; its trace row is instruction (first + pos) - w
  const int ls = lane >> 4, w = 4 * v + ls, f0 = (lane & 15) * 2;
  auto row_of = [&](int64_t row, float (&r)[2]) {
    if (p.codes) {
      const uint32_t code = p.codes[row];
      r[0] = code_feature(code, f0);
      r[1] = code_feature(code, f0 + 1);
    } else {
      const float2 t = *reinterpret_cast<const float2*>(p.feat + row * D + f0);
      r[0] = t.x;
      r[1] = t.y;
    }
  };
  float rowv[2] = {0.f, 0.f};
  auto load_row = [&]() {
    rowv[0] = rowv[1] = 0.f;
    if (RUN_NET && k >= 0 && pos < n_pos && w <= pos) row_of(first + pos - w, rowv);
  };
  load_state();
  load_row();
  uint32_t n_clamped = 0, n_nonfinite = 0, n_mismatch = 0, n_pred = 0;

  for (int it = 0; it < p.n_steps && k >= 0 && pos < n_pos; ++it) {
    const int64_t g = pred_off + pos;
    float nxt[2] = {0.f, 0.f};  // the next step's row for this lane
    if (RUN_NET && pos + 1 < n_pos && w <= pos + 1) row_of(first + pos + 1 - w, nxt);
    float z[2] = {0.f, 0.f};
    if (RUN_NET) {
      // window: slot 0 the current instruction with zero dynamic columns,
      // slot w >= 1 the w-th newest queued one (queue entry count - w)
      {
        float res = 0.f, ex = 0.f;
        bool valid = w == 0;
        if (w >= 1 && w <= count) {
          const int e = (head + count - w) & (QR - 1);
          res = (float)(cur - q_t[e]);
          ex = (float)q_e[e];
          valid = true;
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int c = f0 + e;
          float val = valid ? rowv[e] : 0.f;
          if (c == p.col_res) val = res;
          if (c == p.col_exe) val = ex;
          if (c == p.col_sto) val = 0.f;
          x[v][ls][c] = val;
        }
      }
      wave_lds_sync();
      // conv1: channel c1 at position 2v + pl (slots 2 pl, 2 pl + 1 of the wave)
      {
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int c = 0; c < D; c += 4) {
            const float4 xv = *reinterpret_cast<const float4*>(&x[v][2 * pl + t][c]);
            acc[0] = fmaf(w1[t][c], xv.x, acc[0]);
            acc[1] = fmaf(w1[t][c + 1], xv.y, acc[1]);
            acc[2] = fmaf(w1[t][c + 2], xv.z, acc[2]);
            acc[3] = fmaf(w1[t][c + 3], xv.w, acc[3]);
          }
        float val = b1 + ((acc[0] + acc[1]) + (acc[2] + acc[3]));
        if (relu_mask & 1u) val = fmaxf(val, 0.f);
        a1[v][pl][c1] = val;
      }
      wave_lds_sync();
      // conv2: channel lane at position v, then its share of the final FC
      float part[2];
      {
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int c = 0; c < WV_C1; c += 4) {
            const float4 av = *reinterpret_cast<const float4*>(&a1[v][t][c]);
            acc[0] = fmaf(w2[t][c], av.x, acc[0]);
            acc[1] = fmaf(w2[t][c + 1], av.y, acc[1]);
            acc[2] = fmaf(w2[t][c + 2], av.z, acc[2]);
            acc[3] = fmaf(w2[t][c + 3], av.w, acc[3]);
          }
        float val = b2 + ((acc[0] + acc[1]) + (acc[2] + acc[3]));
        if (relu_mask & 2u) val = fmaxf(val, 0.f);
        part[0] = wf[0] * val;
        part[1] = wf[1] * val;
      }
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        float s = part[o];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
        if (lane == 0) red[v][o] = s;
      }
      lds_barrier();
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        float s = ((red[0][o] + red[1][o]) + red[2][o]) + red[3][o];
        s += bl[o];
        if (relu_mask & 4u) s = fmaxf(s, 0.f);
        z[o] = s;
      }
    }
    // round, or take the injected latencies (every wave alike)
    int32_t lat[2];
    if (RUN_NET) {
      if (p.logits_out && tid == 0)
        for (int o = 0; o < 2; ++o) p.logits_out[g * 2 + o] = z[o];
#pragma unroll
      for (int o = 0; o < 2; ++o) lat[o] = round_latency(z[o], p.lat_max, n_clamped, n_nonfinite);
    }
    ++n_pred;
    if (p.lat_mode != 0) {
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        const int32_t inj = p.lat_table[g * 2 + o];
        if (RUN_NET && inj != lat[o]) ++n_mismatch;
        lat[o] = inj;
      }
    }
    // clock and queue (Sec. 3.2): T = cur + F; the retired prefix (r <= T)
    // leaves; r = max(T + E + 1, r_prev, r_{i-W} + 1); push
    const int64_t Tn = cur + lat[0];
    {
      bool gone = false;
      if (lane < count) gone = q_r[(head + lane) & (QR - 1)] <= Tn;
      const int n_gone = __popcll(__ballot(gone));
      head = (head + n_gone) & (QR - 1);
      count -= n_gone;
    }
    int64_t r = Tn + lat[1] + 1;
    r = r > r_prev ? r : r_prev;
    const int wi = (int)(pos % W);
    if (pos >= W) {
      const int64_t rb = __shfl(rwv, wi) + 1;
      r = r > rb ? r : rb;
    }
    if (lane == wi) rwv = r;
    const int sl = (head + count) & (QR - 1);
    if (count == C) {
      head = (head + 1) & (QR - 1);  // only the newest C stay visible
    } else {
      ++count;
    }
    if (tid == 0) {
      q_e[sl] = lat[1];
      q_t[sl] = Tn;
      q_r[sl] = r;
    }
    r_prev = r;
    cur = Tn;
    ++pos;
    if (pos == warm) t_w = Tn;
    if (pos == n_pos) {  // the drain ends (Eq. 1); the slot takes the next sub-trace
      if (tid == 0) {
        st.fetch[k] = Tn - t_w;
        st.drain[k] = r - Tn;
        st.final_tick[k] = r;
        st.warm_tick[k] = t_w;
        st.pos[k] = pos;
        st.cur[k] = Tn;
        claimed = claim_subtrace(st, p.n_sub);
      }
      __syncthreads();
      k = claimed;
      load_state();
      load_row();
    } else {
      rowv[0] = nxt[0];
      rowv[1] = nxt[1];
      lds_barrier();  // the push is visible to the next step's window
    }
  }

  // the slot's state back to memory, the ring from entry 0 (head 0)
  if (tid == 0) {
    st.slot_kid[slot] = k;
    if (k >= 0) {
      st.cur[k] = cur;
      st.t_w[k] = t_w;
      st.r_prev[k] = r_prev;
      st.pos[k] = pos;
      st.head[k] = 0;
      st.count[k] = count;
    }
    if (n_clamped) atomicAdd(&st.counters[0], (unsigned long long)n_clamped);
    if (n_nonfinite) atomicAdd(&st.counters[1], (unsigned long long)n_nonfinite);
    if (n_mismatch) atomicAdd(&st.counters[2], (unsigned long long)n_mismatch);
    if (n_pred) atomicAdd(&st.counters[3], (unsigned long long)n_pred);
  }
  if (k >= 0 && v == 0) {
    if (lane < count) {
      const int e = (head + lane) & (QR - 1);
      const size_t gq = (size_t)k * C + lane;
      st.q_idx[gq] = (int32_t)(first + pos - count + lane);
      st.q_e[gq] = q_e[e];
      st.q_t[gq] = q_t[e];
      st.q_r[gq] = q_r[e];
    }
    if (lane < W) st.rw[(size_t)k * WMAX + lane] = rwv;
  }
}

// Predictor over explicit windows x [B][L][D] -> logits [B][NOUT]; TRUNK:
// the convolutions only, the last conv's output to trunk_out [B][NB][CH3].
template <class Net, class P, bool TRUNK = false>
__global__ void __launch_bounds__(Net::WAVES * 64)
    forward_kernel(DevWeights wt, uint32_t relu_mask, const float* __restrict__ x, int64_t B,
                   float* __restrict__ logits, void* __restrict__ trunk_out) {
  using G = Geo<Net, P>;
  using T = typename P::T;
  constexpr int NT = G::NT, D = Net::D, DP = G::DP, BS = Net::BS, L = Net::L;
  __shared__ NetSmem<Net, P> sm;
  const int tid = threadIdx.x;
  const int64_t b0 = (int64_t)blockIdx.x * MT;
  constexpr int GSL = G::NG * BS;
  constexpr int ROWS = MT * GSL, TPR = NT / ROWS, CPT = DP / TPR;
  const int row = tid / TPR, part = tid % TPR;
  const int s = row / GSL, t = row % GSL;
  static_assert(NT % ROWS == 0 && DP % TPR == 0 && CPT % 2 == 0 && D % 2 == 0, "gather split");
  if constexpr (P::SCALED)
    for (int c = tid; c < D; c += NT) sm.x_inv[c] = wt.x_inv[c];
  sm.stage_head(wt, tid, NT);
  __syncthreads();
  const int64_t b = b0 + s;
  auto load = [&](int j0, int nb) {
    RowRegs<CPT> r;
    r.valid = b < B && t < nb * BS;
    const float* src = x + ((r.valid ? b : 0) * L + (r.valid ? j0 * BS + t : 0)) * D;
#pragma unroll
    for (int cc = 0; cc < CPT; cc += 2) {
      const int c = part * CPT + cc;
      if (TPR > 1 || cc < D)
        r.v[cc / 2] = *reinterpret_cast<const float2*>(src + (c < D ? c : D - 2));
      else
        r.v[cc / 2] = make_float2(0.f, 0.f);
    }
    return r;
  };
  auto commit = [&](int j0, int nb, const RowRegs<CPT>& r, T* X) {
    (void)j0;
    if (t >= nb * BS) return;
    float v[CPT];
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) {
      const int c = part * CPT + cc;
      v[cc] = (r.valid && c < D) ? (cc & 1 ? r.v[cc / 2].y : r.v[cc / 2].x) : 0.f;
    }
    T e[CPT];
    window_elems<P, CPT, D>(v, sm.x_inv, part * CPT, e);
    store_run<(CPT * sizeof(T)) % 16 == 0 ? 16 : 8>(
        X + s * G::SX + (t >> 1) * G::RX + (t & 1) * DP + part * CPT, e);
  };
  if constexpr (TRUNK) {
    SavePtrs<T> sv{};
    sv.a3 = static_cast<T*>(trunk_out) + b0 * Net::NB * Net::CH3;
    sv.rows = (int)(B - b0 < MT ? B - b0 : MT);
    predict_tile<Net, P, false, true, true>(wt, relu_mask, sm, load, commit, nullptr, nullptr, sv);
  } else {
    predict_tile<Net, P>(wt, relu_mask, sm, load, commit);
    if (tid < MT * Net::NOUT) {
      const int ss = tid / Net::NOUT, o = tid % Net::NOUT;
      if (b0 + ss < B) logits[(b0 + ss) * Net::NOUT + o] = sm.logit[ss][o];
    }
  }
}

// ------------------------------------------------------ residual blocks ---
// A tile of TM rows (window positions at the last conv level, CH3 channels
// each) stays in LDS through all NRES blocks.  Per block the expansion is
// produced EC channels at a time (bias, ReLU, rounded to the form, into one
// of two LDS buffers) and consumed by the projection in the next phase,
// while the following chunk is expanded; the projection's TM x CH3
// accumulators stay in registers for the whole block; then bias, the block
// input and the ReLU, rounded to the form, replace the tile.

// The matrix instruction of a form in the residual blocks: BF16 on
// 32x32x16 tiles, FP32 on 16x16x4.
template <class P>
struct ResMma {
  using M = P;
};
template <>
struct ResMma<PBF16> {
  using M = PBF16W;
};

template <class P>
struct ResGeo {
  using T = typename P::T;
  using M = typename ResMma<P>::M;
  static constexpr int C = NetRB7::CH3, E = NetRB7::EXPAND, EC = 128;
  static constexpr int TM = P::ID == 0 ? 64 : 128, TILE = M::TILE, MTL = TM / TILE;
  static constexpr int PAD = 16 / sizeof(T);
  static constexpr int SXR = C + PAD, SHR = EC + PAD;  // padded LDS rows
  // waves 4 along N x 2 along M in both products
  static constexpr int WAVES = 8, NT = WAVES * 64, WNW = 4, WMW = WAVES / WNW;
  static constexpr int MPW = MTL / WMW, NPE = EC / TILE / WNW, NPP = C / TILE / WNW;
  static_assert(E % EC == 0 && MTL % WMW == 0 && NPE * WNW * TILE == EC &&
                    NPP * WNW * TILE == C,
                "wave split");
};

template <class P>
__global__ void __launch_bounds__(ResGeo<P>::NT)
    resblock_kernel(DevWeights wt, uint32_t relu_mask, typename P::T* __restrict__ x, int64_t rows,
                    const int32_t* __restrict__ active) {
  using RG = ResGeo<P>;
  using M = typename RG::M;
  using T = typename P::T;
  using Acc = typename M::Acc;
  using Net = NetRB7;
  constexpr int C = RG::C, E = RG::E, EC = RG::EC, TM = RG::TM, TILE = RG::TILE;
  constexpr int MPW = RG::MPW, NPE = RG::NPE, NPP = RG::NPP;
  constexpr int NG4 = TILE * TILE / 256;  // 4-column groups per lane and tile
  constexpr int CV = C * (int)sizeof(T) / 16, EPV = 16 / (int)sizeof(T);
  constexpr int KGE = C / M::KG, KGP = EC / M::KG, NCH = E / EC, NTE = E / TILE, NTP = C / TILE;
  __shared__ alignas(16) T xs[TM * RG::SXR];
  __shared__ alignas(16) T hs[2 * TM * RG::SHR];  // two expansion chunks
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t r0 = (int64_t)blockIdx.x * TM;
  const int64_t r1 = r0 + TM < rows ? r0 + TM : rows;  // rows [r0, r1) exist
  if (active) {  // windows none of whose rows is live are skipped
    int a = 0;
    for (int64_t w = r0 / Net::NB + tid; w <= (r1 - 1) / Net::NB; w += RG::NT) a |= active[w];
    if (!__syncthreads_or(a)) return;
  }
  for (int i = tid; i < TM * CV; i += RG::NT) {
    const int r = i / CV, v = i % CV;
    uint4 val = make_uint4(0u, 0u, 0u, 0u);
    if (r0 + r < r1) val = reinterpret_cast<const uint4*>(x + (r0 + r) * C)[v];
    *reinterpret_cast<uint4*>(xs + r * RG::SXR + v * EPV) = val;
  }
  __syncthreads();
  // a wave's A fragments (LDS) serve its NPE or NPP N tiles, its weight
  // fragments its MPW M tiles
  const int wn = wave % RG::WNW, wm = wave / RG::WNW;
  const int row = lane % TILE, ko = (lane / TILE) * (M::KG * TILE / 64);
  const T* apx[MPW];
  const T* aph[MPW];
#pragma unroll
  for (int i = 0; i < MPW; ++i) {
    const int r = (wm * MPW + i) * TILE + row;
    apx[i] = xs + r * RG::SXR + ko;
    aph[i] = hs + r * RG::SHR + ko;
  }
  const size_t half = (size_t)C * E * sizeof(T);
  Acc yacc[MPW][NPP];
#pragma unroll
  for (int i = 0; i < MPW; ++i)
#pragma unroll
    for (int j = 0; j < NPP; ++j) yacc[i][j] = Acc{};
  // Expansion of chunk u into hs buffer u & 1: bias, ReLU, rounded to the form.
  auto expand = [&](int u) {
    const int blk = u / NCH, ch = u % NCH;
    const uint4* We = reinterpret_cast<const uint4*>(static_cast<const char*>(wt.res_w) +
                                                     (size_t)blk * wt.res_stride);
    const float* be = wt.res_b + (size_t)blk * (E + C);
    const bool erelu = relu_mask & (1u << (Net::NCONV + 2 * blk));
    float4 bev[NPE][NG4];  // requested before the weights (loads complete in order)
#pragma unroll
    for (int j = 0; j < NPE; ++j)
#pragma unroll
      for (int g = 0; g < NG4; ++g)
        bev[j][g] = *reinterpret_cast<const float4*>(be + ch * EC + (wn * NPE + j) * TILE +
                                                     M::col4(g, lane));
    Acc hacc[MPW][NPE];
#pragma unroll
    for (int i = 0; i < MPW; ++i)
#pragma unroll
      for (int j = 0; j < NPE; ++j) hacc[i][j] = Acc{};
    mma_stream<M, KGE, NTE, NPE, MPW>(hacc, apx, We, ch * (EC / TILE) + wn * NPE, lane);
    T* hb = hs + (u & 1) * TM * RG::SHR;
#pragma unroll
    for (int j = 0; j < NPE; ++j)
#pragma unroll
      for (int g = 0; g < NG4; ++g) {
        const int hc0 = (wn * NPE + j) * TILE + M::col4(g, lane);  // 4 channels of the chunk
        const float bq[4] = {bev[j][g].x, bev[j][g].y, bev[j][g].z, bev[j][g].w};
#pragma unroll
        for (int i = 0; i < MPW; ++i) {
          T e[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            float v = hacc[i][j][4 * g + q] + bq[q];
            if (erelu) v = fmaxf(v, 0.f);
            e[q] = to_storage<P>(v, 0, nullptr);
          }
          store_run<4 * sizeof(T)>(hb + ((wm * MPW + i) * TILE + row) * RG::SHR + hc0, e);
        }
      }
  };
  // Projection of chunk u from hs buffer u & 1 into yacc.
  auto project = [&](int u) {
    const int blk = u / NCH, ch = u % NCH;
    const uint4* Wp = reinterpret_cast<const uint4*>(static_cast<const char*>(wt.res_w) +
                                                     (size_t)blk * wt.res_stride + half) +
                      (size_t)ch * KGP * NTP * 64;
    const int ho = (u & 1) * TM * RG::SHR;
    const T* aphu[MPW];
#pragma unroll
    for (int i = 0; i < MPW; ++i) aphu[i] = aph[i] + ho;
    mma_stream<M, KGP, NTP, NPP, MPW>(yacc, aphu, Wp, wn * NPP, lane);
  };
  // Chunk u+1's expansion and chunk u's projection share a phase (one
  // barrier per chunk; the two products' chains interleave); a block's first
  // expansion waits for the previous block's output.
  constexpr int TT = Net::NRES * NCH;
  expand(0);
  lds_barrier();
  for (int t = 0; t < TT; ++t) {
    const int blk = t / NCH, ch = t % NCH;
    float4 bpv[NPP][NG4];
    if (ch == NCH - 1) {
      const float* bp = wt.res_b + (size_t)blk * (E + C) + E;
#pragma unroll
      for (int j = 0; j < NPP; ++j)
#pragma unroll
        for (int g = 0; g < NG4; ++g)
          bpv[j][g] = *reinterpret_cast<const float4*>(bp + (wn * NPP + j) * TILE +
                                                       M::col4(g, lane));
    } else {
      expand(t + 1);
    }
    project(t);
    lds_barrier();
    if (ch == NCH - 1) {
      // bias, the block input (as stored) and the activation replace the tile
      const bool orelu = relu_mask & (1u << (Net::NCONV + 2 * blk + 1));
#pragma unroll
      for (int j = 0; j < NPP; ++j)
#pragma unroll
        for (int g = 0; g < NG4; ++g) {
          const int col0 = (wn * NPP + j) * TILE + M::col4(g, lane);
          const float bq[4] = {bpv[j][g].x, bpv[j][g].y, bpv[j][g].z, bpv[j][g].w};
#pragma unroll
          for (int i = 0; i < MPW; ++i) {
            T* xr = xs + ((wm * MPW + i) * TILE + row) * RG::SXR + col0;
            T e[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              float v = yacc[i][j][4 * g + q] + bq[q] + P::val(xr[q]);
              if (orelu) v = fmaxf(v, 0.f);
              e[q] = to_storage<P>(v, 0, nullptr);
            }
            store_run<4 * sizeof(T)>(xr, e);
          }
        }
#pragma unroll
      for (int i = 0; i < MPW; ++i)
#pragma unroll
        for (int j = 0; j < NPP; ++j) yacc[i][j] = Acc{};
      lds_barrier();
      if (t + 1 < TT) {
        expand(t + 1);
        lds_barrier();
      }
    }
  }
  for (int i = tid; i < TM * CV; i += RG::NT) {
    const int r = i / CV, v = i % CV;
    if (r0 + r < r1)
      reinterpret_cast<uint4*>(x + (r0 + r) * C)[v] =
          *reinterpret_cast<const uint4*>(xs + r * RG::SXR + v * EPV);
  }
}

// FC 512 and the hybrid head over x [B][NB][CH3] (the blocks' output):
// each group of the tile's blocks is staged into LDS where the fused step
// keeps its last conv output, then the same hidden-FC and head code runs.
template <class P>
__global__ void __launch_bounds__(NetRB7::WAVES * 64)
    rb_head_kernel(DevWeights wt, uint32_t relu_mask, const typename P::T* __restrict__ x,
                   int64_t B, const int32_t* __restrict__ active, float* __restrict__ logits) {
  using Net = NetRB7;
  using G = Geo<Net, P>;
  using T = typename P::T;
  constexpr int NG = G::NG, NFULL = Net::NB / NG, TAIL = Net::NB % NG;
  constexpr int HT = (Net::HID / 16) / Net::WAVES, V = Net::CH3 * (int)sizeof(T) / 16;
  __shared__ NetSmem<Net, P> sm;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t b0 = (int64_t)blockIdx.x * MT;
  if (active) {
    const int a = tid < MT && b0 + tid < B ? active[b0 + tid] : 0;
    if (!__syncthreads_or(a)) return;
  }
  v4f hacc[HT];
#pragma unroll
  for (int j = 0; j < HT; ++j) hacc[j] = v4f{0.f, 0.f, 0.f, 0.f};
  auto stage = [&](int j0, int nb) {
    for (int i = tid; i < MT * nb * V; i += G::NT) {
      const int s = i / (nb * V), r = i % (nb * V), jb = r / V, v = r % V;
      uint4 val = make_uint4(0u, 0u, 0u, 0u);
      if (b0 + s < B)
        val = reinterpret_cast<const uint4*>(x + ((b0 + s) * Net::NB + j0 + jb) * Net::CH3)[v];
      *reinterpret_cast<uint4*>(sm.a3() + s * G::SAL + jb * Net::CH3 + v * (16 / (int)sizeof(T))) =
          val;
    }
    __syncthreads();
  };
  for (int g = 0; g < NFULL; ++g) {
    stage(g * NG, NG);
    hidden_fc<Net, P, NG>(wt, sm.a3(), g * NG, hacc, wave, lane);
    __syncthreads();
  }
  if constexpr (TAIL > 0) {
    stage(NFULL * NG, TAIL);
    hidden_fc<Net, P, TAIL>(wt, sm.a3(), NFULL * NG, hacc, wave, lane);
    __syncthreads();
  }
  hybrid_head<Net, P, false>(wt, relu_mask, sm, hacc, nullptr, nullptr);
  __syncthreads();
  if (tid < MT * Net::NOUT) {
    const int ss = tid / Net::NOUT, o = tid % Net::NOUT;
    if (b0 + ss < B) logits[(b0 + ss) * Net::NOUT + o] = sm.logit[ss][o];
  }
}

// Training-form forward over explicit windows: the trunk and the hidden
// layer, keeping every activation (the head runs as a GEMM afterwards).
template <class Net, class P>
__global__ void __launch_bounds__(Net::WAVES * 64)
    forward_save_kernel(DevWeights wt, uint32_t relu_mask, const float* __restrict__ x,
                        int64_t B, SaveBlock sb) {
  using G = Geo<Net, P>;
  using T = typename P::T;
  constexpr int NT = G::NT, D = Net::D, DP = G::DP, BS = Net::BS, L = Net::L;
  __shared__ NetSmem<Net, P> sm;
  const int tid = threadIdx.x;
  const int64_t b0 = (int64_t)blockIdx.x * MT;
  constexpr int GSL = G::NG * BS;
  constexpr int ROWS = MT * GSL, TPR = NT / ROWS, CPT = DP / TPR;
  const int row = tid / TPR, part = tid % TPR;
  const int s = row / GSL, t = row % GSL;
  static_assert(NT % ROWS == 0 && DP % TPR == 0 && CPT % 2 == 0 && D % 2 == 0, "gather split");
  if constexpr (P::SCALED)
    for (int c = tid; c < D; c += NT) sm.x_inv[c] = wt.x_inv[c];
  __syncthreads();
  const int64_t b = b0 + s;
  auto load = [&](int j0, int nb) {
    RowRegs<CPT> r;
    r.valid = b < B && t < nb * BS;
    const float* src = x + ((r.valid ? b : 0) * L + (r.valid ? j0 * BS + t : 0)) * D;
#pragma unroll
    for (int cc = 0; cc < CPT; cc += 2) {
      const int c = part * CPT + cc;
      if (TPR > 1 || cc < D)
        r.v[cc / 2] = *reinterpret_cast<const float2*>(src + (c < D ? c : D - 2));
      else
        r.v[cc / 2] = make_float2(0.f, 0.f);
    }
    return r;
  };
  auto commit = [&](int j0, int nb, const RowRegs<CPT>& r, T* X) {
    (void)j0;
    if (t >= nb * BS) return;
    float v[CPT];
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) {
      const int c = part * CPT + cc;
      v[cc] = (r.valid && c < D) ? (cc & 1 ? r.v[cc / 2].y : r.v[cc / 2].x) : 0.f;
    }
    T e[CPT];
    window_elems<P, CPT, D>(v, sm.x_inv, part * CPT, e);
    store_run<(CPT * sizeof(T)) % 16 == 0 ? 16 : 8>(
        X + s * G::SX + (t >> 1) * G::RX + (t & 1) * DP + part * CPT, e);
  };
  SavePtrs<T> sv;
  sv.a1 = static_cast<T*>(sb.a1) + b0 * (Net::NB * BS / 2) * Net::CH1;
  sv.a2 = static_cast<T*>(sb.a2) + b0 * (Net::NB * BS / 4) * Net::CH2;
  sv.a3 = static_cast<T*>(sb.a3) + b0 * Net::NB * Net::CH3;
  sv.h = static_cast<T*>(sb.h) + b0 * Net::HID;
  sv.rows = (int)(B - b0 < MT ? B - b0 : MT);
  predict_tile<Net, P, false, true>(wt, relu_mask, sm, load, commit, nullptr, nullptr, sv);
}

// (the hidden FC's 8-fragment weight chunks requested two ahead, as the step
// kernel's variant 3: 2 % faster than one ahead here, no spills)
template <class P>
static hipError_t launch_fwd_save_t(const DevWeights& w, uint32_t relu, const float* x, int64_t B,
                                    const SaveBlock& sb, hipStream_t stream) {
  const dim3 grid((unsigned)((B + MT - 1) / MT)), block(Geo<NetC3, P>::NT);
  hipLaunchKernelGGL((forward_save_kernel<NetC3V3, P>), grid, block, 0, stream, w, relu, x, B, sb);
  return hipGetLastError();
}

hipError_t launch_forward_save(int prec, const DevWeights& w, uint32_t relu, const float* x,
                               int64_t B, const SaveBlock& sb, hipStream_t stream) {
  return prec == 0 ? launch_fwd_save_t<PF32>(w, relu, x, B, sb, stream)
                   : launch_fwd_save_t<PBF16>(w, relu, x, B, sb, stream);
}

__global__ void reset_kernel(DevState st, int32_t n_sub, int32_t C, int32_t n_slots) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_slots) st.slot_kid[i] = -1;
  if (i == 0) *st.next = 0u;
  if (i < n_sub) {
    st.cur[i] = 0;
    st.t_w[i] = 0;
    st.r_prev[i] = 0;
    st.pos[i] = 0;
    st.head[i] = 0;
    st.count[i] = 0;
    st.fetch[i] = 0;
    st.drain[i] = 0;
    st.final_tick[i] = 0;
    st.warm_tick[i] = 0;
    for (int w = 0; w < WMAX; ++w) st.rw[i * WMAX + w] = 0;
    if (st.m_head) {
      st.m_head[i] = 0;
      st.m_count[i] = 0;
      st.m_inpq[i] = 0;
      st.x_prev[i] = 0;
    }
    for (int e = 0; e < C; ++e) {
      st.q_idx[i * C + e] = 0;
      st.q_e[i * C + e] = 0;
      st.q_t[i * C + e] = 0;
      st.q_r[i * C + e] = 0;
    }
  }
  if (i < NCOUNTERS) st.counters[i] = 0;
}

// total = sum_k (final_tick[k] - warm_tick[k]), one workgroup.
__global__ void __launch_bounds__(256) total_kernel(DevState st, int32_t n_sub, int64_t* total) {
  __shared__ long long part[4];
  long long acc = 0;
  for (int k = threadIdx.x; k < n_sub; k += 256) acc += st.final_tick[k] - st.warm_tick[k];
  for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *total = part[0] + part[1] + part[2] + part[3];
}

template <class Net, class P>
static hipError_t launch_step_t(const DevWeights& w, uint32_t relu, const DevState& s,
                                const StepParams& p, hipStream_t stream) {
  const dim3 grid(p.n_wg), block(Geo<Net, P>::NT);
  if constexpr (std::is_same<Net, NetC3>::value) {
    if (p.lat_mode != 1 && p.col_dep >= 0) {
      hipLaunchKernelGGL((step_kernel<Net, P, true, false, true>), grid, block, 0, stream, w,
                         relu, s, p);
      return hipGetLastError();
    }
  }
  if (p.lat_mode == 1)
    hipLaunchKernelGGL((step_kernel<Net, P, false>), grid, block, 0, stream, w, relu, s, p);
  else
    hipLaunchKernelGGL((step_kernel<Net, P, true>), grid, block, 0, stream, w, relu, s, p);
  return hipGetLastError();
}

template <class Net>
static hipError_t launch_step_n(int prec, const DevWeights& w, uint32_t relu, const DevState& s,
                                const StepParams& p, hipStream_t stream) {
  if (prec == 0) return launch_step_t<Net, PF32>(w, relu, s, p, stream);
  if (prec == 1) return launch_step_t<Net, PBF16>(w, relu, s, p, stream);
  return launch_step_t<Net, PFP8>(w, relu, s, p, stream);
}

template <class Net>
static const void* c3_step_fn(int prec) {
  if (prec == 0) return reinterpret_cast<const void*>(&step_kernel<Net, PF32, true>);
  if (prec == 1) return reinterpret_cast<const void*>(&step_kernel<Net, PBF16, true>);
  return reinterpret_cast<const void*>(&step_kernel<Net, PFP8, true>);
}

hipError_t c3_step_scratch(int prec, int variant, size_t* bytes) {
  const void* f = variant == 1   ? c3_step_fn<NetC3V1>(prec)
                  : variant == 2 ? c3_step_fn<NetC3V2>(prec)
                  : variant == 3 ? c3_step_fn<NetC3V3>(prec)
                                 : c3_step_fn<NetC3>(prec);
  hipFuncAttributes a{};
  const hipError_t e = hipFuncGetAttributes(&a, f);
  *bytes = e == hipSuccess ? a.localSizeBytes : 0;
  return e;
}

hipError_t launch_step(int net, int prec, int variant, const DevWeights& w, uint32_t relu,
                       const DevState& s, const StepParams& p, hipStream_t stream) {
  if (net == 1 && p.lat_mode != 1 && variant == 1)
    return launch_step_n<NetC3V1>(prec, w, relu, s, p, stream);
  if (net == 1 && p.lat_mode != 1 && variant == 2)
    return launch_step_n<NetC3V2>(prec, w, relu, s, p, stream);
  if (net == 1 && p.lat_mode != 1 && variant == 3)
    return launch_step_n<NetC3V3>(prec, w, relu, s, p, stream);
  if (net == 4) {  // store latencies: FP32 and BF16 forms
    if (prec == 0) return launch_step_t<NetC3S, PF32>(w, relu, s, p, stream);
    if (prec == 1) return launch_step_t<NetC3S, PBF16>(w, relu, s, p, stream);
    return hipErrorInvalidValue;
  }
  if (net == 3) {  // hybrid head: FP32 and BF16 forms
    if (prec == 0) return launch_step_t<NetC3Hyb, PF32>(w, relu, s, p, stream);
    if (prec == 1) return launch_step_t<NetC3Hyb, PBF16>(w, relu, s, p, stream);
    return hipErrorInvalidValue;
  }
  if (net == 0 && prec == 0 && variant == WAVE_VARIANT) {
    // one wavefront per slot
    const dim3 grid((unsigned)(p.n_wg * MT)), block(64);
    if (p.lat_mode == 1)
      hipLaunchKernelGGL(wave_step_kernel<false>, grid, block, 0, stream, w, relu, s, p);
    else
      hipLaunchKernelGGL(wave_step_kernel<true>, grid, block, 0, stream, w, relu, s, p);
    return hipGetLastError();
  }
  if (net == 0 && prec == 0 && variant == QUAD_VARIANT) {
    // four wavefronts per slot
    const dim3 grid((unsigned)(p.n_wg * MT)), block(QW * 64);
    if (p.lat_mode == 1)
      hipLaunchKernelGGL(quad_step_kernel<false>, grid, block, 0, stream, w, relu, s, p);
    else
      hipLaunchKernelGGL(quad_step_kernel<true>, grid, block, 0, stream, w, relu, s, p);
    return hipGetLastError();
  }
  return net == 0 ? launch_step_n<NetSmall>(prec, w, relu, s, p, stream)
                  : launch_step_n<NetC3>(prec, w, relu, s, p, stream);
}

template <class Net, class P>
static hipError_t launch_forward_t(const DevWeights& w, uint32_t relu, const float* x, int64_t B,
                                   float* logits, hipStream_t stream) {
  const dim3 grid((unsigned)((B + MT - 1) / MT)), block(Geo<Net, P>::NT);
  hipLaunchKernelGGL((forward_kernel<Net, P>), grid, block, 0, stream, w, relu, x, B, logits,
                     nullptr);
  return hipGetLastError();
}

template <class Net>
static hipError_t launch_forward_n(int prec, const DevWeights& w, uint32_t relu, const float* x,
                                   int64_t B, float* logits, hipStream_t stream) {
  if (prec == 0) return launch_forward_t<Net, PF32>(w, relu, x, B, logits, stream);
  if (prec == 1) return launch_forward_t<Net, PBF16>(w, relu, x, B, logits, stream);
  return launch_forward_t<Net, PFP8>(w, relu, x, B, logits, stream);
}

template <class Net>
static hipError_t launch_cal_t(const DevWeights& w, uint32_t relu, const DevState& s,
                               const StepParams& p, hipStream_t stream) {
  const dim3 grid(p.n_wg), block(Geo<Net, PF32>::NT);
  if constexpr (std::is_same<Net, NetC3>::value) {
    if (p.col_dep >= 0) {
      hipLaunchKernelGGL((step_kernel<Net, PF32, true, true, true>), grid, block, 0, stream, w,
                         relu, s, p);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((step_kernel<Net, PF32, true, true>), grid, block, 0, stream, w, relu, s, p);
  return hipGetLastError();
}

hipError_t launch_calibrate(int net, const DevWeights& w, uint32_t relu, const DevState& s,
                            const StepParams& p, hipStream_t stream) {
  return net == 0 ? launch_cal_t<NetSmall>(w, relu, s, p, stream)
                  : launch_cal_t<NetC3>(w, relu, s, p, stream);
}

int calibration_size(int net) { return net == 0 ? n_cal<NetSmall>() : n_cal<NetC3>(); }

hipError_t launch_forward(int net, int prec, const DevWeights& w, uint32_t relu, const float* x,
                          int64_t B, float* logits, hipStream_t stream) {
  if (net == 4) {
    if (prec == 0) return launch_forward_t<NetC3S, PF32>(w, relu, x, B, logits, stream);
    if (prec == 1) return launch_forward_t<NetC3S, PBF16>(w, relu, x, B, logits, stream);
    return hipErrorInvalidValue;
  }
  if (net == 3) {
    if (prec == 0) return launch_forward_t<NetC3Hyb, PF32>(w, relu, x, B, logits, stream);
    if (prec == 1) return launch_forward_t<NetC3Hyb, PBF16>(w, relu, x, B, logits, stream);
    return hipErrorInvalidValue;
  }
  return net == 0 ? launch_forward_n<NetSmall>(prec, w, relu, x, B, logits, stream)
                  : launch_forward_n<NetC3>(prec, w, relu, x, B, logits, stream);
}

hipError_t launch_reset(const DevState& s, int32_t n_sub, int32_t C, int32_t n_slots,
                        hipStream_t stream) {
  const int threads = 256;
  const int n = n_sub > n_slots ? n_sub : n_slots;
  const int blocks = (n + threads - 1) / threads;
  hipLaunchKernelGGL(reset_kernel, dim3(blocks > 0 ? blocks : 1), dim3(threads), 0, stream, s,
                     n_sub, C, n_slots);
  return hipGetLastError();
}

hipError_t launch_total(const DevState& s, int32_t n_sub, int64_t* total, hipStream_t stream) {
  hipLaunchKernelGGL(total_kernel, dim3(1), dim3(256), 0, stream, s, n_sub, total);
  return hipGetLastError();
}

// The run as a graph of kernel nodes (no memset nodes): the persistent step
// kernel until every slot is empty, then the total.
template <class Net, class P>
static void* step_fn(bool run_net, bool dep = false) {
  if constexpr (std::is_same<Net, NetC3>::value)
    if (run_net && dep) return reinterpret_cast<void*>(&step_kernel<Net, P, true, false, true>);
  return run_net ? reinterpret_cast<void*>(&step_kernel<Net, P, true>)
                 : reinterpret_cast<void*>(&step_kernel<Net, P, false>);
}

hipError_t build_run_graph(int net, int prec, int variant, const DevWeights& w, uint32_t relu,
                           const DevState& s, const StepParams& p, int64_t* total,
                           hipGraph_t* out) {
  const bool run_net = p.lat_mode != 1;
  void* fn;
  int nt;
  int grid_x = p.n_wg;
  if (net == 1 && run_net && variant == 1) {
    fn = prec == 0 ? step_fn<NetC3V1, PF32>(run_net)
         : prec == 1 ? step_fn<NetC3V1, PBF16>(run_net) : step_fn<NetC3V1, PFP8>(run_net);
    nt = Geo<NetC3V1, PF32>::NT;
  } else if (net == 1 && run_net && variant == 2) {
    fn = prec == 0 ? step_fn<NetC3V2, PF32>(run_net)
         : prec == 1 ? step_fn<NetC3V2, PBF16>(run_net) : step_fn<NetC3V2, PFP8>(run_net);
    nt = Geo<NetC3V2, PF32>::NT;
  } else if (net == 1 && run_net && variant == 3) {
    fn = prec == 0 ? step_fn<NetC3V3, PF32>(run_net)
         : prec == 1 ? step_fn<NetC3V3, PBF16>(run_net) : step_fn<NetC3V3, PFP8>(run_net);
    nt = Geo<NetC3V3, PF32>::NT;
  } else if (net == 0 && prec == 0 && variant == WAVE_VARIANT) {
    fn = run_net ? reinterpret_cast<void*>(&wave_step_kernel<true>)
                 : reinterpret_cast<void*>(&wave_step_kernel<false>);
    nt = 64;
    grid_x = p.n_wg * MT;
  } else if (net == 0 && prec == 0 && variant == QUAD_VARIANT) {
    fn = run_net ? reinterpret_cast<void*>(&quad_step_kernel<true>)
                 : reinterpret_cast<void*>(&quad_step_kernel<false>);
    nt = QW * 64;
    grid_x = p.n_wg * MT;
  } else if (net == 0) {
    fn = prec == 0 ? step_fn<NetSmall, PF32>(run_net)
         : prec == 1 ? step_fn<NetSmall, PBF16>(run_net) : step_fn<NetSmall, PFP8>(run_net);
    nt = Geo<NetSmall, PF32>::NT;
  } else if (net == 3) {
    if (prec > 1) return hipErrorInvalidValue;
    fn = prec == 0 ? step_fn<NetC3Hyb, PF32>(run_net) : step_fn<NetC3Hyb, PBF16>(run_net);
    nt = Geo<NetC3Hyb, PF32>::NT;
  } else if (net == 4) {
    if (prec > 1) return hipErrorInvalidValue;
    fn = prec == 0 ? step_fn<NetC3S, PF32>(run_net) : step_fn<NetC3S, PBF16>(run_net);
    nt = Geo<NetC3S, PF32>::NT;
  } else {
    const bool dep = p.col_dep >= 0;
    fn = prec == 0 ? step_fn<NetC3, PF32>(run_net, dep)
         : prec == 1 ? step_fn<NetC3, PBF16>(run_net, dep) : step_fn<NetC3, PFP8>(run_net, dep);
    nt = Geo<NetC3, PF32>::NT;
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipGraphCreate(&g, 0);
  if (e != hipSuccess) return e;
  DevWeights wa = w;
  uint32_t ra = relu;
  DevState sa = s;
  StepParams pa = p;
  void* step_args[] = {&wa, &ra, &sa, &pa};
  hipKernelNodeParams kp{};
  kp.func = fn;
  kp.gridDim = dim3(grid_x);
  kp.blockDim = dim3(nt);
  kp.sharedMemBytes = 0;
  kp.kernelParams = step_args;
  kp.extra = nullptr;
  hipGraphNode_t step_node = nullptr, total_node = nullptr;
  e = hipGraphAddKernelNode(&step_node, g, nullptr, 0, &kp);
  int32_t n_sub = p.n_sub;
  int64_t* tot = total;
  void* total_args[] = {&sa, &n_sub, &tot};
  hipKernelNodeParams kt{};
  kt.func = reinterpret_cast<void*>(&total_kernel);
  kt.gridDim = dim3(1);
  kt.blockDim = dim3(256);
  kt.sharedMemBytes = 0;
  kt.kernelParams = total_args;
  kt.extra = nullptr;
  if (e == hipSuccess) e = hipGraphAddKernelNode(&total_node, g, &step_node, 1, &kt);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return e;
  }
  *out = g;
  return hipSuccess;
}

// ------------------------------------------------------------------ RB7 ---

template <class P>
static hipError_t launch_rb_stage_t(int stage, const DevWeights& w, uint32_t relu,
                                    const DevState& s, const StepParams& p, hipStream_t stream) {
  const dim3 grid(p.n_wg), block(Geo<NetRB7, P>::NT);
  if (stage == 1)
    hipLaunchKernelGGL((step_kernel<NetRB7, P, true, false, false, 1>), grid, block, 0, stream, w,
                       relu, s, p);
  else
    hipLaunchKernelGGL((step_kernel<NetRB7, P, true, false, false, 2>), grid, block, 0, stream, w,
                       relu, s, p);
  return hipGetLastError();
}

hipError_t launch_rb_stage(int prec, int stage, const DevWeights& w, uint32_t relu,
                           const DevState& s, const StepParams& p, hipStream_t stream) {
  if ((stage != 1 && stage != 2) || p.n_steps != 1) return hipErrorInvalidValue;
  if (prec == 0) return launch_rb_stage_t<PF32>(stage, w, relu, s, p, stream);
  if (prec == 1) return launch_rb_stage_t<PBF16>(stage, w, relu, s, p, stream);
  return hipErrorInvalidValue;
}

template <class P>
static hipError_t launch_resblocks_t(const DevWeights& w, uint32_t relu, void* x, int64_t rows,
                                     const int32_t* active, hipStream_t stream) {
  const int64_t tiles = (rows + ResGeo<P>::TM - 1) / ResGeo<P>::TM;
  if (tiles > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((resblock_kernel<P>), dim3((unsigned)tiles), dim3(ResGeo<P>::NT), 0, stream,
                     w, relu, static_cast<typename P::T*>(x), rows, active);
  return hipGetLastError();
}

hipError_t launch_resblocks(int prec, const DevWeights& w, uint32_t relu, void* x, int64_t rows,
                            const int32_t* active, hipStream_t stream) {
  if (rows <= 0) return hipSuccess;
  if (prec == 0) return launch_resblocks_t<PF32>(w, relu, x, rows, active, stream);
  if (prec == 1) return launch_resblocks_t<PBF16>(w, relu, x, rows, active, stream);
  return hipErrorInvalidValue;
}

hipError_t launch_rb_head(int prec, const DevWeights& w, uint32_t relu, const void* x, int64_t B,
                          const int32_t* active, float* logits, hipStream_t stream) {
  if (B <= 0) return hipSuccess;
  const dim3 grid((unsigned)((B + MT - 1) / MT)), block(NetRB7::WAVES * 64);
  if (prec == 0)
    hipLaunchKernelGGL((rb_head_kernel<PF32>), grid, block, 0, stream, w, relu,
                       static_cast<const float*>(x), B, active, logits);
  else if (prec == 1)
    hipLaunchKernelGGL((rb_head_kernel<PBF16>), grid, block, 0, stream, w, relu,
                       static_cast<const PBF16::T*>(x), B, active, logits);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_rb_trunk(int prec, const DevWeights& w, uint32_t relu, const float* x, int64_t B,
                           void* out, hipStream_t stream) {
  if (B <= 0) return hipSuccess;
  const dim3 grid((unsigned)((B + MT - 1) / MT)), block(NetRB7::WAVES * 64);
  if (prec == 0)
    hipLaunchKernelGGL((forward_kernel<NetRB7, PF32, true>), grid, block, 0, stream, w, relu, x, B,
                       nullptr, out);
  else if (prec == 1)
    hipLaunchKernelGGL((forward_kernel<NetRB7, PBF16, true>), grid, block, 0, stream, w, relu, x,
                       B, nullptr, out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace simnet
