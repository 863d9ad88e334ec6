// Training-form kernels of libsimnet.so (gfx950): the pieces of a predictor
// training step that are not the fused trunk forward.
//
//   gemm kernels     C = op(A) x op(B): FP32 form on FP32 MFMA (64x64
//                    tiles), BF16 form on BF16 MFMA (128x128 tiles, operands
//                    rounded to BF16 in LDS); operands in FP32 or BF16 with
//                    arbitrary strides; split-K with an ordered reduction
//                    when the output is small; epilogue with bias, ReLU mask
//                    (a saved activation > 0), accumulation and a column
//                    permutation of C (weight gradients stored in the
//                    parameters' own layout).  Used for the head and for
//                    every input-gradient and weight-gradient product of the
//                    backward pass (a kernel-2 stride-2 convolution is a
//                    GEMM over position pairs); the pipelined BF16 kernel
//                    also sums its left operand's rows (the trunk's bias
//                    gradients).
//   reductions       split-K partials summed in order with the epilogue.
//   loss_kernel      hybrid loss per window (400-bin cross-entropy + L1 on
//                    log1p(latency) per latency type) and its gradient
//                    w.r.t. the head outputs.
//   colsum kernels   bias gradients as chunk partials; sum_partials adds
//                    several lists of partials, each in a fixed order.
//   map_gather_multi weight re-layouts by index maps.
//   pad_rows         a row-major matrix copied with its rows padded.
//   adam kernels     Adam on FP32 master weights (and, fused, the re-layout
//                    of the updated weights).
#include <type_traits>

#include "simnet_internal.h"

namespace simnet {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float ld_elem(const void* p, int bf16, int64_t i) {
  if (bf16) return __uint_as_float((uint32_t)static_cast<const uint16_t*>(p)[i] << 16);
  return static_cast<const float*>(p)[i];
}

// Rows are grouped (row r at (r / grp) * gs + (r % grp) * rs) only where an
// operand skips memory between groups of rows; ungrouped operands carry
// grp >= NO_GROUP and take no division.  Grouped row indices are below
// 2^32 (the host checks), so their division is 32-bit.
__device__ __forceinline__ int64_t grouped_row(int64_t r, int64_t grp, int64_t gs, int64_t rs) {
  if (grp >= NO_GROUP) return r * rs;
  const uint32_t q = (uint32_t)r / (uint32_t)grp;
  return (int64_t)q * gs + (int64_t)((uint32_t)r - q * (uint32_t)grp) * rs;
}

__device__ __forceinline__ int64_t op_index(const GemmOperand& o, int64_t r, int64_t c) {
  return grouped_row(r, o.grp, o.gs, o.rs) + c * o.cs;
}

// Nearest-even BF16 bits of a finite float.
__device__ __forceinline__ uint16_t to_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Column n's offset in a row of C (N below 2^32 when permuted: the host
// checks).
__device__ __forceinline__ int64_t c_col(const GemmArgs& g, int64_t n) {
  if (g.ccg == 0) return n;
  const uint32_t q = (uint32_t)n / (uint32_t)g.ccg;
  return (int64_t)((uint32_t)n - q * (uint32_t)g.ccg) * g.ccm + q;
}

// C(m, n) epilogue shared by every GEMM path: bias, ReLU mask, accumulate,
// grouped row and permuted column addressing, BF16 output.
__device__ __forceinline__ void gemm_store(const GemmArgs& g, int64_t m, int64_t n, float v) {
  if (g.bias) v += g.bias[n];
  if (g.mask.p && !(ld_elem(g.mask.p, g.mask.bf16, op_index(g.mask, m, n)) > 0.f)) v = 0.f;
  const int64_t at = grouped_row(m, g.cgrp, g.cgs, g.ldc) + c_col(g, n);
  if (g.c_bf16) {
    reinterpret_cast<uint16_t*>(g.C)[at] = to_bf16(v);
    return;
  }
  float* c = g.C + at;
  *c = g.beta ? *c + v : v;
}

// The same for the four columns n0 + 16*j (j < 4) of one row m, with the
// row's addresses computed once; the caller has added the bias.
__device__ __forceinline__ void gemm_store_row4(const GemmArgs& g, int64_t m, int64_t n0,
                                                const float (&v)[4]) {
  const int64_t crow = grouped_row(m, g.cgrp, g.cgs, g.ldc);
  const int64_t mrow = g.mask.p ? grouped_row(m, g.mask.grp, g.mask.gs, g.mask.rs) : 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t n = n0 + 16 * j;
    if (n >= g.N) continue;
    float x = v[j];
    if (g.mask.p && !(ld_elem(g.mask.p, g.mask.bf16, mrow + n * g.mask.cs) > 0.f)) x = 0.f;
    const int64_t at = crow + c_col(g, n);
    if (g.c_bf16) {
      reinterpret_cast<uint16_t*>(g.C)[at] = to_bf16(x);
    } else {
      float* c = g.C + at;
      *c = g.beta ? *c + x : x;
    }
  }
}

// Split-K: workgroup z covers k in [z*kc, min(K, (z+1)*kc)) and writes its
// raw partial product to part[z][M][N]; gemm_reduce sums the partials in
// order and applies the epilogue.
__device__ __forceinline__ void k_range(const GemmArgs& g, int step, int64_t* kb, int64_t* ke) {
  const int64_t per = (g.K + g.ksplit - 1) / g.ksplit;
  const int64_t kc = (per + step - 1) / step * step;
  *kb = (int64_t)blockIdx.z * kc;
  *ke = *kb + kc < g.K ? *kb + kc : g.K;
}

__device__ __forceinline__ void gemm_out(const GemmArgs& g, int64_t m, int64_t n, float v) {
  if (g.ksplit > 1)
    g.part[((int64_t)blockIdx.z * g.M + m) * g.N + n] = v;
  else
    gemm_store(g, m, n, v);
}

constexpr int GB = 64, GK = 16, GPAD = 4;

// One thread's four elements of a tile (rows r0.. of R, cols c0.. of C),
// read along whichever dimension is contiguous in memory.
__device__ __forceinline__ void load_tile(const GemmOperand& o, int64_t R, int64_t Cn, int64_t r0,
                                          int64_t c0, bool rows_are_k, int tid, float (&v)[4],
                                          int (&rr)[4], int (&cc)[4]) {
  // tile is GB (non-k) x GK (k); "along" = the contiguous dimension
  const bool k_contig = rows_are_k ? (o.rs == 1 && o.grp >= NO_GROUP) : (o.cs == 1);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    int kk, mm;
    if (k_contig) {
      mm = tid / 4;
      kk = (tid % 4) * 4 + e;
    } else {
      kk = tid / 16;
      mm = (tid % 16) * 4 + e;
    }
    // rows_are_k: operand rows index k (B operand); else rows index m (A)
    const int64_t r = rows_are_k ? r0 + kk : r0 + mm;
    const int64_t c = rows_are_k ? c0 + mm : c0 + kk;
    v[e] = (r < R && c < Cn) ? ld_elem(o.p, o.bf16, op_index(o, r, c)) : 0.f;
    rr[e] = kk;
    cc[e] = mm;
  }
}

// FP32 form: 64x64 tiles on mfma_f32_16x16x4f32, 2x2 waves of 32x32.
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
  __shared__ float As[GK][GB + GPAD];  // [k][m]
  __shared__ float Bs[GK][GB + GPAD];  // [k][n]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t m0 = (int64_t)blockIdx.y * GB, n0 = (int64_t)blockIdx.x * GB;
  const int wm = wave >> 1, wn = wave & 1;
  int64_t kb, ke;
  k_range(g, GK, &kb, &ke);
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  float va[4], vb[4];
  int ka[4], ma[4], kb4[4], nb[4];
  load_tile(g.A, g.M, ke, m0, kb, false, tid, va, ka, ma);
  load_tile(g.B, ke, g.N, kb, n0, true, tid, vb, kb4, nb);
  for (int64_t k0 = kb; k0 < ke; k0 += GK) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      As[ka[e]][ma[e]] = va[e];
      Bs[kb4[e]][nb[e]] = vb[e];
    }
    __syncthreads();
    if (k0 + GK < ke) {  // next tile in flight while this one is multiplied
      load_tile(g.A, g.M, ke, m0, k0 + GK, false, tid, va, ka, ma);
      load_tile(g.B, ke, g.N, k0 + GK, n0, true, tid, vb, kb4, nb);
    }
#pragma unroll
    for (int ks = 0; ks < GK; ks += 4) {
      const int k = ks + (lane >> 4);
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[k][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[k][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  // lane holds C[4*(lane/16) + r][lane % 16] of each 16x16 tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int64_t n = n0 + wn * 32 + j * 16 + (lane & 15);
        if (m < g.M && n < g.N) gemm_out(g, m, n, acc[i][j][r]);
      }
}

// BF16 form: 128x128 tiles, k-steps of 32 on mfma_f32_16x16x32_bf16, 2x2
// waves of 64x64, operands rounded to BF16 (nearest even) into LDS, FP32
// accumulation.  Both LDS tiles are [outer][k] so that a lane's fragment (8
// consecutive k of one row or column) is one 16-byte read.  Each thread
// stages 16 elements of each operand per k-step, read along the operand's
// contiguous dimension: mode 1 = along k (written to LDS as two 16-byte
// runs), mode 2 = along the outer dimension (written as 16 scalars, a
// transpose), mode 0 = no unit stride (scalar reads, k-major mapping).
constexpr int HB = 128, HK = 32, HLD = HK + 8;
static_assert(32 * (HB + 4) * sizeof(float) <= 2 * HB * HLD * sizeof(uint16_t),
              "the epilogue's staging fits one operand's LDS tiles");

typedef __bf16 v8bf_t __attribute__((ext_vector_type(8)));


// One thread's 16 staged elements of an operand: as floats (converted to
// BF16 when stored), or, raw, the 16 BF16 values as loaded (an operand
// already in BF16 needs no conversion: its values round to themselves).
struct Stage {
  union {
    float v[16];
    uint32_t w[8];  // raw: element 2q in the low half of w[q], 2q + 1 in the high
  };
  int raw;
};

// Element (outer, k) of an operand: A is (m, k), B is (k, n).
__device__ __forceinline__ int64_t elem_addr(const GemmOperand& o, bool is_b, int64_t outer,
                                             int64_t k) {
  return is_b ? op_index(o, k, outer) : op_index(o, outer, k);
}

__device__ __forceinline__ void stage_load(const GemmOperand& o, bool is_b, int mode, int vec,
                                           int64_t outer0, int64_t k0, int64_t outer_lim,
                                           int64_t k_lim, int tid, Stage& st) {
  int64_t outer, k;
  int cnt;
  if (mode == 2) {
    k = k0 + tid / 8;
    outer = outer0 + (tid % 8) * 16;
    const int64_t left = outer_lim - outer;
    cnt = k < k_lim ? (left > 16 ? 16 : (left > 0 ? (int)left : 0)) : 0;
  } else {
    outer = outer0 + tid / 2;
    k = k0 + (tid % 2) * 16;
    const int64_t left = k_lim - k;
    cnt = outer < outer_lim ? (left > 16 ? 16 : (left > 0 ? (int)left : 0)) : 0;
  }
  st.raw = 0;
  if (mode != 0 && vec == 1 && cnt == 16) {  // 8-byte vectors
    const int64_t a = elem_addr(o, is_b, outer, k);
    if (o.bf16) {
      const uint2* p = reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(o.p) + a);
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const uint2 w = p[h];
        st.w[2 * h] = w.x;
        st.w[2 * h + 1] = w.y;
      }
      st.raw = 1;
    } else {
      const float2* p = reinterpret_cast<const float2*>(static_cast<const float*>(o.p) + a);
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        const float2 w = p[h];
        st.v[2 * h] = w.x;
        st.v[2 * h + 1] = w.y;
      }
    }
    return;
  }
  if (mode != 0 && vec == 2 && cnt == 16) {  // 16-byte vectors
    const int64_t a = elem_addr(o, is_b, outer, k);
    if (o.bf16) {
      const uint4* p = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(o.p) + a);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint4 w = p[h];
        st.w[4 * h] = w.x;
        st.w[4 * h + 1] = w.y;
        st.w[4 * h + 2] = w.z;
        st.w[4 * h + 3] = w.w;
      }
      st.raw = 1;
    } else {
      const float4* p = reinterpret_cast<const float4*>(static_cast<const float*>(o.p) + a);
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const float4 w = p[h];
        st.v[4 * h] = w.x;
        st.v[4 * h + 1] = w.y;
        st.v[4 * h + 2] = w.z;
        st.v[4 * h + 3] = w.w;
      }
    }
    return;
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    float v = 0.f;
    if (e < cnt)
      v = ld_elem(o.p, o.bf16,
                  mode == 2 ? elem_addr(o, is_b, outer + e, k) : elem_addr(o, is_b, outer, k + e));
    st.v[e] = v;
  }
}

// LDS tiles hold 8-element (16-byte) k-chunks; chunk c of row r sits at
// position c ^ ((r >> 4) & 3), so that the transposing stores of rows 16
// apart (same banks otherwise) spread over four bank groups.
__device__ __forceinline__ int chunk_at(int row, int c) { return c ^ ((row >> 4) & 3); }

__device__ __forceinline__ void stage_store(uint16_t (*S)[HLD], int mode, int tid,
                                            const Stage& st) {
  if (mode == 2) {
    const int k = tid / 8, outer = (tid % 8) * 16;
    if (st.raw) {
#pragma unroll
      for (int e = 0; e < 16; ++e)
        S[outer + e][8 * chunk_at(outer + e, k >> 3) + (k & 7)] =
            (uint16_t)(e & 1 ? st.w[e / 2] >> 16 : st.w[e / 2] & 0xffffu);
      return;
    }
#pragma unroll
    for (int e = 0; e < 16; ++e)
      S[outer + e][8 * chunk_at(outer + e, k >> 3) + (k & 7)] = to_bf16(st.v[e]);
  } else {
    const int outer = tid / 2, c0 = (tid % 2) * 2;
    uint32_t w[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      w[q] = st.raw ? st.w[q]
                    : (uint32_t)to_bf16(st.v[2 * q]) | ((uint32_t)to_bf16(st.v[2 * q + 1]) << 16);
    *reinterpret_cast<uint4*>(&S[outer][8 * chunk_at(outer, c0)]) = uint4{w[0], w[1], w[2], w[3]};
    *reinterpret_cast<uint4*>(&S[outer][8 * chunk_at(outer, c0 + 1)]) =
        uint4{w[4], w[5], w[6], w[7]};
  }
}

// The BF16 kernels' output: the tile's accumulators (wave (wm, wn) holds
// rows wm*64 .., columns wn*64 ..) to C through the epilogue (bias, ReLU
// mask, accumulate, BF16 output), or to the split-K partials.  E: LDS
// scratch of at least 32 x (HB + 4) floats, free once the products end.
__device__ __forceinline__ void gemm_bf16_epilogue(const GemmArgs& g, v4f (&acc)[4][4], float* E,
                                                   int64_t m0, int64_t n0, int wm, int wn, int tid,
                                                   int lane) {
  if (g.evec) {
    // whole 16-byte rows: the tile goes through LDS a quarter at a time (32
    // rows x 128 columns), and each thread finishes 16 consecutive columns
    // of one row with vector reads of the mask and previous C and vector
    // stores (full cache lines per row instead of 64-byte pieces)
    constexpr int ES = HB + 4;  // row stride of the staged quarter, in floats
    const int er = tid / 8, ec = (tid % 8) * 16;
    const int64_t m = m0 + (er / 16) * 64 + (er % 16);  // + i * 16
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          E[(wm * 16 + 4 * (lane >> 4) + r) * ES + wn * 64 + j * 16 + (lane & 15)] = acc[i][j][r];
      __syncthreads();
      const int64_t mi = m + i * 16, n = n0 + ec;
      if (mi < g.M && n < g.N) {
        float v[16];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float4 t = *reinterpret_cast<const float4*>(&E[er * ES + ec + 4 * q]);
          v[4 * q] = t.x;
          v[4 * q + 1] = t.y;
          v[4 * q + 2] = t.z;
          v[4 * q + 3] = t.w;
        }
        if (g.mask.p) {
          const int64_t a = grouped_row(mi, g.mask.grp, g.mask.gs, g.mask.rs) + n;
          float mk[16];
          if (g.mask.bf16) {
            const uint4* mp =
                reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(g.mask.p) + a);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const uint4 w = mp[h];
              const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                mk[8 * h + 2 * q] = __uint_as_float(ws[q] << 16);
                mk[8 * h + 2 * q + 1] = __uint_as_float(ws[q] & 0xffff0000u);
              }
            }
          } else {
            const float4* mp =
                reinterpret_cast<const float4*>(static_cast<const float*>(g.mask.p) + a);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const float4 w = mp[q];
              mk[4 * q] = w.x;
              mk[4 * q + 1] = w.y;
              mk[4 * q + 2] = w.z;
              mk[4 * q + 3] = w.w;
            }
          }
#pragma unroll
          for (int e = 0; e < 16; ++e)
            if (!(mk[e] > 0.f)) v[e] = 0.f;
        }
        const int64_t at = grouped_row(mi, g.cgrp, g.cgs, g.ldc) + n;
        if (g.c_bf16) {
          uint4* cp = reinterpret_cast<uint4*>(reinterpret_cast<uint16_t*>(g.C) + at);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
              w[q] = (uint32_t)to_bf16(v[8 * h + 2 * q]) |
                     ((uint32_t)to_bf16(v[8 * h + 2 * q + 1]) << 16);
            cp[h] = uint4{w[0], w[1], w[2], w[3]};
          }
        } else {
          float4* cp = reinterpret_cast<float4*>(g.C + at);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            float4 o = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
            if (g.beta) {
              const float4 c = cp[q];
              o = make_float4(c.x + o.x, c.y + o.y, c.z + o.z, c.w + o.w);
            }
            cp[q] = o;
          }
        }
      }
      __syncthreads();
    }
    return;
  }
  const int64_t nb = n0 + wn * 64 + (lane & 15);
  // the bias of this lane's four columns, read once (per row the compiler
  // would read it again after every store to C)
  float bj[4] = {0.f, 0.f, 0.f, 0.f};
  if (g.ksplit <= 1 && g.bias)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (nb + 16 * j < g.N) bj[j] = g.bias[nb + 16 * j];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
      if (m >= g.M) continue;
      const float v[4] = {acc[i][0][r] + bj[0], acc[i][1][r] + bj[1], acc[i][2][r] + bj[2],
                          acc[i][3][r] + bj[3]};
      if (g.ksplit > 1) {
        float* prow = g.part + ((int64_t)blockIdx.z * g.M + m) * g.N;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (nb + 16 * j < g.N) prow[nb + 16 * j] = v[j];
      } else {
        gemm_store_row4(g, m, nb, v);
      }
    }
}

__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][HB][HLD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][HB][HLD];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t m0 = (int64_t)blockIdx.y * HB, n0 = (int64_t)blockIdx.x * HB;
  const int wm = wave >> 1, wn = wave & 1;
  int64_t kb, ke;
  k_range(g, HK, &kb, &ke);
  v4f acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  Stage sa, sb;
  stage_load(g.A, false, g.amode, g.avec, m0, kb, g.M, ke, tid, sa);
  stage_load(g.B, true, g.bmode, g.bvec, n0, kb, g.N, ke, tid, sb);
  stage_store(As[0], g.amode, tid, sa);
  stage_store(Bs[0], g.bmode, tid, sb);
  __syncthreads();
  int cur = 0;
  for (int64_t k0 = kb; k0 < ke; k0 += HK) {
    const bool more = k0 + HK < ke;
    if (more) {  // next k-step's operands in flight during this one's MFMAs
      stage_load(g.A, false, g.amode, g.avec, m0, k0 + HK, g.M, ke, tid, sa);
      stage_load(g.B, true, g.bmode, g.bvec, n0, k0 + HK, g.N, ke, tid, sb);
    }
    uint4 af[4], bfr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = wm * 64 + i * 16 + (lane & 15);
      af[i] = *reinterpret_cast<const uint4*>(&As[cur][row][8 * chunk_at(row, lane >> 4)]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = wn * 64 + j * 16 + (lane & 15);
      bfr[j] = *reinterpret_cast<const uint4*>(&Bs[cur][row][8 * chunk_at(row, lane >> 4)]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf_t, af[i]),
                                                           __builtin_bit_cast(v8bf_t, bfr[j]),
                                                           acc[i][j], 0, 0, 0);
    if (more) {
      stage_store(As[cur ^ 1], g.amode, tid, sa);
      stage_store(Bs[cur ^ 1], g.bmode, tid, sb);
    }
    __syncthreads();
    cur ^= 1;
  }
  gemm_bf16_epilogue(g, acc, reinterpret_cast<float*>(&As[0][0][0]), m0, n0, wm, wn, tid, lane);
}

// out[n] = sum_{c < cnt} src[c * stride + n] for n < N, in a fixed order:
// 64 outputs per workgroup, four lanes per output summing every fourth c,
// then the four partial sums in lane order.  Split-K partials (with the
// GEMM epilogue) and column-sum partials both reduce through this.
template <bool GEMM>
__global__ void __launch_bounds__(256) strided_reduce(const float* __restrict__ src, int64_t cnt,
                                                      int64_t stride, int64_t N, GemmArgs g,
                                                      float* __restrict__ out, int beta) {
  __shared__ float red[4][64];
  const int col = threadIdx.x % 64, lane4 = threadIdx.x / 64;
  const int64_t n = (int64_t)blockIdx.x * 64 + col;
  float s = 0.f;
  if (n < N) {
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    int64_t c = lane4;
    for (; c + 12 < cnt; c += 16) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += src[(c + 4 * u) * stride + n];
    }
    for (; c < cnt; c += 4) acc[0] += src[c * stride + n];
    s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  }
  red[lane4][col] = s;
  __syncthreads();
  if (lane4 == 0 && n < N) {
    const float v = (red[0][col] + red[1][col]) + (red[2][col] + red[3][col]);
    if constexpr (GEMM) {
      gemm_store(g, n / g.N, n % g.N, v);
    } else {
      out[n] = beta ? out[n] + v : v;
    }
  }
}

// The same sums for long lists (cnt >= 64 partials): L lanes per output
// (16 or 64, one wave), lane l summing partials c = l, l + L, ... in order,
// then the L lane sums combined by a fixed butterfly (xor L/2, ..., 1), so
// the order is fixed and the latency is that of cnt / L loads, not cnt / 4.
template <bool GEMM>
__global__ void __launch_bounds__(256) strided_reduce_tree(const float* __restrict__ src,
                                                           int64_t cnt, int64_t stride, int64_t N,
                                                           int L, GemmArgs g,
                                                           float* __restrict__ out, int beta) {
  const int per_wg = 256 / L, sub = threadIdx.x % L;
  const int64_t n = (int64_t)blockIdx.x * per_wg + threadIdx.x / L;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  if (n < N) {
    int64_t c = sub;
    for (; c + 3 * L < cnt; c += 4 * L) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += src[(c + u * L) * stride + n];
    }
    for (; c < cnt; c += L) acc[0] += src[c * stride + n];
  }
  float v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  for (int off = L / 2; off >= 1; off /= 2) v += __shfl_xor(v, off);
  if (sub == 0 && n < N) {
    if constexpr (GEMM) {
      gemm_store(g, n / g.N, n % g.N, v);
    } else {
      out[n] = beta ? out[n] + v : v;
    }
  }
}

// 16 waves per 64 outputs (coalesced: a wave reads 64 adjacent outputs of
// one partial), wave w summing partials c = w, w + 16, ... in order, the 16
// wave sums then combined in LDS by a fixed pairwise tree: for long lists
// of partials of many outputs (the split-K weight gradients).
template <bool GEMM>
__global__ void __launch_bounds__(1024) strided_reduce_wide(const float* __restrict__ src,
                                                            int64_t cnt, int64_t stride, int64_t N,
                                                            GemmArgs g, float* __restrict__ out,
                                                            int beta) {
  __shared__ float red[16][64];
  const int col = threadIdx.x % 64, w = threadIdx.x / 64;
  const int64_t n = (int64_t)blockIdx.x * 64 + col;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  if (n < N) {
    int64_t c = w;
    for (; c + 48 < cnt; c += 64) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += src[(c + 16 * u) * stride + n];
    }
    for (; c < cnt; c += 16) acc[0] += src[c * stride + n];
  }
  red[w][col] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  for (int h = 8; h >= 1; h /= 2) {
    if (w < h) red[w][col] += red[w + h][col];
    __syncthreads();
  }
  if (w == 0 && n < N) {
    const float v = red[0][col];
    if constexpr (GEMM) {
      gemm_store(g, n / g.N, n % g.N, v);
    } else {
      out[n] = beta ? out[n] + v : v;
    }
  }
}

// Split-K partials of a GEMM with few parts (cnt < 64) and N a multiple of
// 4: each thread finishes four adjacent outputs of one row, its partials
// read as 16-byte vectors and added in part order, then the epilogue.
__global__ void __launch_bounds__(256) reduce_gemm_vec4(const float* __restrict__ src, int64_t cnt,
                                                        int64_t MN, GemmArgs g) {
  const int64_t q = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (q >= MN) return;
  float4 a = *reinterpret_cast<const float4*>(src + q);
#pragma unroll 4
  for (int64_t c = 1; c < cnt; ++c) {
    const float4 t = *reinterpret_cast<const float4*>(src + c * MN + q);
    a.x += t.x;
    a.y += t.y;
    a.z += t.z;
    a.w += t.w;
  }
  const int64_t m = q / g.N, n = q - m * g.N;
  gemm_store(g, m, n, a.x);
  gemm_store(g, m, n + 1, a.y);
  gemm_store(g, m, n + 2, a.z);
  gemm_store(g, m, n + 3, a.w);
}

// The same for a permuted C (ccg > 0, N = ccg * ccm, no bias, mask or BF16
// output, 16-byte aligned rows): each thread finishes four adjacent outputs
// of one row in C's own order, d -> GEMM column (d % ccm) * ccg + d / ccm,
// so the stores are 16-byte vectors and the permutation falls on the reads
// (a wave's 256 outputs read about two cache lines per part and tap).
__global__ void __launch_bounds__(256) reduce_gemm_perm4(const float* __restrict__ src,
                                                         int64_t cnt, int64_t MN, GemmArgs g) {
  const int64_t q = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (q >= MN) return;
  const int64_t m = q / g.N, d0 = q - m * g.N;
  int64_t col[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t d = d0 + e, t = d / g.ccm;
    col[e] = m * g.N + (d - t * g.ccm) * g.ccg + t;
  }
  float a[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) a[e] = src[col[e]];
#pragma unroll 4
  for (int64_t c = 1; c < cnt; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e) a[e] += src[c * MN + col[e]];
  float4* cp = reinterpret_cast<float4*>(g.C + m * g.ldc + d0);
  float4 o = make_float4(a[0], a[1], a[2], a[3]);
  if (g.beta) {
    const float4 p = *cp;
    o = make_float4(p.x + o.x, p.y + o.y, p.z + o.z, p.w + o.w);
  }
  *cp = o;
}

// Reduce cnt partials of N outputs (see strided_reduce) with the kernel
// that suits the shape: few outputs and a long list (the bias sums): many
// lanes per output; many outputs and a long list: 16 waves per 64 outputs;
// otherwise 4.
template <bool GEMM>
static void launch_reduce(const float* src, int64_t cnt, int64_t stride, int64_t N,
                          const GemmArgs& g, float* out, int beta, hipStream_t stream) {
  if (cnt >= 64 && N <= 1024) {
    const int L = cnt >= 256 ? 64 : 16;
    const int64_t per_wg = 256 / L;
    hipLaunchKernelGGL(strided_reduce_tree<GEMM>, dim3((unsigned)((N + per_wg - 1) / per_wg)),
                       dim3(256), 0, stream, src, cnt, stride, N, L, g, out, beta);
  } else if (cnt >= 64) {
    hipLaunchKernelGGL(strided_reduce_wide<GEMM>, dim3((unsigned)((N + 63) / 64)), dim3(1024), 0,
                       stream, src, cnt, stride, N, g, out, beta);
  } else {
    hipLaunchKernelGGL(strided_reduce<GEMM>, dim3((unsigned)((N + 63) / 64)), dim3(256), 0,
                       stream, src, cnt, stride, N, g, out, beta);
  }
}

// The BF16 kernel for operands that need no edge handling along k: the
// left one in BF16 with 16-byte runs along its contiguous dimension, the
// right one so too or FP32 along n (mode 3 below), rows not grouped (but
// mode 3's), each split-K range a whole number of HK-deep steps, tails of M
// and N filled as fast_op describes.  A thread's requests are then the same
// vectors per operand in every k-step, at addresses that step uniformly, so
// they run NS k-steps ahead of their use in a ring of NS register stages (past
// the end they repeat the last k-step's addresses: a uniform count of
// requests keeps every wait exact; the general kernel's per-thread paths
// force a wait for all of them), and the values go to LDS as loaded.
// AM, BM: the operands' modes (1 = contiguous along k, 2 = along the outer
// dimension, as in gemm_bf16_kernel; 3 = FP32 along n).  Same products in
// the same order as gemm_bf16_kernel, so the same results.  (NS = 3 here.)

// One thread's share of an operand, 16 elements per k-step.  Modes 1 and 2:
// BF16 in 16-byte runs, rows a fixed distance apart (the uint4s between
// consecutive k-steps in `step`).  Mode 3 (the right operand only): FP32
// runs along n in 8-byte pieces, rows (k) possibly grouped, rounded to BF16
// (nearest even, as gemm_bf16_kernel does) on their way to LDS, which then
// takes them as mode 2.  Past the matrix's outer size `dim` the tile is
// filled from rows (mode 1) or runs (modes 2, 3) that exist, the last row or
// the last whole run below the readable extent: they only reach outputs past
// M or N, which the epilogue does not store.
template <int MODE>
struct FastOp {
  static constexpr int W = 8;  // 32-bit words staged per k-step
  const uint4* p;
  int64_t step;
  __device__ __forceinline__ void load(int64_t i, uint32_t (&w)[W]) const {
    const uint4* q = p + i * step;
    const uint4 a = q[0], b = q[1];
    w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
    w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
  }
};

template <>
struct FastOp<3> {
  static constexpr int W = 16;
  const float* p;  // the run's first column, row offset 0
  int64_t k0, grp, gs, rs;
  __device__ __forceinline__ void load(int64_t i, uint32_t (&w)[W]) const {
    const uint2* q = reinterpret_cast<const uint2*>(p + grouped_row(k0 + i * HK, grp, gs, rs));
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const uint2 v = q[h];
      w[2 * h] = v.x;
      w[2 * h + 1] = v.y;
    }
  }
};

template <int MODE>
__device__ __forceinline__ FastOp<MODE> fast_op(const GemmOperand& o, bool is_b, int64_t outer0,
                                                int64_t dim, int64_t kb, int tid) {
  int64_t outer;
  if constexpr (MODE >= 2) {
    const int64_t cap = o.ext ? o.ext : dim;  // a multiple of 16, at least dim
    outer = outer0 + (tid % 8) * 16;
    if (outer > cap - 16) outer = cap - 16;
  } else {
    outer = outer0 + tid / 2;
    if (outer > dim - 1) outer = dim - 1;
  }
  const int64_t k = MODE >= 2 ? kb + tid / 8 : kb + (tid % 2) * 16;
  FastOp<MODE> f;
  if constexpr (MODE == 3) {
    f.p = static_cast<const float*>(o.p) + outer;
    f.k0 = k;
    f.grp = o.grp;
    f.gs = o.gs;
    f.rs = o.rs;
  } else {
    f.step = HK * (is_b ? o.rs : o.cs) / 8;
    f.p = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(o.p) +
                                         elem_addr(o, is_b, outer, k));
  }
  return f;
}

template <int MODE>
__device__ __forceinline__ void fast_store(uint16_t (*S)[HLD], int tid,
                                           const uint32_t (&w)[FastOp<MODE>::W]) {
  if constexpr (MODE == 3) {
    uint32_t h[8];
#pragma unroll
    for (int e = 0; e < 8; ++e)
      h[e] = (uint32_t)to_bf16(__uint_as_float(w[2 * e])) |
             ((uint32_t)to_bf16(__uint_as_float(w[2 * e + 1])) << 16);
    fast_store<2>(S, tid, h);
  } else if constexpr (MODE == 2) {
    const int k = tid / 8, outer = (tid % 8) * 16;
#pragma unroll
    for (int e = 0; e < 16; ++e)
      S[outer + e][8 * chunk_at(outer + e, k >> 3) + (k & 7)] =
          (uint16_t)(e & 1 ? w[e / 2] >> 16 : w[e / 2] & 0xffffu);
  } else {
    const int outer = tid / 2, c0 = (tid % 2) * 2;
    *reinterpret_cast<uint4*>(&S[outer][8 * chunk_at(outer, c0)]) = uint4{w[0], w[1], w[2], w[3]};
    *reinterpret_cast<uint4*>(&S[outer][8 * chunk_at(outer, c0 + 1)]) =
        uint4{w[4], w[5], w[6], w[7]};
  }
}

// k-step i of gemm_bf16_fast_kernel: request step i + 3 into the stage (la,
// lb) that held step i's operands, multiply LDS buffer CUR, store step i +
// 1's stage (sa, sb), requested two steps ago, into the other buffer.
template <int AM, int BM, int CUR>
__device__ __forceinline__ void fast_step(int64_t i, int64_t n_steps, v4f (&acc)[4][4],
                                          uint16_t (*As)[HB][HLD], uint16_t (*Bs)[HB][HLD],
                                          const FastOp<AM>& pa, const FastOp<BM>& pb,
                                          uint32_t (&la)[FastOp<AM>::W],
                                          uint32_t (&lb)[FastOp<BM>::W],
                                          const uint32_t (&sa)[FastOp<AM>::W],
                                          const uint32_t (&sb)[FastOp<BM>::W], int wm, int wn,
                                          int lane, int tid, bool do_rs, float& rs) {
  const int64_t r = i + 3 < n_steps ? i + 3 : n_steps - 1;  // past the end: the last again
  pa.load(r, la);
  pb.load(r, lb);
  uint4 af[4], bfr[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int row = wm * 64 + a * 16 + (lane & 15);
    af[a] = *reinterpret_cast<const uint4*>(&As[CUR][row][8 * chunk_at(row, lane >> 4)]);
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int row = wn * 64 + b * 16 + (lane & 15);
    bfr[b] = *reinterpret_cast<const uint4*>(&Bs[CUR][row][8 * chunk_at(row, lane >> 4)]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf_t, af[a]),
                                                         __builtin_bit_cast(v8bf_t, bfr[b]),
                                                         acc[a][b], 0, 0, 0);
  if (do_rs) {  // this thread's half of row tid / 2 of the A tile, in k order
    const int row = tid >> 1, h = tid & 1;
    const uint4 x0 = *reinterpret_cast<const uint4*>(&As[CUR][row][8 * chunk_at(row, 2 * h)]);
    const uint4 x1 =
        *reinterpret_cast<const uint4*>(&As[CUR][row][8 * chunk_at(row, 2 * h + 1)]);
    const uint32_t w[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      t += __uint_as_float(w[q] << 16);
      t += __uint_as_float(w[q] & 0xffff0000u);
    }
    rs += t;
  }
  if (i + 1 < n_steps) {
    fast_store<AM>(As[CUR ^ 1], tid, sa);
    fast_store<BM>(Bs[CUR ^ 1], tid, sb);
  }
  __syncthreads();
}

// The tile of this workgroup.  Workgroups go to the 8 XCDs in turn (id %
// 8), each XCD with its own L2: when the tiles of a k-split divide evenly,
// XCD x takes the x-th eighth of them in row-major order along the longer
// tile dimension, a band that shares the shorter operand whole and holds an
// eighth of the other, instead of tiles from everywhere.
__device__ __forceinline__ void xcd_tile(int64_t* tm, int64_t* tn) {
  const int64_t nx = gridDim.x, ny = gridDim.y, tiles = nx * ny;
  *tm = blockIdx.y;
  *tn = blockIdx.x;
  if (tiles % 8 != 0 || tiles < 64) return;
  const int64_t id = (int64_t)blockIdx.y * nx + blockIdx.x;
  const int64_t t = (id % 8) * (tiles / 8) + id / 8;
  if (ny >= nx) {
    *tm = t / nx;
    *tn = t % nx;
  } else {
    *tn = t / ny;
    *tm = t % ny;
  }
}

template <int AM, int BM>
__global__ void __launch_bounds__(256, 2) gemm_bf16_fast_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][HB][HLD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][HB][HLD];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  int64_t tm, tn;
  xcd_tile(&tm, &tn);
  const int64_t m0 = tm * HB, n0 = tn * HB;
  const int wm = wave >> 1, wn = wave & 1;
  int64_t kb, ke;
  k_range(g, HK, &kb, &ke);
  v4f acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  const int64_t n = (ke - kb) / HK;
  // the workgroups of the first column of tiles also sum A's rows
  const bool do_rs = g.rowsum != nullptr && tn == 0;
  float rs = 0.f;
  if (n > 0) {
    const FastOp<AM> pa = fast_op<AM>(g.A, false, m0, g.M, kb, tid);
    const FastOp<BM> pb = fast_op<BM>(g.B, true, n0, g.N, kb, tid);
    // three register stages; k-step i's operands are requested into stage
    // i % 3 at the start of step i - 3 (the first three here)
    uint32_t a0[FastOp<AM>::W], a1[FastOp<AM>::W], a2[FastOp<AM>::W];
    uint32_t b0[FastOp<BM>::W], b1[FastOp<BM>::W], b2[FastOp<BM>::W];
    pa.load(0, a0);
    pb.load(0, b0);
    pa.load(n > 1 ? 1 : 0, a1);
    pb.load(n > 1 ? 1 : 0, b1);
    pa.load(n > 2 ? 2 : n - 1, a2);
    pb.load(n > 2 ? 2 : n - 1, b2);
    fast_store<AM>(As[0], tid, a0);
    fast_store<BM>(Bs[0], tid, b0);
    __syncthreads();
    // six steps per iteration, so that stages (i % 3) and LDS buffers (i % 2)
    // are fixed registers and fixed addresses
    // (the guards are nested: a step runs only after the one before it, so
    // the compiler counts the requests in flight exactly)
    for (int64_t i = 0; i < n; i += 6) {
      fast_step<AM, BM, 0>(i, n, acc, As, Bs, pa, pb, a0, b0, a1, b1, wm, wn, lane, tid, do_rs, rs);
      if (i + 1 < n) {
        fast_step<AM, BM, 1>(i + 1, n, acc, As, Bs, pa, pb, a1, b1, a2, b2, wm, wn, lane, tid, do_rs, rs);
        if (i + 2 < n) {
          fast_step<AM, BM, 0>(i + 2, n, acc, As, Bs, pa, pb, a2, b2, a0, b0, wm, wn,
                               lane, tid, do_rs, rs);
          if (i + 3 < n) {
            fast_step<AM, BM, 1>(i + 3, n, acc, As, Bs, pa, pb, a0, b0, a1, b1, wm, wn,
                                 lane, tid, do_rs, rs);
            if (i + 4 < n) {
              fast_step<AM, BM, 0>(i + 4, n, acc, As, Bs, pa, pb, a1, b1, a2, b2, wm, wn,
                                   lane, tid, do_rs, rs);
              if (i + 5 < n)
                fast_step<AM, BM, 1>(i + 5, n, acc, As, Bs, pa, pb, a2, b2, a0, b0, wm,
                                     wn, lane, tid, do_rs, rs);
            }
          }
        }
      }
    }
  }
  if (do_rs) {  // the two halves of each row, then one row sum per row below M
    const float other = __shfl_xor(rs, 1);
    const int64_t m = m0 + (tid >> 1);
    if ((tid & 1) == 0 && m < g.M) g.rowsum[(int64_t)blockIdx.z * g.M + m] = rs + other;
  }
  gemm_bf16_epilogue(g, acc, reinterpret_cast<float*>(&As[0][0][0]), m0, n0, wm, wn, tid, lane);
}

// Operand access mode for the BF16 kernel (see gemm_bf16_kernel) and the
// vector reads a run of 16 elements allows: 2 = 16-byte, 1 = 8-byte (rows
// of an odd multiple of 8 bytes apart, e.g. windows of 111 x 50 FP32
// features), 0 = none.
static void operand_mode(const GemmOperand& o, bool is_b, int32_t* mode, int32_t* vec) {
  const bool grouped = o.grp < NO_GROUP;
  const int64_t k_stride = is_b ? o.rs : o.cs, outer_stride = is_b ? o.cs : o.rs;
  const bool k_is_row = is_b;  // grouping applies to the row index
  if (k_stride == 1 && !(k_is_row && grouped))
    *mode = 1;
  else if (outer_stride == 1 && !(!k_is_row && grouped))
    *mode = 2;
  else
    *mode = 0;
  const int64_t other = *mode == 1 ? outer_stride : k_stride;
  auto fits = [&](int64_t bytes) {
    const int64_t q = bytes / (o.bf16 ? 2 : 4);  // elements per vector
    return *mode != 0 && (reinterpret_cast<uintptr_t>(o.p) % bytes == 0) && other % q == 0 &&
           (!grouped || o.gs % q == 0);
  };
  *vec = fits(16) ? 2 : fits(8) ? 1 : 0;
}

hipError_t launch_gemm(GemmArgs g, int bf16_mma, float* part, int64_t part_cap,
                       hipStream_t stream, int64_t* rowsum_parts) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const int TB = bf16_mma ? HB : GB;
  const int64_t tiles = ((g.M + TB - 1) / TB) * ((g.N + TB - 1) / TB);
  // split K when the output is too small to fill the chip: aim at one round
  // of workgroups (512: two per CU), at least 8 k-steps each, within the
  // partial buffer
  int64_t ks = 1;
  if (part && tiles < 128) {
    ks = 512 / tiles;
    const int64_t steps = g.K / ((bf16_mma ? HK : GK) * 8);
    if (ks > steps) ks = steps;
    if (ks > part_cap / (g.M * g.N)) ks = part_cap / (g.M * g.N);
    if (ks > 65535) ks = 65535;
    if (ks < 2) ks = 1;
  }
  // grouped rows are divided in 32 bits
  const int64_t big = (int64_t)1 << 32;
  if ((g.A.grp < NO_GROUP && g.M >= big) || (g.B.grp < NO_GROUP && g.K >= big) ||
      (g.mask.p && g.mask.grp < NO_GROUP && g.M >= big) || (g.cgrp < NO_GROUP && g.M >= big) ||
      (g.ccg != 0 && (g.ccg < 0 || g.N >= big)))
    return hipErrorInvalidValue;
  g.ksplit = (int32_t)ks;
  g.part = part;
  operand_mode(g.A, false, &g.amode, &g.avec);
  operand_mode(g.B, true, &g.bmode, &g.bvec);
  // the BF16 kernel's vector epilogue: no split, no bias, N whole 16-column
  // runs, C and the mask in 16-byte aligned rows contiguous along n
  {
    const int64_t mq = g.mask.bf16 ? 8 : 4;
    const int64_t cq = g.c_bf16 ? 8 : 4;  // elements per 16 bytes of C
    const bool c_ok = reinterpret_cast<uintptr_t>(g.C) % 16 == 0 && g.ldc % cq == 0 &&
                      (g.cgrp >= NO_GROUP || g.cgs % cq == 0);
    const bool m_ok = !g.mask.p || (g.mask.cs == 1 &&
                                    reinterpret_cast<uintptr_t>(g.mask.p) % 16 == 0 &&
                                    g.mask.rs % mq == 0 &&
                                    (g.mask.grp >= NO_GROUP || g.mask.gs % mq == 0));
    g.evec = bf16_mma && ks == 1 && !g.bias && g.ccg == 0 && g.N % 16 == 0 && c_ok && m_ok;
  }
  const dim3 grid((unsigned)((g.N + TB - 1) / TB), (unsigned)((g.M + TB - 1) / TB), (unsigned)ks);
  // operands with nothing to guard along k: the pipelined kernel (rows
  // along the outer dimension are clamped; runs of 16 along it need a
  // readable extent of whole runs)
  auto whole_runs = [](const GemmOperand& o, int32_t mode, int64_t dim) {
    const int64_t cap = o.ext ? o.ext : dim;
    return mode == 1 || (cap % 16 == 0 && cap >= dim);
  };
  const bool fast_a = bf16_mma && g.A.bf16 && g.avec == 2 && g.amode != 0 &&
                      g.A.grp >= NO_GROUP && whole_runs(g.A, g.amode, g.M) && g.K % HK == 0;
  const bool fast_b = g.B.bf16 && g.bvec == 2 && g.bmode != 0 && g.B.grp >= NO_GROUP &&
                      whole_runs(g.B, g.bmode, g.N);
  // FP32 along n in 8-byte pieces, rows possibly grouped (e.g. the windows)
  const bool fast_b32 = !g.B.bf16 && g.bvec >= 1 && g.bmode == 2 && whole_runs(g.B, 2, g.N);
  if (rowsum_parts) *rowsum_parts = (fast_a && (fast_b32 || fast_b) && g.rowsum) ? ks : 0;
  if (!(fast_a && (fast_b32 || fast_b))) g.rowsum = nullptr;
  if (fast_a && fast_b32) {
    if (g.amode == 1)
      hipLaunchKernelGGL((gemm_bf16_fast_kernel<1, 3>), grid, dim3(256), 0, stream, g);
    else
      hipLaunchKernelGGL((gemm_bf16_fast_kernel<2, 3>), grid, dim3(256), 0, stream, g);
  } else if (fast_a && fast_b) {
    if (g.amode == 1 && g.bmode == 1)
      hipLaunchKernelGGL((gemm_bf16_fast_kernel<1, 1>), grid, dim3(256), 0, stream, g);
    else if (g.amode == 1)
      hipLaunchKernelGGL((gemm_bf16_fast_kernel<1, 2>), grid, dim3(256), 0, stream, g);
    else if (g.bmode == 1)
      hipLaunchKernelGGL((gemm_bf16_fast_kernel<2, 1>), grid, dim3(256), 0, stream, g);
    else
      hipLaunchKernelGGL((gemm_bf16_fast_kernel<2, 2>), grid, dim3(256), 0, stream, g);
  } else if (bf16_mma) {
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, stream, g);
  } else {
    hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, stream, g);
  }
  if (ks > 1) {
    const int64_t MN = g.M * g.N;
    const bool perm4 = g.ccg > 0 && g.N == g.ccg * g.ccm && !g.bias && !g.mask.p && !g.c_bf16 &&
                       g.cgrp >= NO_GROUP && g.ldc % 4 == 0 &&
                       reinterpret_cast<uintptr_t>(g.C) % 16 == 0;
    if (ks < 64 && g.N % 4 == 0 && perm4)
      hipLaunchKernelGGL(reduce_gemm_perm4, dim3((unsigned)((MN / 4 + 255) / 256)), dim3(256), 0,
                         stream, part, ks, MN, g);
    else if (ks < 64 && g.N % 4 == 0)
      hipLaunchKernelGGL(reduce_gemm_vec4, dim3((unsigned)((MN / 4 + 255) / 256)), dim3(256), 0,
                         stream, part, ks, MN, g);
    else
      launch_reduce<true>(part, ks, MN, MN, g, nullptr, 0, stream);
  }
  return hipGetLastError();
}

// Per latency type t the head outputs are n_bins class logits and one
// regression output; loss = CE(class min(lat, n_bins - 1)) + |reg -
// log1p(lat)| summed over t; dz = (softmax - onehot) / B, dreg = sign / B.
// One wavefront per (window, t), its logits held in registers (LOSS_PER per
// lane, lane l taking bins l, l + 64, ...), max and sum of exponentials
// reduced across the wave by a fixed butterfly; four waves (two windows) per
// workgroup, each window's two terms added in t order.
constexpr int LOSS_PER = 8;  // bins per lane: n_bins <= 64 * LOSS_PER
__global__ void __launch_bounds__(256)
    loss_kernel(const float* __restrict__ z, const int32_t* __restrict__ lat, int64_t B,
                int32_t n_bins, float* __restrict__ loss_b, float* __restrict__ dz) {
  __shared__ float part[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t b = (int64_t)blockIdx.x * 2 + (w >> 1);
  const int t = w & 1;
  const int per = n_bins + 1;
  float term = 0.f;
  if (b < B) {
    const float* zt = z + (b * 2 + t) * per;
    const int l = lat[b * 2 + t];
    const int bin = l < n_bins - 1 ? l : n_bins - 1;
    float v[LOSS_PER];
    float m = -INFINITY;
#pragma unroll
    for (int q = 0; q < LOSS_PER; ++q) {
      const int i = lane + 64 * q;
      v[q] = i < n_bins ? zt[i] : -INFINITY;
      m = fmaxf(m, v[q]);
    }
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    float se = 0.f;
#pragma unroll
    for (int q = 0; q < LOSS_PER; ++q)
      if (lane + 64 * q < n_bins) se += expf(v[q] - m);
    for (int o = 32; o >= 1; o >>= 1) se += __shfl_xor(se, o);
    const float lse = m + logf(se);
    const float zr = zt[n_bins], zb = zt[bin];
    const float r = zr - log1pf((float)l);
    const float inv = 1.f / (float)B;
    float* dzt = dz + (b * 2 + t) * per;
#pragma unroll
    for (int q = 0; q < LOSS_PER; ++q) {
      const int i = lane + 64 * q;
      if (i < n_bins) dzt[i] = inv * (expf(v[q] - lse) - (i == bin ? 1.f : 0.f));
    }
    if (lane == 0) dzt[n_bins] = inv * (r > 0.f ? 1.f : (r < 0.f ? -1.f : 0.f));
    term = lse - zb + fabsf(r);
  }
  if (lane == 0) part[w] = term;
  __syncthreads();
  if ((threadIdx.x & 127) == 0 && b < B) loss_b[b] = part[w] + part[w + 1];
}

// loss = mean of per-window losses, summed in a fixed order (one workgroup).
__global__ void __launch_bounds__(256) mean_kernel(const float* __restrict__ v, int64_t n,
                                                   float* __restrict__ out) {
  __shared__ double part[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += v[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (float)(part[0] / (double)n);
}

hipError_t launch_loss(const float* z, const int32_t* lat, int64_t B, int32_t n_bins,
                       float* loss_b, float* loss, float* dz, hipStream_t stream) {
  if (n_bins < 1 || n_bins > 64 * LOSS_PER) return hipErrorInvalidValue;
  hipLaunchKernelGGL(loss_kernel, dim3((unsigned)((B + 1) / 2)), dim3(256), 0, stream, z, lat, B,
                     n_bins, loss_b, dz);
  hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(256), 0, stream, loss_b, B, loss);
  return hipGetLastError();
}

// Column sums of Y [M][ld] over rows in a fixed order: chunks of rows
// summed per workgroup, then the chunk partials through sum_partials.
// Partial column sums (rows without whole vectors): workgroup (x, c) sums rows [c*per, (c+1)*per) of
// columns [x*64*V, (x+1)*64*V), V adjacent columns per lane (V = 2 for BF16
// input, read as one 32-bit word), 4 row lanes per column, in a fixed order.
template <bool BF>
__global__ void __launch_bounds__(256) colsum_partial(const void* __restrict__ yv, int64_t M,
                                                      int64_t N, int64_t ld, int64_t per,
                                                      float* __restrict__ part) {
  constexpr int V = BF ? 2 : 1;
  __shared__ float red[4][64 * V];
  const int col = threadIdx.x % 64, lane4 = threadIdx.x / 64;
  const int64_t n = ((int64_t)blockIdx.x * 64 + col) * V;
  const int64_t c = blockIdx.y, lo = c * per, hi = lo + per < M ? lo + per : M;
  float acc[2][V];
#pragma unroll
  for (int v = 0; v < V; ++v) acc[0][v] = acc[1][v] = 0.f;
  auto add = [&](int slot, int64_t m) {
    if constexpr (BF) {
      const uint16_t* y = static_cast<const uint16_t*>(yv) + m * ld + n;
      if (n + 1 < N) {  // (ld and n even: 4-byte aligned)
        const uint32_t w = *reinterpret_cast<const uint32_t*>(y);
        acc[slot][0] += __uint_as_float(w << 16);
        acc[slot][1] += __uint_as_float(w & 0xffff0000u);
      } else {
        acc[slot][0] += __uint_as_float((uint32_t)y[0] << 16);
      }
    } else {
      acc[slot][0] += static_cast<const float*>(yv)[m * ld + n];
    }
  };
  if (n < N) {
    int64_t m = lo + lane4;
    for (; m + 4 < hi; m += 8) {
      add(0, m);
      add(1, m + 4);
    }
    for (; m < hi; m += 4) add(0, m);
  }
#pragma unroll
  for (int v = 0; v < V; ++v) red[lane4][col * V + v] = acc[0][v] + acc[1][v];
  __syncthreads();
  if (lane4 == 0)
#pragma unroll
    for (int v = 0; v < V; ++v)
      if (n + v < N)
        part[c * N + n + v] = (red[0][col * V + v] + red[1][col * V + v]) +
                              (red[2][col * V + v] + red[3][col * V + v]);
}

// Partial column sums for rows whose columns come in whole VB-byte vectors
// (VW columns each).  Workgroup (x, c) takes column block x (TPR vectors side
// by side) and rows [c*per, min(M, (c+1)*per)): RP = 256 / TPR row lanes,
// lane r summing rows lo + r, lo + r + RP, ... in order, four requests in
// flight; the RP lane sums are combined by a fixed pairwise tree in LDS into
// part[c][n], which sum_partials then adds over c.  (A single launch in
// which the last workgroup of a block adds the partials was slower: the
// device-scope release each workgroup needs before counting writes back its
// XCD's whole L2.)
template <bool BF, int VB>
struct ColVec {
  static constexpr int VW = VB / (BF ? 2 : 4);
  using T = typename std::conditional<VB == 16, uint4, uint2>::type;
  __device__ static __forceinline__ T load(const void* y, int64_t at) {
    return *reinterpret_cast<const T*>(static_cast<const char*>(y) + at * (BF ? 2 : 4));
  }
  __device__ static __forceinline__ void add(float (&a)[VW], const T& t) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(&t);
#pragma unroll
    for (int q = 0; q < VB / 4; ++q) {
      if constexpr (BF) {
        a[2 * q] += __uint_as_float(w[q] << 16);
        a[2 * q + 1] += __uint_as_float(w[q] & 0xffff0000u);
      } else {
        a[q] += __uint_as_float(w[q]);
      }
    }
  }
};

template <int VW>
__device__ __forceinline__ void lane_tree(float (&a)[VW], float* red, int r, int j, int tpr,
                                          int rp) {
#pragma unroll
  for (int v = 0; v < VW; ++v) red[(r * tpr + j) * VW + v] = a[v];
  __syncthreads();
  for (int h = rp / 2; h >= 1; h /= 2) {
    if (r < h)
#pragma unroll
      for (int v = 0; v < VW; ++v)
        red[(r * tpr + j) * VW + v] += red[((r + h) * tpr + j) * VW + v];
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < VW; ++v) a[v] = red[j * VW + v];
}

template <bool BF, int VB>
__global__ void __launch_bounds__(256) colsum_vec(const void* __restrict__ y, int64_t M, int64_t N,
                                                  int64_t ld, int64_t per, int tpr,
                                                  float* __restrict__ part) {
  using V = ColVec<BF, VB>;
  constexpr int VW = V::VW;
  __shared__ float red[256 * VW];
  const int tid = threadIdx.x, j = tid % tpr, r = tid / tpr, rp = 256 / tpr;
  const int64_t n = (int64_t)blockIdx.x * tpr * VW + j * VW;
  const int64_t c = blockIdx.y, lo = c * per, hi = lo + per < M ? lo + per : M;
  const bool on = n < N;
  float a[VW];
#pragma unroll
  for (int v = 0; v < VW; ++v) a[v] = 0.f;
  if (on) {
    int64_t m = lo + r;
    for (; m + 3 * rp < hi; m += 4 * rp) {
      const typename V::T t0 = V::load(y, m * ld + n), t1 = V::load(y, (m + rp) * ld + n),
                          t2 = V::load(y, (m + 2 * rp) * ld + n),
                          t3 = V::load(y, (m + 3 * rp) * ld + n);
      V::add(a, t0);
      V::add(a, t1);
      V::add(a, t2);
      V::add(a, t3);
    }
    for (; m < hi; m += rp) V::add(a, V::load(y, m * ld + n));
  }
  lane_tree<VW>(a, red, r, j, tpr, rp);
  if (r == 0 && on)
#pragma unroll
    for (int v = 0; v < VW; ++v) part[c * N + n + v] = a[v];
}

hipError_t launch_colsum_partial(const void* y, int y_bf16, int64_t M, int64_t N, int64_t ld,
                                 float* work, int64_t* chunks_out, hipStream_t stream) {
  *chunks_out = 0;
  if (N <= 0) return hipSuccess;
  {
    // whole vectors along the rows: 16 bytes, else 8
    const int es = y_bf16 ? 2 : 4;
    const uintptr_t a = reinterpret_cast<uintptr_t>(y);
    auto fits = [&](int vb) {
      const int64_t vw = vb / es;
      return a % vb == 0 && N % vw == 0 && ld % vw == 0;
    };
    const int vb = fits(16) ? 16 : fits(8) ? 8 : 0;
    if (vb && M > 0) {
      const int vw = vb / es;
      int tpr = 1;
      while (tpr < 64 && (int64_t)tpr * vw < N) tpr *= 2;
      const int rp = 256 / tpr;
      const int64_t blocks = (N + (int64_t)tpr * vw - 1) / ((int64_t)tpr * vw);
      if (blocks <= 65535) {
        int64_t chunks = (M + rp * 8 - 1) / (rp * 8);  // about 8 rows per lane
        if (chunks > COLSUM_MAX_CHUNKS) chunks = COLSUM_MAX_CHUNKS;
        const int64_t per = (M + chunks - 1) / chunks;
        chunks = (M + per - 1) / per;
        const dim3 grid((unsigned)blocks, (unsigned)chunks);
#define SIMNET_COLSUM(BF, VB)                                                                   \
  hipLaunchKernelGGL((colsum_vec<BF, VB>), grid, dim3(256), 0, stream, y, M, N, ld, per, tpr, \
                     work)
        if (y_bf16 && vb == 16) SIMNET_COLSUM(true, 16);
        else if (y_bf16) SIMNET_COLSUM(true, 8);
        else if (vb == 16) SIMNET_COLSUM(false, 16);
        else SIMNET_COLSUM(false, 8);
#undef SIMNET_COLSUM
        *chunks_out = chunks;
        return hipGetLastError();
      }
    }
  }
  int64_t chunks = (M + 63) / 64;
  if (chunks > COLSUM_MAX_CHUNKS) chunks = COLSUM_MAX_CHUNKS;
  if (chunks < 1) chunks = 1;
  const int64_t per = (M + chunks - 1) / chunks;
  // (BF16: two adjacent columns per lane, which needs even N and ld)
  if (y_bf16 && N % 2 == 0 && ld % 2 == 0)
    hipLaunchKernelGGL(colsum_partial<true>, dim3((unsigned)((N + 127) / 128), (unsigned)chunks),
                       dim3(256), 0, stream, y, M, N, ld, per, work);
  else if (y_bf16)
    return hipErrorInvalidValue;
  else
    hipLaunchKernelGGL(colsum_partial<false>, dim3((unsigned)((N + 63) / 64), (unsigned)chunks),
                       dim3(256), 0, stream, y, M, N, ld, per, work);
  *chunks_out = chunks;
  return hipGetLastError();
}

// Several lists of partials summed in one launch: workgroup b serves the
// segment whose block range holds b; per segment L lanes per output (16 or
// 64, or 4 for short lists), lane l summing partials c = l, l + L, ... in
// order, then the L lane sums combined by a fixed butterfly.
__global__ void __launch_bounds__(256) sum_partials(SumSegs segs) {
  int s = 0;
  int64_t b = blockIdx.x;
  while (s + 1 < segs.count && b >= segs.seg[s].blocks) {
    b -= segs.seg[s].blocks;
    ++s;
  }
  const SumSeg& q = segs.seg[s];
  const int L = q.lanes, sub = threadIdx.x % L;
  const int64_t n = b * (256 / L) + threadIdx.x / L;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  if (n < q.N) {
    int64_t c = sub;
    for (; c + 3 * L < q.cnt; c += 4 * L) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += q.src[(c + u * L) * q.N + n];
    }
    for (; c < q.cnt; c += L) acc[0] += q.src[c * q.N + n];
  }
  float v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  for (int off = L / 2; off >= 1; off /= 2) v += __shfl_xor(v, off);
  if (sub == 0 && n < q.N) q.out[n] = segs.beta ? q.out[n] + v : v;
}

hipError_t launch_sum_partials(SumSegs segs, hipStream_t stream) {
  if (segs.count < 1 || segs.count > SumSegs::MAX) return hipErrorInvalidValue;
  int64_t blocks = 0;
  for (int s = 0; s < segs.count; ++s) {
    SumSeg& q = segs.seg[s];
    q.lanes = q.cnt >= 256 ? 64 : q.cnt >= 32 ? 16 : 4;
    q.blocks = (q.N + 256 / q.lanes - 1) / (256 / q.lanes);
    blocks += q.blocks;
  }
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(sum_partials, dim3((unsigned)blocks), dim3(256), 0, stream, segs);
  return hipGetLastError();
}

// dst[r][c] = src[r][c] for c < cols, 0 for cols <= c < ld: rows padded to
// a stride whose 16-byte vectors the GEMM operand reads can use.
// One workgroup row per matrix row (grid x), 256 columns per workgroup
// (grid y).
__global__ void pad_rows(const float* __restrict__ src, int64_t cols, int64_t ld,
                         void* __restrict__ dst, int32_t dst_bf16) {
  const int64_t r = blockIdx.x, c = (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (c >= ld) return;
  const float v = c < cols ? src[r * cols + c] : 0.f;
  if (dst_bf16)
    static_cast<uint16_t*>(dst)[r * ld + c] = to_bf16(v);
  else
    static_cast<float*>(dst)[r * ld + c] = v;
}

hipError_t launch_pad_rows(const float* src, int64_t rows, int64_t cols, int64_t ld, void* dst,
                           int32_t dst_bf16, hipStream_t stream) {
  if (rows <= 0) return hipSuccess;
  if (rows > INT32_MAX || (ld + 255) / 256 > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pad_rows, dim3((unsigned)rows, (unsigned)((ld + 255) / 256)), dim3(256), 0,
                     stream, src, cols, ld, dst, dst_bf16);
  return hipGetLastError();
}

// dst[i] = src[map[i]] (0 where map < 0), stored as FP32 or BF16 (nearest
// even), for several (map, n, dst) segments from one source in one launch:
// workgroup b serves the segment whose block range holds b (segments in
// order, each rounded up to whole workgroups).
__global__ void map_gather_multi(const float* __restrict__ src, GatherSegs segs) {
  int s = 0;
  int64_t b = blockIdx.x;
  while (s + 1 < segs.count && b >= (segs.seg[s].n + 255) / 256) {
    b -= (segs.seg[s].n + 255) / 256;
    ++s;
  }
  const GatherSeg& g = segs.seg[s];
  const int64_t i = b * 256 + threadIdx.x;
  if (i >= g.n) return;
  const int32_t k = g.map[i];
  const float v = k < 0 ? 0.f : src[k];
  if (g.bf16) {
    const uint32_t u = __float_as_uint(v);
    static_cast<uint16_t*>(g.dst)[i] = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
  } else {
    static_cast<float*>(g.dst)[i] = v;
  }
}

hipError_t launch_map_gather_multi(const float* src, const GatherSegs& segs, hipStream_t stream) {
  if (segs.count < 1 || segs.count > GatherSegs::MAX) return hipErrorInvalidValue;
  int64_t blocks = 0;
  for (int s = 0; s < segs.count; ++s) blocks += (segs.seg[s].n + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(map_gather_multi, dim3((unsigned)blocks), dim3(256), 0, stream, src, segs);
  return hipGetLastError();
}

__global__ void zero_kernel(float* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

hipError_t launch_zero(float* p, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

// One Adam step (Kingma & Ba, bias corrections c1 = 1 - b1^t, c2 = 1 -
// b2^t, no weight decay) on values: the moments updated in place, the new
// weight returned.  Every Adam kernel here applies this one function with
// contraction into fused multiply-adds off, so they all round alike.
__device__ __forceinline__ float adam_math(float gi, float& mi, float& vi, float wi, float lr,
                                           float b1, float b2, float eps, float c1, float c2) {
#pragma clang fp contract(off)
  mi = b1 * mi + (1.f - b1) * gi;
  vi = b2 * vi + (1.f - b2) * gi * gi;
  return wi - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Adam on FP32 master weights, step t >= 1.
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float mi = m[i], vi = v[i];
  const float wi = adam_math(g[i], mi, vi, w[i], lr, b1, b2, eps, c1, c2);
  m[i] = mi;
  v[i] = vi;
  w[i] = wi;
}

// adam_math on parameter i: moments stored, the new weight returned (and
// not yet stored).
__device__ __forceinline__ float adam_one(const float* __restrict__ w,
                                          const float* __restrict__ g, float* __restrict__ m,
                                          float* __restrict__ v, int64_t i, float lr, float b1,
                                          float b2, float eps, float c1, float c2) {
  float mi = m[i], vi = v[i];
  const float wi = adam_math(g[i], mi, vi, w[i], lr, b1, b2, eps, c1, c2);
  m[i] = mi;
  v[i] = vi;
  return wi;
}

// Adam as adam_kernel, the updated weight also written to a context's
// master copy and, where inv gives byte offsets (-1: none), to its packed and
// permuted copies in the form's precision (BF16 rounded to nearest even, as
// map_gather_multi writes them): the update and the re-layout in one pass.
// Thread t takes parameter t, or t + skip_n from skip_lo on (a range that
// adam_hidden_tiles updates).
__global__ void adam_relayout_kernel(float* __restrict__ w, const float* __restrict__ g,
                                     float* __restrict__ m, float* __restrict__ v, int64_t n,
                                     float lr, float b1, float b2, float eps, float c1, float c2,
                                     float* __restrict__ master, const int2* __restrict__ inv,
                                     char* __restrict__ packed, char* __restrict__ perm,
                                     int32_t bf16, int64_t skip_lo, int64_t skip_n) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= skip_lo) i += skip_n;
  if (i >= n) return;
  const float wi = adam_one(w, g, m, v, i, lr, b1, b2, eps, c1, c2);
  w[i] = wi;
  master[i] = wi;
  const int2 d = inv[i];
  if (bf16) {
    const uint16_t h = to_bf16(wi);
    if (d.x >= 0) *reinterpret_cast<uint16_t*>(packed + d.x) = h;
    if (d.y >= 0) *reinterpret_cast<uint16_t*>(perm + d.y) = h;
  } else {
    if (d.x >= 0) *reinterpret_cast<float*>(packed + d.x) = wi;
    if (d.y >= 0) *reinterpret_cast<float*>(perm + d.y) = wi;
  }
}

// The hidden layer's weights (HO outputs x HC channels x HP positions,
// parameter o*HC*HP + c*HP + p) in tiles of HTO outputs x HTC channels: Adam
// on the tile's rows (contiguous runs of HTC*HP parameters, four requested
// per thread before any is used), the new weights to the master copy and to
// LDS, then from LDS to the permuted copy ([p*HC + c][o]: runs of HTO
// outputs) and the packed copy (per position p the K = HC x N = HO fragment
// order of the forward kernels: k-groups of KG channels, 16-output tiles,
// lane (k % KG) / E * 16 + o % 16, element k % E, E = KG / 4: whole 64 x E
// blocks), in the form's precision.
constexpr int HO = 512, HC = 256, HP = 13, HTO = 16, HTC = 32, HROW = HTC * HP + 1;
__global__ void __launch_bounds__(256)
    adam_hidden_tiles(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                      float* __restrict__ v, float lr, float b1, float b2, float eps, float c1,
                      float c2, float* __restrict__ master, char* __restrict__ packed,
                      char* __restrict__ perm, int32_t bf16, int32_t KG) {
  __shared__ float T[HTO * HROW];  // [o - o0][(c - c0) * HP + p], rows padded by one
  constexpr int NT = HTO * HTC * HP, U = 4;
  const int o0 = blockIdx.x * HTO, c0 = blockIdx.y * HTC;
  for (int base = threadIdx.x; base < NT; base += 256 * U) {
    int64_t ii[U];
    float gv[U], mv[U], vv[U], wv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * 256;
      const int r = idx / (HTC * HP), col = idx - r * (HTC * HP);
      ii[u] = (int64_t)(o0 + r) * (HC * HP) + c0 * HP + col;
      if (idx < NT) {
        gv[u] = g[ii[u]];
        mv[u] = m[ii[u]];
        vv[u] = v[ii[u]];
        wv[u] = w[ii[u]];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * 256;
      if (idx >= NT) continue;
      float mi = mv[u], vi = vv[u];
      const float wi = adam_math(gv[u], mi, vi, wv[u], lr, b1, b2, eps, c1, c2);
      m[ii[u]] = mi;
      v[ii[u]] = vi;
      w[ii[u]] = wi;
      master[ii[u]] = wi;
      const int r = idx / (HTC * HP), col = idx - r * (HTC * HP);
      T[r * HROW + col] = wi;
    }
  }
  __syncthreads();
  // permuted copy: element (p, c, o) at (p*HC + c)*HO + o
  for (int idx = threadIdx.x; idx < NT; idx += 256) {
    const int ol = idx % HTO, rest = idx / HTO, cl = rest % HTC, p = rest / HTC;
    const float x = T[ol * HROW + cl * HP + p];
    const int64_t q = ((int64_t)p * HC + c0 + cl) * HO + o0 + ol;
    if (bf16)
      reinterpret_cast<uint16_t*>(perm)[q] = to_bf16(x);
    else
      reinterpret_cast<float*>(perm)[q] = x;
  }
  // packed copy: per position p, blocks (kg, nt) of 64 lanes x E elements
  const int E = KG / 4, BLK = 64 * E, NKG = HTC / KG, NNT = HTO / 16;
  for (int idx = threadIdx.x; idx < NT; idx += 256) {
    const int blk = idx / BLK, wi = idx - blk * BLK, lane = wi / E, e = wi - lane * E;
    const int ntl = blk % NNT, rest = blk / NNT, kgl = rest % NKG, p = rest / NKG;
    const int kg = c0 / KG + kgl, nt = o0 / 16 + ntl;
    const int c = kg * KG + (lane / 16) * E + e, o = nt * 16 + (lane & 15);
    const float x = T[(o - o0) * HROW + (c - c0) * HP + p];
    const int64_t q = (int64_t)p * (HC * HO) + ((int64_t)(kg * (HO / 16) + nt) * 64 + lane) * E + e;
    if (bf16)
      reinterpret_cast<uint16_t*>(packed)[q] = to_bf16(x);
    else
      reinterpret_cast<float*>(packed)[q] = x;
  }
}

hipError_t launch_adam_relayout(float* w, const float* g, float* m, float* v, int64_t n, float lr,
                                float b1, float b2, float eps, int32_t t, float* master,
                                const int2* inv, void* packed, void* perm, int32_t bf16,
                                int64_t hid_off, void* hid_packed, void* hid_perm,
                                hipStream_t stream) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  const int64_t hn = hid_packed ? (int64_t)HO * HC * HP : 0;
  if (hid_packed && (hid_off < 0 || hid_off + hn > n)) return hipErrorInvalidValue;
  const int64_t rest = n - hn;
  if (rest > 0)
    hipLaunchKernelGGL(adam_relayout_kernel, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0,
                       stream, w, g, m, v, n, lr, b1, b2, eps, c1, c2, master, inv,
                       static_cast<char*>(packed), static_cast<char*>(perm), bf16,
                       hid_packed ? hid_off : n, hn);
  if (hid_packed)
    hipLaunchKernelGGL(adam_hidden_tiles, dim3(HO / HTO, HC / HTC), dim3(256), 0, stream,
                       w + hid_off, g + hid_off, m + hid_off, v + hid_off, lr, b1, b2, eps, c1,
                       c2, master + hid_off, static_cast<char*>(hid_packed),
                       static_cast<char*>(hid_perm), bf16, bf16 ? 32 : 16);
  return hipGetLastError();
}

hipError_t launch_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, int32_t t, hipStream_t stream) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, w, g, m,
                     v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace simnet
