// Training-form kernels of libsimnet.so (gfx950): the pieces of a predictor
// training step that are not the fused trunk forward.
//
//   gemm_kernel      C = op(A) x op(B) on FP32 MFMA, LDS-staged 64x64 tiles;
//                    operands in FP32 or BF16 with arbitrary strides; epilogue
//                    with bias, ReLU mask (a saved activation > 0) and
//                    accumulation.  Used for the head and for every
//                    input-gradient and weight-gradient product of the
//                    backward pass (a kernel-2 stride-2 convolution is a
//                    GEMM over position pairs).
//   loss_kernel      hybrid loss per window (400-bin cross-entropy + L1 on
//                    log1p(latency) per latency type) and its gradient
//                    w.r.t. the head outputs.
//   colsum kernels   bias gradients, summed in a fixed order.
//   map kernels      weight re-layouts and gradient scatters by index maps.
//   adam_kernel      Adam on FP32 master weights.
#include "simnet_internal.h"

namespace simnet {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float ld_elem(const void* p, int bf16, int64_t i) {
  if (bf16) return __uint_as_float((uint32_t)static_cast<const uint16_t*>(p)[i] << 16);
  return static_cast<const float*>(p)[i];
}

__device__ __forceinline__ int64_t op_index(const GemmOperand& o, int64_t r, int64_t c) {
  return (r / o.grp) * o.gs + (r % o.grp) * o.rs + c * o.cs;
}

constexpr int GB = 64, GK = 16, GPAD = 4;

// One thread's four elements of a tile (rows r0.. of R, cols c0.. of C),
// read along whichever dimension is contiguous in memory.
__device__ __forceinline__ void load_tile(const GemmOperand& o, int64_t R, int64_t Cn, int64_t r0,
                                          int64_t c0, bool rows_are_k, int tid, float (&v)[4],
                                          int (&rr)[4], int (&cc)[4]) {
  // tile is GB (non-k) x GK (k); "along" = the contiguous dimension
  const bool k_contig = rows_are_k ? (o.rs == 1 && o.grp > (int64_t)1 << 40) : (o.cs == 1);
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

__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
  __shared__ float As[GK][GB + GPAD];  // [k][m]
  __shared__ float Bs[GK][GB + GPAD];  // [k][n]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t m0 = (int64_t)blockIdx.y * GB, n0 = (int64_t)blockIdx.x * GB;
  const int wm = wave >> 1, wn = wave & 1;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  float va[4], vb[4];
  int ka[4], ma[4], kb[4], nb[4];
  load_tile(g.A, g.M, g.K, m0, 0, false, tid, va, ka, ma);
  load_tile(g.B, g.K, g.N, 0, n0, true, tid, vb, kb, nb);
  for (int64_t k0 = 0; k0 < g.K; k0 += GK) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      As[ka[e]][ma[e]] = va[e];
      Bs[kb[e]][nb[e]] = vb[e];
    }
    __syncthreads();
    if (k0 + GK < g.K) {  // next tile in flight while this one is multiplied
      load_tile(g.A, g.M, g.K, m0, k0 + GK, false, tid, va, ka, ma);
      load_tile(g.B, g.K, g.N, k0 + GK, n0, true, tid, vb, kb, nb);
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
        if (m < g.M && n < g.N) {
          float v = acc[i][j][r];
          if (g.bias) v += g.bias[n];
          if (g.mask.p && !(ld_elem(g.mask.p, g.mask.bf16, op_index(g.mask, m, n)) > 0.f)) v = 0.f;
          float* c = g.C + (m / g.cgrp) * g.cgs + (m % g.cgrp) * g.ldc + n;
          *c = g.beta ? *c + v : v;
        }
      }
}

hipError_t launch_gemm(const GemmArgs& g, hipStream_t stream) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const dim3 grid((unsigned)((g.N + GB - 1) / GB), (unsigned)((g.M + GB - 1) / GB));
  hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, stream, g);
  return hipGetLastError();
}

// One window per workgroup: per latency type t the head outputs are 400
// class logits and one regression output; loss = CE(class min(lat, 399)) +
// |reg - log1p(lat)|; dz = (softmax - onehot) / B, dreg = sign / B.
__global__ void __launch_bounds__(256)
    loss_kernel(const float* __restrict__ z, const int32_t* __restrict__ lat, int64_t B,
                int32_t n_bins, float* __restrict__ loss_b, float* __restrict__ dz) {
  __shared__ float red[4];
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x;
  const int per = n_bins + 1;
  float total = 0.f;
  for (int t = 0; t < 2; ++t) {
    const float* zt = z + (b * 2 + t) * per;
    const int l = lat[b * 2 + t];
    const int bin = l < n_bins - 1 ? l : n_bins - 1;
    float m = -INFINITY;
    for (int i = tid; i < n_bins; i += 256) m = fmaxf(m, zt[i]);
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((tid & 63) == 0) red[tid >> 6] = m;
    __syncthreads();
    m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    __syncthreads();
    float se = 0.f;
    for (int i = tid; i < n_bins; i += 256) se += expf(zt[i] - m);
    for (int o = 32; o >= 1; o >>= 1) se += __shfl_xor(se, o);
    if ((tid & 63) == 0) red[tid >> 6] = se;
    __syncthreads();
    se = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    const float lse = m + logf(se);
    const float r = zt[n_bins] - log1pf((float)l);
    const float inv = 1.f / (float)B;
    float* dzt = dz + (b * 2 + t) * per;
    for (int i = tid; i < n_bins; i += 256)
      dzt[i] = inv * (expf(zt[i] - lse) - (i == bin ? 1.f : 0.f));
    if (tid == 0) dzt[n_bins] = inv * (r > 0.f ? 1.f : (r < 0.f ? -1.f : 0.f));
    total += lse - zt[bin] + fabsf(r);
  }
  if (tid == 0) loss_b[b] = total;
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
  hipLaunchKernelGGL(loss_kernel, dim3((unsigned)B), dim3(256), 0, stream, z, lat, B, n_bins,
                     loss_b, dz);
  hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(256), 0, stream, loss_b, B, loss);
  return hipGetLastError();
}

// Column sums of Y [M][ld] over rows, in two fixed-order passes.
constexpr int CS_CHUNKS = 128;
__global__ void colsum_partial(const float* __restrict__ y, int64_t M, int64_t N, int64_t ld,
                               float* __restrict__ part) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t c = blockIdx.y;
  const int64_t per = (M + CS_CHUNKS - 1) / CS_CHUNKS;
  if (n >= N) return;
  float s = 0.f;
  for (int64_t m = c * per; m < M && m < (c + 1) * per; ++m) s += y[m * ld + n];
  part[c * N + n] = s;
}

__global__ void colsum_final(const float* __restrict__ part, int64_t N, float* __restrict__ out,
                             int beta) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int c = 0; c < CS_CHUNKS; ++c) s += part[c * N + n];
  out[n] = beta ? out[n] + s : s;
}

size_t colsum_workspace(int64_t N) { return sizeof(float) * CS_CHUNKS * (size_t)N; }

hipError_t launch_colsum(const float* y, int64_t M, int64_t N, int64_t ld, float* out, int beta,
                         float* work, hipStream_t stream) {
  const unsigned nb = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL(colsum_partial, dim3(nb, CS_CHUNKS), dim3(256), 0, stream, y, M, N, ld, work);
  hipLaunchKernelGGL(colsum_final, dim3(nb), dim3(256), 0, stream, work, N, out, beta);
  return hipGetLastError();
}

// dst[i] = src[map[i]] (0 where map < 0), stored as FP32 or BF16 (nearest even).
__global__ void map_gather(const float* __restrict__ src, const int32_t* __restrict__ map,
                           int64_t n, void* __restrict__ dst, int bf16) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int32_t k = map[i];
  const float v = k < 0 ? 0.f : src[k];
  if (bf16) {
    const uint32_t u = __float_as_uint(v);
    static_cast<uint16_t*>(dst)[i] = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
  } else {
    static_cast<float*>(dst)[i] = v;
  }
}

// dst[map[i]] (=|+=) src[i] for map[i] >= 0 (the map is one-to-one).
__global__ void map_scatter(const float* __restrict__ src, const int32_t* __restrict__ map,
                            int64_t n, float* __restrict__ dst, int beta) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int32_t k = map[i];
  if (k >= 0) dst[k] = beta ? dst[k] + src[i] : src[i];
}

hipError_t launch_map_gather(const float* src, const int32_t* map, int64_t n, void* dst, int bf16,
                             hipStream_t stream) {
  hipLaunchKernelGGL(map_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, src,
                     map, n, dst, bf16);
  return hipGetLastError();
}

hipError_t launch_map_scatter(const float* src, const int32_t* map, int64_t n, float* dst,
                              int beta, hipStream_t stream) {
  hipLaunchKernelGGL(map_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, src,
                     map, n, dst, beta);
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

// Adam (Kingma & Ba) on FP32 master weights, step t >= 1, no weight decay.
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, int32_t t, hipStream_t stream) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, w, g, m,
                     v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace simnet
