// Peak probes for gfx950, built as libsimnet_peaks.so (measurement only;
// nothing in the simulation path uses them): the matrix-core rate of the
// MFMA instructions the kernels issue, and HBM read and copy bandwidth.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int CHAINS = 8;  // independent accumulators per wave

// prec 0: 16x16x4 FP32 (2,048 FLOP), 1: 16x16x32 BF16 (16,384), 2: 16x16x32
// FP8 e4m3 (16,384), 3: 32x32x16 BF16 (32,768; 4 chains of 16 registers).
// Operands come from the input so nothing folds.
template <int PREC>
__global__ void __launch_bounds__(256) mfma_probe(const uint32_t* __restrict__ seed, int n_iter,
                                                  float* __restrict__ out) {
  const uint32_t s = seed[threadIdx.x & 63];
  v4f acc[CHAINS];
#pragma unroll
  for (int j = 0; j < CHAINS; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
  if constexpr (PREC == 0) {
    const float a = __uint_as_float((s & 0x007fffffu) | 0x3f000000u);
    for (int it = 0; it < n_iter; ++it)
#pragma unroll
      for (int j = 0; j < CHAINS; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, a, acc[j], 0, 0, 0);
  } else if constexpr (PREC == 1) {
    const uint4 u = make_uint4(s, s ^ 0x1234u, s + 7u, s * 3u);
    const v8bf a = __builtin_bit_cast(v8bf, u);
    for (int it = 0; it < n_iter; ++it)
#pragma unroll
      for (int j = 0; j < CHAINS; ++j)
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, a, acc[j], 0, 0, 0);
  } else if constexpr (PREC == 3) {
    const uint4 u = make_uint4(s, s ^ 0x1234u, s + 7u, s * 3u);
    const v8bf a = __builtin_bit_cast(v8bf, u);
    v16f big[CHAINS / 2];
#pragma unroll
    for (int j = 0; j < CHAINS / 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) big[j][e] = 0.f;
    for (int it = 0; it < n_iter; ++it)
#pragma unroll
      for (int j = 0; j < CHAINS / 2; ++j)
        big[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, a, big[j], 0, 0, 0);
#pragma unroll
    for (int j = 0; j < CHAINS / 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[j][e] = big[j][e] + big[j][e + 4] + big[j][e + 8] + big[j][e + 12];
  } else {
    const long a = (long)(((uint64_t)s << 32) | (s ^ 0x5555u));
    for (int it = 0; it < n_iter; ++it)
#pragma unroll
      for (int j = 0; j < CHAINS; ++j)
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, a, acc[j], 0, 0, 0);
  }
  float t = 0.f;
#pragma unroll
  for (int j = 0; j < CHAINS; ++j) t += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = t;
}

// mode 0: read n16 16-byte words and fold them into one word per thread;
// mode 1: copy them to dst; mode 2: every workgroup reads the same first
// n16 words (L2-resident when small) `reps` times (the per-CU read rate
// from L2).
__global__ void __launch_bounds__(256) hbm_probe(const uint4* __restrict__ src,
                                                 uint4* __restrict__ dst, int64_t n16, int mode,
                                                 int reps) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (mode == 2) {
    uint4 f = make_uint4(0u, 0u, 0u, 0u);
    for (int r = 0; r < reps; ++r)
      for (int64_t i = threadIdx.x; i < n16; i += blockDim.x) {
        const uint4 v = src[i];
        f.x ^= v.x + (uint32_t)r;
        f.y ^= v.y;
        f.z ^= v.z;
        f.w ^= v.w;
      }
    dst[i0] = f;
    return;
  }
  if (mode == 1) {
    for (int64_t i = i0; i < n16; i += stride) dst[i] = src[i];
    return;
  }
  uint4 f = make_uint4(0u, 0u, 0u, 0u);
  for (int64_t i = i0; i < n16; i += stride) {
    const uint4 v = src[i];
    f.x ^= v.x;
    f.y ^= v.y;
    f.z ^= v.z;
    f.w ^= v.w;
  }
  dst[i0] = f;
}

int timed(hipStream_t st, float* ms, void (*launch)(hipStream_t, void*), void* arg) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -3;
  hipError_t e = hipEventRecord(e0, st);
  if (e == hipSuccess) {
    launch(st, arg);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e == hipSuccess ? 0 : -3;
}

struct MfmaArg {
  int prec, blocks, n_iter;
  const uint32_t* seed;
  float* out;
};
struct HbmArg {
  const uint4* src;
  uint4* dst;
  int64_t n16;
  int mode, blocks, reps;
};

}  // namespace

extern "C" {

// Matrix-core probe: blocks x 256 threads, each wave n_iter x 8 independent
// MFMAs of the form prec (0 FP32, 1 BF16, 2 FP8; 3: n_iter x 4 of the
// 32x32x16 BF16 one).  seed: DEVICE >= 64 uint32; out: DEVICE >= blocks *
// 256 floats.  *ms = kernel time; FLOP = blocks * 4 * n_iter * 8 * (2,048
// for FP32, else 16,384).  0 or -1 (bad arguments) / -3 (device error).
__attribute__((visibility("default"))) int peaks_mfma(int prec, int blocks, int n_iter,
                                                      const uint32_t* seed, float* out,
                                                      void* stream, float* ms) {
  if (prec < 0 || prec > 3 || blocks < 1 || n_iter < 1 || !seed || !out || !ms) return -1;
  MfmaArg a{prec, blocks, n_iter, seed, out};
  return timed(static_cast<hipStream_t>(stream), ms,
               [](hipStream_t st, void* p) {
                 const MfmaArg& m = *static_cast<MfmaArg*>(p);
                 if (m.prec == 0)
                   hipLaunchKernelGGL(mfma_probe<0>, dim3(m.blocks), dim3(256), 0, st, m.seed,
                                      m.n_iter, m.out);
                 else if (m.prec == 1)
                   hipLaunchKernelGGL(mfma_probe<1>, dim3(m.blocks), dim3(256), 0, st, m.seed,
                                      m.n_iter, m.out);
                 else if (m.prec == 3)
                   hipLaunchKernelGGL(mfma_probe<3>, dim3(m.blocks), dim3(256), 0, st, m.seed,
                                      m.n_iter, m.out);
                 else
                   hipLaunchKernelGGL(mfma_probe<2>, dim3(m.blocks), dim3(256), 0, st, m.seed,
                                      m.n_iter, m.out);
               },
               &a);
}

// HBM probe: mode 0 reads bytes from src (dst: DEVICE >= blocks * 256 * 16
// bytes receives one folded word per thread), mode 1 copies bytes from src
// to dst, mode 2 has every workgroup read the first bytes of src reps times
// (bytes read = blocks * reps * bytes).  bytes a multiple of 16.  *ms =
// kernel time.
__attribute__((visibility("default"))) int peaks_hbm(const void* src, void* dst, int64_t bytes,
                                                     int mode, int blocks, int reps, void* stream,
                                                     float* ms) {
  if (!src || !dst || bytes <= 0 || bytes % 16 || mode < 0 || mode > 2 || blocks < 1 ||
      reps < 1 || !ms)
    return -1;
  HbmArg a{static_cast<const uint4*>(src), static_cast<uint4*>(dst), bytes / 16, mode, blocks,
           reps};
  return timed(static_cast<hipStream_t>(stream), ms,
               [](hipStream_t st, void* p) {
                 const HbmArg& h = *static_cast<HbmArg*>(p);
                 hipLaunchKernelGGL(hbm_probe, dim3(h.blocks), dim3(256), 0, st, h.src, h.dst,
                                    h.n16, h.mode, h.reps);
               },
               &a);
}

}  // extern "C"
