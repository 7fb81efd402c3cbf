// Measured ceilings of this GPU for the rooflines the passes are priced
// against: the matrix-core rate of each instruction the pass kernels issue
// (v_mfma_f32_16x16x4f32, v_mfma_f32_16x16x32_bf16, the scaled
// v_mfma_scale_f32_16x16x128_f8f6f4), and the rate of a plain streaming read
// from HBM.  Operands are hashed from the thread index, so the matrix cores
// see varied bits (their clock depends on the data); results are stored
// only when `write` is set, which callers leave off.
#include "plu_internal.h"

namespace plu {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x;
}

constexpr int kChains = 8;   // independent accumulators per wave

template <int KIND>
__global__ __launch_bounds__(256) void k_peak_mfma(int iters, int write, float* sink) {
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  f32x4 acc[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  if (KIND == 0) {
    // values in [1, 2) with hashed mantissas, scaled so sums stay finite
    const float a = __uint_as_float(0x3F800000u | (mix32(t) >> 9)) * 1e-3f;
    const float b = __uint_as_float(0x3F800000u | (mix32(t + 0x9E3779B9u) >> 9)) * 1e-3f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int j = 0; j < kChains; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[j], 0, 0, 0);
    }
  } else if (KIND == 1) {
    uint32_t w[4], v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      // two bfloat16 in [2^-10, 2^-8) with hashed mantissas
      w[e] = (mix32(t * 8 + e) & 0x007F007Fu) | 0x3A803A80u;
      v[e] = (mix32(t * 8 + 4 + e) & 0x007F007Fu) | 0x3A803A80u;
    }
    const bf16x8 a = __builtin_bit_cast(bf16x8, w);
    const bf16x8 b = __builtin_bit_cast(bf16x8, v);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int j = 0; j < kChains; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
    }
  } else {
    i32x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      // E4M3 codes with exponent field 1..7 (no NaN codes), hashed mantissa
      a[e] = (int)((mix32(t * 16 + e) & 0x07070707u) | 0x08080808u);
      b[e] = (int)((mix32(t * 16 + 8 + e) & 0x07070707u) | 0x18181818u);
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int j = 0; j < kChains; ++j)
        acc[j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc[j], 0, 0, 0, 100, 0, 100);
    }
  }
  if (write) {
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    sink[t] = s;
  }
}

// Every lane reads 4 of the buffer's 16-byte words per iteration, the grid
// striding over the buffer; the words are folded into one value so the
// loads stay live.
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_peak_read(const u32x4v* __restrict__ p, int64_t n,
                                                   int write, uint32_t* sink) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  uint32_t x = 0;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const u32x4v v0 = __builtin_nontemporal_load(p + i);
    const u32x4v v1 = __builtin_nontemporal_load(p + i + stride);
    const u32x4v v2 = __builtin_nontemporal_load(p + i + 2 * stride);
    const u32x4v v3 = __builtin_nontemporal_load(p + i + 3 * stride);
    x ^= (v0.x ^ v1.y) ^ (v2.z ^ v3.w) ^ (v0.w ^ v1.x) ^ (v2.y ^ v3.z);
  }
  for (; i < n; i += stride) {
    const u32x4v v = p[i];
    x ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (write) sink[(int64_t)blockIdx.x * 256 + threadIdx.x] = x;
}

}  // namespace

// Flop of one instruction of each kind (2 m n k).
double peak_flop_per_mfma(int kind) {
  return kind == 0 ? 2.0 * 16 * 16 * 4 : kind == 1 ? 2.0 * 16 * 16 * 32 : 2.0 * 16 * 16 * 128;
}

int peak_chains() { return kChains; }

hipError_t launch_peak_mfma(int kind, int blocks, int iters, hipStream_t s) {
  if (kind == 0)
    hipLaunchKernelGGL(k_peak_mfma<0>, dim3(blocks), dim3(256), 0, s, iters, 0, nullptr);
  else if (kind == 1)
    hipLaunchKernelGGL(k_peak_mfma<1>, dim3(blocks), dim3(256), 0, s, iters, 0, nullptr);
  else if (kind == 2)
    hipLaunchKernelGGL(k_peak_mfma<2>, dim3(blocks), dim3(256), 0, s, iters, 0, nullptr);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_peak_read(const void* buf, int64_t bytes, int blocks, hipStream_t s) {
  if (!buf || bytes < 16 || (reinterpret_cast<uintptr_t>(buf) & 15u)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_peak_read, dim3(blocks), dim3(256), 0, s,
                     reinterpret_cast<const u32x4v*>(buf), bytes / 16, 0, nullptr);
  return hipGetLastError();
}

}  // namespace plu
