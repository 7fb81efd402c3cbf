// Small kernels of the path: the seeded Gaussian test matrix (Sec. 1,
// Alg. 7), operand copies, the U = L2^T gather (Alg. 5 step 8), and the
// float64 error indicator with the Alg. 8 / Alg. 11 stopping rule (Thm 4.3).
#include "plu_internal.h"

namespace plu {

namespace {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// two-multiplier S-box with a Weyl key schedule.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

__device__ __forceinline__ float unit_open0(uint32_t x) {
  // (0, 1]: ((x >> 8) + 1) * 2^-24, exact in float32
  return (float)((x >> 8) + 1u) * 5.9604644775390625e-8f;
}

__global__ __launch_bounds__(256) void k_gaussian(float* out, int64_t ldo, int64_t rows,
                                                 int64_t cols, uint64_t seed) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = rows * cols;
  const int64_t e0 = g * 4;
  if (e0 >= total) return;
  uint32_t c[4] = {(uint32_t)g, (uint32_t)((uint64_t)g >> 32), 0u, 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  float z[4];
  const float two_pi = 6.2831853071795864769f;
  {
    const float r = sqrtf(-2.0f * logf(unit_open0(c[0])));
    const float th = two_pi * unit_open0(c[1]);
    z[0] = r * cosf(th);
    z[1] = r * sinf(th);
  }
  {
    const float r = sqrtf(-2.0f * logf(unit_open0(c[2])));
    const float th = two_pi * unit_open0(c[3]);
    z[2] = r * cosf(th);
    z[3] = r * sinf(th);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t e = e0 + t;
    if (e < total) {
      const int64_t i = e / cols, j = e - i * cols;
      out[i * ldo + j] = z[t];
    }
  }
}

__global__ __launch_bounds__(256) void k_copy_pad(const float* src, int64_t lds, float* dst,
                                                 int64_t ldd, int64_t rows, int64_t cols,
                                                 int64_t cols_pad) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * cols_pad) return;
  const int64_t i = e / cols_pad, j = e - i * cols_pad;
  dst[i * ldd + j] = (j < cols) ? src[i * lds + j] : 0.f;
}

// U[t][r] = V[rowidx[r]][t] for t < k, r < nrows (32 x 32 LDS tiles).
__global__ __launch_bounds__(256) void k_transpose_gather(const float* V, int64_t ldv,
                                                         const int32_t* rowidx, int64_t nrows,
                                                         int k, float* U, int64_t ldu) {
  __shared__ float tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t r0 = (int64_t)blockIdx.x * 32;
  const int t0 = blockIdx.y * 32;
#pragma unroll
  for (int yy = 0; yy < 4; ++yy) {
    const int64_t r = r0 + ty + 8 * yy;
    const int t = t0 + tx;
    if (r < nrows && t < k) tile[ty + 8 * yy][tx] = V[(int64_t)rowidx[r] * ldv + t];
  }
  __syncthreads();
#pragma unroll
  for (int yy = 0; yy < 4; ++yy) {
    const int t = t0 + ty + 8 * yy;
    const int64_t r = r0 + tx;
    if (t < k && r < nrows) U[(int64_t)t * ldu + r] = tile[tx][ty + 8 * yy];
  }
}

// Column norms^2 of G from per-row-block partials, then the indicator
// E_j = ||A||^2 - sum_{i<=j} ||G(:,i)||^2 scanned in column order; k is the
// first column (col_mode) or block end with E <= eps^2 ||A||^2.
// With vsq_part set, each column's energy is divided by the float64 squared
// norm of the corresponding basis column (G(:,j) = A v_j): the indicator of
// Thm 4.3 for the column-normalized basis, which removes the first-order
// effect of storing an orthonormal V in float32.
__global__ __launch_bounds__(256) void k_rank_rule(const double* colsq_part, int nblk, int l,
                                                  const double* vsq_part, int nvblk,
                                                  const double* normA2p, double eps, int b,
                                                  int col_mode, int32_t* kout, double* Eout,
                                                  int32_t* tol, double* colnorm) {
  extern __shared__ double cn[];
  for (int j = threadIdx.x; j < l; j += 256) {
    double s = 0.0;
    for (int k = 0; k < nblk; ++k) s += colsq_part[(int64_t)k * l + j];
    if (vsq_part) {
      double v = 0.0;
      for (int k = 0; k < nvblk; ++k) v += vsq_part[(int64_t)k * l + j];
      if (v > 0.0) s /= v;
    }
    cn[j] = s;
    if (colnorm) colnorm[j] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double nA2 = *normA2p;
  int k = l, ok = 0;
  double E = nA2;
  if (nA2 == 0.0) {
    k = 0;
    ok = 1;
  } else {
    const double acc = eps * eps * nA2;
    for (int t1 = 0; t1 < l && !ok; t1 += b) {
      const int t2 = (t1 + b < l) ? t1 + b : l;
      if (col_mode) {
        for (int j = t1; j < t2; ++j) {
          E -= cn[j];
          if (E <= acc) {
            k = j + 1;
            ok = 1;
            break;
          }
        }
      } else {
        double s = 0.0;
        for (int j = t1; j < t2; ++j) s += cn[j];
        E -= s;
        if (E <= acc) {
          k = t2;
          ok = 1;
        }
      }
    }
  }
  *kout = k;
  *Eout = E;
  *tol = ok;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* p, size_t n, uint32_t v) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_iota(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

}  // namespace

hipError_t launch_gaussian(float* out, int64_t ldo, int64_t rows, int64_t cols, uint64_t seed,
                           hipStream_t s) {
  const int64_t nblk4 = (rows * cols + 3) / 4;
  hipLaunchKernelGGL(k_gaussian, dim3((unsigned)((nblk4 + 255) / 256)), dim3(256), 0, s, out, ldo,
                     rows, cols, seed);
  return hipGetLastError();
}

hipError_t launch_copy_pad(const float* src, int64_t lds, float* dst, int64_t ldd, int64_t rows,
                           int64_t cols, int64_t cols_pad, hipStream_t s) {
  const int64_t tot = rows * cols_pad;
  hipLaunchKernelGGL(k_copy_pad, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, src, lds,
                     dst, ldd, rows, cols, cols_pad);
  return hipGetLastError();
}

hipError_t launch_transpose_gather(const float* V, int64_t ldv, const int32_t* rowidx,
                                   int64_t nrows, int k, float* U, int64_t ldu, hipStream_t s) {
  dim3 grid((unsigned)((nrows + 31) / 32), (unsigned)((k + 31) / 32));
  hipLaunchKernelGGL(k_transpose_gather, grid, dim3(256), 0, s, V, ldv, rowidx, nrows, k, U, ldu);
  return hipGetLastError();
}

hipError_t launch_rank_rule(const double* colsq_part, int nblk, int l, const double* vsq_part,
                            int nvblk, const double* normA2, double eps, int b, int col_mode,
                            int32_t* kout, double* Eout, int32_t* tol, double* colnorm,
                            hipStream_t s) {
  if (l > 8192) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rank_rule, dim3(1), dim3(256), (size_t)l * sizeof(double), s, colsq_part,
                     nblk, l, vsq_part, nvblk, normA2, eps, b, col_mode, kout, Eout, tol, colnorm);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_iota(int32_t* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace plu
