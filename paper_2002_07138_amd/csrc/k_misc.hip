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

struct GaussArgs {
  float* out; int64_t ldo, rows, cols; uint64_t seed;
};

__device__ void b_gaussian(const GaussArgs& a, const Grid& gr) {
  const int64_t g = (int64_t)gr.bx * 256 + threadIdx.x;
  const int64_t total = a.rows * a.cols;
  const int64_t e0 = g * 4;
  if (e0 >= total) return;
  uint32_t c[4] = {(uint32_t)g, (uint32_t)((uint64_t)g >> 32), 0u, 0u};
  philox4x32_10(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
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
      const int64_t i = e / a.cols, j = e - i * a.cols;
      a.out[i * a.ldo + j] = z[t];
    }
  }
}

struct CopyPadArgs {
  const float* src; int64_t lds; float* dst; int64_t ldd, rows, cols, cols_pad;
};

__device__ void b_copy_pad(const CopyPadArgs& a, const Grid& gr) {
  const int64_t e = (int64_t)gr.bx * 256 + threadIdx.x;
  if (e >= a.rows * a.cols_pad) return;
  const int64_t i = e / a.cols_pad, j = e - i * a.cols_pad;
  a.dst[i * a.ldd + j] = (j < a.cols) ? a.src[i * a.lds + j] : 0.f;
}

// dst[rperm[i]][cperm[j]] = src[i][j] for i < rows, j < cols; a null
// permutation is the identity.  Indices outside [0, rows) or [0, cols) are
// skipped, so a malformed permutation leaves entries unwritten but never
// writes outside dst.
struct ScatterArgs {
  const float* src; int64_t lds; float* dst; int64_t ldd, rows, cols;
  const int32_t* rperm; const int32_t* cperm;
};

__device__ void b_scatter_perm(const ScatterArgs& a, const Grid& gr) {
  const int64_t e = (int64_t)gr.bx * 256 + threadIdx.x;
  if (e >= a.rows * a.cols) return;
  const int64_t i = e / a.cols, j = e - i * a.cols;
  const int64_t di = a.rperm ? (int64_t)a.rperm[i] : i;
  const int64_t dj = a.cperm ? (int64_t)a.cperm[j] : j;
  if (di < 0 || di >= a.rows || dj < 0 || dj >= a.cols) return;
  a.dst[di * a.ldd + dj] = a.src[i * a.lds + j];
}

// U[t][r] = V[rowidx[r]][t] for t < k, r < nrows (32 x 32 LDS tiles).
struct TGatherArgs {
  const float* V; int64_t ldv; const int32_t* rowidx; int64_t nrows; int k; float* U;
  int64_t ldu; const int32_t* kcap;
};

__device__ void b_transpose_gather(const TGatherArgs& a, const Grid& gr) {
  __shared__ float tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t r0 = (int64_t)gr.bx * 32;
  const int t0 = gr.by * 32;
  const int kk = a.kcap ? min(a.k, *a.kcap) : a.k;
  if (t0 >= kk) return;
#pragma unroll
  for (int yy = 0; yy < 4; ++yy) {
    const int64_t r = r0 + ty + 8 * yy;
    const int t = t0 + tx;
    if (r < a.nrows && t < kk) tile[ty + 8 * yy][tx] = a.V[(int64_t)a.rowidx[r] * a.ldv + t];
  }
  __syncthreads();
#pragma unroll
  for (int yy = 0; yy < 4; ++yy) {
    const int t = t0 + ty + 8 * yy;
    const int64_t r = r0 + tx;
    if (t < kk && r < a.nrows) a.U[(int64_t)t * a.ldu + r] = tile[tx][ty + 8 * yy];
  }
}

// Column norms^2 of G from per-row-block partials, then the indicator
// E_j = ||A||^2 - sum_{i<=j} ||G(:,i)||^2 scanned in column order; k is the
// first column (col_mode) or block end with E <= eps^2 ||A||^2.
// With vsq_part set, each column's energy is divided by the float64 squared
// norm of the corresponding basis column (G(:,j) = A v_j): the indicator of
// Thm 4.3 for the column-normalized basis, which removes the first-order
// effect of storing an orthonormal V in float32.
struct RankArgs {
  const double* colsq_part; int nblk, l; const double* vsq_part; int nvblk;
  const double* normA2p; double eps; int b, col_mode; int32_t* kout; double* Eout;
  int32_t* tol; double* colnorm;
  const double* E0p;   // nullable: indicator before these columns (default ||A||^2)
};

__device__ void b_rank_rule(const RankArgs& a, const Grid& gr) {
  (void)gr;
  extern __shared__ double cn[];
  const int l = a.l;
  for (int j = threadIdx.x; j < l; j += 256) {
    double s = 0.0;
    for (int k = 0; k < a.nblk; ++k) s += a.colsq_part[(int64_t)k * l + j];
    if (a.vsq_part) {
      double v = 0.0;
      for (int k = 0; k < a.nvblk; ++k) v += a.vsq_part[(int64_t)k * l + j];
      if (v > 0.0) s /= v;
    }
    cn[j] = s;
    if (a.colnorm) a.colnorm[j] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double nA2 = *a.normA2p;
  int k = l, ok = 0;
  double E = a.E0p ? *a.E0p : nA2;
  if (nA2 == 0.0) {
    k = 0;
    ok = 1;
  } else if (!isfinite(nA2)) {
    k = 0;   // non-finite A: nothing is assembled; the caller reports it
  } else {
    const double acc = a.eps * a.eps * nA2;
    for (int t1 = 0; t1 < l && !ok; t1 += a.b) {
      const int t2 = (t1 + a.b < l) ? t1 + a.b : l;
      if (a.col_mode) {
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
  *a.kout = k;
  *a.Eout = E;
  *a.tol = ok;
}

struct FillArgs {
  uint32_t* p; size_t n; uint32_t v;
};

__device__ void b_fill_u32(const FillArgs& a, const Grid& gr) {
  const size_t i = (size_t)gr.bx * 256 + threadIdx.x;
  if (i < a.n) a.p[i] = a.v;
}

struct IotaArgs {
  int32_t* p; int64_t n;
};

__device__ void b_iota(const IotaArgs& a, const Grid& gr) {
  const int64_t i = (int64_t)gr.bx * 256 + threadIdx.x;
  if (i < a.n) a.p[i] = (int32_t)i;
}

struct NegateArgs {
  float* p; int64_t ld, rows, cols;
};

__device__ void b_negate(const NegateArgs& a, const Grid& gr) {
  const int64_t e = (int64_t)gr.bx * 256 + threadIdx.x;
  if (e >= a.rows * a.cols) return;
  const int64_t r = e / a.cols, c = e % a.cols;
  a.p[r * a.ld + c] = -a.p[r * a.ld + c];
}

// X = (R^{-1})^T for the upper triangular k x k factor R (k <= 128), by
// back substitution, one column of R^{-1} per thread, float64 sums; X is
// lower triangular.  One workgroup.
struct TriInvArgs {
  const float* R; int64_t ldr; float* X; int64_t ldx; int k;
};

__device__ void b_tri_inv_t(const TriInvArgs& a, const Grid& gr) {
  (void)gr;
  __shared__ float Rs[128][129];
  __shared__ float Ys[128][129];   // Ys[i][c] = (R^{-1})[i][c]
  const int k = a.k;
  for (int e = threadIdx.x; e < k * k; e += 128) {
    const int i = e / k, j = e % k;
    Rs[i][j] = a.R[(int64_t)i * a.ldr + j];
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < k) {
    for (int i = k - 1; i >= 0; --i) {
      if (i > c) {
        Ys[i][c] = 0.f;
        continue;
      }
      double s = (i == c) ? 1.0 : 0.0;
      for (int j = i + 1; j <= c; ++j) s -= (double)Rs[i][j] * (double)Ys[j][c];
      Ys[i][c] = (float)(s / (double)Rs[i][i]);
    }
    for (int i = 0; i < k; ++i) a.X[(int64_t)c * a.ldx + i] = Ys[i][c];
  }
}

}  // namespace

hipError_t launch_gaussian(float* out, int64_t ldo, int64_t rows, int64_t cols, uint64_t seed,
                           hipStream_t s) {
  const int64_t nblk4 = (rows * cols + 3) / 4;
  return dispatch<GaussArgs, b_gaussian, 256>(GaussArgs{out, ldo, rows, cols, seed},
                                             dim3((unsigned)((nblk4 + 255) / 256)), 0, s);
}

hipError_t launch_copy_pad(const float* src, int64_t lds, float* dst, int64_t ldd, int64_t rows,
                           int64_t cols, int64_t cols_pad, hipStream_t s) {
  const int64_t tot = rows * cols_pad;
  return dispatch<CopyPadArgs, b_copy_pad, 256>(
      CopyPadArgs{src, lds, dst, ldd, rows, cols, cols_pad}, dim3((unsigned)((tot + 255) / 256)),
      0, s);
}

hipError_t launch_scatter_perm(const float* src, int64_t lds, float* dst, int64_t ldd,
                               int64_t rows, int64_t cols, const int32_t* rperm,
                               const int32_t* cperm, hipStream_t s) {
  const int64_t tot = rows * cols;
  if (tot <= 0) return hipSuccess;
  return dispatch<ScatterArgs, b_scatter_perm, 256>(
      ScatterArgs{src, lds, dst, ldd, rows, cols, rperm, cperm},
      dim3((unsigned)((tot + 255) / 256)), 0, s);
}

hipError_t launch_transpose_gather(const float* V, int64_t ldv, const int32_t* rowidx,
                                   int64_t nrows, int k, float* U, int64_t ldu, hipStream_t s,
                                   const int32_t* kcap) {
  dim3 grid((unsigned)((nrows + 31) / 32), (unsigned)((k + 31) / 32));
  return dispatch<TGatherArgs, b_transpose_gather, 256>(
      TGatherArgs{V, ldv, rowidx, nrows, k, U, ldu, kcap}, grid, 0, s);
}

hipError_t launch_rank_rule(const double* colsq_part, int nblk, int l, const double* vsq_part,
                            int nvblk, const double* normA2, double eps, int b, int col_mode,
                            int32_t* kout, double* Eout, int32_t* tol, double* colnorm,
                            hipStream_t s, const double* E0) {
  if (l > 8192) return hipErrorInvalidValue;
  return dispatch<RankArgs, b_rank_rule, 256>(
      RankArgs{colsq_part, nblk, l, vsq_part, nvblk, normA2, eps, b, col_mode, kout, Eout, tol,
               colnorm, E0},
      dim3(1), (size_t)l * sizeof(double), s);
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
  return dispatch<FillArgs, b_fill_u32, 256>(FillArgs{p, n, v},
                                            dim3((unsigned)((n + 255) / 256)), 0, s);
}

hipError_t launch_iota(int32_t* p, int64_t n, hipStream_t s) {
  return dispatch<IotaArgs, b_iota, 256>(IotaArgs{p, n}, dim3((unsigned)((n + 255) / 256)), 0,
                                         s);
}

hipError_t launch_negate(float* p, int64_t ld, int64_t rows, int64_t cols, hipStream_t s) {
  const int64_t tot = rows * cols;
  if (tot == 0) return hipSuccess;
  return dispatch<NegateArgs, b_negate, 256>(NegateArgs{p, ld, rows, cols},
                                            dim3((unsigned)((tot + 255) / 256)), 0, s);
}

hipError_t launch_tri_inv_t(const float* R, int64_t ldr, float* X, int64_t ldx, int k,
                            hipStream_t s) {
  if (k < 1 || k > 128) return hipErrorInvalidValue;
  return dispatch<TriInvArgs, b_tri_inv_t, 128>(TriInvArgs{R, ldr, X, ldx, k}, dim3(1), 0, s);
}


}  // namespace plu
