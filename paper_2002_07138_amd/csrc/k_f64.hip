// Float64 products for the stopping indicator of PowerLU_FP (Thm 4.3 with
// the rule of Alg. 8 / Alg. 11), the PLU_PREC_FP64_INDICATOR form.
//
// The indicator E_j = ||A||_F^2 - sum_{i<=j} ||A q_i||^2 holds for an
// orthonormal basis q_1..q_l.  Its terms are differences of large numbers:
// a rule at eps = 1e-5 decides at 1e-10 ||A||^2, far below what float32
// column energies of G = A V resolve.  This form computes
//   * G64 = A V with float64 products and sums (A and V are float32, so
//     every product is exact in float64),
//   * W = V^T V - I in float64 (the basis' deviation from orthonormality),
//   * per column j, to first order in W (the basis is orthonormal to
//     float32 rounding, |W| ~ 1e-7, so the neglected terms are ~1e-14):
//       c_j = M_jj (1 - W_jj) - 2 sum_{i<j} W_ij M_ij,   M = G64^T G64,
//     the energy ||A q_j||^2 of the basis orthonormalized by Gram-Schmidt in
//     column order (q_j = (v_j - sum_{i<j} q_i R_ij) / R_jj, R from V^T V =
//     R^T R), which keeps Range(q_1..q_j) = Range(v_1..v_j),
// and hands the c_j to the usual prefix-sum rule.
//
// One register-tiled kernel body serves all three products: a 256-thread
// workgroup owns a 128 x 128 output tile (an 8 x 8 block of it per thread,
// rows ty + 16 i and columns tx + 16 j), walking the reduction 16 at a time
// through LDS in float64.  These are FP64 vector FMAs (MI355X's FP64 matrix
// rate is its vector rate); the kernels are bound by FP64 issue.
#include "plu_internal.h"

namespace plu {

namespace {

constexpr int FT = 128;   // output tile edge
constexpr int FK = 16;    // reduction depth per LDS stage

// acc[i][j] = sum_r op(A)(p0 + ty + 16 i, r) * B(r, c0 + tx + 16 j) over
// r < R; op(A)(p, r) = A[p * lda + r] (MODE 0) or A[r * lda + p] (MODE 1);
// entries outside P x R, R x C read as zero.
template <int MODE, typename TA, typename TB>
__device__ __forceinline__ void f64_tile(const TA* __restrict__ A, int64_t lda,
                                         const TB* __restrict__ B, int64_t ldb, int64_t P,
                                         int64_t R, int64_t C, int64_t p0, int64_t c0,
                                         double (&acc)[8][8], double* As, double* Bs) {
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = 0.0;
  for (int64_t r0 = 0; r0 < R; r0 += FK) {
    if (MODE == 0) {
      // row p of the tile: 8 consecutive reduction indices per thread
      const int p = tid >> 1, k0 = (tid & 1) * 8;
      const int64_t gp = p0 + p;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t gr = r0 + k0 + e;
        As[(k0 + e) * FT + p] = (gp < P && gr < R) ? (double)A[gp * lda + gr] : 0.0;
      }
    } else {
      const int k = tid >> 4, pc = (tid & 15) * 8;
      const int64_t gr = r0 + k;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t gp = p0 + pc + e;
        As[k * FT + pc + e] = (gp < P && gr < R) ? (double)A[gr * lda + gp] : 0.0;
      }
    }
    {
      const int k = tid >> 4, cc = (tid & 15) * 8;
      const int64_t gr = r0 + k;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t gc = c0 + cc + e;
        Bs[k * FT + cc + e] = (gc < C && gr < R) ? (double)B[gr * ldb + gc] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < FK; ++k) {
      double a[8], b[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i] = As[k * FT + ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 8; ++j) b[j] = Bs[k * FT + tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
}

// out (P x C, float64, ld ldo) = op(A) B, A and B float32.
struct F64GemmArgs {
  const float* A; int64_t lda;
  const float* B; int64_t ldb;
  int64_t P, R, C;
  double* out; int64_t ldo;
  int mode;
};

template <int MODE>
__device__ void b_f64_gemm(const F64GemmArgs& a, const Grid& gr) {
  __shared__ double As[FK * FT];
  __shared__ double Bs[FK * FT];
  const int64_t p0 = (int64_t)gr.bx * FT, c0 = (int64_t)gr.by * FT;
  double acc[8][8];
  f64_tile<MODE>(a.A, a.lda, a.B, a.ldb, a.P, a.R, a.C, p0, c0, acc, As, Bs);
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int64_t p = p0 + ty + 16 * i;
    if (p >= a.P) continue;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t c = c0 + tx + 16 * j;
      if (c < a.C) a.out[p * a.ldo + c] = acc[i][j];
    }
  }
}

// W = X^T X - I over the tiles on and above the diagonal (X: R x l float32,
// ld ldx); tiles below it are left untouched (never read).
struct F64GramArgs {
  const float* X; int64_t ldx;
  int64_t R, l;
  double* W; int64_t ldw;
};

__device__ void b_f64_gram_w(const F64GramArgs& a, const Grid& gr) {
  if (gr.bx > gr.by) return;
  __shared__ double As[FK * FT];
  __shared__ double Bs[FK * FT];
  const int64_t p0 = (int64_t)gr.bx * FT, c0 = (int64_t)gr.by * FT;
  double acc[8][8];
  f64_tile<1>(a.X, a.ldx, a.X, a.ldx, a.l, a.R, a.l, p0, c0, acc, As, Bs);
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int64_t p = p0 + ty + 16 * i;
    if (p >= a.l) continue;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t c = c0 + tx + 16 * j;
      if (c < a.l) a.W[p * a.ldw + c] = acc[i][j] - (p == c ? 1.0 : 0.0);
    }
  }
}

// Per tile (row block bx, column block by) of M = Y^T Y (Y: R x l, ld ldy,
// float64 or float32): part[bx * l + j] = sum over the tile's rows i of
//   i <  j: -2 W_ij M_ij,   i == j: M_jj (1 - W_jj),   i > j: 0.
// Tiles below the diagonal write zeros.  The rule then sums part over the
// row blocks in order.
template <typename TY>
struct F64CorrArgs {
  const TY* Y; int64_t ldy;
  int64_t R, l;
  const double* W; int64_t ldw;
  double* part;
};

template <typename TY>
__device__ void b_f64_corr(const F64CorrArgs<TY>& a, const Grid& gr) {
  __shared__ double As[FK * FT];
  __shared__ double Bs[FK * FT];
  const int64_t p0 = (int64_t)gr.bx * FT, c0 = (int64_t)gr.by * FT;
  const int tid = threadIdx.x;
  if (gr.bx > gr.by) {
    if (tid < FT && c0 + tid < a.l) a.part[(int64_t)gr.bx * a.l + c0 + tid] = 0.0;
    return;
  }
  double acc[8][8];
  f64_tile<1>(a.Y, a.ldy, a.Y, a.ldy, a.l, a.R, a.l, p0, c0, acc, As, Bs);
  const int ty = tid >> 4, tx = tid & 15;
  double colsum[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) colsum[j] = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int64_t p = p0 + ty + 16 * i;
    if (p >= a.l) continue;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t c = c0 + tx + 16 * j;
      if (c >= a.l) continue;
      double v = 0.0;
      if (p < c) v = -2.0 * a.W[p * a.ldw + c] * acc[i][j];
      else if (p == c) v = acc[i][j] * (1.0 - a.W[c * a.ldw + c]);
      colsum[j] += v;
    }
  }
  // column sums over the 16 row groups, in a fixed order (LDS reused)
  double* red = As;   // 16 x 128 doubles = FK * FT
#pragma unroll
  for (int j = 0; j < 8; ++j) red[ty * FT + tx + 16 * j] = colsum[j];
  __syncthreads();
  if (tid < FT && c0 + tid < a.l) {
    double s = 0.0;
    for (int t = 0; t < 16; ++t) s += red[t * FT + tid];
    a.part[(int64_t)gr.bx * a.l + c0 + tid] = s;
  }
}

}  // namespace

hipError_t launch_f64_gemm(int mode, const float* A, int64_t lda, const float* B, int64_t ldb,
                           int64_t P, int64_t R, int64_t C, double* out, int64_t ldo,
                           hipStream_t s) {
  if (P <= 0 || C <= 0) return hipSuccess;
  const dim3 grid((unsigned)((P + FT - 1) / FT), (unsigned)((C + FT - 1) / FT));
  const F64GemmArgs args{A, lda, B, ldb, P, R, C, out, ldo, mode};
  if (mode == 0) return dispatch<F64GemmArgs, b_f64_gemm<0>, 256, 2>(args, grid, 0, s);
  return dispatch<F64GemmArgs, b_f64_gemm<1>, 256, 2>(args, grid, 0, s);
}

hipError_t launch_f64_gram_w(const float* X, int64_t ldx, int64_t R, int64_t l, double* W,
                             int64_t ldw, hipStream_t s) {
  if (l <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((l + FT - 1) / FT);
  return dispatch<F64GramArgs, b_f64_gram_w, 256, 2>(F64GramArgs{X, ldx, R, l, W, ldw},
                                                     dim3(nb, nb), 0, s);
}

hipError_t launch_f64_corr(const double* Y, const float* Y32, int64_t ldy, int64_t R, int64_t l,
                           const double* W, int64_t ldw, double* part, hipStream_t s) {
  if (l <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((l + FT - 1) / FT);
  if (Y)
    return dispatch<F64CorrArgs<double>, b_f64_corr<double>, 256, 2>(
        F64CorrArgs<double>{Y, ldy, R, l, W, ldw, part}, dim3(nb, nb), 0, s);
  return dispatch<F64CorrArgs<float>, b_f64_corr<float>, 256, 2>(
      F64CorrArgs<float>{Y32, ldy, R, l, W, ldw, part}, dim3(nb, nb), 0, s);
}

int f64_row_blocks(int64_t l) { return (int)((l + FT - 1) / FT); }

}  // namespace plu
