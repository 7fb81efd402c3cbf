// Thin QR of a tall M x c iterate (the paper's [V, ~] = qr(X) in Alg. 6/7).
//
// Method: X = P^T L U (LU with partial pivoting, rows in place) gives
// V0 = P^T L = X U^{-1}, a unit lower trapezoidal basis of the same column
// space whose conditioning does not inherit X's (the ill-conditioning goes
// to U).  V0 is then orthonormalized by block classical Gram-Schmidt with
// reorthogonalization (BCGS2) over column blocks of 128, each block by
// CholeskyQR2: Gram matrix accumulated in float64, Cholesky and triangular
// inverse in float64 inside one workgroup, and the basis update V R^{-1} on
// the FP32 MFMA pass kernel.  Every factor applied from the right is upper
// triangular, so Range(Q(:,1:j)) = Range(X(:,1:j)) for all j: Q is the thin
// Q factor of X up to column signs.
#include "plu_internal.h"

#include <cfloat>

namespace plu {

namespace {

constexpr int QB = 128;   // column block of the Gram-Schmidt sweep

// part[chunk][a][b] = sum over the chunk's rows of V[i][a] V[i][b] (float64),
// for a / 16 <= b / 16 only (the Gram is symmetric: b_gram_reduce reads the
// other entries from their mirror, which the same products in the same
// order give bit for bit).
struct GramArgs {
  const float* V; int64_t ldv, M; int bw; int64_t rows_per_chunk; double* part;
  const int32_t* run_if;   // nullable: nothing is done when it reads 0
};

__device__ void b_gram(const GramArgs& ga, const Grid& gr) {
  const float* __restrict__ V = ga.V;
  const int64_t ldv = ga.ldv, M = ga.M;
  const int bw = ga.bw;
  const int64_t rows_per_chunk = ga.rows_per_chunk;
  double* part = ga.part;
  if (ga.run_if && *ga.run_if == 0) return;
  __shared__ float S[64][QB + 1];
  const int t = threadIdx.x;
  const int ta = t >> 4, tb = t & 15;
  double acc[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = 0.0;
  const int64_t r0 = (int64_t)gr.bx * rows_per_chunk;
  const int64_t r1 = (r0 + rows_per_chunk < M) ? r0 + rows_per_chunk : M;
  for (int64_t rb = r0; rb < r1; rb += 64) {
    __syncthreads();
    for (int e = t; e < 64 * QB; e += 256) {
      const int rr = e / QB, cc = e % QB;
      const int64_t row = rb + rr;
      S[rr][cc] = (row < r1 && cc < bw) ? V[row * ldv + cc] : 0.f;
    }
    __syncthreads();
    // the tile's rows past the chunk are zeros: adding their products would
    // change no sum, so they are skipped
    const int nr = (r1 - rb < 64) ? (int)(r1 - rb) : 64;
    for (int rr = 0; rr < nr; ++rr) {
      double av[8], bv[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) av[i] = S[rr][ta + 16 * i];
#pragma unroll
      for (int j = 0; j < 8; ++j) bv[j] = S[rr][tb + 16 * j];
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = i; j < 8; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
  }
  double* out = part + (int64_t)gr.bx * bw * bw;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int a = ta + 16 * i;
    if (a >= bw) continue;
#pragma unroll
    for (int j = i; j < 8; ++j) {
      const int b = tb + 16 * j;
      if (b < bw) out[a * bw + b] = acc[i][j];
    }
  }
}

struct GramReduceArgs {
  const double* part; int nchunk, bw; double* W; const int32_t* run_if;
};

__device__ void b_gram_reduce(const GramReduceArgs& ga, const Grid& gr) {
  const double* part = ga.part;
  const int nchunk = ga.nchunk, bw = ga.bw;
  double* W = ga.W;
  if (ga.run_if && *ga.run_if == 0) return;
  const int e = gr.bx * 256 + threadIdx.x;
  if (e >= bw * bw) return;
  // b_gram keeps entry (a, b) only for a / 16 <= b / 16; the thread of such
  // an entry also writes its mirror
  const int a = e / bw, b = e % bw;
  if (a / 16 > b / 16) return;
  // eight independent partial sums keep eight loads in flight; fixed order
  double s8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int64_t st = (int64_t)bw * bw;
  int c = 0;
  for (; c + 8 <= nchunk; c += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) s8[u] += part[(int64_t)(c + u) * st + e];
  }
  for (int u = 0; c < nchunk; ++c, ++u) s8[u] += part[(int64_t)c * st + e];
  const double t = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
  W[e] = t;
  if (a / 16 < b / 16) W[b * bw + a] = t;
}

// Cholesky W = L L^T and Y = L^{-1} in float64 inside one workgroup; R^{-1}
// = Y^T is written as float32 (upper triangular, bw x bw, leading dimension
// ldr) and, when Rinv64 is set, as float64.
struct CholArgs {
  const double* W; int bw; float* Rinv; int64_t ldr; double* Rinv64; int32_t* status;
  int32_t* need_lu;   // nullable: set to 1 when the Cholesky factor shows X ill-conditioned
  const int32_t* run_if;   // nullable: nothing is done when it reads 0
};

// Below this ratio of the smallest to the largest diagonal entry of the
// Cholesky factor (a lower bound of 1/cond(X)), X is orthonormalized after
// the LU reorthogonalization: CholeskyQR2 with a float64 Gram is accurate for
// cond(X) well below 1e7, and the ratio underestimates cond(X).
constexpr double kCholRatioMin = 1e-4;

constexpr int CHOL_NB = 16;    // block size of the blocked Cholesky
constexpr int CHOL_QS = 17;    // row stride (doubles) of the block-column buffer
constexpr int CHOL_T = 512;    // threads of the Cholesky workgroup (two waves per SIMD)

// A lane's double from lane src of the wave (src is a constant after unrolling).
__device__ __forceinline__ double readlane_f64(double v, int src) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// 1/sqrt(d) for a positive normal d: the hardware estimate and two Newton
// steps y <- y + y (1 - d y^2) / 2 (each squares the relative error, so the
// estimate's ~2^-22 ends below double rounding).
__device__ __forceinline__ double rsqrt_f64(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-(d * y), y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

__device__ void b_chol_inv(const CholArgs& ca, const Grid& gr) {
  // Right-looking blocked Cholesky (blocks of 16) that carries the inverse
  // along: Y = L^{-1} is the product of the elimination steps applied to I,
  // so block row J of Y is X_JJ T(J, :) (X_JJ = L_JJ^{-1}, T the running
  // right-hand side) and the rows below lose L(I, J) Y(J, :).  Per block:
  //   (1) one wave factors the 16 x 16 diagonal block and inverts it in
  //       registers (lane r holds row r of L_JJ and column r of X_JJ; the
  //       pivot column is broadcast with readlane) -- for block J + 1 this
  //       runs during step (3) of block J, right after that wave has updated
  //       the block, while the other waves update the rest;
  //   (2) the panel L(I, J) = A(I, J) X_JJ^T (a product, not a triangular
  //       solve) and Y(J, :J) = X_JJ T(J, :J), one row or column per thread
  //       with the same arithmetic, into a block-column buffer Q:
  //       Q[i] = L(i, J) for rows below the block, Q[c] = Y(J, c)^T for
  //       columns up to it;
  //   (3) one symmetric rank-16 update out(r, c) -= Q[r] . Q[c] for every
  //       row r below the block and c <= r: the trailing matrix for c below
  //       the block, T for c up to it; 4 x 4 register tiles.
  // S holds A / L in its lower triangle and Y transposed above it: Y[r][c]
  // (c <= r) at S[c][r + 1].  Entries of S that no later step reads (the
  // factored block column, rows and columns past bw) take whatever the
  // branch-free loads and stores put there; every access stays inside S.
  (void)gr;
  const double* W = ca.W;
  const int bw = ca.bw;
  float* Rinv = ca.Rinv;
  const int64_t ldr = ca.ldr;
  double* Rinv64 = ca.Rinv64;
  int32_t* status = ca.status;
  if (ca.run_if && *ca.run_if == 0) return;
  constexpr int NB = CHOL_NB;
  __shared__ int bad;
  __shared__ double S[QB][QB + 1];
  // Q rows QB .. QB + 15 hold the 16 x 16 identity (read as rows, so the
  // per-lane unit vectors are reloaded each block instead of held live)
  __shared__ double Q[QB + NB][CHOL_QS];
  __shared__ __align__(16) double XdT[NB][NB];   // XdT[m][c] = X_JJ[c][m]
  __shared__ double QD[NB][CHOL_QS];             // Q rows of the diagonal block
  __shared__ double Dg[QB];                      // diagonal of L
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  if (t == 0) bad = 0;
  if (t < NB * NB) Q[QB + t / NB][t % NB] = (t / NB == t % NB) ? 1.0 : 0.0;
  {
    // S[r][c] = W[r][c] for c <= r < bw, 0 elsewhere in rows and columns
    // 0 .. 127 (the running T / Y above the diagonal); column 128 is zero.
    // Thread (ry, cx) of 32 x 16 covers rows ry + 32 p and columns cx + 16 u;
    // every load is issued before the first store (clamped addresses).
    const int cx = t & 15, ry = t >> 4;
    double v[4][8];
#pragma unroll
    for (int p4 = 0; p4 < 4; ++p4)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int r = ry + 32 * p4, c = cx + 16 * u;
        const int rr = (r < bw) ? r : bw - 1, cc = (c < rr) ? c : rr;
        const double w = W[rr * bw + cc];
        v[p4][u] = (r < bw && c <= r) ? w : 0.0;
      }
#pragma unroll
    for (int p4 = 0; p4 < 4; ++p4)
#pragma unroll
      for (int u = 0; u < 8; ++u) S[ry + 32 * p4][cx + 16 * u] = v[p4][u];
    if (t < QB) S[t][QB] = 0.0;
  }
  __syncthreads();
  const int nblk = (bw + NB - 1) / NB;
  // (1) for block J, by wave 0: the diagonal block, padded to 16 x 16 with
  // the identity.  Lane r < nb holds row r of the block (entries above the
  // diagonal are never combined with those below it, so they are left as they
  // come); lanes nb .. 15 hold identity rows, other lanes row 0 of the
  // identity.  Writes X_JJ to XdT and QD, Y_JJ into S, the pivots into Dg.
  auto diag_block = [&](int J) {
    const int nb = (bw - J < NB) ? bw - J : NB;
    const int r = lane;
    const int rs = (r < NB) ? r : 0;
    const double* arow = (r < nb) ? &S[J + r][J] : &Q[QB + rs][0];
    const double* irow = &Q[QB + rs][0];
    double a[NB], x[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      a[c] = arow[c];
      x[c] = irow[c];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      double d = readlane_f64(a[j], j);
      if (!(d > 0.0)) {
        if (lane == 0) {
          status[2] = 1;
          bad = 1;
        }
        d = DBL_MIN;
        a[j] = (r == j) ? d : a[j];
      }
      const double rp = rsqrt_f64(d);
      // column j of L: the pivot lane gets d / sqrt(d) = sqrt(d), the rows
      // below their multipliers
      a[j] *= rp;
      if (lane == 0) Dg[J + j] = d * rp;
      x[j] *= rp;
#pragma unroll
      for (int c = j + 1; c < NB; ++c) {
        const double lc = readlane_f64(a[j], c);   // L(J + c, J + j)
        a[c] = fma(-a[j], lc, a[c]);
        x[c] = fma(-lc, x[j], x[c]);
      }
      // finish the step's updates here (an empty asm that takes the
      // registers in and out; no instruction): the compiler would otherwise
      // sink them to their next use and keep every broadcast multiplier of
      // the block live in scalar registers
#pragma unroll
      for (int c = j + 1; c < NB; ++c) asm volatile("" : "+v"(a[c]), "+v"(x[c]));
    }
    if (r < NB) {
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        XdT[r][c] = x[c];
        QD[r][c] = x[c];                              // Y(J + c, J + r)
      }
    }
    if (r < nb) {
      // Y(J + rr, J + r) = x[rr]; for rr < r the slot is in the factored
      // (dead) lower part and receives the zero x[rr]
#pragma unroll
      for (int rr = 0; rr < NB; ++rr) S[J + r][J + 1 + rr] = x[rr];
    }
  };
  if (wave == 0) diag_block(0);
  __syncthreads();
  for (int J = 0; J < bw; J += NB) {
    const int nb = (bw - J < NB) ? bw - J : NB;
    // (2) out = v X_JJ^T for a source vector v: the row of the panel
    // (v = A(i, J:J+16), x = i, y0 = J) or the column of T (v = T(J:J+nb, c),
    // x = c, y0 = J + 1), four threads per vector, each the outputs
    // c' = q, q + 4, q + 8, q + 12; Q[x][c'] = S[x][y0 + c'] = out[c'].  In
    // the last block (nb < 16) out[c'] = 0 for c' >= nb lands in columns past
    // bw.  The four threads of a vector are lanes of one wave, which reads
    // all of v before any of them stores.  The diagonal block's rows of Q
    // come from QD.
    const int r0 = J + nb, nrow = bw - r0;
    if (t < 4 * (nrow + J)) {
      const int src = t >> 2, q = t & 3;
      const bool panel = src < nrow;
      const int x0 = panel ? r0 + src : src - nrow;
      const int y0 = panel ? J : J + 1;
      double v[NB];
#pragma unroll
      for (int m = 0; m < NB; ++m) {
        const double sv = S[x0][y0 + m];
        v[m] = (m < nb) ? sv : 0.0;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int c = q + 4 * k;
        double o = 0.0;
#pragma unroll
        for (int m = 0; m < 4 * k + 4; ++m) o = fma(v[m], XdT[m][c], o);   // XdT[m][c] = 0 for m > c
        Q[x0][c] = o;
        S[x0][y0 + c] = o;
      }
    }
    if (t < NB * NB) Q[J + t / NB][t % NB] = QD[t / NB][t % NB];   // rows past bw are never read
    __syncthreads();
    if (nrow <= 0) break;
    // (3) out(r, c) -= Q[r] . Q[c], r >= r0, c <= r, over 16 x 16 tiles
    // (R, C), R a row block below the diagonal one, C <= R.  Rows past bw and
    // c > r in a diagonal tile are computed too and land in slots no later
    // step reads.  Wave 0 takes the tile (Rb0, Rb0), the next diagonal block,
    // in 2 x 2 pieces and then factors it (look-ahead); waves 1 .. 7 take
    // the other tiles in 4 x 4 pieces.
    const int Rb0 = J / NB + 1;
    if (wave == 0) {
      const int rb = Rb0 * NB + 2 * (lane >> 3), cb = Rb0 * NB + 2 * (lane & 7);
      double acc[2][2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = S[rb + i][cb + j];
#pragma unroll
      for (int kk = 0; kk < NB; ++kk) {
        const double qa0 = Q[rb][kk], qa1 = Q[rb + 1][kk];
        const double qb0 = Q[cb][kk], qb1 = Q[cb + 1][kk];
        acc[0][0] = fma(-qa0, qb0, acc[0][0]);
        acc[0][1] = fma(-qa0, qb1, acc[0][1]);
        acc[1][0] = fma(-qa1, qb0, acc[1][0]);
        acc[1][1] = fma(-qa1, qb1, acc[1][1]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) S[rb + i][cb + j] = acc[i][j];
      // a wave's LDS operations complete in issue order; keep the compiler
      // from moving the block's loads above these stores
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      diag_block(Rb0 * NB);
    } else {
      const int ntiles = (nblk * (nblk + 1) - Rb0 * (Rb0 + 1)) / 2 - 1;   // without (Rb0, Rb0)
      for (int w = t - 64; w < ntiles * 16; w += CHOL_T - 64) {
        int tile = w >> 4;
        const int sub = w & 15;
        if (tile >= Rb0) ++tile;             // skip (Rb0, Rb0), the Rb0-th tile
        int R = Rb0;
        while (tile > R) {
          tile -= R + 1;
          ++R;
        }
        const int C = tile;
        const bool tpart = C < Rb0;          // columns of T (transposed storage)
        const int rb = R * NB + 4 * (sub >> 2), cb = C * NB + 4 * (sub & 3);
        double* dst[4][4];
        double acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int r = rb + i, c = cb + j;
            dst[i][j] = tpart ? &S[c][r + 1] : &S[r][c];
            acc[i][j] = *dst[i][j];
          }
        double qa[2][4], qb[2][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          qa[0][i] = Q[rb + i][0];
          qb[0][i] = Q[cb + i][0];
        }
#pragma unroll
        for (int kk = 0; kk < NB; ++kk) {
          const int cur = kk & 1, nxt = cur ^ 1;
          if (kk + 1 < NB) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              qa[nxt][i] = Q[rb + i][kk + 1];
              qb[nxt][i] = Q[cb + i][kk + 1];
            }
          }
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = fma(-qa[cur][i], qb[cur][j], acc[i][j]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) *dst[i][j] = acc[i][j];
      }
    }
    __syncthreads();
  }
  if (ca.need_lu && t == 0) {
    double mn = Dg[0], mx = Dg[0];
    for (int j = 1; j < bw; ++j) {
      mn = fmin(mn, Dg[j]);
      mx = fmax(mx, Dg[j]);
    }
    *ca.need_lu = (bad || !(mn > kCholRatioMin * mx)) ? 1 : 0;
  }
  // Rinv[r][c] = Y[c][r] = S[r][c + 1] for r <= c, 0 below the diagonal
  {
    const int cx = t & 15, ry = t >> 4;
#pragma unroll
    for (int p4 = 0; p4 < 4; ++p4) {
      const int r = ry + 32 * p4;
      if (r >= bw) break;
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = cx + 16 * u;
        const double sv = S[r][c + 1];
        v[u] = (r <= c) ? sv : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = cx + 16 * u;
        if (c < bw) {
          Rinv[(int64_t)r * ldr + c] = (float)v[u];
          if (Rinv64) Rinv64[(int64_t)r * ldr + c] = v[u];
        }
      }
    }
  }
}

// dst = src R^{-1} with float64 products and sums, rounded once to float32.
// R^{-1} (upper triangular, bw x bw <= 128 x 128) is staged in LDS as float32
// with its diagonal kept in float64 (in the last CholeskyQR round R is close
// to I, so the off-diagonal entries are tiny and their float32 rounding is a
// second-order effect); each thread owns two rows (r and r + 64) and 16
// interleaved columns of a block of 128 rows.  A block takes about 131 KB of
// LDS, one per CU: 128 rows keep a 20000-row product to one round of the
// device's CUs (64-row blocks took two).
constexpr int APPLY_ROWS = 128;
constexpr size_t APPLY_LDS = (size_t)QB * QB * sizeof(float) + QB * sizeof(double) +
                             (size_t)APPLY_ROWS * (QB + 1) * sizeof(float);

struct ApplyArgs {
  const float* src; int64_t lds, M; int bw; const double* rinv; int64_t ldr; float* dst;
  int64_t ldd;
};

__device__ void b_apply_rinv64(const ApplyArgs& aa, const Grid& gr) {
  const float* __restrict__ src = aa.src;
  const int64_t lds = aa.lds, M = aa.M;
  const int bw = aa.bw;
  const double* __restrict__ rinv = aa.rinv;
  const int64_t ldr = aa.ldr;
  float* dst = aa.dst;
  const int64_t ldd = aa.ldd;
  extern __shared__ double smem[];
  double* Dg = smem;                                           // [QB] diagonal, float64
  float* R = reinterpret_cast<float*>(smem + QB);              // [QB][QB]
  float* Vs = R + QB * QB;                                     // [APPLY_ROWS][QB+1]
  const int t = threadIdx.x;
  for (int r = t >> 5; r < bw; r += 16)
    for (int c = t & 31; c < QB; c += 32)
      R[r * QB + c] = (c < bw && c != r) ? (float)rinv[(int64_t)r * ldr + c] : 0.f;
  if (t < bw) Dg[t] = rinv[(int64_t)t * ldr + t];
  const int64_t r0 = (int64_t)gr.bx * APPLY_ROWS;
  for (int rr = t >> 5; rr < APPLY_ROWS; rr += 16) {
    const int64_t row = r0 + rr;
    for (int c = t & 31; c < bw; c += 32) Vs[rr * (QB + 1) + c] = (row < M) ? src[row * lds + c] : 0.f;
  }
  __syncthreads();
  const int rr = t & 63;          // rows rr and rr + 64 of the block
  const int cg = t >> 6;          // column group: columns cg, cg+8, ...
  double acc[2][QB / 8];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int jj = 0; jj < QB / 8; ++jj) acc[h][jj] = 0.0;
  // R^{-1} is upper triangular (its diagonal applied below): column j takes
  // the terms tt < j only.  Segment s covers the tt with columns jj >= s of
  // this thread's group still open; every column's chain keeps the order of
  // tt, and the skipped terms are exact zeros, so the sums are those of the
  // full loop.
#pragma unroll
  for (int sg = 0; sg < QB / 8; ++sg) {
    const int lo = sg == 0 ? 0 : cg + 8 * (sg - 1);
    const int hi = (cg + 8 * sg < bw) ? cg + 8 * sg : bw;
    for (int tt = lo; tt < hi; ++tt) {
      const double v0 = Vs[rr * (QB + 1) + tt];
      const double v1 = Vs[(rr + 64) * (QB + 1) + tt];
      const float* Rr = R + tt * QB + cg;
#pragma unroll
      for (int jj = sg; jj < QB / 8; ++jj) {
        const double rv = (double)Rr[8 * jj];
        acc[0][jj] = fma(v0, rv, acc[0][jj]);
        acc[1][jj] = fma(v1, rv, acc[1][jj]);
      }
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int rb = rr + 64 * h;
    const int64_t row = r0 + rb;
    if (row >= M) continue;
#pragma unroll
    for (int jj = 0; jj < QB / 8; ++jj) {
      const int j = cg + 8 * jj;
      if (j < bw) dst[row * ldd + j] = (float)fma((double)Vs[rb * (QB + 1) + j], Dg[j], acc[h][jj]);
    }
  }
}

hipError_t gemm_any(int mode, int epi, GemmArgs g, const QrWork& qw, hipStream_t s) {
  // EPI_STORE with automatic split-K through qw.part
  const GemmPlan pl = plan_gemm(g.P, g.R, g.C, 64, 1024);
  hipError_t e;
  if (pl.nsplit > 1 && epi == EPI_STORE) {
    if ((int64_t)pl.nsplit * g.P * g.ldo > qw.part_cap) return hipErrorInvalidValue;
    float* out = g.out;
    g.out = qw.part;
    g.part_stride = g.P * g.ldo;
    if ((e = launch_gemm(mode, EPI_PART, 0, g, pl, s)) != hipSuccess) return e;
    return launch_splitk_reduce(qw.part, g.P * g.ldo, pl.nsplit, out, g.ldo, g.P, g.C, nullptr, 64,
                                s);
  }
  GemmPlan p1 = pl;
  if (epi != EPI_STORE) p1 = plan_gemm(g.P, g.R, g.C, 1, 1);
  return launch_gemm(mode, epi, 0, g, p1, s);
}

hipError_t cholqr_round(const float* src, int64_t lds, int64_t M, int bw, float* dst, int64_t ldd,
                        const QrWork& qw, bool fp64_apply, hipStream_t s,
                        const int32_t* factor_if = nullptr) {
  // factor_if (nullable): the Gram and Cholesky steps run only when it reads
  // nonzero (otherwise the R^{-1} already in qw.rinv is applied)
  int nchunk = (int)((M + 63) / 64);
  if (nchunk > qw.max_chunks) nchunk = qw.max_chunks;
  int64_t rpc = (M + nchunk - 1) / nchunk;
  rpc = ((rpc + 63) / 64) * 64;
  nchunk = (int)((M + rpc - 1) / rpc);
  hipError_t e;
  if ((e = dispatch<GramArgs, b_gram, 256>(GramArgs{src, lds, M, bw, rpc, qw.gram_part, factor_if},
                                           dim3(nchunk), 0, s)) != hipSuccess)
    return e;
  if ((e = dispatch<GramReduceArgs, b_gram_reduce, 256>(
           GramReduceArgs{qw.gram_part, nchunk, bw, qw.gram, factor_if},
           dim3((bw * bw + 255) / 256), 0, s)) != hipSuccess)
    return e;
  if ((e = dispatch<CholArgs, b_chol_inv, CHOL_T>(
           CholArgs{qw.gram, bw, qw.rinv, (int64_t)QB, fp64_apply ? qw.rinv64 : nullptr,
                    qw.status, nullptr, factor_if},
           dim3(1), 0, s)) != hipSuccess)
    return e;
  if (fp64_apply) {
    return dispatch<ApplyArgs, b_apply_rinv64, 512>(
        ApplyArgs{src, lds, M, bw, qw.rinv64, (int64_t)QB, dst, ldd},
        dim3((unsigned)((M + APPLY_ROWS - 1) / APPLY_ROWS)), APPLY_LDS, s);
  }
  GemmArgs g;
  g.A = src; g.lda = lds;
  g.X = qw.rinv; g.ldx = QB;
  g.out = dst; g.ldo = ldd;
  g.P = M; g.R = bw; g.C = bw;
  return gemm_any(0, EPI_STORE, g, qw, s);
}

// Whether X (one block) is well enough conditioned for CholeskyQR2 alone:
// its float64 Gram, Cholesky and the diagonal test write qw.status[4].
hipError_t cholqr_probe(const float* X, int64_t ldx, int64_t M, int bw, const QrWork& qw,
                        hipStream_t s) {
  int nchunk = (int)((M + 63) / 64);
  if (nchunk > qw.max_chunks) nchunk = qw.max_chunks;
  int64_t rpc = (M + nchunk - 1) / nchunk;
  rpc = ((rpc + 63) / 64) * 64;
  nchunk = (int)((M + rpc - 1) / rpc);
  hipError_t e;
  if ((e = dispatch<GramArgs, b_gram, 256>(GramArgs{X, ldx, M, bw, rpc, qw.gram_part, nullptr},
                                           dim3(nchunk), 0, s)) != hipSuccess)
    return e;
  if ((e = dispatch<GramReduceArgs, b_gram_reduce, 256>(
           GramReduceArgs{qw.gram_part, nchunk, bw, qw.gram, nullptr},
           dim3((bw * bw + 255) / 256), 0, s)) != hipSuccess)
    return e;
  // R^{-1} of X itself is kept in qw.rinv: the first CholeskyQR round reuses
  // it when the LU is skipped
  return dispatch<CholArgs, b_chol_inv, CHOL_T>(
      CholArgs{qw.gram, bw, qw.rinv, (int64_t)QB, nullptr, qw.status, qw.status + 4, nullptr},
      dim3(1), 0, s);
}

}  // namespace

hipError_t thin_qr_run(float* X, int64_t ldx, int64_t M, int c, const GetrfWork& gw0,
                       const QrWork& qw, hipStream_t s) {
  hipError_t e;
  // Block classical Gram-Schmidt with reorthogonalization over blocks of QB
  // columns.  Each block, once projected off the earlier ones, is probed:
  // the Cholesky factor of its float64 Gram decides whether it first takes
  // the LU reorthogonalization V_J <- P^T L (the LU kernels read the flag on
  // the device and run or return at once).  Both steps multiply the block by
  // upper triangular matrices, so Range(Q(:,1:j)) = Range(X(:,1:j)).
  GetrfWork gw = gw0;
  gw.run_if = qw.status + 4;
  for (int j0 = 0; j0 < c; j0 += QB) {
    const int bw = (c - j0 < QB) ? c - j0 : QB;
    float* VJ = X + j0;
    if (j0 > 0) {
      for (int rep = 0; rep < 2; ++rep) {
        // W = Q(:, :j0)^T V_J
        GemmArgs g;
        g.A = qw.q; g.lda = qw.ldq;
        g.X = VJ; g.ldx = ldx;
        g.out = qw.wproj; g.ldo = QB;
        g.P = j0; g.R = M; g.C = bw;
        if ((e = gemm_any(1, EPI_STORE, g, qw, s)) != hipSuccess) return e;
        // V_J -= Q(:, :j0) W
        GemmArgs h;
        h.A = qw.q; h.lda = qw.ldq;
        h.X = qw.wproj; h.ldx = QB;
        h.out = VJ; h.ldo = ldx;
        h.P = M; h.R = j0; h.C = bw;
        if ((e = gemm_any(0, EPI_SUB, h, qw, s)) != hipSuccess) return e;
      }
    }
    if ((e = cholqr_probe(VJ, ldx, M, bw, qw, s)) != hipSuccess) return e;
    if ((e = getrf_run(VJ, ldx, M, bw, gw, nullptr, nullptr, 0, 0, s)) != hipSuccess) return e;
    // first round on the MFMA pass kernel; the second (R nearly I) in float64
    // so that the stored basis is orthonormal to about one fp32 rounding.  The
    // first round reuses the probe's factor unless the LU changed the block.
    if ((e = cholqr_round(VJ, ldx, M, bw, qw.tmp, QB, qw, false, s, qw.status + 4)) !=
        hipSuccess)
      return e;
    if ((e = cholqr_round(qw.tmp, QB, M, bw, qw.q + j0, qw.ldq, qw, true, s)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

hipError_t gram_inverse_run(const float* X, int64_t ldx, int64_t M, int c, const QrWork& qw,
                            hipStream_t s) {
  if (c < 1 || c > QB || M < c) return hipErrorInvalidValue;
  // the Cholesky factor's diagonal test (qw.status[4]) is not used here
  return cholqr_probe(X, ldx, M, c, qw, s);
}

}  // namespace plu
