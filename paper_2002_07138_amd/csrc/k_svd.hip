// SVD of a small square matrix R (l x l, l <= 128): the deterministic step of
// RandSVD (Alg. 1 step 5) once B^T = Q_b R is reduced by a thin QR, so that
// B = V_r S (Q_b U_r)^T for R = U_r S V_r^T.
//
// Method: one-sided (Hestenes) Jacobi in one workgroup.  Column pairs (i, j)
// of X = R J are rotated until every pair is orthogonal to the tolerance;
// then S = the column norms of X, U_r = X S^{-1} and V_r = J.  The pairs of a
// sweep follow the round-robin (circle) order, l/2 disjoint pairs per round,
// one pair per quad of lanes (up to 32 contiguous rows each, 16-byte LDS
// accesses); per-lane float32 partial dot products are summed in float64
// across the quad by DPP, the rotation angle is float64, and X and J are
// stored and rotated as float32 in LDS (two 66 KB tiles at l = 128).
#include "plu_internal.h"

namespace plu {

namespace {

constexpr int SVD_MAX = 128;
constexpr int SVD_LPP = 4;                    // lanes per column pair (one quad)
constexpr int SVD_T = SVD_MAX / 2 * SVD_LPP;  // 256: 64 pairs
constexpr int SVD_RPL = SVD_MAX / SVD_LPP;    // 32 contiguous rows per lane
constexpr int SVD_LD = SVD_MAX + 4;           // column stride (floats) of the LDS tiles

struct JacobiArgs {
  const float* R; int64_t ldr; int l;
  float* Ur; int64_t ldur;     // U_r, columns in non-increasing order of S
  float* Vr; int64_t ldvr;     // V_r, same order
  float* S; int kout;          // the kout largest singular values
  int32_t* sweeps_out;         // nullable: sweeps taken
  int max_sweeps;
  double tol;                  // rotate while |x_i . x_j| > tol ||x_i|| ||x_j|| (1e-6: above
                               // the float32 tiles' rounding floor, about 2 u32)
};

// A double from lane (lane ^ 1) or (lane ^ 2) of the quad: DPP quad_perm
// [1,0,3,2] (0xB1) or [2,3,0,1] (0x4E) on both 32-bit halves.
template <int CTRL>
__device__ __forceinline__ double quad_swap(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const unsigned hi =
      (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum over the four lanes of a quad; the butterfly's additions are the same
// pairs in every lane, so all four get the same total.
__device__ __forceinline__ double quad_sum(double v) {
  v += quad_swap<0xB1>(v);
  return v + quad_swap<0x4E>(v);
}

__device__ void b_jacobi_svd(const JacobiArgs& a, const Grid& gr) {
  (void)gr;
  __shared__ __align__(16) float X[SVD_MAX][SVD_LD];    // X[j][r]: column j of R J
  __shared__ __align__(16) float Jm[SVD_MAX][SVD_LD];   // Jm[j][r]: column j of J
  __shared__ double sig[SVD_MAX];
  __shared__ int rk[SVD_MAX];
  __shared__ int rotated;
  const int l = a.l;
  const int t = threadIdx.x;
  const int g = t >> 2, q = t & 3;
  const int nu = (l + 15) / 16;               // float4 groups of rows per lane
  const int r0 = q * 4 * nu;                  // this lane's rows r0 .. r0 + 4 nu - 1
  // rows past l are zero in both tiles, so the fixed-trip loops below need
  // no row mask
  for (int e = t; e < SVD_MAX * SVD_MAX; e += SVD_T) {
    const int c = e / SVD_MAX, r = e - c * SVD_MAX;
    X[c][r] = (r < l && c < l) ? a.R[(int64_t)r * a.ldr + c] : 0.f;
    Jm[c][r] = (r == c && r < l) ? 1.f : 0.f;
  }
  const int le = (l + 1) & ~1;             // column l is a dummy when l is odd
  const double tol2 = a.tol * a.tol;
  int sweep = 0;
  while (sweep < a.max_sweeps) {
    __syncthreads();                       // every thread has read the last flag
    if (t == 0) rotated = 0;
    __syncthreads();
    for (int rnd = 0; rnd < le - 1; ++rnd) {
      if (g < le / 2) {
        // circle method: position 0 fixed, positions 1 .. le-1 turn by rnd
        const int p0 = g, p1 = le - 1 - g;
        int i = (p0 == 0) ? 0 : ((p0 - 1 + rnd) % (le - 1)) + 1;
        int j = ((p1 - 1 + rnd) % (le - 1)) + 1;
        if (i > j) {
          const int tmp = i;
          i = j;
          j = tmp;
        }
        if (j < l) {
          // rows past l are zero, and past 4 nu lanes' ranges are never read
          float4 xi[SVD_RPL / 4], xj[SVD_RPL / 4];
#pragma unroll
          for (int u = 0; u < SVD_RPL / 4; ++u) {
            if (u < nu) {
              xi[u] = *reinterpret_cast<const float4*>(&X[i][r0 + 4 * u]);
              xj[u] = *reinterpret_cast<const float4*>(&X[j][r0 + 4 * u]);
            } else {
              xi[u] = make_float4(0.f, 0.f, 0.f, 0.f);
              xj[u] = xi[u];
            }
          }
          // per-lane partial sums in float32 (at most 32 terms: error about
          // sqrt(32) u32 of sum |x_i x_j|, below the tolerance), then float64
          float al[2] = {0.f, 0.f}, be[2] = {0.f, 0.f}, ga[2] = {0.f, 0.f};
#pragma unroll
          for (int u = 0; u < SVD_RPL / 4; ++u) {
            if (u < nu) {
              const float av[4] = {xi[u].x, xi[u].y, xi[u].z, xi[u].w};
              const float bv[4] = {xj[u].x, xj[u].y, xj[u].z, xj[u].w};
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const int h = e & 1;
                al[h] = fmaf(av[e], av[e], al[h]);
                be[h] = fmaf(bv[e], bv[e], be[h]);
                ga[h] = fmaf(av[e], bv[e], ga[h]);
              }
            }
          }
          const double A2 = quad_sum((double)al[0] + (double)al[1]);
          const double B2 = quad_sum((double)be[0] + (double)be[1]);
          const double G = quad_sum((double)ga[0] + (double)ga[1]);
          if (A2 > 0.0 && B2 > 0.0 && G * G > tol2 * A2 * B2) {
            // x_i' = c x_i - s x_j, x_j' = s x_i + c x_j with x_i' . x_j' = 0:
            // t = s / c is the smaller root of t^2 + 2 zeta t - 1 = 0, in
            // float64; c and s are rounded to float32, the tiles' format
            const double zeta = (B2 - A2) / (2.0 * G);
            const double tn = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const float cs = (float)(1.0 / sqrt(1.0 + tn * tn));
            const float sn = cs * (float)tn;
#pragma unroll
            for (int u = 0; u < SVD_RPL / 4; ++u) {
              if (u >= nu) break;
              float4 ni, nj;
              ni.x = fmaf(cs, xi[u].x, -sn * xj[u].x);
              ni.y = fmaf(cs, xi[u].y, -sn * xj[u].y);
              ni.z = fmaf(cs, xi[u].z, -sn * xj[u].z);
              ni.w = fmaf(cs, xi[u].w, -sn * xj[u].w);
              nj.x = fmaf(sn, xi[u].x, cs * xj[u].x);
              nj.y = fmaf(sn, xi[u].y, cs * xj[u].y);
              nj.z = fmaf(sn, xi[u].z, cs * xj[u].z);
              nj.w = fmaf(sn, xi[u].w, cs * xj[u].w);
              *reinterpret_cast<float4*>(&X[i][r0 + 4 * u]) = ni;
              *reinterpret_cast<float4*>(&X[j][r0 + 4 * u]) = nj;
            }
#pragma unroll
            for (int u = 0; u < SVD_RPL / 4; ++u) {
              if (u >= nu) break;
              const float4 vi = *reinterpret_cast<const float4*>(&Jm[i][r0 + 4 * u]);
              const float4 vj = *reinterpret_cast<const float4*>(&Jm[j][r0 + 4 * u]);
              float4 ni, nj;
              ni.x = fmaf(cs, vi.x, -sn * vj.x);
              ni.y = fmaf(cs, vi.y, -sn * vj.y);
              ni.z = fmaf(cs, vi.z, -sn * vj.z);
              ni.w = fmaf(cs, vi.w, -sn * vj.w);
              nj.x = fmaf(sn, vi.x, cs * vj.x);
              nj.y = fmaf(sn, vi.y, cs * vj.y);
              nj.z = fmaf(sn, vi.z, cs * vj.z);
              nj.w = fmaf(sn, vi.w, cs * vj.w);
              *reinterpret_cast<float4*>(&Jm[i][r0 + 4 * u]) = ni;
              *reinterpret_cast<float4*>(&Jm[j][r0 + 4 * u]) = nj;
            }
            if (q == 0) rotated = 1;
          }
        }
      }
      __syncthreads();
    }
    ++sweep;
    if (!rotated) break;                   // read after the last round's barrier
  }
  if (t == 0 && a.sweeps_out) *a.sweeps_out = sweep;
  // singular values (column norms of X) and their non-increasing order
  for (int j = g; j < l; j += SVD_T / SVD_LPP) {
    double ss = 0.0;
    for (int r = r0; r < r0 + 4 * nu; ++r) ss = fma((double)X[j][r], (double)X[j][r], ss);
    ss = quad_sum(ss);
    if (q == 0) sig[j] = sqrt(ss);
  }
  __syncthreads();
  if (t < l) {
    const double sj = sig[t];
    int rank = 0;
    for (int i = 0; i < l; ++i) rank += (sig[i] > sj || (sig[i] == sj && i < t)) ? 1 : 0;
    rk[t] = rank;
    if (rank < a.kout) a.S[rank] = (float)sj;
  }
  __syncthreads();
  for (int e = t; e < l * l; e += SVD_T) {
    const int j = e / l, r = e - j * l;
    const int c = rk[j];
    const double sj = sig[j];
    a.Ur[(int64_t)r * a.ldur + c] = (sj > 0.0) ? (float)((double)X[j][r] / sj) : 0.f;
    a.Vr[(int64_t)r * a.ldvr + c] = Jm[j][r];
  }
}

}  // namespace

hipError_t launch_jacobi_svd(const float* R, int64_t ldr, int l, float* Ur, int64_t ldur,
                             float* Vr, int64_t ldvr, float* S, int kout, int32_t* sweeps_out,
                             hipStream_t s) {
  if (l < 1 || l > SVD_MAX || kout < 0 || kout > l) return hipErrorInvalidValue;
  return dispatch<JacobiArgs, b_jacobi_svd, SVD_T>(
      JacobiArgs{R, ldr, l, Ur, ldur, Vr, ldvr, S, kout, sweeps_out, 40, 1e-6}, dim3(1), 0, s);
}

}  // namespace plu
