// Pass kernels: one streaming pass over A producing A X or A^T X (the matrix
// products of Alg. 7 and of Alg. 5 step 3 / Alg. 8 step 3), on FP32 MFMA.
//
// Work decomposition (per workgroup of 256 threads = 4 waves):
//   * 128 rows of the kept dimension P (32 per wave, 2 MFMA row tiles), or
//     64 rows (1 tile per wave) in the variant the autotuner may pick; the
//     small register footprint lets 4 (or 6) workgroups share a CU, which is
//     what hides the HBM latency of the streamed A tiles,
//   * NT*16 columns of the sketch (NT <= 8 MFMA column tiles),
//   * a contiguous range of the reduced dimension R, walked 16 (direct
//     passes) or 32 at a time through LDS with the next stage prefetched into
//     registers; the prefetch is issued before the barrier that follows the
//     LDS store.
// v_mfma_f32_16x16x4f32 is fed with a permuted reduction order: lane (r, g)
// of a 16x16x4 step s uses reduction index 4g + s inside a 16-wide group, so
// one 16-byte LDS read of A gives a lane its operands for four consecutive
// MFMAs in mode N.  Both operands use the same permutation, so the sum is
// unchanged.  Split partials are reduced by a second kernel in a fixed order,
// so results do not depend on scheduling.
#include "plu_internal.h"

#include <algorithm>

namespace plu {

namespace {

constexpr int BP = GEMM_BP;     // rows per workgroup of the default variant
constexpr int BK = GEMM_BK;     // reduction depth per stage of the default variant

__device__ __forceinline__ double block_sum_double(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = (red[0] + red[1]) + (red[2] + red[3]);
  return t;
}

__device__ __forceinline__ f32x4 load4(const float* src, int64_t idx, int64_t lim, int vec) {
  // src[idx .. idx+3], entries at or beyond lim read as zero.  vec (uniform)
  // says src + idx is 16-byte aligned, so the full case is one vector load.
  f32x4 v = {0.f, 0.f, 0.f, 0.f};
  if (vec && idx + 3 < lim) {
    v = *reinterpret_cast<const f32x4*>(src + idx);
  } else {
    if (idx + 0 < lim) v.x = src[idx + 0];
    if (idx + 1 < lim) v.y = src[idx + 1];
    if (idx + 2 < lim) v.z = src[idx + 2];
    if (idx + 3 < lim) v.w = src[idx + 3];
  }
  return v;
}

// RT: 16-row MFMA tiles per wave (the workgroup covers BP = 64 RT rows);
// BKT: reduction depth per LDS stage.  DYN: the grouped form, where the
// column-tile count (g.nt <= NT) is read at run time; all NT tiles are
// multiplied (columns past C load as zeros, columns of the next block are
// computed and dropped) and only g.nt are stored.
template <int MODE, int NT, int EPI, int RT = GEMM_BP / 64, int BKT = GEMM_BK, bool DYN = false>
__device__ __forceinline__ void pass_body(const GemmArgs& g, const Grid& gr) {
  if (g.run_if && *g.run_if == 0) return;
  constexpr int BP = 64 * RT;
  constexpr int BK = BKT;
  constexpr int AST_N = BK + 4;   // mode N A tile: [BP][BK+4]  (row p, reduction r)
  constexpr int AST_T = BP + 4;   // mode T A tile: [BK][BP+4]  (reduction r, row p)
  constexpr int XC = NT * 16;
  constexpr int XST = XC + 4;
  constexpr int A_ELEMS = (MODE == 0) ? BP * AST_N : BK * AST_T;
  constexpr int AV = BP * BK / 4;            // float4 slots in the A tile
  constexpr int AIT = AV / 256;
  constexpr int XV = BK * NT * 4;            // float4 slots in the X tile
  constexpr int XIT = (XV + 255) / 256;
  static_assert(AV % 256 == 0, "A tile must split evenly over 256 threads");
  __shared__ __attribute__((aligned(16))) float As[A_ELEMS];
  __shared__ __attribute__((aligned(16))) float Xs[BK * XST];
  __shared__ double red[4];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, pr = lane & 15, g4 = lane >> 4;
  // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous range of logical ids, ordered split-major, so the workgroups
  // sharing an L2 also share the rows of X they stream.
  const int nwg = gr.gx;
  const int xcd = gr.bx & 7, idx = gr.bx >> 3;
  const int per = nwg >> 3, rem = nwg & 7;
  const int lid = (xcd < rem) ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
  const int npb = nwg / g.nsplit;
  const int split = lid / npb;
  const int64_t p0 = (int64_t)(lid % npb) * BP;
  const int ntr = DYN ? g.nt : NT;                 // column tiles of this problem
  const int64_t c0 = (int64_t)gr.by * (DYN ? ntr * 16 : XC);
  const int64_t rb = (int64_t)split * g.rsplit;
  int64_t re = (rb + g.rsplit < g.R) ? rb + g.rsplit : g.R;
  if (g.kcap) {   // a rank known only on the device (uniform over the workgroup)
    const int64_t kc = *g.kcap;
    if (c0 >= kc - g.kc_col_off) return;
    if (g.kc_red_off >= 0 && re > kc - g.kc_red_off) re = kc - g.kc_red_off;
  }
  const bool do_ss = (g.sumsq_part != nullptr) && gr.by == 0;
  constexpr int epi = EPI;
  double ss = 0.0;

  f32x4 ra[AIT];
  f32x4 rx[XIT];
  f32x4 acc[RT][NT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  auto gload = [&](int64_t r) {
    if (MODE == 0) {
      constexpr int TPR = BK / 4;            // threads per A row
      constexpr int RPP = 256 / TPR;         // rows per pass
#pragma unroll
      for (int it = 0; it < AIT; ++it) {
        const int row = it * RPP + tid / TPR;
        const int col = (tid % TPR) * 4;
        const int64_t p = p0 + row;
        f32x4 v = {0.f, 0.f, 0.f, 0.f};
        if (p < g.P) {
          const int64_t srow = g.arow ? (int64_t)g.arow[p] : p;
          v = load4(g.A + srow * g.lda, r + col, re, g.avec);
        }
        ra[it] = v;
      }
    } else {
      constexpr int TPR = BP / 4;
      constexpr int RPP = 256 / TPR;
#pragma unroll
      for (int it = 0; it < AIT; ++it) {
        const int row = it * RPP + tid / TPR;
        const int col = (tid % TPR) * 4;
        const int64_t rr = r + row;
        f32x4 v = {0.f, 0.f, 0.f, 0.f};
        if (rr < re) v = load4(g.A + rr * g.lda, p0 + col, g.P, g.avec);
        ra[it] = v;
      }
    }
    if (do_ss) {
#pragma unroll
      for (int it = 0; it < AIT; ++it) {
        const double a0 = ra[it].x, a1 = ra[it].y, a2 = ra[it].z, a3 = ra[it].w;
        ss = fma(a0, a0, ss); ss = fma(a1, a1, ss); ss = fma(a2, a2, ss); ss = fma(a3, a3, ss);
      }
    }
#pragma unroll
    for (int it = 0; it < XIT; ++it) {
      const int idx = it * 256 + tid;
      f32x4 v = {0.f, 0.f, 0.f, 0.f};
      if (idx < XV) {
        const int row = idx / (NT * 4);
        const int col = (idx % (NT * 4)) * 4;
        const int64_t rr = r + row;
        if (rr < re) v = load4(g.X + rr * g.ldx, c0 + col, g.C, g.xvec);
      }
      rx[it] = v;
    }
  };

  auto sstore = [&]() {
#pragma unroll
    for (int it = 0; it < AIT; ++it) {
      if (MODE == 0) {
        constexpr int TPR = BK / 4, RPP = 256 / TPR;
        const int row = it * RPP + tid / TPR;
        const int col = (tid % TPR) * 4;
        *reinterpret_cast<f32x4*>(&As[row * AST_N + col]) = ra[it];
      } else {
        constexpr int TPR = BP / 4, RPP = 256 / TPR;
        const int row = it * RPP + tid / TPR;
        const int col = (tid % TPR) * 4;
        *reinterpret_cast<f32x4*>(&As[row * AST_T + col]) = ra[it];
      }
    }
#pragma unroll
    for (int it = 0; it < XIT; ++it) {
      const int idx = it * 256 + tid;
      if (idx < XV) {
        const int row = idx / (NT * 4);
        const int col = (idx % (NT * 4)) * 4;
        *reinterpret_cast<f32x4*>(&Xs[row * XST + col]) = rx[it];
      }
    }
  };

  auto compute = [&]() {
#pragma unroll
    for (int kk = 0; kk < BK / 16; ++kk) {
      if (MODE == 0) {
        f32x4 a[RT];
#pragma unroll
        for (int i = 0; i < RT; ++i)
          a[i] = *reinterpret_cast<const f32x4*>(
              &As[(wave * 16 * RT + i * 16 + pr) * AST_N + kk * 16 + g4 * 4]);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          float b[NT];
#pragma unroll
          for (int j = 0; j < NT; ++j) b[j] = Xs[(kk * 16 + g4 * 4 + s) * XST + j * 16 + pr];
#pragma unroll
          for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][s], b[j], acc[i][j], 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          float a[RT], b[NT];
#pragma unroll
          for (int i = 0; i < RT; ++i)
            a[i] = As[(kk * 16 + g4 * 4 + s) * AST_T + wave * 16 * RT + i * 16 + pr];
#pragma unroll
          for (int j = 0; j < NT; ++j) b[j] = Xs[(kk * 16 + g4 * 4 + s) * XST + j * 16 + pr];
#pragma unroll
          for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
      }
    }
  };

  if (rb < re) {
    gload(rb);
    for (int64_t r = rb; r < re; r += BK) {
      __syncthreads();
      sstore();
      // the next stage's loads go out before the barrier: its wait then
      // overlaps them too
      if (r + BK < re) gload(r + BK);
      __syncthreads();
      compute();
    }
  }

  // Epilogue: acc[i][j][e] is out[p][c] with p = p0 + 16 RT wave + 16 i + 4 g4 + e,
  // c = c0 + 16 j + pr (the 16x16 MFMA output layout).
  double rs = 0.0, as = 0.0;
#pragma unroll
  for (int i = 0; i < RT; ++i) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t p = p0 + wave * 16 * RT + i * 16 + g4 * 4 + e;
      if (p >= g.P) continue;
      bool rowok = true;
      if (epi == EPI_SUB && g.rowmask) rowok = g.rowmask[p] < 0;
      if (!rowok) continue;
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        if (DYN && j >= ntr) continue;
        const int64_t c = c0 + j * 16 + pr;
        if (c >= g.C) continue;
        const float v = acc[i][j][e];
        if (epi == EPI_STORE) {
          g.out[p * g.ldo + c] = v;
        } else if (epi == EPI_PART) {
          g.out[(int64_t)split * g.part_stride + p * g.ldo + c] = v;
        } else if (epi == EPI_SUB) {
          g.out[p * g.ldo + c] -= v;
        } else {
          // every entry of Aref is read by exactly one (p, c), so
          // ||Aref||_F^2 comes along
          const double a = (double)g.Aref[p * g.ldaref + c * g.aref_cs];
          const double d = a - (double)v;
          rs = fma(d, d, rs);
          as = fma(a, a, as);
        }
      }
    }
  }
  const int64_t wg = (int64_t)gr.by * gr.gx + gr.bx;
  if (g.sumsq_part != nullptr && gr.by == 0) {
    const double t = block_sum_double(ss, red);
    if (tid == 0) g.sumsq_part[gr.bx] = t;
  }
  if (epi == EPI_RESID) {
    const double t = block_sum_double(rs, red);
    if (tid == 0) g.resid_part[wg] = t;
    if (g.aref_sq_part) {
      const double ta = block_sum_double(as, red);
      if (tid == 0) g.aref_sq_part[wg] = ta;
    }
  }
}

// The direct passes (store or split partials) stage 16 of the reduced
// dimension per LDS step: fewer registers in flight per thread, so 4
// workgroups of 128 rows (or 6 of 64 rows) share a CU, and the waiting on
// the streamed tiles of one is covered by the multiplies of the others.  The
// summation order of each output element is that of 32 per step (two steps
// of 16 are the same MFMA sequence), so the bits do not change.
constexpr int PASS_BK_DIRECT = 16;

template <int EPI>
constexpr int pass_bk() { return (EPI == EPI_STORE || EPI == EPI_PART) ? PASS_BK_DIRECT : GEMM_BK; }

// The one-tile-per-wave variant (64 rows per workgroup): half the registers,
// so more workgroups share a CU; the autotuner tries it beside the default.
template <int MODE, int NT, int EPI>
__device__ void b_pass64(const GemmArgs& g, const Grid& gr) {
  pass_body<MODE, NT, EPI, 1, pass_bk<EPI>()>(g, gr);
}

template <int MODE, int NT, int EPI>
__device__ void b_pass(const GemmArgs& g, const Grid& gr) {
  pass_body<MODE, NT, EPI, GEMM_BP / 64, pass_bk<EPI>()>(g, gr);
}

// The grouped pass: either direction and up to 8 column tiles, read from the
// problem's arguments, so one launch serves every pass of a batch that has
// the same epilogue.  Its direct forms also stage 16 per step (3 waves per
// SIMD instead of 2).
template <int EPI>
__device__ void b_pass_any64(const GemmArgs& g, const Grid& gr) {
  if (g.mode == 0) pass_body<0, 8, EPI, 1, pass_bk<EPI>(), true>(g, gr);
  else pass_body<1, 8, EPI, 1, pass_bk<EPI>(), true>(g, gr);
}

template <int EPI>
__device__ void b_pass_any(const GemmArgs& g, const Grid& gr) {
  if (g.mode == 0) pass_body<0, 8, EPI, GEMM_BP / 64, pass_bk<EPI>(), true>(g, gr);
  else pass_body<1, 8, EPI, GEMM_BP / 64, pass_bk<EPI>(), true>(g, gr);
}

template <int MODE, int EPI>
hipError_t launch_nt64(int nt, dim3 grid, const GemmArgs& a, hipStream_t s) {
  if (thread_recorder()) {
    GemmArgs b = a;
    b.mode = MODE;
    b.nt = nt;
    return dispatch<GemmArgs, b_pass_any64<EPI>, 256, 2>(b, grid, 0, s);
  }
  switch (nt) {
#define PLU_NT_CASE(N) \
  case N: return dispatch<GemmArgs, b_pass64<MODE, N, EPI>, 256, 4>(a, grid, 0, s);
    PLU_NT_CASE(1) PLU_NT_CASE(2) PLU_NT_CASE(3) PLU_NT_CASE(4)
    PLU_NT_CASE(5) PLU_NT_CASE(6) PLU_NT_CASE(7) PLU_NT_CASE(8)
#undef PLU_NT_CASE
    default: return hipErrorInvalidValue;
  }
}

template <int MODE, int EPI>
hipError_t launch_nt(int nt, dim3 grid, const GemmArgs& a, hipStream_t s) {
  if (thread_recorder()) {
    // recorded launches use the grouped form so that every pass of a batch
    // can share one launch
    GemmArgs b = a;
    b.mode = MODE;
    b.nt = nt;
    return dispatch<GemmArgs, b_pass_any<EPI>, 256, 1>(b, grid, 0, s);
  }
  switch (nt) {
#define PLU_NT_CASE(N) \
  case N:                                                                         \
    return dispatch<GemmArgs, b_pass<MODE, N, EPI>, 256,                          \
                    (pass_bk<EPI>() == PASS_BK_DIRECT && N < 8) ? 4 : 2>(a, grid, 0, s);
    PLU_NT_CASE(1) PLU_NT_CASE(2) PLU_NT_CASE(3) PLU_NT_CASE(4)
    PLU_NT_CASE(5) PLU_NT_CASE(6) PLU_NT_CASE(7) PLU_NT_CASE(8)
#undef PLU_NT_CASE
    default: return hipErrorInvalidValue;
  }
}

// out = sum over splits of the partials (fixed order), one thread per 4
// consecutive columns of a row; optional per-column float64 sums of squares
// over each block of rows_per_block rows (deterministic: fixed order).
struct ReduceArgs {
  const float* part; int64_t pld, part_stride; int nsplit; float* out; int64_t ldo, P, C;
  double* colsq_part; int rb;
};

constexpr int RED_T = 1024;   // threads of the split-K reduction workgroup

__device__ void b_splitk_reduce(const ReduceArgs& ra, const Grid& gr) {
  // One workgroup per block of rb rows and 64 float4 column groups; each
  // thread sums its rows' partials over the splits in split order (up to
  // sixteen splits in flight), so the sums do not depend on the thread
  // layout.
  const float* __restrict__ part = ra.part;
  const int64_t pld = ra.pld;                      // row stride of the partials
  const int64_t part_stride = ra.part_stride;
  const int nsplit = ra.nsplit;
  float* out = ra.out;
  const int64_t ldo = ra.ldo, P = ra.P, C = ra.C;
  double* colsq_part = ra.colsq_part;
  const int rb = ra.rb;
  const int64_t c4n = (C + 3) / 4;                 // float4 groups per row
  const int lanes_per_row = (int)((c4n < 64) ? c4n : 64);
  const int rows_per_pass = RED_T / lanes_per_row;
  const int tid = threadIdx.x;
  const int rsub = tid / lanes_per_row, cl = tid % lanes_per_row;
  const int64_t pb = gr.bx;
  const int64_t pe = (pb * rb + rb < P) ? pb * rb + rb : P;
  const bool active = rsub < rows_per_pass;
  const int64_t cgi = (int64_t)gr.by * 64 + cl;   // this thread's float4 column group
  double cs[4] = {0.0, 0.0, 0.0, 0.0};
  if (active && cgi < c4n) {
    const int64_t c0 = cgi * 4;
    // whole float4 reads wherever they stay inside a row of the partials;
    // entries at columns >= C are read but not used
    const bool v4ok = ((reinterpret_cast<uintptr_t>(part) & 15u) == 0) && ((pld & 3) == 0) &&
                      ((part_stride & 3) == 0) && (c0 + 3 < pld);
    for (int64_t p = pb * rb + rsub; p < pe; p += rows_per_pass) {
      float s[4] = {0.f, 0.f, 0.f, 0.f};
      const float* src0 = part + p * pld + c0;
      if (v4ok) {
        int k = 0;
        for (; k + 16 <= nsplit; k += 16) {
          f32x4 v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u)
            v[u] = *reinterpret_cast<const f32x4*>(src0 + (int64_t)(k + u) * part_stride);
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            s[0] += v[u].x; s[1] += v[u].y; s[2] += v[u].z; s[3] += v[u].w;
          }
        }
        if (k + 8 <= nsplit) {
          f32x4 v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u)
            v[u] = *reinterpret_cast<const f32x4*>(src0 + (int64_t)(k + u) * part_stride);
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            s[0] += v[u].x; s[1] += v[u].y; s[2] += v[u].z; s[3] += v[u].w;
          }
          k += 8;
        }
        for (; k < nsplit; ++k) {
          const f32x4 v = *reinterpret_cast<const f32x4*>(src0 + (int64_t)k * part_stride);
          s[0] += v.x; s[1] += v.y; s[2] += v.z; s[3] += v.w;
        }
      } else {
        for (int k = 0; k < nsplit; ++k) {
          const float* src = src0 + (int64_t)k * part_stride;
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (c0 + e < C) s[e] += src[e];
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (c0 + e < C) {
          if (out) out[p * ldo + c0 + e] = s[e];
          const double d = s[e];
          cs[e] = fma(d, d, cs[e]);
        }
      }
    }
  }
  if (!colsq_part) return;
  // combine the rows_per_pass partial sums of each column group in a fixed order
  __shared__ double acc[RED_T][4];
#pragma unroll
  for (int e = 0; e < 4; ++e) acc[tid][e] = cs[e];
  __syncthreads();
  if (rsub == 0 && cgi < c4n) {
    double tsum[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = 0; r < rows_per_pass; ++r)
#pragma unroll
      for (int e = 0; e < 4; ++e) tsum[e] += acc[r * lanes_per_row + cl][e];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (cgi * 4 + e < C) colsq_part[pb * C + cgi * 4 + e] = tsum[e];
  }
}

struct SumArgs {
  const double* in; int64_t n; double* out;
};

__device__ void b_sum_doubles(const SumArgs& a, const Grid& gr) {
  (void)gr;
  const double* in = a.in;
  const int64_t n = a.n;
  double* out = a.out;
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += in[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

struct SumsqArgs {
  const float* A; int64_t lda, m, n; double* part;
};

__device__ void b_sumsq_matrix(const SumsqArgs& a, const Grid& gr) {
  const float* A = a.A;
  const int64_t lda = a.lda, m = a.m, n = a.n;
  double* part = a.part;
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = gr.bx; i < m; i += gr.gx) {
    const float* row = A + i * lda;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
      const double d = row[j];
      s = fma(d, d, s);
    }
  }
  const double t = block_sum_double(s, red);
  if (threadIdx.x == 0) part[gr.bx] = t;
}

}  // namespace

GemmPlan plan_gemm(int64_t P, int64_t R, int64_t C, int max_split, int slots, int kalign,
                   int bp) {
  // slots: workgroups the device runs at once.  The split of R is chosen so
  // that the grid fills whole rounds of slots (the last round nearly full),
  // with at least 256 of R per split.  bp: rows per workgroup (GEMM_BP, or
  // 64 for the one-tile-per-wave variant of the direct passes).
  GemmPlan pl;
  pl.bp = (bp == 64) ? 64 : BP;
  pl.pblocks = (int)((P + pl.bp - 1) / pl.bp);
  const int64_t cb = (C + 127) / 128;
  pl.cblocks = (int)cb;
  const int64_t cpb = (C + cb - 1) / cb;          // columns per block, balanced
  pl.nt = (int)((cpb + 15) / 16);
  if (pl.nt < 1) pl.nt = 1;
  const int64_t base = (int64_t)pl.pblocks * pl.cblocks;
  const int64_t max_by_depth = std::max<int64_t>(1, R / 256);
  const int64_t hi = std::max<int64_t>(1, std::min<int64_t>(max_split, max_by_depth));
  int64_t best_ns = 1;
  double best_eff = -1.0;
  for (int64_t ns = 1; ns <= hi; ++ns) {
    const int64_t tot = base * ns;
    const int64_t rounds = (tot + slots - 1) / slots;
    // efficiency of the last-round fill, discounted when the grid is tiny
    double eff = (double)tot / (double)(rounds * slots);
    if (tot < slots) eff = (double)tot / (double)slots;
    if (eff > best_eff + 0.02) {
      best_eff = eff;
      best_ns = ns;
    }
  }
  int64_t rs = (R + best_ns - 1) / best_ns;
  rs = ((rs + kalign - 1) / kalign) * kalign;
  int64_t ns = (R + rs - 1) / rs;
  if (ns < 1) ns = 1;
  pl.nsplit = (int)ns;
  pl.rsplit = rs > 0 ? rs : kalign;
  return pl;
}

hipError_t launch_gemm(int mode, int epi, int bf16, const GemmArgs& a, const GemmPlan& pl,
                       hipStream_t s) {
  if (bf16) return hipErrorInvalidValue;
  GemmArgs g = a;
  g.avec = ((reinterpret_cast<uintptr_t>(g.A) & 15u) == 0 && (g.lda & 3) == 0) ? 1 : 0;
  g.xvec = ((reinterpret_cast<uintptr_t>(g.X) & 15u) == 0 && (g.ldx & 3) == 0) ? 1 : 0;
  g.nsplit = pl.nsplit;
  g.rsplit = pl.rsplit;
  // column blocks of nt*16 columns each
  dim3 grid(pl.pblocks * pl.nsplit, pl.cblocks);
  if ((int64_t)pl.cblocks * pl.nt * 16 < g.C) return hipErrorInvalidValue;
  if (pl.bp == 64) {
    // planned for the one-tile-per-wave kernels: the direct passes only
    if (epi != EPI_STORE && epi != EPI_PART) return hipErrorInvalidValue;
    if (mode == 0)
      return epi == EPI_STORE ? launch_nt64<0, EPI_STORE>(pl.nt, grid, g, s)
                              : launch_nt64<0, EPI_PART>(pl.nt, grid, g, s);
    return epi == EPI_STORE ? launch_nt64<1, EPI_STORE>(pl.nt, grid, g, s)
                            : launch_nt64<1, EPI_PART>(pl.nt, grid, g, s);
  }
  if (mode == 0) {
    switch (epi) {
      case EPI_STORE: return launch_nt<0, EPI_STORE>(pl.nt, grid, g, s);
      case EPI_PART: return launch_nt<0, EPI_PART>(pl.nt, grid, g, s);
      case EPI_SUB: return launch_nt<0, EPI_SUB>(pl.nt, grid, g, s);
      case EPI_RESID: return launch_nt<0, EPI_RESID>(pl.nt, grid, g, s);
    }
  } else {
    switch (epi) {
      case EPI_STORE: return launch_nt<1, EPI_STORE>(pl.nt, grid, g, s);
      case EPI_PART: return launch_nt<1, EPI_PART>(pl.nt, grid, g, s);
      case EPI_SUB: return launch_nt<1, EPI_SUB>(pl.nt, grid, g, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_splitk_reduce_ld(const float* part, int64_t pld, int64_t part_stride,
                                   int nsplit, float* out, int64_t ldo, int64_t P, int64_t C,
                                   double* colsq_part, int rows_per_block, hipStream_t s) {
  if (pld < C || (nsplit > 1 && part_stride < P * pld)) return hipErrorInvalidValue;
  dim3 grid((unsigned)((P + rows_per_block - 1) / rows_per_block),
            (unsigned)(((C + 3) / 4 + 63) / 64));
  return dispatch<ReduceArgs, b_splitk_reduce, RED_T>(
      ReduceArgs{part, pld, part_stride, nsplit, out, ldo, P, C, colsq_part, rows_per_block},
      grid, 0, s);
}

hipError_t launch_splitk_reduce(const float* part, int64_t part_stride, int nsplit, float* out,
                                int64_t ldo, int64_t P, int64_t C, double* colsq_part,
                                int rows_per_block, hipStream_t s) {
  return launch_splitk_reduce_ld(part, ldo, part_stride, nsplit, out, ldo, P, C, colsq_part,
                                 rows_per_block, s);
}

hipError_t launch_sum_doubles(const double* in, int64_t n, double* out, hipStream_t s) {
  return dispatch<SumArgs, b_sum_doubles, 256>(SumArgs{in, n, out}, dim3(1), 0, s);
}

hipError_t launch_sumsq_matrix(const float* A, int64_t lda, int64_t m, int64_t n, double* part,
                               int nblocks, hipStream_t s) {
  return dispatch<SumsqArgs, b_sumsq_matrix, 256>(SumsqArgs{A, lda, m, n, part}, dim3(nblocks),
                                                  0, s);
}

}  // namespace plu
