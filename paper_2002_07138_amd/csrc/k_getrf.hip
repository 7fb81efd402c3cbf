// Tall-skinny LU with partial pivoting: the paper's lu(.) applied to the
// m x l (or n x l) iterates of Alg. 7 and to Y and B^T in Alg. 5 steps 4/6.
//
// Design (gfx950):
//  * Rows never move.  Row i keeps its storage; a pivoted row is marked with
//    the step that chose it (piv_step[i]) and holds its U row, every other row
//    holds its multipliers.  LAPACK's "current position" of each row is
//    tracked (pos[i]) so that exact ties are broken exactly as getrf does
//    (first maximum in the current row order).  The final factor in this
//    storage is V = P^T L -- the form Alg. 6/7 ask for -- so no gather is
//    needed between power passes.
//  * A panel of up to NB = 64 columns is factored by one cooperative grid.
//    Each wave owns 64*RPT rows whose panel entries live in VGPRs (RPT x NB
//    floats per lane).  Each pivot step costs one all-to-all exchange: every
//    wave publishes its best candidate (value, row, position, runner-up) and,
//    a little later, that candidate row's trailing entries; every wave polls
//    all headers, picks the same winner, reads the winner's row and updates
//    its own rows.  Message words are 64-bit {payload, tag} pairs written and
//    read with agent-scope atomics; the tag names the step, so no fences or
//    resets are needed between steps.  Every wait is bounded by a wall-clock
//    limit; on expiry the grid raises a flag and all waves exit.
//  * Wider matrices are factored panel by panel (right-looking): a small
//    triangular solve forms U12 for the panel's pivot rows and an MFMA pass
//    applies the rank-NB update to the rows that are still unpivoted.
#include "plu_internal.h"

#include <climits>
#include <type_traits>
#include <utility>

namespace plu {

namespace {

constexpr int MSGH = 4;   // header words per message

struct PanelArgs {
  float* F;
  int64_t ldf;
  int64_t M;
  int jb;
  int nbw;
  int32_t* piv_step;
  int32_t* pos;
  int32_t* piv_row;
  float* gaps;
  int32_t* zstep;           // first zero-pivot step (atomic min)
  int32_t* abortf;          // raised on timeout; every wait gives up once it is set
  unsigned long long* msg;
  uint32_t tagbase;
  int nwaves;
  int msgw;                 // words per message = MSGH + NB
  uint64_t timeout_ticks;
};

__device__ __forceinline__ void st_word(unsigned long long* p, uint32_t payload, uint32_t tag) {
  const unsigned long long w = ((unsigned long long)tag << 32) | (unsigned long long)payload;
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long ld_word(unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until *p carries `tag`; returns false on timeout or abort.
__device__ __forceinline__ bool wait_word(unsigned long long* p, uint32_t tag, uint32_t& payload,
                                          int32_t* abortf, uint64_t t0, uint64_t limit) {
  int it = 0;
  while (true) {
    const unsigned long long w = ld_word(p);
    if ((uint32_t)(w >> 32) == tag) {
      payload = (uint32_t)w;
      return true;
    }
    if ((++it & 127) == 0) {
      if (wall_clock64() - t0 > limit) {
        __hip_atomic_store(abortf, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
      if (__hip_atomic_load(abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
        return false;
    }
  }
}

// Candidate ordering key: larger |value| first, then smaller position.
// key 0 means "no candidate".
__device__ __forceinline__ unsigned long long cand_key(float a, int pos) {
  return ((unsigned long long)__float_as_uint(a) << 32) |
         (unsigned long long)(0xFFFFFFFFu - (uint32_t)pos);
}

struct Cand {
  unsigned long long key;
  int row;        // -1 if none
  float sv;       // signed value
  int src;        // publishing wave (global winner search) or q (local search)
  float sec;      // runner-up |value| among merged candidates, -1 if none
};

__device__ __forceinline__ float key_abs(unsigned long long key) {
  return key == 0ull ? -1.f : __uint_as_float((uint32_t)(key >> 32));
}

__device__ __forceinline__ void merge(Cand& x, const Cand& y) {
  if (y.key > x.key) {
    const float la = key_abs(x.key);
    float s = y.sec > la ? y.sec : la;
    s = s > x.sec ? s : x.sec;
    x.key = y.key; x.row = y.row; x.sv = y.sv; x.src = y.src; x.sec = s;
  } else {
    const float la = key_abs(y.key);
    float s = x.sec > la ? x.sec : la;
    s = s > y.sec ? s : y.sec;
    x.sec = s;
  }
}

__device__ __forceinline__ Cand wave_reduce(Cand c) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    Cand y;
    y.key = __shfl_xor(c.key, o, 64);
    y.row = __shfl_xor(c.row, o, 64);
    y.sv = __shfl_xor(c.sv, o, 64);
    y.src = __shfl_xor(c.src, o, 64);
    y.sec = __shfl_xor(c.sec, o, 64);
    merge(c, y);
  }
  return c;
}

template <int NB, int RPT>
__global__ __launch_bounds__(256) void k_getrf_panel(PanelArgs a) {
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint64_t t0 = wall_clock64();

  float x[RPT][NB];
  bool act[RPT], live0[RPT];
  int rpos[RPT], pstep[RPT];
  int rowid[RPT];

#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t r = ((int64_t)gw * RPT + q) * 64 + lane;
    rowid[q] = (int)r;
    act[q] = false;
    rpos[q] = INT_MAX;
    pstep[q] = -1;
#pragma unroll
    for (int jj = 0; jj < NB; ++jj) x[q][jj] = 0.f;
    if (r < a.M) {
      act[q] = a.piv_step[r] < 0;
      rpos[q] = a.pos[r];
      if (act[q]) {
        const float* src = a.F + r * a.ldf + a.jb;
        const bool vec = (reinterpret_cast<uintptr_t>(src) & 15u) == 0;
#pragma unroll
        for (int jj = 0; jj < NB; jj += 4) {
          if (vec && jj + 3 < a.nbw) {
            const f32x4 v = *reinterpret_cast<const f32x4*>(src + jj);
            x[q][jj] = v.x; x[q][jj + 1] = v.y; x[q][jj + 2] = v.z; x[q][jj + 3] = v.w;
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (jj + e < a.nbw) x[q][jj + e] = src[jj + e];
          }
        }
      }
    }
    live0[q] = act[q];
  }

  auto slot = [&](int J, int w) __attribute__((always_inline)) -> unsigned long long* {
    return a.msg + ((size_t)(J & 1) * a.nwaves + w) * a.msgw;
  };

  // Local best over this wave's rows for column j (compile-time j).
  auto local_cand = [&](auto jc) __attribute__((always_inline)) -> Cand {
    constexpr int j = decltype(jc)::value;
    Cand c{0ull, -1, 0.f, -1, -1.f};
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (act[q]) {
        Cand y{cand_key(fabsf(x[q][j]), rpos[q]), rowid[q], x[q][j], q, -1.f};
        merge(c, y);
      }
    }
    return c;
  };

  bool ok = true;
  // Publishes the header of this wave's candidate for step J and returns the
  // wave-level winner (for the later data publication).
  auto publish_header = [&](const Cand& wb, int J) __attribute__((always_inline)) {
    const uint32_t tag = a.tagbase + (uint32_t)J + 1u;
    unsigned long long* s = slot(J, gw);
    if (lane < MSGH) {
      uint32_t payload = 0;
      if (lane == 0) payload = __float_as_uint(wb.sv);
      if (lane == 1) payload = (uint32_t)wb.row;
      if (lane == 2) payload = 0xFFFFFFFFu - (uint32_t)wb.key;   // candidate's position
      if (lane == 3) payload = __float_as_uint(wb.sec);
      st_word(s + lane, payload, tag);
    }
  };

  // Publishes the trailing entries (columns > j) of the wave's candidate row.
  auto publish_data = [&](auto jc, const Cand& wb, int J) __attribute__((always_inline)) {
    constexpr int j = decltype(jc)::value;
    const uint32_t tag = a.tagbase + (uint32_t)J + 1u;
    unsigned long long* s = slot(J, gw) + MSGH;
    const int owner = wb.row >= 0 ? (int)(wb.row - (((int64_t)gw * RPT + wb.src) * 64)) : 0;
    const int qsel = wb.row >= 0 ? wb.src : 0;
    float mine = 0.f;
#pragma unroll
    for (int jj = j + 1; jj < NB; ++jj) {
      float t = x[0][jj];
#pragma unroll
      for (int q = 1; q < RPT; ++q) t = (qsel == q) ? x[q][jj] : t;
      const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t), owner));
      mine = (lane == jj) ? v : mine;
    }
    if (lane > j && lane < NB) st_word(s + lane, __float_as_uint(mine), tag);
  };

  // step 0 candidate
  {
    Cand wb = wave_reduce(local_cand(std::integral_constant<int, 0>{}));
    publish_header(wb, a.jb);
    publish_data(std::integral_constant<int, 0>{}, wb, a.jb);
  }

  auto step = [&](auto jc) __attribute__((always_inline)) {
    constexpr int j = decltype(jc)::value;
    if (!ok || j >= a.nbw) return;
    const int J = a.jb + j;
    const uint32_t tag = a.tagbase + (uint32_t)J + 1u;
    // ---- gather every wave's candidate header and agree on the winner
    Cand best{0ull, -1, 0.f, -1, -1.f};
    for (int w = lane; w < a.nwaves; w += 64) {
      unsigned long long* s = slot(J, w);
      uint32_t h0, h1, h2, h3;
      if (!wait_word(s + 0, tag, h0, a.abortf, t0, a.timeout_ticks) ||
          !wait_word(s + 1, tag, h1, a.abortf, t0, a.timeout_ticks) ||
          !wait_word(s + 2, tag, h2, a.abortf, t0, a.timeout_ticks) ||
          !wait_word(s + 3, tag, h3, a.abortf, t0, a.timeout_ticks)) {
        ok = false;
        break;
      }
      const int row = (int)h1;
      if (row >= 0) {
        const float sv = __uint_as_float(h0);
        Cand y{cand_key(fabsf(sv), (int)h2), row, sv, w, __uint_as_float(h3)};
        merge(best, y);
      }
    }
    ok = __all(ok);
    if (!ok) return;
    best = wave_reduce(best);
    // ---- the winner's trailing entries: lane jj (j < jj < NB) holds u[jj]
    float uv = 0.f;
    bool dok = true;
    if (lane > j && lane < NB && best.row >= 0) {
      uint32_t w;
      dok = wait_word(slot(J, best.src) + MSGH + lane, tag, w, a.abortf, t0, a.timeout_ticks);
      uv = __uint_as_float(w);
    }
    ok = __all(dok);
    if (!ok) return;
    const float piv = best.sv;
    const float aw = key_abs(best.key);
    const int wpos = (int)(0xFFFFFFFFu - (uint32_t)best.key);
    if (gw == 0 && lane == 0) {
      a.piv_row[J] = best.row;
      const float sec = best.sec > 0.f ? best.sec : 0.f;
      a.gaps[J] = aw > 0.f ? (aw - sec) / aw : 0.f;
      if (!(aw > 0.f)) atomicMin(a.zstep, J);
    }
    const float rinv = (piv != 0.f) ? 1.0f / piv : 0.f;
    // ---- bookkeeping and multipliers; update column j+1 first
    float lmul[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      lmul[q] = 0.f;
      if (act[q]) {
        if (rowid[q] == best.row) {
          act[q] = false;
          pstep[q] = J;
          rpos[q] = J;
        } else {
          if (rpos[q] == J) rpos[q] = wpos;
          const float l = (piv != 0.f) ? x[q][j] * rinv : x[q][j];
          x[q][j] = l;
          lmul[q] = l;
        }
      }
    }
    if constexpr (j + 1 < NB) {
      const float u1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(uv), j + 1));
#pragma unroll
      for (int q = 0; q < RPT; ++q)
        if (act[q]) x[q][j + 1] = fmaf(-lmul[q], u1, x[q][j + 1]);
      // ---- next step's candidate header goes out before the rest of the update
      Cand wb{0ull, -1, 0.f, -1, -1.f};
      const bool more = (j + 1 < a.nbw);
      if (more) {
        wb = wave_reduce(local_cand(std::integral_constant<int, j + 1>{}));
        publish_header(wb, J + 1);
      }
#pragma unroll
      for (int jj = j + 2; jj < NB; ++jj) {
        const float u = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(uv), jj));
#pragma unroll
        for (int q = 0; q < RPT; ++q)
          if (act[q]) x[q][jj] = fmaf(-lmul[q], u, x[q][jj]);
      }
      if (more) publish_data(std::integral_constant<int, j + 1>{}, wb, J + 1);
    }
  };

  [&]<int... Js>(std::integer_sequence<int, Js...>) __attribute__((always_inline)) {
    (step(std::integral_constant<int, Js>{}), ...);
  }(std::make_integer_sequence<int, NB>{});

  if (!ok) return;
  // ---- write back this panel's columns and the row bookkeeping
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t r = rowid[q];
    if (r < a.M && live0[q]) {
      float* dst = a.F + r * a.ldf + a.jb;
#pragma unroll
      for (int jj = 0; jj < NB; ++jj)
        if (jj < a.nbw) dst[jj] = x[q][jj];
      a.pos[r] = rpos[q];
      if (pstep[q] >= 0) a.piv_step[r] = pstep[q];
    }
  }
}

struct TrsmArgs {
  float* F;
  int64_t ldf;
  int jb, nbw, c;
  const int32_t* piv_row;
  float* u12;
  int64_t ldu12;
};

// U12 = L11^{-1} F[pivot rows of the panel, right columns]; written back into
// the pivot rows and into a compact nbw x (c - jb - nbw) buffer.
__global__ __launch_bounds__(64) void k_getrf_trsm(TrsmArgs a) {
  __shared__ float L11[64][65];
  __shared__ float us[64][65];
  __shared__ int rows[64];
  const int t = threadIdx.x;
  if (t < a.nbw) rows[t] = a.piv_row[a.jb + t];
  __syncthreads();
  for (int s = 0; s < a.nbw; ++s) {
    L11[s][t] = (t < s) ? a.F[(int64_t)rows[s] * a.ldf + a.jb + t] : 0.f;
  }
  __syncthreads();
  const int cs = a.jb + a.nbw;
  const int64_t cc = (int64_t)cs + (int64_t)blockIdx.x * 64 + t;
  if (cc >= a.c) return;
  for (int s = 0; s < a.nbw; ++s) {
    float v = a.F[(int64_t)rows[s] * a.ldf + cc];
    for (int k = 0; k < s; ++k) v = fmaf(-L11[s][k], us[k][t], v);
    us[s][t] = v;
    a.F[(int64_t)rows[s] * a.ldf + cc] = v;
    a.u12[(int64_t)s * a.ldu12 + (cc - cs)] = v;
  }
}

__global__ __launch_bounds__(256) void k_getrf_init(int32_t* piv_step, int32_t* pos, int64_t M,
                                                   int32_t* zstep) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < M) {
    piv_step[i] = -1;
    pos[i] = (int32_t)i;
  }
  if (i == 0) *zstep = INT_MAX;
}

// Turns the in-place factor into V = P^T L (unit diagonal on each pivot row,
// zeros to its right), extracts U (or U^T) and the row order perm.
__global__ __launch_bounds__(256) void k_getrf_finalize(float* F, int64_t ldf, int64_t M, int c,
                                                       const int32_t* piv_step, const int32_t* pos,
                                                       int32_t* perm, float* Uout, int64_t ldu,
                                                       int utrans) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= M * (int64_t)c) return;
  const int64_t i = e / c;
  const int t = (int)(e - i * c);
  const int s = piv_step[i];
  float* f = F + i * ldf + t;
  if (s >= 0) {
    const float v = *f;
    if (t >= s) {
      if (Uout) {
        if (utrans) Uout[(int64_t)t * ldu + s] = v;
        else Uout[(int64_t)s * ldu + t] = v;
      }
      *f = (t == s) ? 1.f : 0.f;
    } else if (Uout) {
      if (utrans) Uout[(int64_t)t * ldu + s] = 0.f;
      else Uout[(int64_t)s * ldu + t] = 0.f;
    }
  }
  if (t == 0 && perm) perm[pos[i]] = (int32_t)i;
}

template <int NB, int RPT>
hipError_t launch_panel(const PanelArgs& pa, int nblocks, hipStream_t s) {
  void* args[] = {const_cast<PanelArgs*>(&pa)};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_getrf_panel<NB, RPT>),
                                    dim3(nblocks), dim3(256), args, 0, s);
}

}  // namespace

size_t getrf_msg_words(int64_t M) {
  // worst case: RPT = 1 rows per lane -> one wave per 64 rows, rounded to 4 waves
  const int64_t waves = ((M + 255) / 256) * 4;
  return (size_t)2 * waves * (MSGH + 64);
}

hipError_t getrf_run(float* F, int64_t ldf, int64_t M, int c, const GetrfWork& w, int32_t* perm,
                     float* Uout, int64_t ldu, int utrans, hipStream_t s) {
  if (c <= 0 || M < c) return hipErrorInvalidValue;
  hipError_t e;
  hipLaunchKernelGGL(k_getrf_init, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, w.piv_step,
                     w.pos, M, w.zstep);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  constexpr int NB = 64, RPT = 2;
  const int64_t waves = (M + 64 * RPT - 1) / (64 * RPT);
  const int nblocks = (int)((waves + 3) / 4);
  if ((int64_t)nblocks * 4 > w.max_waves) return hipErrorInvalidValue;
  const int nw = nblocks * 4;
  if ((size_t)2 * nw * (MSGH + NB) > w.msg_words) return hipErrorInvalidValue;
  for (int jb = 0; jb < c; jb += NB) {
    PanelArgs pa;
    pa.F = F; pa.ldf = ldf; pa.M = M; pa.jb = jb; pa.nbw = (c - jb < NB) ? c - jb : NB;
    pa.piv_step = w.piv_step; pa.pos = w.pos; pa.piv_row = w.piv_row; pa.gaps = w.gaps;
    pa.zstep = w.zstep; pa.abortf = w.abortf; pa.msg = w.msg;
    const uint32_t seq = (*w.tag_counter)++;
    if (seq % 500000u == 0u) {
      if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(w.msg), w.msg_words * 2, 0u, s)) !=
          hipSuccess)
        return e;
    }
    pa.tagbase = (seq % 500000u) * 8192u;
    pa.nwaves = nw;
    pa.msgw = MSGH + NB;
    pa.timeout_ticks = w.timeout_ticks;
    e = launch_panel<NB, RPT>(pa, nblocks, s);
    if (e != hipSuccess) return e;
    const int cs = jb + pa.nbw;
    if (cs < c) {
      TrsmArgs ta{F, ldf, jb, pa.nbw, c, w.piv_row, w.u12, w.ldu12};
      hipLaunchKernelGGL(k_getrf_trsm, dim3((unsigned)((c - cs + 63) / 64)), dim3(64), 0, s, ta);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      GemmArgs g;
      g.A = F + jb; g.lda = ldf;
      g.X = w.u12; g.ldx = w.ldu12;
      g.out = F + cs; g.ldo = ldf;
      g.P = M; g.R = pa.nbw; g.C = c - cs;
      g.rowmask = w.piv_step;
      GemmPlan pl = plan_gemm(M, pa.nbw, c - cs, 1, 1);
      if ((e = launch_gemm(0, EPI_SUB, 0, g, pl, s)) != hipSuccess) return e;
    }
  }
  const int64_t tot = M * (int64_t)c;
  hipLaunchKernelGGL(k_getrf_finalize, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, F,
                     ldf, M, c, w.piv_step, w.pos, perm, Uout, ldu, utrans);
  return hipGetLastError();
}

}  // namespace plu
