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
#include <cstdlib>
#include <type_traits>
#include <utility>

namespace plu {

namespace {

constexpr int MSGH = 8;   // header words per message slot (the look-ahead panel uses 5)

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
  const int32_t* run_if;    // the panel does nothing when it reads 0 (nullable)
  const int32_t* kcap;      // nullable: steps at or beyond column *kcap are not taken
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

__device__ __forceinline__ float key_abs(unsigned long long key) {
  return key == 0ull ? -1.f : __uint_as_float((uint32_t)(key >> 32));
}

// Wave-wide reductions: rotations inside each row of 16 lanes (DPP), then
// the two cross-row exchanges.
template <int R>
__device__ __forceinline__ uint32_t dpp_ror(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x120 + R, 0xF, 0xF, false);
}

__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}

template <int R>
__device__ __forceinline__ unsigned long long dpp_ror64(unsigned long long v) {
  const uint32_t lo = dpp_ror<R>((uint32_t)v), hi = dpp_ror<R>((uint32_t)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// The cross-row steps use gfx950's row swaps (VALU, no LDS round trip).  A
// value swapped with itself comes back as the pair (lower row's, upper row's)
// in every lane: rows 16 apart for the 16-lane swap, halves 32 apart for the
// 32-lane one.  Both entries of the pair go into the reduction, so the result
// covers the lane and its partner whatever the lane's side.
//
// Wave-wide top two in one pass: k becomes the largest key, s the largest
// |value| among all other candidates.  Each lane enters its key and its own
// runner-up |value| (-1 if none); a key that loses a comparison passes its
// |value| on to s.
__device__ __forceinline__ void top2_merge(unsigned long long& k, float& s, unsigned long long k2,
                                           float s2) {
  const unsigned long long lo = k < k2 ? k : k2;
  k = k < k2 ? k2 : k;
  s = fmaxf(fmaxf(s, s2), key_abs(lo));
}

template <int W>
__device__ __forceinline__ void xrow_top2(unsigned long long& k, float& s) {
  const uint32_t lo = (uint32_t)k, hi = (uint32_t)(k >> 32), su = __float_as_uint(s);
  const auto a = W == 16 ? __builtin_amdgcn_permlane16_swap(lo, lo, false, false)
                         : __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = W == 16 ? __builtin_amdgcn_permlane16_swap(hi, hi, false, false)
                         : __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const auto c = W == 16 ? __builtin_amdgcn_permlane16_swap(su, su, false, false)
                         : __builtin_amdgcn_permlane32_swap(su, su, false, false);
  k = ((unsigned long long)b[0] << 32) | a[0];
  s = __uint_as_float(c[0]);
  top2_merge(k, s, ((unsigned long long)b[1] << 32) | a[1], __uint_as_float(c[1]));
}

__device__ __forceinline__ void wave_top2(unsigned long long& k, float& s) {
  top2_merge(k, s, dpp_ror64<1>(k), __uint_as_float(dpp_ror<1>(__float_as_uint(s))));
  top2_merge(k, s, dpp_ror64<2>(k), __uint_as_float(dpp_ror<2>(__float_as_uint(s))));
  top2_merge(k, s, dpp_ror64<4>(k), __uint_as_float(dpp_ror<4>(__float_as_uint(s))));
  top2_merge(k, s, dpp_ror64<8>(k), __uint_as_float(dpp_ror<8>(__float_as_uint(s))));
  xrow_top2<16>(k, s);
  xrow_top2<32>(k, s);
}

// One cooperative grid factors a panel of up to NB columns.  A workgroup of
// NWAVE waves owns NWAVE*64*RPT consecutive rows; each lane keeps a window of
// NB panel columns of its RPT rows in VGPRs.  Steps are processed in groups
// of S (unrolled, so the window is indexed at compile time); after each
// group the window shifts left by S columns, which keeps the code small
// enough for the instruction cache.  Multipliers and the pivot row's U
// entries are stored to F as soon as they are final.
//
// Pivot step: (1) each wave finds its best candidate and runner-up (one
// top-two reduction of the 64-bit key |value|, position), the workgroup
// combines them in LDS; (2) the owner
// of the workgroup's candidate publishes one message: header (value, row,
// position, runner-up) and the candidate's window entries to the right of
// the pivot column; (3) the waves of every workgroup share the polling of all
// messages into LDS; (4) every wave picks the same winner and updates.
template <int NB, int RPT, int NWAVE, int S>
__device__ void b_panel(const PanelArgs& a, const Grid& gr) {
  if (a.run_if && *a.run_if == 0) return;   // uniform over the grid: every workgroup leaves
  // steps of this panel: all of its columns, or those below a device-side
  // column count (the same value in every workgroup)
  int nbw = a.nbw;
  if (a.kcap) {
    const int kc = *a.kcap - a.jb;
    if (kc <= 0) return;
    if (kc < nbw) nbw = kc;
  }
  constexpr int MAXG = 64;                 // message slots (workgroups) at most
  constexpr int kFirstPollSleep = 24;      // s_sleep units of 64 clocks: about 0.7 us
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int G = gr.gx;
  const int wg = gr.bx;
  const uint64_t t0 = wall_clock64();

  __shared__ unsigned long long wck[NWAVE];            // wave best keys
  __shared__ float wcs[NWAVE];                         // wave runner-up |value|
  __shared__ uint32_t hdr[MAXG][MSGH];                 // polled headers
  __shared__ __attribute__((aligned(16))) float dat[MAXG][NB];   // polled windows
  __shared__ __attribute__((aligned(16))) float rowbuf[NWAVE][NB];
  __shared__ int flag_abort;

  float x[RPT][NB];
  bool act[RPT];
  int rpos[RPT], pstep[RPT], rowid[RPT];
  const int64_t wave_base = ((int64_t)wg * NWAVE + wv) * RPT * 64;

#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t r = wave_base + q * 64 + lane;
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
          if (vec && jj + 3 < nbw) {
            const f32x4 v = *reinterpret_cast<const f32x4*>(src + jj);
            x[q][jj] = v.x; x[q][jj + 1] = v.y; x[q][jj + 2] = v.z; x[q][jj + 3] = v.w;
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (jj + e < nbw) x[q][jj + e] = src[jj + e];
          }
        }
      }
    }
  }
  const bool live_any = act[0] || (RPT > 1 && act[RPT - 1]);
  (void)live_any;
  bool live0[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) live0[q] = act[q];
  if (threadIdx.x == 0) flag_abort = 0;
  __syncthreads();

  auto slot = [&](int J, int g) __attribute__((always_inline)) -> unsigned long long* {
    return a.msg + ((size_t)(J & 1) * G + g) * a.msgw;
  };

  bool ok = true;
  uint32_t lmask[RPT];      // window columns of the current group that hold multipliers

  // one pivot step on window column s (compile time); jcur = window origin
  auto step = [&](auto sc, int jcur) __attribute__((always_inline)) {
    constexpr int s = decltype(sc)::value;
    const int j = jcur + s;
    const int J = a.jb + j;
    const uint32_t tag = a.tagbase + (uint32_t)J + 1u;
    // ---- (1) candidates
    unsigned long long mykey = 0ull;
    int myq = 0;
    float mysec = -1.f;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (act[q]) {
        const float av = fabsf(x[q][s]);
        const unsigned long long k = cand_key(av, rpos[q]);
        if (k > mykey) {
          mysec = fmaxf(mysec, key_abs(mykey));
          mykey = k;
          myq = q;
        } else {
          mysec = fmaxf(mysec, av);
        }
      }
    }
    unsigned long long wk = mykey;
    float wsec = mysec;
    wave_top2(wk, wsec);
    const unsigned long long bal = __ballot(wk != 0ull && mykey == wk);
    const int wl = bal ? (int)__ffsll((long long)bal) - 1 : 0;
    const int wq = __builtin_amdgcn_readlane(myq, wl);
    if (lane == 0) {
      wck[wv] = wk;
      wcs[wv] = wsec;
    }
    __syncthreads();
    unsigned long long bk = 0ull;
    int bw = 0;
#pragma unroll
    for (int v = 0; v < NWAVE; ++v) {
      const unsigned long long k = wck[v];
      if (k > bk) {
        bk = k;
        bw = v;
      }
    }
    float bsec = -1.f;
#pragma unroll
    for (int v = 0; v < NWAVE; ++v) bsec = fmaxf(bsec, (v == bw) ? wcs[v] : key_abs(wck[v]));
    // ---- (2) publish the workgroup's candidate: a message to every
    // workgroup, or, when the grid is one workgroup, straight into the LDS
    // copy the polling would fill
    const bool local = (G == 1);
    auto put_h = [&](uint32_t v) __attribute__((always_inline)) {
      if (local) hdr[0][lane] = v;
      else st_word(slot(J, wg) + lane, v, tag);
    };
    auto put_d = [&](uint32_t v) __attribute__((always_inline)) {
      if (local) dat[0][lane] = __uint_as_float(v);
      else st_word(slot(J, wg) + MSGH + lane, v, tag);
    };
    if (bk != 0ull && wv == bw) {
      if (lane == wl) {
#pragma unroll
        for (int jj = 0; jj < NB; jj += 4) {
          f32x4 v4;
          v4.x = x[0][jj]; v4.y = x[0][jj + 1]; v4.z = x[0][jj + 2]; v4.w = x[0][jj + 3];
#pragma unroll
          for (int q = 1; q < RPT; ++q) {
            if (wq == q) {
              v4.x = x[q][jj]; v4.y = x[q][jj + 1]; v4.z = x[q][jj + 2]; v4.w = x[q][jj + 3];
            }
          }
          *reinterpret_cast<f32x4*>(&rowbuf[wv][jj]) = v4;
        }
      }
      const float mine = rowbuf[wv][lane < NB ? lane : 0];
      if (lane > s && lane < NB) put_d(__float_as_uint(mine));
      if (lane < MSGH) {
        uint32_t pl = 0;
        if (lane == 0) pl = __float_as_uint(rowbuf[wv][s]);
        if (lane == 1) pl = (uint32_t)(wave_base + wq * 64 + wl);
        if (lane == 2) pl = 0xFFFFFFFFu - (uint32_t)bk;
        if (lane == 3) pl = __float_as_uint(bsec);
        put_h(pl);
      }
    } else if (bk == 0ull && wv == 0) {              // no candidate in this workgroup
      if (lane < MSGH) put_h(lane == 1 ? 0xFFFFFFFFu : 0u);
      if (lane > s && lane < NB) put_d(0u);
    }
    // ---- (3) poll the messages of workgroups wv, wv+NWAVE, ... into LDS;
    // all of a wave's slots are in flight together.  A poll costs one
    // round trip to memory (about 1 us across XCDs); the first one waits
    // about 0.7 us for the other workgroups' messages to land, so most
    // steps need one poll instead of two.
    if (!local) {
      __builtin_amdgcn_s_sleep(kFirstPollSleep);
      constexpr int TS = MAXG / NWAVE;
      uint32_t pend_h = 0, pend_d = 0;
#pragma unroll
      for (int t = 0; t < TS; ++t) {
        if (wv + NWAVE * t < G) {
          if (lane < MSGH) pend_h |= 1u << t;
          if (lane > s && lane < NB) pend_d |= 1u << t;
        }
      }
      int it = 0;
      while (true) {
        unsigned long long vh[TS], vd[TS];
#pragma unroll
        for (int t = 0; t < TS; ++t) {
          unsigned long long* sl = slot(J, wv + NWAVE * t);
          if (pend_h & (1u << t)) vh[t] = ld_word(sl + lane);
          if (pend_d & (1u << t)) vd[t] = ld_word(sl + MSGH + lane);
        }
#pragma unroll
        for (int t = 0; t < TS; ++t) {
          const int g = wv + NWAVE * t;
          if ((pend_h & (1u << t)) && (uint32_t)(vh[t] >> 32) == tag) {
            hdr[g][lane] = (uint32_t)vh[t];
            pend_h &= ~(1u << t);
          }
          if ((pend_d & (1u << t)) && (uint32_t)(vd[t] >> 32) == tag) {
            dat[g][lane] = __uint_as_float((uint32_t)vd[t]);
            pend_d &= ~(1u << t);
          }
        }
        if (__all((pend_h | pend_d) == 0u)) break;
        if ((++it & 63) == 0) {
          bool stop = false;
          if (wall_clock64() - t0 > a.timeout_ticks) {
            __hip_atomic_store(a.abortf, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            stop = true;
          } else if (__hip_atomic_load(a.abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            stop = true;
          }
          if (__any(stop)) {
            if (lane == 0) flag_abort = 1;
            break;
          }
        }
      }
    }
    __syncthreads();
    if (flag_abort) {
      ok = false;
      return;
    }
    // ---- (4) every wave agrees on the winner
    unsigned long long gkey = 0ull;
    float gabs = -1.f, gsec = -1.f;
    if (lane < G) {
      const int row = (int)hdr[lane][1];
      if (row >= 0) {
        gabs = fabsf(__uint_as_float(hdr[lane][0]));
        gkey = cand_key(gabs, (int)hdr[lane][2]);
        gsec = __uint_as_float(hdr[lane][3]);
      }
    }
    unsigned long long best = gkey;
    float runner = gsec;
    wave_top2(best, runner);
    const unsigned long long gb = __ballot(best != 0ull && gkey == best);
    const int gs = gb ? (int)__ffsll((long long)gb) - 1 : 0;
    const float piv = __uint_as_float(hdr[gs][0]);
    const int prow = (best != 0ull) ? (int)hdr[gs][1] : -1;
    const float aw = key_abs(best);
    const int wpos = (int)(0xFFFFFFFFu - (uint32_t)best);
    if (wg == 0 && wv == 0 && lane == 0) {
      a.piv_row[J] = prow;
      const float sec = runner > 0.f ? runner : 0.f;
      a.gaps[J] = aw > 0.f ? (aw - sec) / aw : 0.f;
      if (!(aw > 0.f)) atomicMin(a.zstep, J);
    }
    // the pivot row's U entries (its window was staged in rowbuf by its wave)
    if (prow >= wave_base && prow < wave_base + RPT * 64) {
      if (lane >= s && lane < NB && jcur + lane < nbw)
        a.F[(int64_t)prow * a.ldf + a.jb + jcur + lane] = rowbuf[wv][lane];
    }
    const float rinv = (piv != 0.f) ? 1.0f / piv : 0.f;
    float lm[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      lm[q] = 0.f;
      if (act[q]) {
        if (rowid[q] == prow) {
          act[q] = false;
          pstep[q] = J;
          rpos[q] = J;
        } else {
          if (rpos[q] == J) rpos[q] = wpos;
          const float l = (piv != 0.f) ? x[q][s] * rinv : x[q][s];
          x[q][s] = l;
          lm[q] = l;
          lmask[q] |= 1u << s;
        }
      }
    }
    const float* ug = &dat[gs][0];
#pragma unroll
    for (int j4 = (s + 1) / 4; j4 < NB / 4; ++j4) {
      const f32x4 u4 = *reinterpret_cast<const f32x4*>(ug + 4 * j4);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int jj = 4 * j4 + e;
        if (jj > s) {
#pragma unroll
          for (int q = 0; q < RPT; ++q)
            // rows no longer active have lm = 0; their window is not read again
            x[q][jj] = fmaf(-lm[q], u4[e], x[q][jj]);
        }
      }
    }
  };

  for (int jcur = 0; jcur < nbw; jcur += S) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) lmask[q] = 0u;
    [&]<int... Ss>(std::integer_sequence<int, Ss...>) __attribute__((always_inline)) {
      ((ok && jcur + Ss < nbw ? step(std::integral_constant<int, Ss>{}, jcur) : void()), ...);
    }(std::make_integer_sequence<int, S>{});
    if (!ok) break;
    // the group's multipliers, one store batch per row
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (lmask[q]) {
        float* dst = a.F + (int64_t)rowid[q] * a.ldf + a.jb + jcur;
        if (S == 4 && lmask[q] == 0xFu && (reinterpret_cast<uintptr_t>(dst) & 15u) == 0) {
          f32x4 v4;
          v4.x = x[q][0]; v4.y = x[q][1]; v4.z = x[q][2]; v4.w = x[q][3];
          *reinterpret_cast<f32x4*>(dst) = v4;
        } else {
#pragma unroll
          for (int e = 0; e < S; ++e)
            if (lmask[q] & (1u << e)) dst[e] = x[q][e];
        }
      }
    }
    // shift the window left by S columns
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
#pragma unroll
      for (int jj = 0; jj < NB - S; ++jj) x[q][jj] = x[q][jj + S];
#pragma unroll
      for (int jj = NB - S; jj < NB; ++jj) x[q][jj] = 0.f;
    }
  }

  if (!ok) return;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t r = rowid[q];
    if (r < a.M && live0[q]) {
      a.pos[r] = rpos[q];
      if (pstep[q] >= 0) a.piv_step[r] = pstep[q];
    }
  }
}

// The same panel with one step of look-ahead.  A step's critical path used to
// run: candidate, barrier, message, poll, barrier, agree, full rank-1 update
// -- and only then the next candidate.  Here the update of a step is split:
// once the winner of step J is agreed, every row first updates only column
// J+1, the next candidate is found and published at once, and the rest of
// step J's update runs while that message is in flight.  The candidate's
// message therefore carries its row *before* step J's update together with
// its multiplier l_r of step J; every receiver forms the pivot row of step
// J+1 as fma(-l_r, u_J, row) -- the very operation the owner would have
// applied -- so the factors are bit-identical to the plain panel's.  A
// message is written in the window coordinates of the step it serves (after
// the window shift when it crosses a group of S steps).  Header words: the
// candidate's |value| source value, its row, its position key, the runner-up
// |value|, and l_r.
template <int NB, int RPT, int NWAVE, int S, int SLP>
__device__ void b_panel_la(const PanelArgs& a, const Grid& gr) {
  if (a.run_if && *a.run_if == 0) return;   // uniform over the grid: every workgroup leaves
  int nbw = a.nbw;
  if (a.kcap) {
    const int kc = *a.kcap - a.jb;
    if (kc <= 0) return;
    if (kc < nbw) nbw = kc;
  }
  constexpr int MAXG = 64;                 // message slots (workgroups) at most
  constexpr int HW = 5;                    // header words used
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int G = gr.gx;
  const int wg = gr.bx;
  const uint64_t t0 = wall_clock64();

  __shared__ unsigned long long wck[NWAVE];            // wave best keys
  __shared__ float wcs[NWAVE];                         // wave runner-up |value|
  __shared__ uint32_t hdr[MAXG][HW];                   // polled headers
  __shared__ __attribute__((aligned(16))) float dat[MAXG][NB];   // polled windows
  __shared__ __attribute__((aligned(16))) float rowbuf[NWAVE][NB];
  __shared__ __attribute__((aligned(16))) float urow[NWAVE][NB];  // pivot row, per wave
  __shared__ int flag_abort;

  float x[RPT][NB];
  bool act[RPT];
  int rpos[RPT], pstep[RPT], rowid[RPT];
  const int64_t wave_base = ((int64_t)wg * NWAVE + wv) * RPT * 64;

#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t r = wave_base + q * 64 + lane;
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
          if (vec && jj + 3 < nbw) {
            const f32x4 v = *reinterpret_cast<const f32x4*>(src + jj);
            x[q][jj] = v.x; x[q][jj + 1] = v.y; x[q][jj + 2] = v.z; x[q][jj + 3] = v.w;
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (jj + e < nbw) x[q][jj + e] = src[jj + e];
          }
        }
      }
    }
  }
  bool live0[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) live0[q] = act[q];
  if (threadIdx.x == 0) flag_abort = 0;

  auto slot = [&](int J, int g) __attribute__((always_inline)) -> unsigned long long* {
    return a.msg + ((size_t)(J & 1) * G + g) * a.msgw;
  };
  const bool local = (G == 1);

  bool ok = true;
  uint32_t lmask[RPT];      // window columns of the current group that hold multipliers
  float lm[RPT];            // multipliers of the step just agreed
#pragma unroll
  for (int q = 0; q < RPT; ++q) lm[q] = 0.f;
  float uprev = 0.f;        // this lane's column of the last pivot row (window coordinates)

  // Candidate of step J on window column C (compile time) and its message,
  // written with data columns shifted left by SH (0, or S when step J is the
  // first of the next group).  Every wave takes part (one barrier).
  auto publish = [&](auto cc, auto shc, int J) __attribute__((always_inline)) {
    constexpr int C = decltype(cc)::value;
    constexpr int SH = decltype(shc)::value;
    constexpr int CN = C - SH;                       // the column in the message's coordinates
    const uint32_t tag = a.tagbase + (uint32_t)J + 1u;
    unsigned long long mykey = 0ull;
    int myq = 0;
    float mysec = -1.f, mylm = 0.f;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (act[q]) {
        const float av = fabsf(x[q][C]);
        const unsigned long long k = cand_key(av, rpos[q]);
        if (k > mykey) {
          mysec = fmaxf(mysec, key_abs(mykey));
          mykey = k;
          myq = q;
          mylm = lm[q];
        } else {
          mysec = fmaxf(mysec, av);
        }
      }
    }
    unsigned long long wk = mykey;
    float wsec = mysec;
    wave_top2(wk, wsec);
    const unsigned long long bal = __ballot(wk != 0ull && mykey == wk);
    const int wl = bal ? (int)__ffsll((long long)bal) - 1 : 0;
    const int wq = __builtin_amdgcn_readlane(myq, wl);
    const float wlm = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(mylm), wl));
    if (lane == 0) {
      wck[wv] = wk;
      wcs[wv] = wsec;
    }
    __syncthreads();
    unsigned long long bk = 0ull;
    int bw = 0;
#pragma unroll
    for (int v = 0; v < NWAVE; ++v) {
      const unsigned long long k = wck[v];
      if (k > bk) {
        bk = k;
        bw = v;
      }
    }
    float bsec = -1.f;
#pragma unroll
    for (int v = 0; v < NWAVE; ++v) bsec = fmaxf(bsec, (v == bw) ? wcs[v] : key_abs(wck[v]));
    auto put_h = [&](uint32_t v) __attribute__((always_inline)) {
      if (local) hdr[0][lane] = v;
      else st_word(slot(J, wg) + lane, v, tag);
    };
    auto put_d = [&](uint32_t v) __attribute__((always_inline)) {
      if (local) dat[0][lane] = __uint_as_float(v);
      else st_word(slot(J, wg) + MSGH + lane, v, tag);
    };
    if (bk != 0ull && wv == bw) {
      if (lane == wl) {
        // the row before this step's update, in the message's coordinates
#pragma unroll
        for (int jj = 0; jj < NB; jj += 4) {
          f32x4 v4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int q = 0; q < RPT; ++q) {
            if (wq == q) {
#pragma unroll
              for (int e = 0; e < 4; ++e)
                if (jj + e + SH < NB) v4[e] = x[q][jj + e + SH];
            }
          }
          *reinterpret_cast<f32x4*>(&rowbuf[wv][jj]) = v4;
        }
      }
      __builtin_amdgcn_wave_barrier();
      const float mine = rowbuf[wv][lane < NB ? lane : 0];
      if (lane > CN && lane < NB) put_d(__float_as_uint(mine));
      if (lane < HW) {
        uint32_t pl = 0;
        if (lane == 0) pl = __float_as_uint(rowbuf[wv][CN]);
        if (lane == 1) pl = (uint32_t)(wave_base + wq * 64 + wl);
        if (lane == 2) pl = 0xFFFFFFFFu - (uint32_t)bk;
        if (lane == 3) pl = __float_as_uint(bsec);
        if (lane == 4) pl = __float_as_uint(wlm);
        put_h(pl);
      }
    } else if (bk == 0ull && wv == 0) {              // no candidate in this workgroup
      if (lane < HW) put_h(lane == 1 ? 0xFFFFFFFFu : 0u);
      if (lane > CN && lane < NB) put_d(0u);
    }
  };

  // One pivot step on window column s (compile time); jcur = window origin.
  auto step = [&](auto sc, int jcur) __attribute__((always_inline)) {
    constexpr int s = decltype(sc)::value;
    const int j = jcur + s;
    const int J = a.jb + j;
    const uint32_t tag = a.tagbase + (uint32_t)J + 1u;
    // ---- poll the messages of step J (published a step earlier)
    if (!local) {
      if (SLP > 0) __builtin_amdgcn_s_sleep(SLP);
      constexpr int TS = MAXG / NWAVE;
      uint32_t pend_h = 0, pend_d = 0;
#pragma unroll
      for (int t = 0; t < TS; ++t) {
        if (wv + NWAVE * t < G) {
          if (lane < HW) pend_h |= 1u << t;
          if (lane > s && lane < NB) pend_d |= 1u << t;
        }
      }
      int it = 0;
      while (true) {
        unsigned long long vh[TS], vd[TS];
#pragma unroll
        for (int t = 0; t < TS; ++t) {
          unsigned long long* sl = slot(J, wv + NWAVE * t);
          if (pend_h & (1u << t)) vh[t] = ld_word(sl + lane);
          if (pend_d & (1u << t)) vd[t] = ld_word(sl + MSGH + lane);
        }
#pragma unroll
        for (int t = 0; t < TS; ++t) {
          const int g = wv + NWAVE * t;
          if ((pend_h & (1u << t)) && (uint32_t)(vh[t] >> 32) == tag) {
            hdr[g][lane] = (uint32_t)vh[t];
            pend_h &= ~(1u << t);
          }
          if ((pend_d & (1u << t)) && (uint32_t)(vd[t] >> 32) == tag) {
            dat[g][lane] = __uint_as_float((uint32_t)vd[t]);
            pend_d &= ~(1u << t);
          }
        }
        if (__all((pend_h | pend_d) == 0u)) break;
        if ((++it & 63) == 0) {
          bool stop = false;
          if (wall_clock64() - t0 > a.timeout_ticks) {
            __hip_atomic_store(a.abortf, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            stop = true;
          } else if (__hip_atomic_load(a.abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            stop = true;
          }
          if (__any(stop)) {
            if (lane == 0) flag_abort = 1;
            break;
          }
        }
      }
    }
    __syncthreads();
    if (flag_abort) {
      ok = false;
      return;
    }
    // ---- every wave agrees on the winner of step J
    unsigned long long gkey = 0ull;
    float gabs = -1.f, gsec = -1.f;
    if (lane < G) {
      const int row = (int)hdr[lane][1];
      if (row >= 0) {
        gabs = fabsf(__uint_as_float(hdr[lane][0]));
        gkey = cand_key(gabs, (int)hdr[lane][2]);
        gsec = __uint_as_float(hdr[lane][3]);
      }
    }
    unsigned long long best = gkey;
    float runner = gsec;
    wave_top2(best, runner);
    const unsigned long long gb = __ballot(best != 0ull && gkey == best);
    const int gs = gb ? (int)__ffsll((long long)gb) - 1 : 0;
    const float piv = __uint_as_float(hdr[gs][0]);
    const float lr = __uint_as_float(hdr[gs][4]);
    const int prow = (best != 0ull) ? (int)hdr[gs][1] : -1;
    const float aw = key_abs(best);
    const int wpos = (int)(0xFFFFFFFFu - (uint32_t)best);
    if (wg == 0 && wv == 0 && lane == 0) {
      a.piv_row[J] = prow;
      const float sec = runner > 0.f ? runner : 0.f;
      a.gaps[J] = aw > 0.f ? (aw - sec) / aw : 0.f;
      if (!(aw > 0.f)) atomicMin(a.zstep, J);
    }
    // the pivot row of step J: the winner's row brought through its own
    // update of the previous step
    float uc = 0.f;
    if (lane == s) uc = piv;
    else if (lane > s) uc = fmaf(-lr, uprev, dat[gs][lane]);
    uprev = uc;
    urow[wv][lane] = uc;
    __builtin_amdgcn_wave_barrier();
    if (prow >= wave_base && prow < wave_base + RPT * 64) {
      if (lane >= s && jcur + lane < nbw) a.F[(int64_t)prow * a.ldf + a.jb + jcur + lane] = uc;
    }
    const float rinv = (piv != 0.f) ? 1.0f / piv : 0.f;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      lm[q] = 0.f;
      if (act[q]) {
        if (rowid[q] == prow) {
          act[q] = false;
          pstep[q] = J;
          rpos[q] = J;
        } else {
          if (rpos[q] == J) rpos[q] = wpos;
          const float l = (piv != 0.f) ? x[q][s] * rinv : x[q][s];
          x[q][s] = l;
          lm[q] = l;
          lmask[q] |= 1u << s;
        }
      }
    }
    // column J+1 first, then the next step's candidate goes out, then the
    // rest of this step's update while its message travels
    if (s + 1 < NB) {
      const float u1 = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(uc), s + 1));
#pragma unroll
      for (int q = 0; q < RPT; ++q) x[q][s + 1] = fmaf(-lm[q], u1, x[q][s + 1]);
    }
    if (j + 1 < nbw) {
      if constexpr (s + 1 < S) publish(std::integral_constant<int, s + 1>{},
                                       std::integral_constant<int, 0>{}, J + 1);
      else publish(std::integral_constant<int, s + 1>{}, std::integral_constant<int, S>{}, J + 1);
    }
    const float* ug = &urow[wv][0];
#pragma unroll
    for (int j4 = (s + 2) / 4; j4 < NB / 4; ++j4) {
      const f32x4 u4 = *reinterpret_cast<const f32x4*>(ug + 4 * j4);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int jj = 4 * j4 + e;
        if (jj > s + 1) {
#pragma unroll
          for (int q = 0; q < RPT; ++q)
            // rows no longer active have lm = 0; their window is not read again
            x[q][jj] = fmaf(-lm[q], u4[e], x[q][jj]);
        }
      }
    }
  };

  // the first step's candidate, from the window as loaded
  __syncthreads();
  publish(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{}, a.jb);
  for (int jcur = 0; jcur < nbw; jcur += S) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) lmask[q] = 0u;
    [&]<int... Ss>(std::integer_sequence<int, Ss...>) __attribute__((always_inline)) {
      ((ok && jcur + Ss < nbw ? step(std::integral_constant<int, Ss>{}, jcur) : void()), ...);
    }(std::make_integer_sequence<int, S>{});
    if (!ok) break;
    // the group's multipliers, one store batch per row
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (lmask[q]) {
        float* dst = a.F + (int64_t)rowid[q] * a.ldf + a.jb + jcur;
        if (S == 4 && lmask[q] == 0xFu && (reinterpret_cast<uintptr_t>(dst) & 15u) == 0) {
          f32x4 v4;
          v4.x = x[q][0]; v4.y = x[q][1]; v4.z = x[q][2]; v4.w = x[q][3];
          *reinterpret_cast<f32x4*>(dst) = v4;
        } else {
#pragma unroll
          for (int e = 0; e < S; ++e)
            if (lmask[q] & (1u << e)) dst[e] = x[q][e];
        }
      }
    }
    // shift the window (and this lane's pivot-row column) left by S columns
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
#pragma unroll
      for (int jj = 0; jj < NB - S; ++jj) x[q][jj] = x[q][jj + S];
#pragma unroll
      for (int jj = NB - S; jj < NB; ++jj) x[q][jj] = 0.f;
    }
    {
      const float t = __shfl(uprev, (lane + S) & 63, 64);
      uprev = (lane + S < NB) ? t : 0.f;
    }
  }

  if (!ok) return;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t r = rowid[q];
    if (r < a.M && live0[q]) {
      a.pos[r] = rpos[q];
      if (pstep[q] >= 0) a.piv_step[r] = pstep[q];
    }
  }
}

// The look-ahead panel for grids of up to 16 workgroups: no barrier after
// the poll.  Every wave reads all headers itself (lane g: workgroup g's) and
// decides the winner on its own; the windows are still polled by one wave per
// workgroup into LDS, each flagged there with the step's tag, and a wave
// waits only for the winner's flag.  The LDS buffers are double-buffered by
// step parity, since a wave may now run a step ahead of the others.  Waves
// that give up a wait report it before the candidate barrier, where all of
// them decide together to stop.  With more workgroups the extra header reads
// cost more than the barrier they save (measured: 6.3 against 5.8 us per
// step at 40 workgroups, 5.3 against 5.4 at 10).
template <int NB, int RPT, int NWAVE, int S, int SLP>
__device__ void b_panel_lw(const PanelArgs& a, const Grid& gr) {
  if (a.run_if && *a.run_if == 0) return;   // uniform over the grid: every workgroup leaves
  int nbw = a.nbw;
  if (a.kcap) {
    const int kc = *a.kcap - a.jb;
    if (kc <= 0) return;
    if (kc < nbw) nbw = kc;
  }
  constexpr int MAXG = 64;                 // message slots (workgroups) at most
  constexpr int HW = 5;                    // header words used
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int G = gr.gx;
  const int wg = gr.bx;
  const uint64_t t0 = wall_clock64();

  // Double-buffered by step parity: a wave may run one step ahead of the
  // others (nothing but the candidate barrier holds the waves together)
  __shared__ unsigned long long wck[2][NWAVE];         // wave best keys
  __shared__ float wcs[2][NWAVE];                      // wave runner-up |value|
  __shared__ uint32_t hloc[2][HW];                     // header, one-workgroup grid
  __shared__ __attribute__((aligned(16))) float dat[2][MAXG][NB];   // polled windows
  __shared__ uint32_t dflag[2][MAXG];                  // tag of the step whose window is in dat
  __shared__ int wab[3][NWAVE];                        // a wave gave up waiting (per parity; final)
  __shared__ __attribute__((aligned(16))) float rowbuf[NWAVE][NB];
  __shared__ __attribute__((aligned(16))) float urow[NWAVE][NB];  // pivot row, per wave
  __shared__ int flag_abort;

  float x[RPT][NB];
  bool act[RPT];
  int rpos[RPT], pstep[RPT], rowid[RPT];
  const int64_t wave_base = ((int64_t)wg * NWAVE + wv) * RPT * 64;

#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t r = wave_base + q * 64 + lane;
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
          if (vec && jj + 3 < nbw) {
            const f32x4 v = *reinterpret_cast<const f32x4*>(src + jj);
            x[q][jj] = v.x; x[q][jj + 1] = v.y; x[q][jj + 2] = v.z; x[q][jj + 3] = v.w;
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (jj + e < nbw) x[q][jj + e] = src[jj + e];
          }
        }
      }
    }
  }
  bool live0[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) live0[q] = act[q];
  if (threadIdx.x == 0) flag_abort = 0;
  for (int t = threadIdx.x; t < 2 * MAXG; t += 64 * NWAVE) dflag[t / MAXG][t % MAXG] = 0u;

  auto slot = [&](int J, int g) __attribute__((always_inline)) -> unsigned long long* {
    return a.msg + ((size_t)(J & 1) * G + g) * a.msgw;
  };
  const bool local = (G == 1);

  bool ok = true;
  uint32_t lmask[RPT];      // window columns of the current group that hold multipliers
  float lm[RPT];            // multipliers of the step just agreed
#pragma unroll
  for (int q = 0; q < RPT; ++q) lm[q] = 0.f;
  float uprev = 0.f;        // this lane's column of the last pivot row (window coordinates)
  // this wave gave up a wait in the current step (timeout or an abort seen):
  // reported before the next barrier, where all waves decide together
  bool stop = false;

  // Candidate of step J on window column C (compile time) and its message,
  // written with data columns shifted left by SH (0, or S when step J is the
  // first of the next group).  Every wave takes part (one barrier).
  auto publish = [&](auto cc, auto shc, int J) __attribute__((always_inline)) {
    constexpr int C = decltype(cc)::value;
    constexpr int SH = decltype(shc)::value;
    constexpr int CN = C - SH;                       // the column in the message's coordinates
    const uint32_t tag = a.tagbase + (uint32_t)J + 1u;
    const int par = J & 1;
    unsigned long long mykey = 0ull;
    int myq = 0;
    float mysec = -1.f, mylm = 0.f;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (act[q]) {
        const float av = fabsf(x[q][C]);
        const unsigned long long k = cand_key(av, rpos[q]);
        if (k > mykey) {
          mysec = fmaxf(mysec, key_abs(mykey));
          mykey = k;
          myq = q;
          mylm = lm[q];
        } else {
          mysec = fmaxf(mysec, av);
        }
      }
    }
    unsigned long long wk = mykey;
    float wsec = mysec;
    wave_top2(wk, wsec);
    const unsigned long long bal = __ballot(wk != 0ull && mykey == wk);
    const int wl = bal ? (int)__ffsll((long long)bal) - 1 : 0;
    const int wq = __builtin_amdgcn_readlane(myq, wl);
    const float wlm = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(mylm), wl));
    if (lane == 0) {
      wck[par][wv] = wk;
      wcs[par][wv] = wsec;
      wab[par][wv] = stop ? 1 : 0;
    }
    __syncthreads();
    // a wave that gave up is seen by all of them here, from values written
    // before the barrier (the same decision in every wave)
    {
      int any = 0;
#pragma unroll
      for (int v = 0; v < NWAVE; ++v) any |= wab[par][v];
      if (any) {
        ok = false;
        return;
      }
    }
    unsigned long long bk = 0ull;
    int bw = 0;
#pragma unroll
    for (int v = 0; v < NWAVE; ++v) {
      const unsigned long long k = wck[par][v];
      if (k > bk) {
        bk = k;
        bw = v;
      }
    }
    float bsec = -1.f;
#pragma unroll
    for (int v = 0; v < NWAVE; ++v)
      bsec = fmaxf(bsec, (v == bw) ? wcs[par][v] : key_abs(wck[par][v]));
    auto put_h = [&](uint32_t v) __attribute__((always_inline)) {
      if (local) hloc[par][lane] = v;
      else st_word(slot(J, wg) + lane, v, tag);
    };
    auto put_d = [&](uint32_t v) __attribute__((always_inline)) {
      if (local) dat[par][0][lane] = __uint_as_float(v);
      else st_word(slot(J, wg) + MSGH + lane, v, tag);
    };
    if (bk != 0ull && wv == bw) {
      if (lane == wl) {
        // the row before this step's update, in the message's coordinates
#pragma unroll
        for (int jj = 0; jj < NB; jj += 4) {
          f32x4 v4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int q = 0; q < RPT; ++q) {
            if (wq == q) {
#pragma unroll
              for (int e = 0; e < 4; ++e)
                if (jj + e + SH < NB) v4[e] = x[q][jj + e + SH];
            }
          }
          *reinterpret_cast<f32x4*>(&rowbuf[wv][jj]) = v4;
        }
      }
      __builtin_amdgcn_wave_barrier();
      const float mine = rowbuf[wv][lane < NB ? lane : 0];
      if (lane > CN && lane < NB) put_d(__float_as_uint(mine));
      if (lane < HW) {
        uint32_t pl = 0;
        if (lane == 0) pl = __float_as_uint(rowbuf[wv][CN]);
        if (lane == 1) pl = (uint32_t)(wave_base + wq * 64 + wl);
        if (lane == 2) pl = 0xFFFFFFFFu - (uint32_t)bk;
        if (lane == 3) pl = __float_as_uint(bsec);
        if (lane == 4) pl = __float_as_uint(wlm);
        put_h(pl);
      }
      if (local) {
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) dflag[par][0] = tag;
      }
    } else if (bk == 0ull && wv == 0) {              // no candidate in this workgroup
      if (lane < HW) put_h(lane == 1 ? 0xFFFFFFFFu : 0u);
      if (lane > CN && lane < NB) put_d(0u);
      if (local) {
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) dflag[par][0] = tag;
      }
    }
  };

  // One pivot step on window column s (compile time); jcur = window origin.
  auto step = [&](auto sc, int jcur) __attribute__((always_inline)) {
    constexpr int s = decltype(sc)::value;
    const int j = jcur + s;
    const int J = a.jb + j;
    const uint32_t tag = a.tagbase + (uint32_t)J + 1u;
    const int par = J & 1;
    // ---- poll the messages of step J (published a step earlier): every
    // wave reads all headers itself (lane g: workgroup g's), and the windows
    // of its share of the workgroups into LDS, flagging each one there
    uint32_t hv[HW];
#pragma unroll
    for (int e = 0; e < HW; ++e) hv[e] = 0u;
    auto spin_ok = [&](int it) __attribute__((always_inline)) -> bool {
      // every 64th spin: the wall-clock bound, another workgroup's abort, or
      // another wave's (the caller then leaves its wait)
      if ((it & 63) != 0) return true;
      bool bad = false;
      if (wall_clock64() - t0 > a.timeout_ticks) {
        __hip_atomic_store(a.abortf, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bad = true;
      } else if (__hip_atomic_load(a.abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                 __hip_atomic_load(&flag_abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0) {
        bad = true;
      }
      return !__any(bad);
    };
    if (!local) {
      if (SLP > 0) __builtin_amdgcn_s_sleep(SLP);
      constexpr int TS = MAXG / NWAVE;
      uint32_t pend_d = 0;
#pragma unroll
      for (int t = 0; t < TS; ++t)
        if (wv + NWAVE * t < G && lane > s && lane < NB) pend_d |= 1u << t;
      bool hpend = lane < G;
      int it = 0;
      while (true) {
        unsigned long long wh[HW], vd[TS];
        unsigned long long* hs = slot(J, lane < G ? lane : 0);
        if (hpend) {
#pragma unroll
          for (int e = 0; e < HW; ++e) wh[e] = ld_word(hs + e);
        }
#pragma unroll
        for (int t = 0; t < TS; ++t) {
          unsigned long long* sl = slot(J, wv + NWAVE * t);
          if (pend_d & (1u << t)) vd[t] = ld_word(sl + MSGH + lane);
        }
        if (hpend) {
          bool all = true;
#pragma unroll
          for (int e = 0; e < HW; ++e) all = all && (uint32_t)(wh[e] >> 32) == tag;
          if (all) {
#pragma unroll
            for (int e = 0; e < HW; ++e) hv[e] = (uint32_t)wh[e];
            hpend = false;
          }
        }
#pragma unroll
        for (int t = 0; t < TS; ++t) {
          const int g = wv + NWAVE * t;
          if ((pend_d & (1u << t)) && (uint32_t)(vd[t] >> 32) == tag) {
            dat[par][g][lane] = __uint_as_float((uint32_t)vd[t]);
            pend_d &= ~(1u << t);
          }
        }
        if (__all(!hpend && pend_d == 0u)) break;
        if (!spin_ok(++it)) {
          stop = true;
          break;
        }
      }
      if (!stop) {
        // this wave's windows are in LDS: flag them for the other waves
        __builtin_amdgcn_wave_barrier();
        if (lane < TS && wv + NWAVE * lane < G) dflag[par][wv + NWAVE * lane] = tag;
      }
    }
    if (stop) {
      if (lane == 0) flag_abort = 1;
    }
    // ---- the local grid's header (one workgroup: straight from LDS)
    if (local && !stop) {
      int it = 0;
      while (__hip_atomic_load(&dflag[par][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != tag) {
        if (!spin_ok(++it)) {
          stop = true;
          break;
        }
      }
      if (lane == 0) {
#pragma unroll
        for (int e = 0; e < HW; ++e) hv[e] = hloc[par][e];
      }
    }
    // ---- every wave agrees on the winner of step J
    unsigned long long gkey = 0ull;
    float gabs = -1.f, gsec = -1.f;
    if (lane < G) {
      const int row = (int)hv[1];
      if (row >= 0) {
        gabs = fabsf(__uint_as_float(hv[0]));
        gkey = cand_key(gabs, (int)hv[2]);
        gsec = __uint_as_float(hv[3]);
      }
    }
    unsigned long long best = gkey;
    float runner = gsec;
    wave_top2(best, runner);
    const unsigned long long gb = __ballot(best != 0ull && gkey == best);
    const int gs = gb ? (int)__ffsll((long long)gb) - 1 : 0;
    const float piv = __uint_as_float(__builtin_amdgcn_readlane(hv[0], gs));
    const float lr = __uint_as_float(__builtin_amdgcn_readlane(hv[4], gs));
    const int prow = (best != 0ull) ? (int)__builtin_amdgcn_readlane(hv[1], gs) : -1;
    const float aw = key_abs(best);
    const int wpos = (int)(0xFFFFFFFFu - (uint32_t)best);
    // the winner's window: polled by wave gs % NWAVE of this workgroup
    if (!local && !stop) {
      int it = 0;
      while (__hip_atomic_load(&dflag[par][gs], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != tag) {
        if (!spin_ok(++it)) {
          stop = true;
          break;
        }
      }
      if (stop && lane == 0) flag_abort = 1;
    }
    if (wg == 0 && wv == 0 && lane == 0) {
      a.piv_row[J] = prow;
      const float sec = runner > 0.f ? runner : 0.f;
      a.gaps[J] = aw > 0.f ? (aw - sec) / aw : 0.f;
      if (!(aw > 0.f)) atomicMin(a.zstep, J);
    }
    // the pivot row of step J: the winner's row brought through its own
    // update of the previous step
    float uc = 0.f;
    if (lane == s) uc = piv;
    else if (lane > s) uc = fmaf(-lr, uprev, dat[par][gs][lane]);
    uprev = uc;
    urow[wv][lane] = uc;
    __builtin_amdgcn_wave_barrier();
    if (prow >= wave_base && prow < wave_base + RPT * 64) {
      if (lane >= s && jcur + lane < nbw) a.F[(int64_t)prow * a.ldf + a.jb + jcur + lane] = uc;
    }
    const float rinv = (piv != 0.f) ? 1.0f / piv : 0.f;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      lm[q] = 0.f;
      if (act[q]) {
        if (rowid[q] == prow) {
          act[q] = false;
          pstep[q] = J;
          rpos[q] = J;
        } else {
          if (rpos[q] == J) rpos[q] = wpos;
          const float l = (piv != 0.f) ? x[q][s] * rinv : x[q][s];
          x[q][s] = l;
          lm[q] = l;
          lmask[q] |= 1u << s;
        }
      }
    }
    // column J+1 first, then the next step's candidate goes out, then the
    // rest of this step's update while its message travels
    if (s + 1 < NB) {
      const float u1 = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(uc), s + 1));
#pragma unroll
      for (int q = 0; q < RPT; ++q) x[q][s + 1] = fmaf(-lm[q], u1, x[q][s + 1]);
    }
    if (j + 1 < nbw) {
      if constexpr (s + 1 < S) publish(std::integral_constant<int, s + 1>{},
                                       std::integral_constant<int, 0>{}, J + 1);
      else publish(std::integral_constant<int, s + 1>{}, std::integral_constant<int, S>{}, J + 1);
    }
    const float* ug = &urow[wv][0];
#pragma unroll
    for (int j4 = (s + 2) / 4; j4 < NB / 4; ++j4) {
      const f32x4 u4 = *reinterpret_cast<const f32x4*>(ug + 4 * j4);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int jj = 4 * j4 + e;
        if (jj > s + 1) {
#pragma unroll
          for (int q = 0; q < RPT; ++q)
            // rows no longer active have lm = 0; their window is not read again
            x[q][jj] = fmaf(-lm[q], u4[e], x[q][jj]);
        }
      }
    }
  };

  // the first step's candidate, from the window as loaded
  __syncthreads();
  publish(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{}, a.jb);
  for (int jcur = 0; jcur < nbw; jcur += S) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) lmask[q] = 0u;
    [&]<int... Ss>(std::integer_sequence<int, Ss...>) __attribute__((always_inline)) {
      ((ok && jcur + Ss < nbw ? step(std::integral_constant<int, Ss>{}, jcur) : void()), ...);
    }(std::make_integer_sequence<int, S>{});
    if (!ok) break;
    // the group's multipliers, one store batch per row
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (lmask[q]) {
        float* dst = a.F + (int64_t)rowid[q] * a.ldf + a.jb + jcur;
        if (S == 4 && lmask[q] == 0xFu && (reinterpret_cast<uintptr_t>(dst) & 15u) == 0) {
          f32x4 v4;
          v4.x = x[q][0]; v4.y = x[q][1]; v4.z = x[q][2]; v4.w = x[q][3];
          *reinterpret_cast<f32x4*>(dst) = v4;
        } else {
#pragma unroll
          for (int e = 0; e < S; ++e)
            if (lmask[q] & (1u << e)) dst[e] = x[q][e];
        }
      }
    }
    // shift the window (and this lane's pivot-row column) left by S columns
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
#pragma unroll
      for (int jj = 0; jj < NB - S; ++jj) x[q][jj] = x[q][jj + S];
#pragma unroll
      for (int jj = NB - S; jj < NB; ++jj) x[q][jj] = 0.f;
    }
    {
      const float t = __shfl(uprev, (lane + S) & 63, 64);
      uprev = (lane + S < NB) ? t : 0.f;
    }
  }

  if (lane == 0) wab[2][wv] = stop ? 1 : 0;
  __syncthreads();
  {
    int any = 0;
#pragma unroll
    for (int v = 0; v < NWAVE; ++v) any |= wab[2][v];
    if (!ok || any) return;
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t r = rowid[q];
    if (r < a.M && live0[q]) {
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
  const int32_t* run_if;
  const int32_t* kcap;      // nullable: columns at or beyond *kcap are not solved
};

// U12 = L11^{-1} F[pivot rows of the panel, right columns]; written back into
// the pivot rows and into a compact nbw x (c - jb - nbw) buffer.  One wave per
// right-hand column, lane r holding row r: at step s row s is final, its value
// is broadcast from lane s (readlane, no LDS round trip) and every lane
// subtracts its multiple, the next step's multiplier already loaded.  The
// strictly lower L11 is staged in LDS (zeros on and above the diagonal, so
// rows at or above s are left exactly as they are).  Each entry sees the same
// fmaf sequence as a left-looking substitution (its terms in ascending s).
__device__ void b_trsm(const TrsmArgs& a, const Grid& gr) {
  if (a.run_if && *a.run_if == 0) return;
  int c = a.c;
  if (a.kcap) {   // the panel stopped at column *kcap: nothing right of it is needed
    const int kc = *a.kcap;
    if (a.jb + a.nbw >= kc) return;
    if (kc < c) c = kc;
  }
  __shared__ float L11[64][65];
  __shared__ int rows[64];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int nbw = a.nbw;
  if (t < 64) rows[t] = t < nbw ? a.piv_row[a.jb + t] : 0;
  __syncthreads();
  {
    // every load issued before the first is waited for
    float lv[16];
#pragma unroll
    for (int it = 0; it < 16; ++it) {
      const int e = it * 256 + t, r = e >> 6, s = e & 63;
      lv[it] = (r < nbw && s < r) ? a.F[(int64_t)rows[r] * a.ldf + a.jb + s] : 0.f;
    }
#pragma unroll
    for (int it = 0; it < 16; ++it) {
      const int e = it * 256 + t;
      L11[e >> 6][e & 63] = lv[it];
    }
  }
  __syncthreads();
  const int cs = a.jb + nbw;
  const int64_t cc = (int64_t)cs + (int64_t)gr.bx * 4 + wave;
  if (cc >= c) return;   // uniform over the wave; no barrier follows
  float x = (lane < nbw) ? a.F[(int64_t)rows[lane] * a.ldf + cc] : 0.f;
  float lnext = L11[lane][0];
  for (int s = 0; s < nbw - 1; ++s) {
    const float lcur = lnext;
    lnext = L11[lane][s + 1];
    const float xs = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), s));
    x = fmaf(-lcur, xs, x);
  }
  if (lane < nbw) {
    a.F[(int64_t)rows[lane] * a.ldf + cc] = x;
    a.u12[(int64_t)lane * a.ldu12 + (cc - cs)] = x;
  }
}

struct InitArgs {
  int32_t* piv_step; int32_t* pos; int64_t M; int32_t* zstep; const int32_t* run_if;
};

__device__ void b_getrf_init(const InitArgs& a, const Grid& gr) {
  if (a.run_if && *a.run_if == 0) return;
  const int64_t i = (int64_t)gr.bx * 256 + threadIdx.x;
  if (i < a.M) {
    a.piv_step[i] = -1;
    a.pos[i] = (int32_t)i;
  }
  if (i == 0) *a.zstep = INT_MAX;
}

// Turns the in-place factor into V = P^T L (unit diagonal on each pivot row,
// zeros to its right), extracts U (or U^T) and the row order perm.
struct FinalizeArgs {
  float* F; int64_t ldf, M; int c; const int32_t* piv_step; const int32_t* pos; int32_t* perm;
  float* Uout; int64_t ldu; int utrans; const int32_t* run_if;
  const int32_t* kcap;      // nullable: U entries outside the leading *kcap square are zeros
};

__device__ void b_getrf_finalize(const FinalizeArgs& fa, const Grid& gr) {
  if (fa.run_if && *fa.run_if == 0) return;
  float* F = fa.F;
  const int64_t ldf = fa.ldf, M = fa.M;
  const int c = fa.c;
  const int32_t* piv_step = fa.piv_step;
  const int32_t* pos = fa.pos;
  int32_t* perm = fa.perm;
  float* Uout = fa.Uout;
  const int64_t ldu = fa.ldu;
  const int utrans = fa.utrans;
  const int64_t e = (int64_t)gr.bx * 256 + threadIdx.x;
  if (e >= M * (int64_t)c) return;
  const int kc = fa.kcap ? *fa.kcap : c;
  if (fa.kcap && Uout && e < (int64_t)c * c) {
    // the rows and columns of U past the steps taken
    const int s2 = (int)(e / c), t2 = (int)(e % c);
    if (s2 >= kc || t2 >= kc) Uout[(int64_t)s2 * ldu + t2] = 0.f;
  }
  const int64_t i = e / c;
  const int t = (int)(e - i * c);
  const int s = piv_step[i];
  float* f = F + i * ldf + t;
  if (s >= 0) {
    const float v = (t < kc) ? *f : 0.f;
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

template <int NB, int RPT, int NWAVE, int S>
hipError_t launch_panel(const PanelArgs& pa, int nblocks, hipStream_t s) {
  // PLU_PANEL_LA=0 selects the panel without look-ahead (same factors)
  static const int la = [] {
    const char* v = std::getenv("PLU_PANEL_LA");
    return v ? std::atoi(v) : 1;
  }();
  if (la == 0)
    return dispatch<PanelArgs, b_panel<NB, RPT, NWAVE, S>, 64 * NWAVE>(pa, dim3(nblocks), 0, s,
                                                                        true);
  if (nblocks <= 16)
    return dispatch<PanelArgs, b_panel_lw<NB, RPT, NWAVE, S, 8>, 64 * NWAVE>(pa, dim3(nblocks), 0,
                                                                              s, true);
  return dispatch<PanelArgs, b_panel_la<NB, RPT, NWAVE, S, 8>, 64 * NWAVE>(pa, dim3(nblocks), 0,
                                                                            s, true);
}

}  // namespace

size_t getrf_msg_words(int64_t M) {
  // one message slot per panel workgroup (at most 64), two parities
  (void)M;
  return (size_t)2 * 64 * (MSGH + 64);
}

hipError_t getrf_run(float* F, int64_t ldf, int64_t M, int c, const GetrfWork& w, int32_t* perm,
                     float* Uout, int64_t ldu, int utrans, hipStream_t s) {
  if (c <= 0 || M < c) return hipErrorInvalidValue;
  hipError_t e;
  if ((e = dispatch<InitArgs, b_getrf_init, 256>(InitArgs{w.piv_step, w.pos, M, w.zstep, w.run_if},
                                                 dim3((unsigned)((M + 255) / 256)), 0, s)) !=
      hipSuccess)
    return e;
  constexpr int NB = 64, NWAVE = 8, S = 4;
  // one row per lane while 64 workgroups of 512 rows suffice, else two;
  // PLU_PANEL_RPT=2 forces two rows per lane (half the workgroups)
  static const int rpt_env = [] {
    const char* v = std::getenv("PLU_PANEL_RPT");
    return v ? std::atoi(v) : 0;
  }();
  int rpt = (M <= 64LL * NWAVE * 64) ? 1 : 2;
  if (rpt_env == 2) rpt = 2;
  const int64_t rows_per_wg = (int64_t)NWAVE * 64 * rpt;
  const int nblocks = (int)((M + rows_per_wg - 1) / rows_per_wg);
  if (nblocks > 64 || (int64_t)nblocks * NWAVE > w.max_waves) return hipErrorInvalidValue;
  if ((size_t)2 * nblocks * (MSGH + NB) > w.msg_words) return hipErrorInvalidValue;
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
    pa.nwaves = nblocks;
    pa.msgw = MSGH + NB;
    pa.timeout_ticks = w.timeout_ticks;
    pa.run_if = w.run_if;
    pa.kcap = w.kcap;
    e = (rpt == 1) ? launch_panel<NB, 1, NWAVE, S>(pa, nblocks, s)
                   : launch_panel<NB, 2, NWAVE, S>(pa, nblocks, s);
    if (e != hipSuccess) return e;
    const int cs = jb + pa.nbw;
    if (cs < c) {
      TrsmArgs ta{F, ldf, jb, pa.nbw, c, w.piv_row, w.u12, w.ldu12, w.run_if, w.kcap};
      if ((e = dispatch<TrsmArgs, b_trsm, 256>(ta, dim3((unsigned)((c - cs + 3) / 4)), 0, s)) !=
          hipSuccess)
        return e;
      GemmArgs g;
      g.A = F + jb; g.lda = ldf;
      g.X = w.u12; g.ldx = w.ldu12;
      g.out = F + cs; g.ldo = ldf;
      g.P = M; g.R = pa.nbw; g.C = c - cs;
      g.rowmask = w.piv_step;
      g.run_if = w.run_if;
      // with a device column count: columns from cs on, panel rows from jb
      g.kcap = w.kcap;
      g.kc_col_off = cs;
      g.kc_red_off = jb;
      GemmPlan pl = plan_gemm(M, pa.nbw, c - cs, 1, 1);
      if ((e = launch_gemm(0, EPI_SUB, 0, g, pl, s)) != hipSuccess) return e;
    }
  }
  const int64_t tot = M * (int64_t)c;
  return dispatch<FinalizeArgs, b_getrf_finalize, 256>(
      FinalizeArgs{F, ldf, M, c, w.piv_step, w.pos, perm, Uout, ldu, utrans, w.run_if, w.kcap},
      dim3((unsigned)((tot + 255) / 256)), 0, s);
}

}  // namespace plu
