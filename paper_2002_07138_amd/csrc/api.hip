// C ABI of libpowerlu and the drivers that sequence the kernels:
//   * fixed rank: Alg. 5 with Alg. 7 as its steps 1-2 (Sec. 3.1, 3.4);
//   * fixed precision: Alg. 9 on Alg. 8 / Alg. 11 with the Thm 4.3 indicator.
// The host only enqueues work on the handle's stream; it synchronizes only to
// fill a plu_info, to read the fixed-precision rank, or for plu_residual.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <tuple>
#include <cstring>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <array>
#include <vector>

#include "../../include/powerlu.h"
#include "plu_internal.h"

using namespace plu;

// The workspace of plu_fixed_rank_static: one array per device, in the code
// object's device memory, held until the process ends.  Host code never uses
// the name itself (on the host it is not a device address): plu_create looks
// up its address on each device once (scratch_ptr) and every launch gets that.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct plu_handle_s {
  int device = 0;
  void* scratch_dev = nullptr;   // this device's address of `scratch`
  hipStream_t stream = nullptr;
  int cu_count = 256;
  uint64_t timeout_ticks = 0;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  // the rounded copies of A at the start of the arena (precision form): which
  // A they hold (base == nullptr: none)
  struct {
    const float* A = nullptr;
    const char* base = nullptr;
    int64_t m = 0, n = 0, lda = 0;
    int fmt = 0;
    bool acol = false;
  } lowp;
  uint32_t tag_counter = 0;   // LU panel launches on the arena's message buffer
  uint32_t call_tags = 0;     // the same for a call on a caller workspace or under capture
  size_t msg_off = 0, msg_words = 0;
  // batched path: one workspace region per problem, merged-launch tables,
  // and the graph of the last captured batch with the requests it was built for
  char* batch_arena = nullptr;
  size_t batch_bytes = 0;
  plu::MergeBuffers mbuf;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<unsigned char> gsig;
  plu::MergeBuffers gbuf;
  hipStream_t gstream = nullptr;   // capture stream (the handle's may be the null stream)
  // batched path: the streams a batch's problems run on side by side, forked
  // from and joined back into the caller's stream, with the merged-launch
  // tables of each (eager, and kept for the captured graph)
  static constexpr int kSide = 4;
  hipStream_t side[kSide] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kSide] = {};
  plu::MergeBuffers sbuf[kSide];
  plu::MergeBuffers sgbuf[kSide];
  // pivot trace of the last call (plu_set_pivot_trace / plu_pivot_trace):
  // device copies of every GETRF's pivot rows and gaps, in order
  int32_t* trace_piv = nullptr;
  float* trace_gaps = nullptr;
  int64_t trace_cap = 0, trace_n = 0, trace_need = 0;
};

namespace {

constexpr int kQB = 128;
constexpr int kMaxGramChunks = 256;
constexpr int kTargetWgs = 1024;  // concurrent pass workgroups: 4 per CU on 256 CUs
constexpr int kMaxSplit = 16;
constexpr int kLowpWgs = 512;     // 2 per CU: kLowpWgs / 2 is the CU count the
                                  // workspace sizing of the precision form assumes

inline int64_t ru4(int64_t x) { return (x + 3) & ~int64_t(3); }

inline bool valid_layout(int32_t layout) { return layout == PLU_ROW_MAJOR || layout == PLU_COL_MAJOR; }

// PLU_FP64_IND_G32=1: the float64 indicator's correction applied to the
// float32 G (no float64 pass), for measuring what each part contributes
bool fp64_ind_on_g32() {
  static const bool on = [] {
    const char* e = std::getenv("PLU_FP64_IND_G32");
    return e && e[0] == '1';
  }();
  return on;
}

bool valid_prec(int prec) {
  const int fmt = prec & PLU_PREC_FORMAT_MASK;
  if ((prec & PLU_PREC_REFINE_LAST) && (prec & PLU_PREC_REFINE_TWO)) return false;
  return fmt >= PLU_PREC_FP32 && fmt <= PLU_PREC_FP8_E4M3 &&
         (prec & ~(PLU_PREC_FORMAT_MASK | PLU_PREC_REFINE_LAST | PLU_PREC_REFINE_TWO |
                   PLU_PREC_A_UNCHANGED | PLU_PREC_FP64_INDICATOR)) == 0;
}
inline int64_t ru(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

#define PLU_TRY_HIP(expr)                \
  do {                                   \
    hipError_t e__ = (expr);             \
    if (e__ != hipSuccess) {             \
      std::fprintf(stderr, "libpowerlu: %s failed: %s\n", #expr, hipGetErrorString(e__)); \
      return PLU_ERR_HIP;                \
    }                                    \
  } while (0)

// Bump layout over the handle's arena.  A first pass with base == nullptr
// measures the size.
struct Layout {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = ru(off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct Ws {
  float *om, *ym, *zn, *qb, *tmp, *bt, *part, *u12, *rinv, *wproj, *ut1, *ut2;
  int64_t part_cap, lp;
  int32_t *piv_step, *pos, *piv_row1, *piv_row2, *piv_row0, *status;
  float *gaps0, *gaps1, *gaps2;
  unsigned long long* msg;
  size_t msg_words;
  double *gram_part, *gram, *rinv64, *sumsq_part, *colsq_part, *vsq_part, *colnorm, *scal;
  int32_t* iscal;
  // float64 indicator: G = A V in float64 (m x lp), V^T V - I (lp x lp), and
  // the per-row-block column terms of the corrected energies
  double *g64 = nullptr, *w64 = nullptr, *ind_part = nullptr;
  int64_t sumsq_cap, colsq_cap;
  // precision form: bfloat16 copies of A (row-major and transposed) and of the
  // sketch (transposed), padded to multiples of 64 along the contraction index
  uint16_t *ab, *abt, *xt;
  int64_t ldab, ldabt, ldxt, xt_rows;
  double* cvt_part;
  int64_t cvt_cap;
  // FP8 form: codes and E8M0 scales of A (both layouts) and of the sketch
  uint8_t *a8, *a8s, *a8t, *a8ts, *x8, *x8s;
  int64_t lda8, lda8t, ldx8, x8_rows;
  // A is stored column-major (lda >= m): it is then the row-major n x m
  // matrix A^T, so A X is the transposed-direction pass over that storage
  // and A^T Y the direct one
  bool acol = false;
  // restarted fixed precision: the kept basis V (n x lp) and G = A V (m x lp)
  float *vall = nullptr, *gall = nullptr;
  // sparse A: the passes run on its compressed rows / columns instead
  const SparseMat* sp = nullptr;
  // counter of this call's LU panel launches (tags of their messages)
  uint32_t* tags = nullptr;
  // the handle's stream is being captured into a graph: no autotuning runs
  bool capturing = false;
  // a call that must not allocate (plu_fixed_rank_static): no autotuning runs
  bool no_tune = false;
  // the workspace is the handle's arena (the rounded copies of A may persist)
  bool on_arena = false;
  double* anorm = nullptr;   // ||A||_F^2 of the rounded copies' A (precision form)
};

int64_t part_need(int64_t m, int64_t n, int64_t l) {
  // largest nsplit * P * ldo over the passes and the QR projections
  const int64_t lp = ru4(l);
  int64_t need = 0;
  for (int tr = 0; tr < 2; ++tr) {
    const int64_t P = tr ? n : m, R = tr ? m : n;
    GemmPlan pl = plan_gemm(P, R, l, kMaxSplit, kTargetWgs);
    if (pl.nsplit > 1) need = std::max(need, (int64_t)pl.nsplit * P * lp);
  }
  const int64_t Mx = std::max(m, n);
  for (int64_t j0 = kQB; j0 < l; j0 += kQB) {
    GemmPlan pl = plan_gemm(j0, Mx, kQB, 64, kTargetWgs);
    if (pl.nsplit > 1) need = std::max(need, (int64_t)pl.nsplit * j0 * kQB);
  }
  {
    GemmPlan pl = plan_gemm(Mx, kQB, kQB, 64, kTargetWgs);
    if (pl.nsplit > 1) need = std::max(need, (int64_t)pl.nsplit * Mx * kQB);
  }
  return need;
}

// Split plan of the reduced-precision passes: workgroups of `rows` rows
// (256 for bfloat16, 192 for FP8), one per CU (their LDS), splits on
// multiples of the stage depth ka along K, at most max_split.  A sketch of
// more than 8 column tiles (128 columns) up to wide_max tiles takes the wide
// kernel (one column block of 192 rows, A streamed once) instead of several
// column blocks.  The pass is bound by the bytes of A (bpe per entry), so
// the split weighs the rounds of cu_count workgroups it needs (idle CUs in
// the last round) against the bytes its float32 partials add (written and
// read back: 8 P l per split, against bpe P K for A).
GemmPlan plan_lowp(int64_t P, int64_t K, int64_t C, int cu_count, int max_split, int rows,
                   int64_t ka, double bpe, int wide_max) {
  GemmPlan pl = plan_gemm(P, K, C, 1, 1, 64);          // column blocks and tiles
  if (pl.cblocks > 1 && (C + 15) / 16 <= wide_max) {
    pl.cblocks = 1;
    pl.nt = (int)((C + 15) / 16);
    rows = 192;
  }
  pl.pblocks = (int)((P + rows - 1) / rows);
  const int64_t base = (int64_t)pl.pblocks * pl.cblocks;
  const int64_t hi =
      std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(kMaxSplit, max_split), K / 256));
  int64_t best_ns = 1;
  double best_cost = 1e30;
  for (int64_t ns = 1; ns <= hi; ++ns) {
    const int64_t tot = base * ns, rounds = (tot + cu_count - 1) / cu_count;
    const double cost = (double)(rounds * cu_count) / (double)tot +
                        (ns > 1 ? (double)ns * 8.0 * C / (bpe * K) : 0.0);
    if (cost < best_cost) {
      best_cost = cost;
      best_ns = ns;
    }
  }
  const int64_t rs = ru((K + best_ns - 1) / best_ns, ka);
  pl.nsplit = (int)((K + rs - 1) / rs);
  pl.rsplit = rs;
  return pl;
}

GemmPlan plan_lowp(int prec, int64_t P, int64_t K, int64_t C, int cu_count, int max_split) {
  return prec == PLU_PREC_BF16
             ? plan_lowp(P, K, C, cu_count, max_split, 256, 128, 2.0, 16)
             : plan_lowp(P, K, C, cu_count, max_split, 192, 256, 33.0 / 32.0, 14);
}

// Contraction padding of the reduced-precision copies (the depth of one
// stage of the pass kernel).
inline int64_t lowp_kalign(int prec) { return prec == PLU_PREC_FP8_E4M3 ? 256 : 128; }

// Rows of the transposed sketch a reduced-precision pass over C columns
// reads (both pass kernels take plan_gemm's column blocking).
int64_t lowp_xt_rows(int64_t P, int64_t K, int64_t C) {
  const GemmPlan pl = plan_gemm(P, K, C, 1, 1, 64);
  return ru((int64_t)pl.cblocks * pl.nt * 16, 64);
}

// Float32 partials of the split passes of the precision form, on a device of
// kLowpWgs / 2 CUs (the passes take a smaller split where they must).
int64_t lowp_part_need(int64_t m, int64_t n, int64_t l, int prec) {
  int64_t need = 0;
  const int64_t lp = ru4(l), ka = lowp_kalign(prec);
  for (int tr = 0; tr < 2; ++tr) {
    const int64_t P = tr ? n : m, K = ru(tr ? m : n, ka);
    const GemmPlan pl = plan_lowp(prec, P, K, l, kLowpWgs / 2, kMaxSplit);
    if (pl.nsplit > 1) need = std::max(need, (int64_t)pl.nsplit * P * lp);
  }
  return need;
}

Ws layout(Layout& L, int64_t m, int64_t n, int64_t l, int prec = PLU_PREC_FP32,
          bool basis_store = false) {
  const bool ind64 = (prec & PLU_PREC_FP64_INDICATOR) != 0;
  prec &= PLU_PREC_FORMAT_MASK;
  Ws w{};
  const int64_t Mx = std::max(m, n);
  const int64_t lp = ru4(std::max<int64_t>(l, 4));
  w.lp = lp;
  // the rounded copies of A first: their place depends on m, n and the
  // format only, so calls of other sketch widths find them where they are
  if (prec == PLU_PREC_BF16) {
    w.ldab = ru(n, 128);
    w.ldabt = ru(m, 128);
    w.ab = L.take<uint16_t>((size_t)m * w.ldab);
    w.abt = L.take<uint16_t>((size_t)n * w.ldabt);
    w.anorm = L.take<double>(1);
  } else if (prec == PLU_PREC_FP8_E4M3) {
    w.lda8 = ru(n, 256);
    w.lda8t = ru(m, 256);
    w.a8 = L.take<uint8_t>((size_t)m * w.lda8);
    w.a8s = L.take<uint8_t>((size_t)m * (w.lda8 / 32));
    w.a8t = L.take<uint8_t>((size_t)n * w.lda8t);
    w.a8ts = L.take<uint8_t>((size_t)n * (w.lda8t / 32));
    w.anorm = L.take<double>(1);
  }
  w.om = L.take<float>(Mx * lp);
  w.ym = L.take<float>(m * lp);
  w.zn = L.take<float>(n * lp);
  w.qb = L.take<float>(Mx * lp);
  w.tmp = L.take<float>(Mx * kQB);
  w.bt = L.take<float>(n * lp);
  w.part_cap = std::max<int64_t>(part_need(m, n, l), 1);
  if (prec != PLU_PREC_FP32) w.part_cap = std::max(w.part_cap, lowp_part_need(m, n, l, prec));
  w.part = L.take<float>(w.part_cap);
  w.u12 = L.take<float>(64 * lp);
  w.rinv = L.take<float>(kQB * kQB);
  w.wproj = L.take<float>(std::max<int64_t>(lp, kQB) * kQB);
  w.ut1 = L.take<float>(lp * lp);
  w.ut2 = L.take<float>(lp * lp);
  w.piv_step = L.take<int32_t>(Mx);
  w.pos = L.take<int32_t>(Mx);
  w.piv_row0 = L.take<int32_t>(lp);
  w.piv_row1 = L.take<int32_t>(lp);
  w.piv_row2 = L.take<int32_t>(lp);
  w.gaps0 = L.take<float>(lp);
  w.gaps1 = L.take<float>(lp);
  w.gaps2 = L.take<float>(lp);
  w.status = L.take<int32_t>(64);
  w.msg_words = getrf_msg_words(Mx);
  w.msg = L.take<unsigned long long>(w.msg_words);
  // the thin QR's float64 Gram partials: one per 64 rows, at most
  // kMaxGramChunks (the chunking itself does not depend on this size)
  w.gram_part = L.take<double>((size_t)std::min<int64_t>(kMaxGramChunks, (Mx + 63) / 64) * kQB * kQB);
  w.gram = L.take<double>(kQB * kQB);
  w.rinv64 = L.take<double>(kQB * kQB);
  w.sumsq_cap = 65536;
  w.sumsq_part = L.take<double>(w.sumsq_cap);
  w.colsq_cap = ((m + 63) / 64) * lp;
  w.colsq_part = L.take<double>(w.colsq_cap);
  w.vsq_part = L.take<double>(((n + 63) / 64) * lp);
  w.colnorm = L.take<double>(lp);
  w.scal = L.take<double>(16);
  w.iscal = L.take<int32_t>(16);
  if (prec == PLU_PREC_BF16) {
    w.ldxt = ru(Mx, 128);
    w.xt_rows = std::max(lowp_xt_rows(m, ru(n, 128), l), lowp_xt_rows(n, ru(m, 128), l));
    w.xt = L.take<uint16_t>((size_t)w.xt_rows * w.ldxt);
    w.cvt_cap = ((std::max(ru(m, 128), ru(n, 128)) + 63) / 64) * 8;   // either storage order
    w.cvt_part = L.take<double>(w.cvt_cap);
  } else if (prec == PLU_PREC_FP8_E4M3) {
    w.ldx8 = ru(Mx, 256);
    w.x8_rows = std::max(lowp_xt_rows(m, w.lda8, l), lowp_xt_rows(n, w.lda8t, l));
    w.x8 = L.take<uint8_t>((size_t)w.x8_rows * w.ldx8);
    w.x8s = L.take<uint8_t>((size_t)w.x8_rows * (w.ldx8 / 32));
    w.cvt_cap = ((std::max(ru(m, 256), ru(n, 256)) + 63) / 64) * 8;   // either storage order
    w.cvt_part = L.take<double>(w.cvt_cap);
  }
  if (basis_store) {
    w.vall = L.take<float>(n * lp);
    w.gall = L.take<float>(m * lp);
  }
  if (ind64) {
    w.g64 = L.take<double>(m * lp);
    w.w64 = L.take<double>(lp * lp);
    w.ind_part = L.take<double>((size_t)f64_row_blocks(l) * lp);
  }
  return w;
}

// Status of ensure_ws when a caller workspace is smaller than the call needs.
constexpr int kWsTooSmall = -1000;

bool stream_capturing(hipStream_t s) {
  if (!s) return false;   // the null stream cannot be captured
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &st) == hipSuccess && st == hipStreamCaptureStatusActive;
}

// Lays out the workspace of a call: on the caller's `work` (work_bytes long)
// when given, else on the handle's arena, grown on demand (never while the
// stream is captured: PLU_ERR_OOM then).  A call on a caller workspace or
// under capture numbers its LU panel launches from zero, so its first panel
// clears the message buffer in the call's own launch sequence (a replayed
// graph then never sees the messages of an earlier replay).
int ensure_ws(plu_handle h, int64_t m, int64_t n, int64_t l, Ws* out,
              int prec = PLU_PREC_FP32, bool basis_store = false, void* work = nullptr,
              size_t work_bytes = 0, bool init_status = true) {
  Layout dry;
  layout(dry, m, n, l, prec, basis_store);
  const size_t need = dry.off + 256;
  const bool capturing = stream_capturing(h->stream);
  if (work) {
    const uintptr_t a = (reinterpret_cast<uintptr_t>(work) + 255) & ~uintptr_t(255);
    const size_t skew = a - reinterpret_cast<uintptr_t>(work);
    if (work_bytes < skew || work_bytes - skew < dry.off) return kWsTooSmall;
    Layout L;
    L.base = reinterpret_cast<char*>(a);
    *out = layout(L, m, n, l, prec, basis_store);
    h->call_tags = 0;
    out->tags = &h->call_tags;
    out->on_arena = false;
  } else {
    if (need > h->arena_bytes && capturing) {
      std::fprintf(stderr, "libpowerlu: the workspace must exist before graph capture "
                           "(an eager call of the same shape, or a caller workspace)\n");
      return PLU_ERR_OOM;
    }
    if (need > h->arena_bytes) {
      if (h->arena) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(h->arena);
        h->arena = nullptr;
        h->arena_bytes = 0;
      }
      const size_t alloc = need + need / 8;
      if (hipMalloc(reinterpret_cast<void**>(&h->arena), alloc) != hipSuccess) {
        (void)hipGetLastError();
        return PLU_ERR_OOM;
      }
      h->arena_bytes = alloc;
      h->tag_counter = 0;   // next panel launch clears the message buffer
      h->lowp.base = nullptr;
    }
    Layout L;
    L.base = h->arena;
    *out = layout(L, m, n, l, prec, basis_store);
    out->on_arena = true;
    // a call that lays out the arena differently overwrites the rounded copies
    const int fmt = prec & PLU_PREC_FORMAT_MASK;
    if (fmt == PLU_PREC_FP32 || h->lowp.m != m || h->lowp.n != n || h->lowp.fmt != fmt)
      h->lowp.base = nullptr;
    if (capturing) {
      h->call_tags = 0;
      out->tags = &h->call_tags;
    } else {
      out->tags = &h->tag_counter;
    }
  }
  out->capturing = capturing;
  // per-call status words (read by the LU steps): zero-pivot slots to
  // "none", flags to 0
  if (init_status &&
      (launch_fill_u32(reinterpret_cast<uint32_t*>(out->status), 32, 0x7FFFFFFFu, h->stream) !=
           hipSuccess ||
       launch_fill_u32(reinterpret_cast<uint32_t*>(out->status + 32), 32, 0u, h->stream) !=
           hipSuccess))
    return PLU_ERR_HIP;
  return PLU_OK;
}

GetrfWork getrf_work(plu_handle h, const Ws& w, int which) {
  GetrfWork g;
  g.piv_step = w.piv_step;
  g.pos = w.pos;
  g.piv_row = which == 1 ? w.piv_row1 : which == 2 ? w.piv_row2 : w.piv_row0;
  g.gaps = which == 1 ? w.gaps1 : which == 2 ? w.gaps2 : w.gaps0;
  g.zstep = w.status + 4 * which;
  g.abortf = w.status + 32;
  g.msg = w.msg;
  g.msg_words = w.msg_words;
  g.u12 = w.u12;
  g.ldu12 = w.lp;
  g.tag_counter = w.tags ? w.tags : &h->tag_counter;
  g.timeout_ticks = h->timeout_ticks;
  g.max_waves = h->cu_count * 8;
  return g;
}

// Appends the pivot rows and gaps of the GETRF just queued with work g (c
// steps) to the handle's pivot trace, when tracing is on.
hipError_t trace_getrf(plu_handle h, const GetrfWork& g, int c) {
  if (!h->trace_cap || thread_recorder()) return hipSuccess;
  const int64_t at = h->trace_need;
  h->trace_need += c;
  if (at + c > h->trace_cap) return hipSuccess;   // reported by plu_pivot_trace
  hipError_t e = hipMemcpyAsync(h->trace_piv + at, g.piv_row, c * sizeof(int32_t),
                                hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->trace_gaps + at, g.gaps, c * sizeof(float), hipMemcpyDeviceToDevice,
                       h->stream);
  h->trace_n = at + c;
  return e;
}

void trace_reset(plu_handle h) { h->trace_n = h->trace_need = 0; }

QrWork qr_work(const Ws& w, float* q, int64_t ldq) {
  QrWork r;
  r.q = q;
  r.ldq = ldq;
  r.tmp = w.tmp;
  r.gram_part = w.gram_part;
  r.max_chunks = kMaxGramChunks;
  r.gram = w.gram;
  r.rinv = w.rinv;
  r.rinv64 = w.rinv64;
  r.wproj = w.wproj;
  r.part = w.part;
  r.part_cap = w.part_cap;
  r.status = w.status + 48;
  return r;
}

// One pass over A: out = A X (trans 0) or A^T X (trans 1).  Optional fused
// ||A||_F^2 into normA2_dev and column norms^2 partials into colsq (then
// *colsq_blocks receives the number of row blocks).
// Autotuned split of the passes over A.  The first pass of a shape (direction,
// P, R, C, leading dimension of the output) on a device times the candidate
// plans -- 128 or 64 rows per workgroup, each with the split that fills whole
// rounds of 512, 768, 1024, 1280, 1536 or 2048 resident workgroups -- with
// events on the handle's stream and keeps the fastest for the process, so
// every later pass of that shape (single calls and batches alike) runs the
// same plan and gives the same bits.  The row-block size leaves every output
// element's summation order unchanged; the split does not.
// The tuner's choices are kept per size class: the kept and reduced
// dimensions in half-octave buckets, the sketch width exactly (it sets the
// kernel's column tiles), so that a stream of requests of ever new shapes
// tunes once per class, not once per shape.
struct TuneKey {
  int device, trans, pb, rb, only_bp;
  int64_t C;
  bool operator<(const TuneKey& o) const {
    return std::tie(device, trans, pb, rb, only_bp, C) <
           std::tie(o.device, o.trans, o.pb, o.rb, o.only_bp, o.C);
  }
};
int size_bucket(int64_t x) {
  return (int)std::floor(2.0 * std::log2((double)std::max<int64_t>(x, 1)));
}
// a tuned choice: row-block size and the concurrent-workgroup count the split
// is planned for (plan_gemm turns them into the plan of any shape of the class)
struct TunedChoice {
  int bp, slots;
};
std::mutex g_tune_mu;
std::map<TuneKey, TunedChoice> g_tuned;

// row stride of the split partials of a pass whose output has row stride ldo
int64_t part_ld(int64_t ldo) { return (ldo + 3) & ~int64_t(3); }

hipError_t pass_launch(plu_handle h, const Ws& w, int trans, const GemmArgs& g0, const GemmPlan& pl,
                       float* out, int64_t ldo, double* colsq, hipStream_t s);

bool tune_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("PLU_AUTOTUNE");
    return !(e && e[0] == '0');
  }();
  return on;
}

GemmPlan pass_plan(plu_handle h, const Ws& w, int trans, const GemmArgs& g, float* out, int64_t ldo) {
  const int64_t P = g.P, R = g.R, C = g.C;
  // split boundaries on whole 128-byte lines of A's rows (32 floats), so no
  // line is fetched by two workgroups of adjacent splits
  constexpr int kLineAlign = 32;
  const GemmPlan def = plan_gemm(P, R, C, kMaxSplit, kTargetWgs, kLineAlign);
  auto fits = [&](const GemmPlan& p) {
    return (p.nsplit == 1 || (int64_t)p.nsplit * P * part_ld(ldo) <= w.part_cap) &&
           (int64_t)p.pblocks * p.nsplit <= w.sumsq_cap;
  };
  // PLU_AUTOTUNE_ROWS=64 or 128 holds the tuner to one row-block size
  int only_bp = 0;
  if (const char* rows = std::getenv("PLU_AUTOTUNE_ROWS")) only_bp = std::atoi(rows);
  const TuneKey key{h->device, trans, size_bucket(P), size_bucket(R), only_bp, C};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      const GemmPlan p = plan_gemm(P, R, C, kMaxSplit, it->second.slots, kLineAlign, it->second.bp);
      if (fits(p)) return p;
      return fits(def) ? def : plan_gemm(P, R, C, 1, 1);
    }
  }
  // small passes, recorded (batched) launches and launches under graph
  // capture use the default plan
  if (!tune_enabled() || thread_recorder() || w.capturing || w.no_tune || 2.0 * P * R * C < 2e10)
    return fits(def) ? def : plan_gemm(P, R, C, 1, 1);
  std::vector<GemmPlan> cands;
  std::vector<int> cand_slots;
  for (int bp : {GEMM_BP, 64}) {
    if (only_bp == 64 || only_bp == GEMM_BP) {
      if (bp != only_bp) continue;
    }
    for (int slots : {512, 768, 1024, 1280, 1536, 2048}) {
      GemmPlan p = plan_gemm(P, R, C, kMaxSplit, slots, kLineAlign, bp);
      if (!fits(p)) continue;
      bool dup = false;
      for (auto& c : cands) dup |= c.nsplit == p.nsplit && c.bp == p.bp;
      if (dup) continue;
      cands.push_back(p);
      cand_slots.push_back(slots);
    }
  }
  if (cands.empty()) return plan_gemm(P, R, C, 1, 1);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return cands[0];
  // three rounds over all candidates in turn, keeping each one's fastest
  // round, so that a clock still rising during the first launches favours
  // none of them
  std::vector<float> cand_ms(cands.size(), 1e30f);
  std::vector<char> cand_ok(cands.size(), 1);
  // a few launches first to bring the clocks up (the first timed round
  // would otherwise favour the candidates timed last), then every candidate
  // once to warm up its code and caches
  for (int r = 0; r < 2; ++r)
    (void)pass_launch(h, w, trans, g, cands[0], out, ldo, nullptr, h->stream);
  for (size_t c = 0; c < cands.size(); ++c)
    cand_ok[c] = pass_launch(h, w, trans, g, cands[c], out, ldo, nullptr, h->stream) == hipSuccess;
  for (int round = 0; round < 3; ++round) {
    for (size_t c = 0; c < cands.size(); ++c) {
      if (!cand_ok[c]) continue;
      float ms = 0.f;
      bool ok = hipEventRecord(e0, h->stream) == hipSuccess;
      for (int r = 0; r < 2 && ok; ++r)
        ok = pass_launch(h, w, trans, g, cands[c], out, ldo, nullptr, h->stream) == hipSuccess;
      ok = ok && hipEventRecord(e1, h->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
           hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
      if (!ok) cand_ok[c] = 0;
      else cand_ms[c] = std::min(cand_ms[c], ms);
    }
  }
  // the fastest, or among the candidates within 2% of it the one with the
  // fewest splits: fewer split partials written and read back (each split
  // adds 8 P l bytes of traffic to the pass)
  GemmPlan best = cands[0];
  int best_slots = cand_slots[0];
  float best_ms = 1e30f;
  for (size_t c = 0; c < cands.size(); ++c)
    if (cand_ok[c]) best_ms = std::min(best_ms, cand_ms[c]);
  float kept_ms = 1e30f;
  int kept_split = 1 << 30;
  for (size_t c = 0; c < cands.size(); ++c) {
    if (!cand_ok[c] || cand_ms[c] > best_ms * 1.02f) continue;
    if (cands[c].nsplit < kept_split || (cands[c].nsplit == kept_split && cand_ms[c] < kept_ms)) {
      kept_split = cands[c].nsplit;
      kept_ms = cand_ms[c];
      best = cands[c];
      best_slots = cand_slots[c];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (const char* lg = std::getenv("PLU_AUTOTUNE_LOG"); lg && lg[0] == '1') {
    for (size_t c = 0; c < cands.size(); ++c)
      std::fprintf(stderr, "plu autotune: %s P %lld R %lld C %lld ldo %lld: rows %d split %d: %.4f ms%s\n",
                   trans ? "T" : "N", (long long)P, (long long)R, (long long)C, (long long)ldo,
                   cands[c].bp, cands[c].nsplit, cand_ms[c] / 2, (cands[c].bp == best.bp &&
                   cands[c].nsplit == best.nsplit) ? "  <- kept" : "");
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = TunedChoice{best.bp, best_slots};
  return best;
}

hipError_t pass_launch(plu_handle h, const Ws& w, int trans, const GemmArgs& g0, const GemmPlan& pl,
                       float* out, int64_t ldo, double* colsq, hipStream_t s) {
  GemmArgs g = g0;
  const int64_t P = g.P;
  const int rb = 64;
  hipError_t e;
  if (pl.nsplit > 1) {
    // the partials' rows padded to whole float4s, so the reduction reads
    // every column group, the last one too, as whole float4s
    const int64_t pld = part_ld(ldo);
    if ((int64_t)pl.nsplit * P * pld > w.part_cap) return hipErrorInvalidValue;
    g.out = w.part; g.ldo = pld; g.part_stride = P * pld;
    if ((e = launch_gemm(trans, EPI_PART, 0, g, pl, s)) != hipSuccess) return e;
    return launch_splitk_reduce_ld(w.part, pld, P * pld, pl.nsplit, out, ldo, P, g.C, colsq, rb, s);
  }
  g.out = out; g.ldo = ldo;
  if ((e = launch_gemm(trans, EPI_STORE, 0, g, pl, s)) != hipSuccess) return e;
  if (colsq) return launch_splitk_reduce(out, 0, 1, nullptr, ldo, P, g.C, colsq, rb, s);
  return hipSuccess;
}

// Tunes (when it has not been tuned yet, and only eagerly: never while
// recording or capturing) the split of a pass run_pass would make with these
// arguments, so that launches recorded later for a batch or a graph take the
// same plan as the single calls and give the same bits.
void pretune_pass(plu_handle h, const Ws& w, int trans, int64_t m, int64_t n, const float* A,
                  int64_t lda, const float* X, int64_t ldx, int64_t l, float* out, int64_t ldo) {
  if (w.sp || thread_recorder() || w.capturing || w.no_tune) return;
  if (w.acol) {
    trans ^= 1;
    std::swap(m, n);
  }
  GemmArgs g0;
  g0.A = A; g0.lda = lda; g0.X = X; g0.ldx = ldx;
  g0.P = trans ? n : m; g0.R = trans ? m : n; g0.C = l;
  (void)pass_plan(h, w, trans, g0, out, ldo);
}

// Whether pretune_pass with these arguments would still time candidates (a
// large pass whose size class has no tuned choice yet).
bool pass_needs_tuning(plu_handle h, const Ws& w, int trans, int64_t m, int64_t n, int64_t l) {
  if (w.sp || !tune_enabled()) return false;
  if (w.acol) {
    trans ^= 1;
    std::swap(m, n);
  }
  const int64_t P = trans ? n : m, R = trans ? m : n;
  if (2.0 * P * R * l < 2e10) return false;
  int only_bp = 0;
  if (const char* rows = std::getenv("PLU_AUTOTUNE_ROWS")) only_bp = std::atoi(rows);
  const TuneKey key{h->device, trans, size_bucket(P), size_bucket(R), only_bp, l};
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_tuned.find(key) == g_tuned.end();
}

hipError_t run_pass(plu_handle h, const Ws& w, int trans, int64_t m, int64_t n, const float* A,
                    int64_t lda, const float* X, int64_t ldx, int64_t l, float* out, int64_t ldo,
                    double* normA2_dev, double* colsq, int* colsq_blocks) {
  if (w.sp) {   // sparse A: a gather over the compressed rows (A X) or columns (A^T Y)
    const SparseMat& S = *w.sp;
    const int64_t P = trans ? S.n : S.m;
    hipError_t e = trans ? launch_spmm(S.colptr, S.rowidx, S.valsT, S.n, X, ldx, (int)l, out, ldo,
                                       h->stream)
                         : launch_spmm(S.rowptr, S.colidx, S.vals, S.m, X, ldx, (int)l, out, ldo,
                                       h->stream);
    if (e != hipSuccess) return e;
    if (colsq && (e = launch_splitk_reduce(out, 0, 1, nullptr, ldo, P, l, colsq, 64, h->stream)) !=
                     hipSuccess)
      return e;
    if (colsq_blocks) *colsq_blocks = (int)((P + 63) / 64);
    if (normA2_dev)
      return hipMemcpyAsync(normA2_dev, S.normA2, sizeof(double), hipMemcpyDeviceToDevice,
                            h->stream);
    return hipSuccess;
  }
  if (w.acol) {   // the storage is A^T, row-major
    trans ^= 1;
    std::swap(m, n);
  }
  const int64_t P = trans ? n : m, R = trans ? m : n;
  GemmArgs g0;
  g0.A = A; g0.lda = lda; g0.X = X; g0.ldx = ldx;
  g0.P = P; g0.R = R; g0.C = l;
  const GemmPlan pl = pass_plan(h, w, trans, g0, out, ldo);
  GemmArgs g = g0;
  if (normA2_dev) {
    if ((int64_t)pl.pblocks * pl.nsplit > w.sumsq_cap) return hipErrorInvalidValue;
    g.sumsq_part = w.sumsq_part;
  }
  hipError_t e;
  const int rb = 64;
  if ((e = pass_launch(h, w, trans, g, pl, out, ldo, colsq, h->stream)) != hipSuccess) return e;
  if (colsq_blocks) *colsq_blocks = (int)((P + rb - 1) / rb);
  if (normA2_dev) {
    if ((e = launch_sum_doubles(w.sumsq_part, (int64_t)pl.pblocks * pl.nsplit, normA2_dev,
                                h->stream)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

// bfloat16 copies of A for the precision form (both layouts), with ||A||_F^2
// accumulated in float64 from the fp32 values.
hipError_t convert_a_bf16(plu_handle h, const Ws& w, int64_t m, int64_t n, const float* A,
                          int64_t lda, double* normA2_dev) {
  hipError_t e;
  int64_t np = 0;
  if (w.acol)   // the storage is A^T: its row-major copy is the transposed one
    e = launch_cvt_bf16(A, lda, n, m, w.abt, w.ldabt, w.ab, w.ldab, m, w.cvt_part, &np,
                        h->stream);
  else
    e = launch_cvt_bf16(A, lda, m, n, w.ab, w.ldab, w.abt, w.ldabt, n, w.cvt_part, &np,
                        h->stream);
  if (e != hipSuccess) return e;
  if (np > w.cvt_cap) return hipErrorInvalidValue;
  if (normA2_dev) return launch_sum_doubles(w.cvt_part, np, normA2_dev, h->stream);
  return hipSuccess;
}

// One pass of the precision form: out = A X (trans 0) or A^T X (trans 1) with
// both operands rounded to bfloat16 (A from the copies made by
// convert_a_bf16), fp32 accumulation.
hipError_t run_pass_bf16(plu_handle h, const Ws& w, int trans, int64_t m, int64_t n,
                         const float* X, int64_t ldx, int64_t l, float* out, int64_t ldo) {
  const int64_t P = trans ? n : m, Kl = trans ? m : n;
  const uint16_t* M = trans ? w.abt : w.ab;
  const int64_t ldm = trans ? w.ldabt : w.ldab;
  const int64_t pld = part_ld(ldo);
  // the kernel walks K 128 at a time: the copies are padded to that (zeros
  // past the logical K in A's copies and in the sketch's)
  const int64_t K = ru(Kl, 128);
  // the split the partials buffer holds (it is sized for the plan on a
  // device of kLowpWgs / 2 CUs; on others a smaller split may be taken)
  const int cap = (int)std::max<int64_t>(1, w.part_cap / std::max<int64_t>(1, P * pld));
  const GemmPlan pl = plan_lowp(PLU_PREC_BF16, P, K, l, h->cu_count, cap);
  const int64_t ct = ru((int64_t)pl.cblocks * pl.nt * 16, 64);
  if (ct > w.xt_rows || K > w.ldxt || K > ldm) return hipErrorInvalidValue;
  hipError_t e;
  if ((e = launch_cvt_bf16(X, ldx, Kl, l, nullptr, 0, w.xt, K, ct, nullptr, nullptr,
                           h->stream)) != hipSuccess)
    return e;
  if (pl.nsplit > 1) {
    if ((e = launch_pass_bf16(EPI_PART, M, ldm, w.xt, K, w.part, pld, P * pld, P, K, l, pl,
                              h->stream)) != hipSuccess)
      return e;
    return launch_splitk_reduce_ld(w.part, pld, P * pld, pl.nsplit, out, ldo, P, l, nullptr, 64,
                                   h->stream);
  }
  return launch_pass_bf16(EPI_STORE, M, ldm, w.xt, K, out, ldo, 0, P, K, l, pl, h->stream);
}

// Block-scaled FP8 copies of A for the precision form (both layouts) and
// ||A||_F^2 (float64, from the fp32 values: one extra read of A).
hipError_t convert_a_fp8(plu_handle h, const Ws& w, int64_t m, int64_t n, const float* A,
                         int64_t lda, double* normA2_dev) {
  hipError_t e;
  int64_t np = 0;
  double* part = normA2_dev ? w.cvt_part : nullptr;
  if (w.acol)   // the storage is A^T: its row-major copy is the transposed one
    e = launch_cvt_fp8(A, lda, n, m, w.a8t, w.a8ts, w.lda8t, w.a8, w.a8s, w.lda8, m, part, &np,
                       h->stream);
  else
    e = launch_cvt_fp8(A, lda, m, n, w.a8, w.a8s, w.lda8, w.a8t, w.a8ts, w.lda8t, n, part, &np,
                       h->stream);
  if (e != hipSuccess) return e;
  if (np > w.cvt_cap) return hipErrorInvalidValue;
  if (normA2_dev) return launch_sum_doubles(w.cvt_part, np, normA2_dev, h->stream);
  return hipSuccess;
}

// The rounded copies of A for the precision form (both storage orders), and
// ||A||_F^2 (float64, from the fp32 values) into normA2_dev (nullable).  With
// `reuse` -- the caller's PLU_PREC_A_UNCHANGED -- and copies of this very A
// (same pointer, shape, leading dimension, storage order and format) still in
// the handle's arena, nothing is converted again.
hipError_t lowp_copies(plu_handle h, const Ws& w, int fmt, int64_t m, int64_t n, const float* A,
                       int64_t lda, bool reuse, double* normA2_dev) {
  const char* base = fmt == PLU_PREC_BF16 ? reinterpret_cast<const char*>(w.ab)
                                          : reinterpret_cast<const char*>(w.a8);
  auto& c = h->lowp;
  const bool hit = reuse && w.on_arena && c.base == base && c.A == A && c.m == m && c.n == n &&
                   c.lda == lda && c.fmt == fmt && c.acol == w.acol;
  hipError_t e;
  if (!hit) {
    e = fmt == PLU_PREC_BF16 ? convert_a_bf16(h, w, m, n, A, lda, w.anorm)
                             : convert_a_fp8(h, w, m, n, A, lda, w.anorm);
    if (e != hipSuccess) return e;
    if (w.on_arena) {
      c.A = A; c.base = base; c.m = m; c.n = n; c.lda = lda; c.fmt = fmt; c.acol = w.acol;
    }
  }
  if (normA2_dev)
    return hipMemcpyAsync(normA2_dev, w.anorm, sizeof(double), hipMemcpyDeviceToDevice, h->stream);
  return hipSuccess;
}

// One pass of the FP8 form: both operands block-scaled E4M3, fp32 accumulation.
hipError_t run_pass_fp8(plu_handle h, const Ws& w, int trans, int64_t m, int64_t n,
                        const float* X, int64_t ldx, int64_t l, float* out, int64_t ldo) {
  // the kernel walks K 256 at a time (the copies are padded to that)
  const int64_t P = trans ? n : m, Kl = trans ? m : n, K = ru(Kl, 256);
  const uint8_t* M = trans ? w.a8t : w.a8;
  const uint8_t* Ms = trans ? w.a8ts : w.a8s;
  const int64_t ldm = trans ? w.lda8t : w.lda8;
  const int64_t pld = part_ld(ldo);
  const int cap = (int)std::max<int64_t>(1, w.part_cap / std::max<int64_t>(1, P * pld));
  const GemmPlan pl = plan_lowp(PLU_PREC_FP8_E4M3, P, K, l, h->cu_count, cap);
  const int64_t ct = ru((int64_t)pl.cblocks * pl.nt * 16, 64);
  if (ct > w.x8_rows || K > w.ldx8 || K > ldm) return hipErrorInvalidValue;
  hipError_t e;
  if ((e = launch_cvt_fp8(X, ldx, Kl, l, nullptr, nullptr, 0, w.x8, w.x8s, K, ct, nullptr,
                         nullptr, h->stream)) !=
      hipSuccess)
    return e;
  if (pl.nsplit > 1) {
    if ((e = launch_pass_fp8(EPI_PART, M, Ms, ldm, w.x8, w.x8s, K, w.part, pld, P * pld, P, K,
                             l, pl, h->stream)) != hipSuccess)
      return e;
    return launch_splitk_reduce_ld(w.part, pld, P * pld, pl.nsplit, out, ldo, P, l, nullptr, 64,
                                   h->stream);
  }
  return launch_pass_fp8(EPI_STORE, M, Ms, ldm, w.x8, w.x8s, K, out, ldo, 0, P, K, l, pl,
                         h->stream);
}

// W (P x l, ldw) = C^T X for C rc x P (ldc) and X rc x l (ldx): a short wide
// product whose reduction over the rc rows is split through the workspace
// partials.
hipError_t small_tn(plu_handle h, const Ws& w, const float* C, int64_t ldc, const float* X,
                    int64_t ldx, int64_t P, int64_t rc, int64_t l, float* W, int64_t ldw) {
  hipError_t e;
  GemmArgs g;
  g.A = C; g.lda = ldc; g.X = X; g.ldx = ldx;
  g.P = P; g.R = rc; g.C = l;
  int max_split = (int)std::min<int64_t>(64, w.part_cap / std::max<int64_t>(P * ldw, 1));
  if (max_split < 1) max_split = 1;
  const GemmPlan pl = plan_gemm(P, rc, l, max_split, 1024);
  if (pl.nsplit > 1) {
    g.out = w.part; g.ldo = ldw; g.part_stride = P * ldw;
    if ((e = launch_gemm(1, EPI_PART, 0, g, pl, h->stream)) != hipSuccess) return e;
    return launch_splitk_reduce(w.part, P * ldw, pl.nsplit, W, ldw, P, l, nullptr, 64, h->stream);
  }
  g.out = W; g.ldo = ldw;
  return launch_gemm(1, EPI_STORE, 0, g, pl, h->stream);
}

// out -= B (C^T X) with C (rc x Ld), B (rb x Ld), both leading dimension
// ldd; X rc x l (ldx); W (Ld x l, ldw) is scratch.
hipError_t project_out(plu_handle h, const Ws& w, const float* C, const float* B, int64_t ldd,
                       int64_t Ld, int64_t rc, int64_t rb, const float* X, int64_t ldx, int64_t l,
                       float* out, int64_t ldo, float* W, int64_t ldw) {
  hipError_t e;
  if ((e = small_tn(h, w, C, ldd, X, ldx, Ld, rc, l, W, ldw)) != hipSuccess) return e;
  GemmArgs u;
  u.A = B; u.lda = ldd; u.X = W; u.ldx = ldw; u.out = out; u.ldo = ldo;
  u.P = rb; u.R = Ld; u.C = l;
  return launch_gemm(0, EPI_SUB, 0, u, plan_gemm(rb, Ld, l, 1, 1), h->stream);
}

// Alg. 7.  Leaves the orthonormal n x l basis in *Vout (one of the workspace
// buffers, leading dimension w.lp); passes counted in *passes.  With Ld > 0
// it runs on the remainder A (I - Vd Vd^T) of the kept basis Vd (n x Ld)
// with Gd = A Vd (m x Ld), both of leading dimension w.lp: each pass A X
// becomes A X - Gd (Vd^T X) and each A^T Y becomes A^T Y - Vd (Gd^T Y).
hipError_t range_basis(plu_handle h, const Ws& w, int64_t m, int64_t n, const float* A, int64_t lda,
                       int l, int v, const float* Omega, uint64_t seed, float** Vout,
                       int* passes, int prec = PLU_PREC_FP32, const float* Vd = nullptr,
                       const float* Gd = nullptr, int64_t Ld = 0) {
  const int64_t lp = w.lp;
  const int64_t rows = (v % 2 == 0) ? m : n;
  hipError_t e;
  if (Omega) {
    if ((e = launch_copy_pad(Omega, l, w.om, lp, rows, l, l, h->stream)) != hipSuccess) return e;
  } else {
    if ((e = launch_gaussian(w.om, lp, rows, l, seed, h->stream)) != hipSuccess) return e;
  }
  double* normA2 = w.scal + 0;
  bool first = true;
  int np = 0;
  float* V = nullptr;
  const int P = (v - 1) / 2;
  const GetrfWork gw = getrf_work(h, w, 0);
  const QrWork qw = qr_work(w, w.qb, lp);
  const int fmt = prec & PLU_PREC_FORMAT_MASK;
  // the last `exact_tail` of the v - 1 passes run on the fp32 A
  const int exact_tail = (prec & PLU_PREC_REFINE_TWO) ? 2 : (prec & PLU_PREC_REFINE_LAST) ? 1 : 0;
  // the rounded copies are needed only if some pass is rounded
  const bool any_rounded = fmt != PLU_PREC_FP32 && v - 1 > exact_tail;
  if (any_rounded) {
    if ((e = lowp_copies(h, w, fmt, m, n, A, lda, (prec & PLU_PREC_A_UNCHANGED) != 0, normA2)) !=
        hipSuccess)
      return e;
    first = false;
  }
  // one of the v - 1 passes of Alg. 7 (the first one also yields ||A||_F^2);
  // with a refinement flag the last one or two of them run on the fp32 A
  int pidx = 0;
  auto pass = [&](int trans, const float* X, float* out) -> hipError_t {
    const bool rounded = any_rounded && pidx < v - 1 - exact_tail;
    ++pidx;
    hipError_t r;
    if (rounded && fmt == PLU_PREC_BF16) {
      r = run_pass_bf16(h, w, trans, m, n, X, lp, l, out, lp);
    } else if (rounded && fmt == PLU_PREC_FP8_E4M3) {
      r = run_pass_fp8(h, w, trans, m, n, X, lp, l, out, lp);
    } else {
      r = run_pass(h, w, trans, m, n, A, lda, X, lp, l, out, lp, first ? normA2 : nullptr, nullptr,
                   nullptr);
      first = false;
    }
    if (r != hipSuccess || Ld == 0) return r;
    // the remainder's pass (w.bt, n x lp, holds the small Ld x l product)
    return trans == 0 ? project_out(h, w, Vd, Gd, lp, Ld, n, m, X, lp, l, out, lp, w.bt, lp)
                      : project_out(h, w, Gd, Vd, lp, Ld, m, n, X, lp, l, out, lp, w.bt, lp);
  };
  if (v % 2 == 0) {
    if ((e = pass(1, w.om, w.zn)) != hipSuccess) return e;
    ++np;
    if (v > 2) {
      if ((e = getrf_run(w.zn, lp, n, l, gw, nullptr, nullptr, 0, 0, h->stream)) != hipSuccess)
        return e;
      if ((e = trace_getrf(h, gw, l)) != hipSuccess) return e;
      V = w.zn;
    } else {
      if ((e = thin_qr_run(w.zn, lp, n, l, gw, qw, h->stream)) != hipSuccess) return e;
      V = w.qb;
    }
  } else {
    V = w.om;
  }
  for (int i = 1; i <= P; ++i) {
    if ((e = pass(0, V, w.ym)) != hipSuccess) return e;
    ++np;
    if ((e = getrf_run(w.ym, lp, m, l, gw, nullptr, nullptr, 0, 0, h->stream)) != hipSuccess ||
        (e = trace_getrf(h, gw, l)) != hipSuccess)
      return e;
    if ((e = pass(1, w.ym, w.zn)) != hipSuccess) return e;
    ++np;
    if (i == P) {
      if ((e = thin_qr_run(w.zn, lp, n, l, gw, qw, h->stream)) != hipSuccess) return e;
      V = w.qb;
    } else {
      if ((e = getrf_run(w.zn, lp, n, l, gw, nullptr, nullptr, 0, 0, h->stream)) != hipSuccess)
        return e;
      if ((e = trace_getrf(h, gw, l)) != hipSuccess) return e;
      V = w.zn;
    }
  }
  *Vout = V;
  *passes = np;
  return hipSuccess;
}

// Alg. 5 steps 4-8 given Y = A V(:, :k) (leading dimension lp; w.ym unless Yin
// is given) and V.  Y is overwritten.  With kdev (device int32) the rank is
// *kdev <= k, read by the kernels: every launch is sized for k columns and
// stops at *kdev (the LUs take *kdev steps, the products reduce over *kdev
// terms), so the host never needs the rank; L columns and U rows from *kdev
// on are left unspecified.
hipError_t assemble(plu_handle h, const Ws& w, int64_t m, int64_t n, int k, const float* V,
                    int32_t* p, int32_t* q, float* L, int64_t ldl, float* U, int64_t ldu,
                    float* Yin = nullptr, const int32_t* kdev = nullptr) {
  const int64_t lp = w.lp;
  float* const Y = Yin ? Yin : w.ym;
  hipError_t e;
  GetrfWork g1 = getrf_work(h, w, 1);
  GetrfWork g2 = getrf_work(h, w, 2);
  g1.kcap = kdev;
  g2.kcap = kdev;
  // [L1, U1, P] = lu(Y): Y <- P^T L1, ut1 <- U1^T
  if ((e = getrf_run(Y, lp, m, k, g1, p, w.ut1, lp, 1, h->stream)) != hipSuccess) return e;
  if ((e = trace_getrf(h, g1, k)) != hipSuccess) return e;
  // B^T = V(:, :k) U1^T  (n x k)
  {
    GemmArgs g;
    g.A = V; g.lda = lp; g.X = w.ut1; g.ldx = lp; g.out = w.bt; g.ldo = lp;
    g.P = n; g.R = k; g.C = k;
    g.kcap = kdev; g.kc_red_off = 0;
    if ((e = launch_gemm(0, EPI_STORE, 0, g, plan_gemm(n, k, k, 1, 1), h->stream)) != hipSuccess)
      return e;
  }
  // [L2, U2, Q] = lu(B^T): bt <- Q^T L2, ut2 <- U2^T
  if ((e = getrf_run(w.bt, lp, n, k, g2, q, w.ut2, lp, 1, h->stream)) != hipSuccess) return e;
  if ((e = trace_getrf(h, g2, k)) != hipSuccess) return e;
  // L = L1 U2^T with L1 = (P^T L1)[p]
  {
    GemmArgs g;
    g.A = Y; g.lda = lp; g.arow = p; g.X = w.ut2; g.ldx = lp; g.out = L; g.ldo = ldl;
    g.P = m; g.R = k; g.C = k;
    g.kcap = kdev; g.kc_red_off = 0;
    if ((e = launch_gemm(0, EPI_STORE, 0, g, plan_gemm(m, k, k, 1, 1), h->stream)) != hipSuccess)
      return e;
  }
  // U = L2^T with L2 = (Q^T L2)[q]
  return launch_transpose_gather(w.bt, lp, q, n, k, U, ldu, h->stream, kdev);
}

// Host image of the small device results a call reports (status words,
// scalars, rank-rule integers, pivot gaps): offsets in bytes.
constexpr size_t kStageSt = 0, kStageSc = 160, kStageIs = 192, kStageGaps = 256;
size_t stage_bytes(int rank) { return kStageGaps + 8 * (size_t)std::max(rank, 0); }

// Queues the copies of that image into host memory `host` on stream s; the
// pivot gaps of the two final LUs take `rank` entries each (an upper bound
// on the rank when it is known only on the device).
hipError_t stage_info(const Ws& w, int rank, unsigned char* host, hipStream_t s) {
  hipError_t e;
  if ((e = hipMemcpyAsync(host + kStageSt, w.status, 40 * sizeof(int32_t), hipMemcpyDeviceToHost,
                          s)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(host + kStageSc, w.scal, 4 * sizeof(double), hipMemcpyDeviceToHost,
                          s)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(host + kStageIs, w.iscal, 2 * sizeof(int32_t), hipMemcpyDeviceToHost,
                          s)) != hipSuccess)
    return e;
  if (rank > 0) {
    if ((e = hipMemcpyAsync(host + kStageGaps, w.gaps1, rank * sizeof(float),
                            hipMemcpyDeviceToHost, s)) != hipSuccess)
      return e;
    if ((e = hipMemcpyAsync(host + kStageGaps + 4 * (size_t)rank, w.gaps2, rank * sizeof(float),
                            hipMemcpyDeviceToHost, s)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

// Fills *info from a host image of the results (see stage_info) holding
// nstage gaps per final LU, of which the first `rank` count.
int info_from_stage(const unsigned char* host, int status, int rank, int nstage, int passes, int l,
                    bool fp, plu_info* info) {
  int32_t st[40];
  double sc[4];
  std::memcpy(st, host + kStageSt, sizeof(st));
  std::memcpy(sc, host + kStageSc, sizeof(sc));
  std::memset(info, 0, sizeof(*info));
  info->rank = rank;
  info->passes = passes;
  info->l = l;
  info->normA2 = sc[0];
  info->E_final = fp ? sc[1] : 0.0;
  info->tol_reached = fp ? 1 : 0;
  int zp = INT32_MAX;
  const bool timeout = st[32] != 0;
  for (int wch = 1; wch <= 2; ++wch) zp = std::min(zp, st[4 * wch]);
  info->zero_pivot_step = (zp == INT32_MAX) ? -1 : zp;
  float mg = 1.f;
  for (int w = 0; w < 2; ++w)
    for (int i = 0; i < rank; ++i) {
      float x;
      std::memcpy(&x, host + kStageGaps + 4 * ((size_t)w * nstage + i), sizeof(x));
      mg = std::min(mg, x);
    }
  info->min_pivot_gap = mg;
  if (timeout) status = PLU_ERR_TIMEOUT;
  else if (!std::isfinite(sc[0])) status = PLU_ERR_NONFINITE;
  else if (status == PLU_OK && info->zero_pivot_step >= 0) status = PLU_WARN_ZERO_PIVOT;
  info->status = status;
  return status;
}

// Synchronizes and fills *info (nothing when info is NULL).  rank < 0: the
// rank is the device-side one of the fixed-precision rule (w.iscal), and the
// status is derived from it (TOL_NOT_REACHED when the rule did not stop).
int finish_info(plu_handle h, const Ws& w, int status, int rank, int passes, int l, bool fp,
                plu_info* info) {
  if (!info) return status;
  PLU_TRY_HIP(hipStreamSynchronize(h->stream));
  int32_t ks[2] = {0, 1};
  if (rank < 0) {
    PLU_TRY_HIP(hipMemcpy(ks, w.iscal, sizeof(ks), hipMemcpyDeviceToHost));
    rank = ks[0];
    if (status == PLU_OK && !ks[1]) status = PLU_TOL_NOT_REACHED;
  }
  // the fixed part of the image on the stack; the gaps' minimum in chunks
  // (no heap memory: plu_fixed_rank_static allocates nothing)
  unsigned char img[kStageGaps];
  PLU_TRY_HIP(hipMemcpy(img + kStageSt, w.status, 40 * sizeof(int32_t), hipMemcpyDeviceToHost));
  PLU_TRY_HIP(hipMemcpy(img + kStageSc, w.scal, 4 * sizeof(double), hipMemcpyDeviceToHost));
  float mg = 1.f;
  for (const float* gp : {w.gaps1, w.gaps2}) {
    float buf[512];
    for (int i0 = 0; i0 < rank; i0 += 512) {
      const int c = std::min(512, rank - i0);
      PLU_TRY_HIP(hipMemcpy(buf, gp + i0, c * sizeof(float), hipMemcpyDeviceToHost));
      for (int i = 0; i < c; ++i) mg = std::min(mg, buf[i]);
    }
  }
  const int st = info_from_stage(img, status, 0, 0, passes, l, fp, info);
  info->rank = rank;
  info->min_pivot_gap = mg;
  if (fp) info->tol_reached = ks[1] ? 1 : 0;
  return st;
}

void drop_graph(plu_handle h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->gexec = nullptr;
  h->graph = nullptr;
  h->gsig.clear();
  h->gbuf.destroy();
  for (auto& b : h->sgbuf) b.destroy();
}

// Checks one batched request; returns 0 or -(field index, from 1, in the
// declaration order of plu_request) and the sketch width in *l_out.
int check_request(const plu_request& r, int64_t* l_out) {
  if (r.mode != 0 && r.mode != 1) return -1;
  if (r.m <= 0) return -3;
  if (r.n <= 0) return -4;
  if (!valid_layout(r.layout)) return -22;
  if (r.lda < (r.layout == PLU_COL_MAJOR ? r.m : r.n)) return -5;
  if (!r.A || (reinterpret_cast<uintptr_t>(r.A) & 3u)) return -6;
  const int64_t mn = std::min(r.m, r.n);
  int64_t l = 0;
  if (r.mode == 0) {
    if (r.k < 1) return -7;
    if (r.p_over < 0) return -8;
    l = (int64_t)r.k + r.p_over;
    if (l >= mn) return -8;
  } else {
    if (r.b < 1) return -10;
    l = r.l ? r.l : std::min<int64_t>(50LL * r.b, r.b * ((mn - 1) / r.b));
    if (l <= 0 || l % r.b != 0 || l >= mn) return -11;
    if (!(r.eps > 0.0)) return -12;
  }
  if (r.v < 2) return -9;
  if (!valid_prec(r.prec)) return -13;
  if (!r.p) return -16;
  if (!r.q) return -17;
  if (!r.L) return -18;
  if (r.ldl < (r.mode == 0 ? r.k : l)) return -19;
  if (!r.U) return -20;
  if (r.ldu < r.n) return -21;
  *l_out = l;
  return 0;
}

// One problem of a batch: its own workspace region and launch record.
struct BatchProblem {
  plu_request* r = nullptr;
  int64_t l = 0;
  int prec = PLU_PREC_FP32;   // the request's precision form (its rounded
                              // copies are made in the problem's workspace)
  size_t off = 0, bytes = 0;
  plu_handle_s hs;
  Ws w{};
  Recorder rec;
  float* V = nullptr;
  int np = 0, nblk = 0, k = 0;
  bool ok = true;
};

// Steps of plu_fixed_rank or of plu_fixed_precision (its assembly at the
// rank the rule leaves on the device), recorded on the calling thread's
// recorder.
hipError_t batch_phase_a(BatchProblem& b) {
  plu_request& r = *b.r;
  plu_handle hs = &b.hs;
  hipError_t e;
  int st = ensure_ws(hs, r.m, r.n, b.l, &b.w, b.prec);
  if (st) return hipErrorOutOfMemory;
  b.w.acol = r.layout == PLU_COL_MAJOR;
  if ((e = range_basis(hs, b.w, r.m, r.n, r.A, r.lda, (int)b.l, r.v, r.Omega, r.seed, &b.V,
                       &b.np, b.prec)) != hipSuccess)
    return e;
  if (r.mode == 0) {
    if ((e = run_pass(hs, b.w, 0, r.m, r.n, r.A, r.lda, b.V, b.w.lp, r.k, b.w.ym, b.w.lp, nullptr,
                      nullptr, nullptr)) != hipSuccess)
      return e;
    ++b.np;
    return assemble(hs, b.w, r.m, r.n, r.k, b.V, r.p, r.q, r.L, r.ldl, r.U, r.ldu);
  }
  if ((e = run_pass(hs, b.w, 0, r.m, r.n, r.A, r.lda, b.V, b.w.lp, b.l, b.w.ym, b.w.lp, nullptr,
                    b.w.colsq_part, &b.nblk)) != hipSuccess)
    return e;
  ++b.np;
  if ((e = launch_splitk_reduce(b.V, 0, 1, nullptr, b.w.lp, r.n, b.l, b.w.vsq_part, 64,
                                hs->stream)) != hipSuccess)
    return e;
  if ((e = launch_rank_rule(b.w.colsq_part, b.nblk, (int)b.l, b.w.vsq_part, (int)((r.n + 63) / 64),
                            b.w.scal + 0, r.eps, r.b, r.column_exact ? 1 : 0, b.w.iscal + 0,
                            b.w.scal + 1, b.w.iscal + 1, b.w.colnorm, hs->stream)) != hipSuccess)
    return e;
  return assemble(hs, b.w, r.m, r.n, (int)b.l, b.V, r.p, r.q, r.L, r.ldl, r.U, r.ldu, nullptr,
                  b.w.iscal);
}

// Records fn(b) for every problem (each on its own recorder) and runs the
// merged sequence.
template <class F>
hipError_t record_and_run(plu_handle h, std::vector<BatchProblem*>& ps, F fn, MergeBuffers& buf,
                          bool dry_size_only, size_t* table_bytes) {
  std::vector<const Recorder*> lists;
  for (BatchProblem* b : ps) {
    b->rec.ops.clear();
    thread_recorder() = &b->rec;
    hipError_t e = fn(*b);
    thread_recorder() = nullptr;
    if (e != hipSuccess) return e;
    lists.push_back(&b->rec);
  }
  (void)dry_size_only;
  (void)table_bytes;
  return run_merged(lists, h->stream, h->cu_count, buf, nullptr);
}

hipError_t ensure_side_streams(plu_handle h) {
  if (h->fork_ev) return hipSuccess;
  hipError_t e;
  for (int i = 0; i < plu_handle_s::kSide; ++i) {
    if (!h->side[i] && (e = hipStreamCreateWithFlags(&h->side[i], hipStreamNonBlocking)) != hipSuccess)
      return e;
    if (!h->join_ev[i] &&
        (e = hipEventCreateWithFlags(&h->join_ev[i], hipEventDisableTiming)) != hipSuccess)
      return e;
  }
  return hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming);
}

// The problems of a batch side by side on up to kSide streams forked from
// the caller's stream (and joined back into it): the longest problem first,
// each to the least loaded stream (work estimated as m n l v).  A stream with
// one problem launches its kernels directly; a stream with several runs their
// merged launch sequence, unless one of them is in a rounded precision form:
// the reduced-precision kernels are launched directly (they are not recorded
// for merging), so such a stream runs its problems directly, one after the
// other.  The LU panels' workgroups wait on each other, so the merged panels
// of one stream are held to cu_count / streams workgroups at a time, and a
// direct problem's panel has at most 64: the panels in flight at once always
// fit on the device.
struct SidePlan {
  int S = 0;
  std::vector<std::vector<BatchProblem*>> groups;
  std::vector<std::vector<const Recorder*>> lists;
  std::vector<char> direct;
};

bool rounded_form(const BatchProblem* b) {
  return (b->prec & PLU_PREC_FORMAT_MASK) != PLU_PREC_FP32;
}

// Partition, recording of the merged streams' launches, and (for a graph
// capture, which may allocate nothing) their table buffers: all before any
// launch or capture.
hipError_t side_prepare(plu_handle h, std::vector<BatchProblem*>& all, bool capture,
                        SidePlan& sp) {
  hipError_t e;
  if ((e = ensure_side_streams(h)) != hipSuccess) return e;
  sp.S = (int)std::min<size_t>(plu_handle_s::kSide, all.size());
  std::vector<BatchProblem*> order(all);
  auto work = [](const BatchProblem* b) {
    return (double)b->r->m * (double)b->r->n * (double)b->l * (double)b->r->v;
  };
  std::stable_sort(order.begin(), order.end(),
                   [&](const BatchProblem* a, const BatchProblem* b) { return work(a) > work(b); });
  sp.groups.assign((size_t)sp.S, {});
  sp.lists.assign((size_t)sp.S, {});
  std::vector<double> load((size_t)sp.S, 0.0);
  for (BatchProblem* b : order) {
    const size_t g = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
    sp.groups[g].push_back(b);
    load[g] += work(b);
  }
  sp.direct.assign((size_t)sp.S, 0);
  for (int g = 0; g < sp.S; ++g) {
    const auto& grp = sp.groups[(size_t)g];
    sp.direct[(size_t)g] =
        grp.size() < 2 || std::any_of(grp.begin(), grp.end(), rounded_form) ? 1 : 0;
    if (sp.direct[(size_t)g]) continue;
    for (BatchProblem* b : sp.groups[(size_t)g]) {
      b->rec.ops.clear();
      thread_recorder() = &b->rec;
      e = batch_phase_a(*b);
      thread_recorder() = nullptr;
      if (e != hipSuccess) return e;
      sp.lists[(size_t)g].push_back(&b->rec);
    }
    if (capture &&
        (e = h->sgbuf[g].reserve(merged_table_bytes(sp.lists[(size_t)g], h->cu_count / sp.S))) !=
            hipSuccess)
      return e;
  }
  return hipSuccess;
}

// The launches of a prepared batch, forked from and joined into stream s
// (capture: s is capturing a graph; the merged tables live in the buffers
// kept for it).
hipError_t side_launch(plu_handle h, hipStream_t s, SidePlan& sp, bool capture) {
  hipError_t e;
  if ((e = hipEventRecord(h->fork_ev, s)) != hipSuccess) return e;
  for (int g = 0; g < sp.S; ++g)
    if ((e = hipStreamWaitEvent(h->side[g], h->fork_ev, 0)) != hipSuccess) return e;
  for (int g = 0; g < sp.S; ++g) {
    if (sp.direct[(size_t)g]) {
      for (BatchProblem* b : sp.groups[(size_t)g]) {
        b->hs.stream = h->side[g];
        if ((e = batch_phase_a(*b)) != hipSuccess) return e;
      }
    } else {
      MergeBuffers& buf = capture ? h->sgbuf[g] : h->sbuf[g];
      buf.capturing = capture;
      e = run_merged(sp.lists[(size_t)g], h->side[g], h->cu_count / sp.S, buf, nullptr);
      buf.capturing = false;
      if (e != hipSuccess) return e;
    }
  }
  for (int g = 0; g < sp.S; ++g) {
    if ((e = hipEventRecord(h->join_ev[g], h->side[g])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s, h->join_ev[g], 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Inputs of a batch that decide its launch sequence (for graph reuse).
std::vector<unsigned char> batch_signature(const plu_request* reqs, int count) {
  std::vector<unsigned char> sig;
  const size_t in_bytes = offsetof(plu_request, rank);
  sig.resize((size_t)count * in_bytes);
  for (int i = 0; i < count; ++i)
    std::memcpy(sig.data() + (size_t)i * in_bytes, &reqs[i], in_bytes);
  return sig;
}

// ---------------------------------------------------------------------------
// Serving loop.
// ---------------------------------------------------------------------------
double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// First-fit sub-allocator over one device block (the HBM budget).
struct Pool {
  char* base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_;   // offset -> length
  bool init(size_t bytes) {
    if (hipMalloc(reinterpret_cast<void**>(&base), bytes) != hipSuccess) {
      (void)hipGetLastError();
      base = nullptr;
      return false;
    }
    size = bytes;
    free_[0] = bytes;
    return true;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, o = it->first + bytes;
        free_.erase(it);
        if (rest) free_[o] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct ServerJob {
  uint64_t ticket = 0;
  plu_request host{};          // the client's request (host pointers)
  plu_request dev{};           // the same problem on device copies
  int64_t cap = 0;             // columns of L / rows of U
  size_t pool_off = 0, pool_bytes = 0, ws_off = 0, ws_bytes = 0;
  BatchProblem bp;
  size_t head = 0;
  uint64_t done_seq = 0;       // the launch batch holding its last step
  bool waiting = false;        // all recorded steps issued, waiting for ev
  int slot = -1;               // its slot: index of its pinned result image
  hipEvent_t up = nullptr;     // recorded after the copy of A on the upload stream
  bool uploaded = false;       // that copy has landed: its steps may be issued
  double t_up = 0, t_issued = 0, t_computed = 0;   // server-side timestamps
  int lane = 0;                // the stream its launches go to
  double work = 0;             // m n l v: its share of that lane's load
  bool direct = false;         // a rounded precision form: not recorded; all
                               // its launches go out at its first issue
  plu_result res{};
};

// Elements of the device copy of A when it is the whole span of a strided
// host block (from its first to its last element, one contiguous copy, kept
// with the host's stride), else 0 (the block's own m n entries).  Strided
// host-to-device copies run at about a fifth of the contiguous rate
// (measured 11.7 against 57 GB/s from pinned memory), so a stride up to 3x
// the row length is cheaper to copy whole.
int64_t a_span_elems(const plu_request& r) {
  const bool col = r.layout == PLU_COL_MAJOR;
  const int64_t inner = col ? r.m : r.n, outer = col ? r.n : r.m;
  if (r.lda > inner && r.lda <= 3 * inner) return (outer - 1) * r.lda + inner;
  return 0;
}

size_t server_footprint(const plu_request& r, int64_t l, int64_t cap, size_t* ws_bytes) {
  Layout dry;
  layout(dry, r.m, r.n, l, r.prec & ~PLU_PREC_A_UNCHANGED);
  *ws_bytes = (size_t)ru((int64_t)(dry.off + 256), 256);
  auto a = [](size_t x) { return (x + 255) & ~size_t(255); };
  const int64_t span = a_span_elems(r);
  const size_t abytes = span ? (size_t)span * 4 : (size_t)r.m * r.n * 4;
  return a(abytes) + a((size_t)r.m * 4) + a((size_t)r.n * 4) +
         a((size_t)r.m * cap * 4) + a((size_t)cap * r.n * 4) + *ws_bytes;
}

}  // namespace

// A sparse matrix bound to a device: the caller's compressed rows and the
// compressed columns and ||A||_F^2 built from them.
struct plu_sparse_s {
  int device = 0;
  SparseMat mat;
  void* mem = nullptr;
};

struct plu_server_s {
  plu_handle h = nullptr;
  hipStream_t stream = nullptr;    // compute stream (all recorded steps)
  hipStream_t ustream = nullptr;   // upload stream (copies of A)
  // finisher threads, each with its copy-out stream and pinned staging of
  // strided results
  struct Finisher {
    hipStream_t cs = nullptr;
    unsigned char* ostage = nullptr;
    size_t cap = 0;
    std::thread th;
  };
  std::vector<Finisher> fins;
  Pool pool;
  // per slot: pinned host image of a problem's small results (stage_info),
  // written by copies queued on the compute stream behind its last step
  std::vector<unsigned char*> stage;
  std::vector<size_t> stage_cap;
  std::vector<int> free_slots;
  int max_slots = 1;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_fin;
  std::deque<std::unique_ptr<ServerJob>> pending;
  std::vector<std::unique_ptr<ServerJob>> active;    // admitted, steps in flight
  std::deque<ServerJob*> finishing;                  // all steps done, copy-out queued
  int nfinishing = 0;                                // in finishing or being copied out
  std::map<uint64_t, plu_result> done;
  std::vector<hipEvent_t> events;                    // free event objects
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  int device = 0;
  int fatal = 0;
  MergeStats stats;       // grouped launches and the steps they carried
  size_t batches = 0;
  // worker-thread time (seconds): idle, waiting for the device, recording
  // admitted problems, planning and issuing launch groups; and the sum over
  // batches of the problems with steps left
  double t_idle = 0, t_devwait = 0, t_record = 0, t_issue = 0;
  double t_copyout = 0;   // finisher thread: copying results out
  // sums over problems: admission to upload landed, to last step issued, to
  // last step complete, to copied out
  double s_up = 0, s_issue = 0, s_compute = 0, s_out = 0;
  size_t n_done = 0;
  size_t sum_ready = 0, sum_active = 0, sum_pending = 0, budget_stops = 0;
};

namespace {

hipEvent_t take_event(plu_server S) {
  std::lock_guard<std::mutex> lk(S->mu);
  if (!S->events.empty()) {
    hipEvent_t e = S->events.back();
    S->events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

// Admits requests, records their steps and keeps the compute stream fed with
// merged launch groups; finished requests go to the finisher thread.  At most
// two launch batches are queued ahead of the device, so arrivals join soon.
void server_loop(plu_server S) {
  (void)hipSetDevice(S->device);
  plu_handle h = S->h;
  constexpr size_t kGroupsPerIter = 32;
  // Admitted problems are spread over lanes, one stream each (the handle's
  // side streams), least loaded first: one lane's LU panels and thin QRs
  // overlap the passes of the others.  Within a lane the problems' launch
  // sequences are merged continuously.  A lane's merged LU panels are held
  // to cu_count / lanes workgroups, so all panels in flight fit at once.
  constexpr int kLanes = plu_handle_s::kSide;
  if (ensure_side_streams(h) != hipSuccess) {
    std::fprintf(stderr, "libpowerlu server: could not create its streams\n");
    std::lock_guard<std::mutex> lk(S->mu);
    S->fatal = PLU_ERR_HIP;
  }
  auto lane_stream = [&](int ln) { return h->side[ln] ? h->side[ln] : S->stream; };
  // per lane: issued launch batches (sequence number, event recorded after
  // it), oldest first; a lane's batches complete in order on its stream
  std::array<std::deque<std::pair<uint64_t, hipEvent_t>>, kLanes> inflight;
  std::array<uint64_t, kLanes> seq{}, completed{};
  std::array<double, kLanes> load{};
  // retires a lane's completed batches; with block, waits for its oldest
  // first.  An event goes back to the pool only here, once nothing refers to it.
  auto retire = [&](int ln, bool block) {
    bool first = true;
    bool any = false;
    while (!inflight[ln].empty()) {
      hipEvent_t e = inflight[ln].front().second;
      if (!e) {   // no event could be recorded (reported as fatal)
        completed[ln] = inflight[ln].front().first;
        inflight[ln].pop_front();
        any = true;
        continue;
      }
      if (block && first) {
        const auto tw = std::chrono::steady_clock::now();
        (void)hipEventSynchronize(e);
        S->t_devwait += std::chrono::duration<double>(std::chrono::steady_clock::now() - tw).count();
      } else if (hipEventQuery(e) != hipSuccess) {
        break;
      }
      first = false;
      any = true;
      completed[ln] = inflight[ln].front().first;
      inflight[ln].pop_front();
      std::lock_guard<std::mutex> lk(S->mu);
      S->events.push_back(e);
    }
    return any;
  };
  auto inflight_any = [&] {
    for (auto& q : inflight)
      if (!q.empty()) return true;
    return false;
  };
  auto ready = [](const ServerJob* j) { return j->uploaded && !j->waiting; };
  for (;;) {
    // copies of A that have landed (only this thread changes `active`)
    hipEvent_t upwait = nullptr;
    for (auto& up : S->active) {
      ServerJob* j = up.get();
      if (j->uploaded) continue;
      if (!j->up) {   // the upload failed (reported as fatal)
        j->uploaded = true;
        continue;
      }
      if (hipEventQuery(j->up) == hipSuccess) {
        j->uploaded = true;
        j->t_up = now_s(S->t0);
        std::lock_guard<std::mutex> lk(S->mu);
        S->events.push_back(j->up);
        j->up = nullptr;
      } else if (!upwait) {
        upwait = j->up;
      }
    }
    std::vector<ServerJob*> admitted;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      bool runnable = false;
      for (auto& up : S->active)
        if (ready(up.get())) runnable = true;
      if (!runnable && !inflight_any() && !upwait) {
        const auto tw = std::chrono::steady_clock::now();
        S->cv_work.wait(lk, [&] {
          bool r = false;
          for (auto& up : S->active)
            if (ready(up.get())) r = true;
          return S->stop || r ||
                 (!S->pending.empty() &&
                  (int)S->active.size() + S->nfinishing < S->max_slots);
        });
        S->t_idle += std::chrono::duration<double>(std::chrono::steady_clock::now() - tw).count();
      }
      if (S->stop && S->pending.empty() && S->active.empty() && S->nfinishing == 0 &&
          !inflight_any())
        return;
      // a slot is held from admission until the result is copied out
      while (!S->pending.empty() && (int)S->active.size() + S->nfinishing < S->max_slots) {
        ServerJob* j = S->pending.front().get();
        size_t off = 0;
        if (!S->pool.alloc(j->pool_bytes, &off)) {
          ++S->budget_stops;
          break;
        }
        j->pool_off = off;
        j->slot = S->free_slots.back();
        S->free_slots.pop_back();
        j->res.t_admit = now_s(S->t0);
        S->active.push_back(std::move(S->pending.front()));
        S->pending.pop_front();
        admitted.push_back(j);
      }
    }
    const auto trec = std::chrono::steady_clock::now();
    for (ServerJob* j : admitted) {
      char* b = S->pool.base + j->pool_off;
      auto take = [&](size_t bytes) {
        char* p = b;
        b += (bytes + 255) & ~size_t(255);
        return p;
      };
      plu_request& r = j->host;
      plu_request& d = j->dev;
      d = r;
      // the device copy keeps the request's storage order, packed, or the
      // whole span of a strided block with the host's stride
      const int64_t span = a_span_elems(r);
      d.A = reinterpret_cast<float*>(take(span ? (size_t)span * 4 : (size_t)r.m * r.n * 4));
      const bool col = r.layout == PLU_COL_MAJOR;
      const int64_t inner = col ? r.m : r.n, outer = col ? r.n : r.m;
      d.lda = span ? r.lda : inner;
      d.p = reinterpret_cast<int32_t*>(take((size_t)r.m * 4));
      d.q = reinterpret_cast<int32_t*>(take((size_t)r.n * 4));
      d.L = reinterpret_cast<float*>(take((size_t)r.m * j->cap * 4));
      d.ldl = j->cap;
      d.U = reinterpret_cast<float*>(take((size_t)j->cap * r.n * 4));
      d.ldu = r.n;
      d.Omega = nullptr;
      char* ws = take(j->ws_bytes);
      const size_t sneed = stage_bytes((int)j->cap);
      if (S->stage_cap[j->slot] < sneed) {
        // the slot is free: no copy into its old image is in flight
        if (S->stage[j->slot]) (void)hipHostFree(S->stage[j->slot]);
        S->stage[j->slot] = nullptr;
        S->stage_cap[j->slot] = 0;
        const size_t c = std::max<size_t>(sneed + sneed / 2, 16384);
        if (hipHostMalloc(reinterpret_cast<void**>(&S->stage[j->slot]), c,
                          hipHostMallocDefault) == hipSuccess)
          S->stage_cap[j->slot] = c;
        else {
          S->stage[j->slot] = nullptr;
          std::lock_guard<std::mutex> lk(S->mu);
          S->fatal = PLU_ERR_OOM;
        }
      }
      // A goes up on its own stream, overlapping the steps of other problems
      hipError_t eu;
      if (span)
        eu = hipMemcpyAsync(const_cast<float*>(d.A), r.A, (size_t)span * 4,
                            hipMemcpyHostToDevice, S->ustream);
      else if (r.lda == inner)
        eu = hipMemcpyAsync(const_cast<float*>(d.A), r.A, (size_t)r.m * r.n * 4,
                            hipMemcpyHostToDevice, S->ustream);
      else
        eu = hipMemcpy2DAsync(const_cast<float*>(d.A), (size_t)inner * 4, r.A,
                              (size_t)r.lda * 4, (size_t)inner * 4, (size_t)outer,
                              hipMemcpyHostToDevice, S->ustream);
      j->up = take_event(S);
      j->uploaded = false;
      if (eu == hipSuccess && j->up) eu = hipEventRecord(j->up, S->ustream);
      if (eu != hipSuccess || !j->up) {
        std::fprintf(stderr, "libpowerlu server: upload: %s\n", hipGetErrorString(eu));
        std::lock_guard<std::mutex> lk(S->mu);
        S->fatal = PLU_ERR_HIP;
      }
      BatchProblem& bp = j->bp;
      bp.r = &d;
      bp.hs = *h;
      bp.hs.stream = S->stream;
      bp.hs.arena = ws;
      bp.hs.arena_bytes = j->ws_bytes;
      bp.hs.tag_counter = 0;
      bp.hs.batch_arena = nullptr;
      bp.hs.graph = nullptr;
      bp.hs.gexec = nullptr;
      bp.hs.gstream = nullptr;
      bp.hs.trace_cap = 0;
      bp.hs.mbuf = MergeBuffers();
      bp.hs.gbuf = MergeBuffers();
      int64_t l = 0;
      (void)check_request(d, &l);
      bp.l = l;
      // a rounded form makes its copies of A in its own workspace each time
      bp.prec = d.prec & ~PLU_PREC_A_UNCHANGED;
      j->direct = rounded_form(&bp);
      j->work = (double)d.m * (double)d.n * (double)l * (double)d.v;
      j->lane = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[(size_t)j->lane] += j->work;
      {
        // splits of large passes tuned eagerly (on this problem's workspace,
        // once A has landed), so the recorded launches equal the single calls
        Layout L;
        L.base = ws;
        Ws w = layout(L, d.m, d.n, l, bp.prec);
        w.acol = d.layout == PLU_COL_MAJOR;
        // (only a size class not tuned yet waits for the copy of A)
        if (pass_needs_tuning(&bp.hs, w, 0, d.m, d.n, l) ||
            pass_needs_tuning(&bp.hs, w, 1, d.m, d.n, l) ||
            (d.mode == 0 && pass_needs_tuning(&bp.hs, w, 0, d.m, d.n, d.k))) {
          if (j->up) (void)hipEventSynchronize(j->up);
          pretune_pass(&bp.hs, w, 0, d.m, d.n, d.A, d.lda, w.om, w.lp, l, w.ym, w.lp);
          pretune_pass(&bp.hs, w, 1, d.m, d.n, d.A, d.lda, w.om, w.lp, l, w.zn, w.lp);
          if (d.mode == 0)
            pretune_pass(&bp.hs, w, 0, d.m, d.n, d.A, d.lda, w.om, w.lp, d.k, w.ym, w.lp);
        }
      }
      bp.rec.ops.clear();
      hipError_t e = hipSuccess;
      if (!j->direct) {
        thread_recorder() = &bp.rec;
        e = batch_phase_a(bp);
        thread_recorder() = nullptr;
      }
      j->head = 0;
      j->waiting = false;
      if (e != hipSuccess) j->res.status = PLU_ERR_HIP;
    }
    S->t_record += std::chrono::duration<double>(std::chrono::steady_clock::now() - trec).count();
    // per lane: issue one batch of merged groups over its problems with
    // steps left
    bool issued = false;
    for (int ln = 0; ln < kLanes; ++ln) {
      std::vector<const Recorder*> lists;
      std::vector<size_t> heads;
      std::vector<ServerJob*> js, direct;
      for (auto& up : S->active)
        if (up->lane == ln && ready(up.get())) {
          if (up->direct) {
            direct.push_back(up.get());
            continue;
          }
          lists.push_back(&up->bp.rec);
          heads.push_back(up->head);
          js.push_back(up.get());
        }
      if (js.empty() && direct.empty()) continue;
      issued = true;
      const hipStream_t ls = lane_stream(ln);
      // bound the lane's queue: wait for its batch before last
      while (inflight[ln].size() >= 2) retire(ln, true);
      const auto ti = std::chrono::steady_clock::now();
      hipError_t e = hipSuccess;
      // rounded-form problems: every launch of the single call, in order, on
      // the lane's stream (their kernels are not recorded for merging)
      for (ServerJob* j : direct) {
        j->bp.hs.stream = ls;
        if ((e = batch_phase_a(j->bp)) != hipSuccess) break;
      }
      if (e == hipSuccess && !js.empty())
        e = run_merged_steps(lists, heads, ls, h->cu_count / kLanes, kGroupsPerIter, h->sbuf[ln],
                             &S->stats);
      // problems with all steps issued: queue the copies of their small
      // results behind them, so that the event below covers those too
      for (ServerJob* j : direct) {
        if (e != hipSuccess || !S->stage[j->slot]) continue;
        const int nst = j->dev.mode == 0 ? j->dev.k : (int)j->bp.l;
        e = stage_info(j->bp.w, nst, S->stage[j->slot], ls);
      }
      for (size_t i = 0; i < js.size() && e == hipSuccess; ++i) {
        ServerJob* j = js[i];
        if (heads[i] < j->bp.rec.ops.size() || !S->stage[j->slot]) continue;
        // the gaps of both final LUs: k steps, or up to l for a rank on the device
        const int nst = j->dev.mode == 0 ? j->dev.k : (int)j->bp.l;
        e = stage_info(j->bp.w, nst, S->stage[j->slot], ls);
      }
      S->t_issue += std::chrono::duration<double>(std::chrono::steady_clock::now() - ti).count();
      ++S->batches;
      S->sum_ready += js.size() + direct.size();
      S->sum_active += S->active.size();
      {
        std::lock_guard<std::mutex> lk(S->mu);
        S->sum_pending += S->pending.size();
      }
      hipEvent_t ev = take_event(S);
      if (e == hipSuccess && ev) e = hipEventRecord(ev, ls);
      if (e != hipSuccess || !ev) {
        std::fprintf(stderr, "libpowerlu server: %s\n", hipGetErrorString(e));
        std::lock_guard<std::mutex> lk(S->mu);
        S->fatal = PLU_ERR_HIP;
      }
      inflight[ln].push_back({++seq[ln], ev});
      for (ServerJob* j : direct) {
        j->waiting = true;
        j->done_seq = seq[ln];
        j->t_issued = now_s(S->t0);
      }
      for (size_t i = 0; i < js.size(); ++i) {
        js[i]->head = heads[i];
        if (js[i]->head >= js[i]->bp.rec.ops.size()) {
          js[i]->waiting = true;
          js[i]->done_seq = seq[ln];
          js[i]->t_issued = now_s(S->t0);
        }
      }
    }
    if (!issued) {
      if (inflight_any()) {
        // nothing to issue: wait until some lane's oldest batch completes
        const auto tw = std::chrono::steady_clock::now();
        for (;;) {
          bool any = false;
          for (int ln = 0; ln < kLanes; ++ln) any |= retire(ln, false);
          if (any || !inflight_any()) break;
          std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        S->t_devwait += std::chrono::duration<double>(std::chrono::steady_clock::now() - tw).count();
      } else if (upwait) {
        // nothing to issue until a copy of A lands
        const auto tw = std::chrono::steady_clock::now();
        (void)hipEventSynchronize(upwait);
        S->t_devwait += std::chrono::duration<double>(std::chrono::steady_clock::now() - tw).count();
      }
    }
    // problems whose steps are all complete
    for (int ln = 0; ln < kLanes; ++ln) retire(ln, false);
    std::vector<ServerJob*> to_finish;
    for (auto& up : S->active) {
      ServerJob* j = up.get();
      if (!j->waiting) continue;
      if (!S->fatal && completed[(size_t)j->lane] < j->done_seq) continue;
      to_finish.push_back(j);
      load[(size_t)j->lane] -= j->work;
    }
    if (!to_finish.empty()) {
      std::lock_guard<std::mutex> lk(S->mu);
      for (ServerJob* j : to_finish) {
        for (auto it = S->active.begin(); it != S->active.end(); ++it)
          if (it->get() == j) {
            it->release();
            S->active.erase(it);
            break;
          }
        j->t_computed = now_s(S->t0);
        S->finishing.push_back(j);
        ++S->nfinishing;
      }
      S->cv_fin.notify_all();
    }
  }
}

// Copies finished problems out (host buffers of the client), fills their
// results and frees their device memory, off the launch thread.
void server_finisher(plu_server S, int idx) {
  plu_server_s::Finisher& F = S->fins[idx];
  (void)hipSetDevice(S->device);
  for (;;) {
    ServerJob* j = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_fin.wait(lk, [&] { return !S->finishing.empty() || (S->stop && S->active.empty() &&
                                                                 S->pending.empty()); });
      if (S->finishing.empty()) return;
      j = S->finishing.front();
      S->finishing.pop_front();
    }
    const plu_request& d = j->dev;
    const plu_request& r = j->host;
    BatchProblem& bp = j->bp;
    int k = d.mode == 0 ? d.k : 0;
    int fatal = 0;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      fatal = S->fatal;
    }
    const auto tc = std::chrono::steady_clock::now();
    if (!fatal) {
      const unsigned char* img = S->stage[j->slot];
      int st = PLU_OK;
      if (d.mode == 1) {
        int32_t ks[2];
        double sc;
        std::memcpy(ks, img + kStageIs, sizeof(ks));
        std::memcpy(&sc, img + kStageSc, sizeof(sc));
        st = !std::isfinite(sc) ? PLU_ERR_NONFINITE : ks[1] ? PLU_OK : PLU_TOL_NOT_REACHED;
        k = std::min<int>(ks[0], (int)j->cap);
      }
      const int nst = d.mode == 0 ? k : (int)bp.l;
      j->res.status = info_from_stage(img, st, k, nst, d.v, (int)bp.l, d.mode == 1, &j->res.info);
      if (d.mode == 1) j->res.info.tol_reached = st == PLU_OK ? 1 : 0;
      j->res.rank = k;
      // p, q and contiguous blocks straight into the client's memory; a
      // strided block (fewer than ld columns) through pinned staging: copies
      // of strided rows into pageable memory go row by row
      hipError_t e = hipMemcpyAsync(r.p, d.p, (size_t)r.m * 4, hipMemcpyDeviceToHost, F.cs);
      if (e == hipSuccess)
        e = hipMemcpyAsync(r.q, d.q, (size_t)r.n * 4, hipMemcpyDeviceToHost, F.cs);
      struct Blk {
        float* dst;
        int64_t ldd;
        const float* src;
        int64_t lds, rows, cols;
      };
      const Blk blks[2] = {{r.L, r.ldl, d.L, d.ldl, r.m, k}, {r.U, r.ldu, d.U, d.ldu, k, r.n}};
      for (const Blk& bk : blks) {
        if (k <= 0 || e != hipSuccess) break;
        const size_t row = (size_t)bk.cols * 4, bytes = row * (size_t)bk.rows;
        if (bk.ldd == bk.cols && bk.lds == bk.cols) {
          e = hipMemcpyAsync(bk.dst, bk.src, bytes, hipMemcpyDeviceToHost, F.cs);
          continue;
        }
        if (F.cap < bytes) {
          if ((e = hipStreamSynchronize(F.cs)) != hipSuccess) break;
          if (F.ostage) (void)hipHostFree(F.ostage);
          F.ostage = nullptr;
          F.cap = 0;
          const size_t c = bytes + bytes / 2;
          if ((e = hipHostMalloc(reinterpret_cast<void**>(&F.ostage), c, hipHostMallocDefault)) !=
              hipSuccess) {
            F.ostage = nullptr;
            break;
          }
          F.cap = c;
        }
        e = hipMemcpy2DAsync(F.ostage, row, bk.src, (size_t)bk.lds * 4, row, (size_t)bk.rows,
                             hipMemcpyDeviceToHost, F.cs);
        if (e == hipSuccess) e = hipStreamSynchronize(F.cs);
        if (e != hipSuccess) break;
        for (int64_t i = 0; i < bk.rows; ++i)
          std::memcpy(bk.dst + i * bk.ldd, F.ostage + i * row, row);
      }
      if (e == hipSuccess) e = hipStreamSynchronize(F.cs);
      if (e != hipSuccess) j->res.status = PLU_ERR_HIP;
    } else {
      j->res.status = fatal;
    }
    j->res.t_done = now_s(S->t0);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->t_copyout += std::chrono::duration<double>(std::chrono::steady_clock::now() - tc).count();
      S->done[j->ticket] = j->res;
      S->s_up += j->t_up - j->res.t_admit;
      S->s_issue += j->t_issued - j->t_up;
      S->s_compute += j->t_computed - j->t_issued;
      S->s_out += j->res.t_done - j->t_computed;
      ++S->n_done;
      S->pool.release(j->pool_off, j->pool_bytes);
      S->free_slots.push_back(j->slot);
      --S->nfinishing;
      S->cv_done.notify_all();
      S->cv_work.notify_one();   // memory freed: admission may proceed
    }
    delete j;
  }
}


// PowerLU_FP with restarts (the Remark after Alg. 8): when a round's l
// columns miss the tolerance, the next round draws a fresh Gaussian matrix
// (on the device, from seed + round) and runs Alg. 7 on the remainder
// A (I - V V^T) of the basis V kept so far.  The new block is projected out
// of V twice and re-orthonormalized, its G block is A times it, and the
// Thm 4.3 indicator continues over the concatenated columns.  V and G
// accumulate in w.vall and w.gall; the assembly (Alg. 9 steps 2-6) runs on
// their first k columns.  One synchronization per round reads its rank.
int fixed_precision_rounds(plu_handle h, const Ws& w, int64_t m, int64_t n, const float* A,
                           int64_t lda, double eps, int b, int l, int v, int column_exact,
                           int rounds, int prec, const float* Omega, uint64_t seed, int32_t* p,
                           int32_t* q, float* L, int64_t ldl, float* U, int64_t ldu,
                           int32_t* rank_dev, plu_info* info) {
  const int64_t lp = w.lp;
  const GetrfWork gw = getrf_work(h, w, 0);
  const QrWork qw = qr_work(w, w.qb, lp);
  const size_t rowb = (size_t)l * sizeof(float), pitch = (size_t)lp * sizeof(float);
  int np = 0, k = 0;
  bool tol_ok = false;
  int64_t off = 0;
  double sc[2] = {0.0, 0.0};
  for (int r = 0; r < rounds; ++r) {
    float* V = nullptr;
    int npr = 0;
    // later rounds keep the rounded copies of A the first one made
    PLU_TRY_HIP(range_basis(h, w, m, n, A, lda, l, v, r == 0 ? Omega : nullptr,
                            seed + (uint64_t)r, &V, &npr, r == 0 ? prec : prec | PLU_PREC_A_UNCHANGED,
                            w.vall, w.gall, off));
    np += npr;
    float* Vr = w.vall + off;
    PLU_TRY_HIP(hipMemcpy2DAsync(Vr, pitch, V, pitch, rowb, n, hipMemcpyDeviceToDevice,
                                 h->stream));
    if (off > 0) {
      for (int rep = 0; rep < 2; ++rep)
        PLU_TRY_HIP(project_out(h, w, w.vall, w.vall, lp, off, n, n, Vr, lp, l, Vr, lp, w.bt, lp));
      PLU_TRY_HIP(thin_qr_run(Vr, lp, n, l, gw, qw, h->stream));   // orthonormal block in w.qb
      PLU_TRY_HIP(hipMemcpy2DAsync(Vr, pitch, w.qb, pitch, rowb, n, hipMemcpyDeviceToDevice,
                                   h->stream));
    }
    // G block = A V_r with float64 column energies, and the basis columns' norms
    int nblk = 0;
    PLU_TRY_HIP(run_pass(h, w, 0, m, n, A, lda, Vr, lp, l, w.gall + off, lp, nullptr,
                         w.colsq_part, &nblk));
    ++np;
    PLU_TRY_HIP(launch_splitk_reduce(Vr, 0, 1, nullptr, lp, n, l, w.vsq_part, 64, h->stream));
    PLU_TRY_HIP(launch_rank_rule(w.colsq_part, nblk, l, w.vsq_part, (int)((n + 63) / 64),
                                 w.scal + 0, eps, b, column_exact ? 1 : 0, w.iscal + 0, w.scal + 1,
                                 w.iscal + 1, w.colnorm, h->stream, r == 0 ? nullptr : w.scal + 1));
    PLU_TRY_HIP(hipStreamSynchronize(h->stream));
    int32_t ks[2];
    PLU_TRY_HIP(hipMemcpy(ks, w.iscal, sizeof(ks), hipMemcpyDeviceToHost));
    PLU_TRY_HIP(hipMemcpy(sc, w.scal, sizeof(sc), hipMemcpyDeviceToHost));
    if (!std::isfinite(sc[0])) {
      if (info) {
        std::memset(info, 0, sizeof(*info));
        info->status = PLU_ERR_NONFINITE;
        info->normA2 = sc[0];
      }
      return PLU_ERR_NONFINITE;
    }
    tol_ok = ks[1] != 0;
    k = (int)off + ks[0];
    if (tol_ok) break;
    off += l;
  }
  if (rank_dev)
    PLU_TRY_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(rank_dev), 1, (uint32_t)k, h->stream));
  const int status = tol_ok ? PLU_OK : PLU_TOL_NOT_REACHED;
  if (k == 0) {
    PLU_TRY_HIP(launch_iota(p, m, h->stream));
    PLU_TRY_HIP(launch_iota(q, n, h->stream));
  } else {
    PLU_TRY_HIP(assemble(h, w, m, n, k, w.vall, p, q, L, ldl, U, ldu, w.gall));
  }
  int rs = finish_info(h, w, status, k, np, l, true, info);
  if (info) info->tol_reached = tol_ok ? 1 : 0;
  return info ? rs : status;
}

}  // namespace

extern "C" {

const char* plu_status_string(int status) {
  switch (status) {
    case PLU_OK: return "ok";
    case PLU_WARN_ZERO_PIVOT: return "zero pivot met (result still produced)";
    case PLU_TOL_NOT_REACHED: return "tolerance not reached with l columns";
    case PLU_ERR_NONFINITE: return "input holds NaN or Inf";
    case PLU_ERR_OOM: return "device workspace allocation failed";
    case PLU_ERR_HIP: return "HIP runtime error";
    case PLU_ERR_NOT_IMPLEMENTED: return "not implemented";
    case PLU_ERR_TIMEOUT: return "device-side wait exceeded its bound";
    case PLU_PENDING: return "pending";
    case PLU_ERR_TOO_LARGE: return "the problem needs more workspace than the static scratch holds";
    default: return status < 0 ? "invalid argument" : "unknown status";
  }
}

int plu_create(plu_handle* out, int device, void* hip_stream) {
  if (!out) return -1;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return -2;
  plu_handle h = new plu_handle_s();
  h->device = device;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  PLU_TRY_HIP(hipSetDevice(device));
  int cus = 0, coop = 0, clk_khz = 0;
  PLU_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  PLU_TRY_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device));
  PLU_TRY_HIP(hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, device));
  if (!coop) {
    delete h;
    return PLU_ERR_NOT_IMPLEMENTED;
  }
  h->cu_count = cus > 0 ? cus : 256;
  {
    // this device's copy of `scratch`, looked up once per device (with the
    // device current) and kept for the process
    static std::mutex mu;
    static void* addr[256] = {};
    std::lock_guard<std::mutex> lk(mu);
    if (device < 256 && !addr[device]) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) {
        std::fprintf(stderr, "libpowerlu: hipGetSymbolAddress(scratch) failed: %s\n",
                     hipGetErrorString(e));
        (void)hipGetLastError();
      } else {
        addr[device] = ptr;
      }
    }
    h->scratch_dev = device < 256 ? addr[device] : nullptr;
  }
  // bound on any device-side wait: 5 seconds of the constant-rate wall clock
  h->timeout_ticks = (uint64_t)(clk_khz > 0 ? clk_khz : 100000) * 1000ull * 5ull;
  *out = h;
  return PLU_OK;
}

int plu_destroy(plu_handle h) {
  if (!h) return -1;
  (void)hipStreamSynchronize(h->stream);
  drop_graph(h);
  if (h->gstream) (void)hipStreamDestroy(h->gstream);
  for (int i = 0; i < plu_handle_s::kSide; ++i) {
    if (h->side[i]) (void)hipStreamDestroy(h->side[i]);
    if (h->join_ev[i]) (void)hipEventDestroy(h->join_ev[i]);
    h->sbuf[i].destroy();
  }
  if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
  h->mbuf.destroy();
  if (h->arena) (void)hipFree(h->arena);
  if (h->batch_arena) (void)hipFree(h->batch_arena);
  if (h->trace_piv) (void)hipFree(h->trace_piv);
  if (h->trace_gaps) (void)hipFree(h->trace_gaps);
  delete h;
  return PLU_OK;
}

int plu_set_stream(plu_handle h, void* hip_stream) {
  if (!h) return -1;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return PLU_OK;
}

int plu_workspace_size(plu_handle h, int64_t m, int64_t n, int32_t l, int32_t max_rounds,
                       int32_t prec, size_t* bytes) {
  if (!h) return -1;
  if (m <= 0) return -2;
  if (n <= 0) return -3;
  if (l <= 0) return -4;
  if (max_rounds < 1) return -5;
  if (!valid_prec(prec)) return -6;
  if (!bytes) return -7;
  Layout dry;
  layout(dry, m, n, (int64_t)l * max_rounds, prec, max_rounds > 1);
  *bytes = dry.off + 256;   // 256: room to align an unaligned caller buffer
  return PLU_OK;
}

int plu_gaussian(plu_handle h, int64_t rows, int64_t cols, uint64_t seed, float* out,
                 int64_t ldo) {
  if (!h) return -1;
  if (rows < 0) return -2;
  if (cols < 0) return -3;
  if (!out && rows * cols > 0) return -5;
  if (ldo < cols) return -6;
  if (rows * cols == 0) return PLU_OK;
  PLU_TRY_HIP(hipSetDevice(h->device));
  PLU_TRY_HIP(launch_gaussian(out, ldo, rows, cols, seed, h->stream));
  return PLU_OK;
}

int plu_pass(plu_handle h, int32_t trans, int64_t m, int64_t n, const float* A, int64_t lda,
             int32_t l, const float* X, int64_t ldx, float* out, int64_t ldo, int32_t prec,
             double* normA2_out) {
  if (!h) return -1;
  if (trans != 0 && trans != 1) return -2;
  if (m <= 0) return -3;
  if (n <= 0) return -4;
  if (!A || (reinterpret_cast<uintptr_t>(A) & 3u)) return -5;
  if (lda < n) return -6;
  if (l <= 0) return -7;
  if (!X || (reinterpret_cast<uintptr_t>(X) & 3u)) return -8;
  if (ldx < l) return -9;
  if (!out) return -10;
  if (ldo < l) return -11;
  const int fmt = prec & ~PLU_PREC_A_UNCHANGED;
  if (fmt != PLU_PREC_FP32 && fmt != PLU_PREC_BF16 && fmt != PLU_PREC_FP8_E4M3) return -12;
  PLU_TRY_HIP(hipSetDevice(h->device));
  Ws w;
  // a pass alone runs no LU step: no status words to initialize
  int st = ensure_ws(h, m, n, std::max<int64_t>(l, ru4(ldo)), &w, fmt, false, nullptr, 0, false);
  if (st) return st;
  if (fmt != PLU_PREC_FP32) {
    PLU_TRY_HIP(lowp_copies(h, w, fmt, m, n, A, lda, (prec & PLU_PREC_A_UNCHANGED) != 0,
                            normA2_out));
    if (fmt == PLU_PREC_BF16) PLU_TRY_HIP(run_pass_bf16(h, w, trans, m, n, X, ldx, l, out, ldo));
    else PLU_TRY_HIP(run_pass_fp8(h, w, trans, m, n, X, ldx, l, out, ldo));
    return PLU_OK;
  }
  PLU_TRY_HIP(run_pass(h, w, trans, m, n, A, lda, X, ldx, l, out, ldo, normA2_out, nullptr,
                       nullptr));
  return PLU_OK;
}

int plu_quantize(plu_handle h, int32_t fmt, int64_t rows, int64_t cols, const float* src,
                 int64_t lds, int32_t transpose, void* dst, int64_t ldd, void* scales) {
  if (!h) return -1;
  if (fmt != PLU_PREC_BF16 && fmt != PLU_PREC_FP8_E4M3) return -2;
  if (rows <= 0) return -3;
  if (cols <= 0) return -4;
  if (!src || (reinterpret_cast<uintptr_t>(src) & 3u)) return -5;
  if (lds < cols) return -6;
  if (transpose != 0 && transpose != 1) return -7;
  if (!dst || (reinterpret_cast<uintptr_t>(dst) & 15u)) return -8;
  const int64_t align = fmt == PLU_PREC_BF16 ? 64 : 128;
  if (ldd % align != 0 || ldd < (transpose ? rows : cols)) return -9;
  if (fmt == PLU_PREC_FP8_E4M3 && !scales) return -10;
  PLU_TRY_HIP(hipSetDevice(h->device));
  if (fmt == PLU_PREC_FP8_E4M3) {
    uint8_t* d = reinterpret_cast<uint8_t*>(dst);
    uint8_t* sc = reinterpret_cast<uint8_t*>(scales);
    if (transpose)
      PLU_TRY_HIP(launch_cvt_fp8(src, lds, rows, cols, nullptr, nullptr, 0, d, sc, ldd, cols,
                                 nullptr, nullptr, h->stream));
    else
      PLU_TRY_HIP(launch_cvt_fp8(src, lds, rows, cols, d, sc, ldd, nullptr, nullptr, 0, 0,
                                 nullptr, nullptr, h->stream));
    return PLU_OK;
  }
  uint16_t* d = reinterpret_cast<uint16_t*>(dst);
  if (transpose)
    PLU_TRY_HIP(launch_cvt_bf16(src, lds, rows, cols, nullptr, 0, d, ldd, cols, nullptr, nullptr,
                                h->stream));
  else
    PLU_TRY_HIP(launch_cvt_bf16(src, lds, rows, cols, d, ldd, nullptr, 0, 0, nullptr, nullptr,
                                h->stream));
  return PLU_OK;
}

int plu_getrf(plu_handle h, int64_t M, int32_t c, float* F, int64_t ldf, int32_t* perm,
              float* Ufac, int64_t ldu, plu_info* info) {
  if (!h) return -1;
  if (M <= 0) return -2;
  if (c <= 0 || c > M) return -3;
  if (!F || (reinterpret_cast<uintptr_t>(F) & 3u)) return -4;
  if (ldf < c) return -5;
  if (Ufac && ldu < c) return -8;
  PLU_TRY_HIP(hipSetDevice(h->device));
  Ws w;
  int st = ensure_ws(h, M, c + 1, c, &w);
  if (st) return st;
  const GetrfWork g = getrf_work(h, w, 1);
  trace_reset(h);
  PLU_TRY_HIP(getrf_run(F, ldf, M, c, g, perm, Ufac, ldu, 0, h->stream));
  PLU_TRY_HIP(trace_getrf(h, g, c));
  if (info) {
    PLU_TRY_HIP(hipStreamSynchronize(h->stream));
    int32_t s[2];
    PLU_TRY_HIP(hipMemcpy(&s[0], g.zstep, sizeof(int32_t), hipMemcpyDeviceToHost));
    PLU_TRY_HIP(hipMemcpy(&s[1], g.abortf, sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<float> gp(c);
    PLU_TRY_HIP(hipMemcpy(gp.data(), g.gaps, c * sizeof(float), hipMemcpyDeviceToHost));
    std::memset(info, 0, sizeof(*info));
    info->rank = c;
    info->zero_pivot_step = (s[0] == INT32_MAX) ? -1 : s[0];
    float mg = 1.f;
    for (float x : gp) mg = std::min(mg, x);
    info->min_pivot_gap = mg;
    int status = PLU_OK;
    if (s[1]) status = PLU_ERR_TIMEOUT;
    else if (info->zero_pivot_step >= 0) status = PLU_WARN_ZERO_PIVOT;
    info->status = status;
    return status;
  }
  return PLU_OK;
}

int plu_thin_qr(plu_handle h, int64_t M, int32_t c, float* X, int64_t ldx) {
  if (!h) return -1;
  if (M <= 0) return -2;
  if (c <= 0 || c >= M) return -3;
  if (!X || (reinterpret_cast<uintptr_t>(X) & 3u)) return -4;
  if (ldx < c) return -5;
  PLU_TRY_HIP(hipSetDevice(h->device));
  Ws w;
  int st = ensure_ws(h, M, M, c, &w);
  if (st) return st;
  const GetrfWork g = getrf_work(h, w, 0);
  const QrWork q = qr_work(w, w.qb, w.lp);
  PLU_TRY_HIP(thin_qr_run(X, ldx, M, c, g, q, h->stream));
  PLU_TRY_HIP(hipMemcpy2DAsync(X, ldx * sizeof(float), w.qb, w.lp * sizeof(float),
                               c * sizeof(float), M, hipMemcpyDeviceToDevice, h->stream));
  return PLU_OK;
}

int plu_range_basis(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A,
                    int64_t lda, int32_t l, int32_t v, int32_t prec, const float* Omega,
                    uint64_t seed, float* V, int64_t ldv) {
  if (!h) return -1;
  if (!valid_layout(layout)) return -2;
  if (m <= 0) return -3;
  if (n <= 0) return -4;
  if (!A || (reinterpret_cast<uintptr_t>(A) & 3u)) return -5;
  if (lda < (layout == PLU_COL_MAJOR ? m : n)) return -6;
  if (l <= 0 || l >= std::min(m, n)) return -7;
  if (v < 2) return -8;
  if (!valid_prec(prec) || (prec & PLU_PREC_FP64_INDICATOR)) return -9;
  if (!V) return -12;
  if (ldv < l) return -13;
  PLU_TRY_HIP(hipSetDevice(h->device));
  Ws w;
  int st = ensure_ws(h, m, n, l, &w, prec);
  if (st) return st;
  w.acol = layout == PLU_COL_MAJOR;
  trace_reset(h);
  float* Vw = nullptr;
  int np = 0;
  PLU_TRY_HIP(range_basis(h, w, m, n, A, lda, l, v, Omega, seed, &Vw, &np, prec));
  PLU_TRY_HIP(hipMemcpy2DAsync(V, ldv * sizeof(float), Vw, w.lp * sizeof(float),
                               l * sizeof(float), n, hipMemcpyDeviceToDevice, h->stream));
  return PLU_OK;
}

static int fixed_rank_impl(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A,
                           int64_t lda, const SparseMat* sp, int off, int32_t k, int32_t p_over,
                           int32_t v, int32_t prec, const float* Omega, uint64_t seed, int32_t* p,
                           int32_t* q, float* L, int64_t ldl, float* U, int64_t ldu,
                           void* work, size_t work_bytes, plu_info* info, bool no_tune = false) {
  if (!h) return -1;
  if (!sp && !valid_layout(layout)) return -2;
  if (!sp && m <= 0) return -3;
  if (!sp && n <= 0) return -4;
  if (!sp && (!A || (reinterpret_cast<uintptr_t>(A) & 3u))) return -5;
  if (!sp && lda < (layout == PLU_COL_MAJOR ? m : n)) return -6;
  if (k < 1) return -(7 - off);
  if (p_over < 0) return -(8 - off);
  const int64_t l = (int64_t)k + p_over;
  if (l >= std::min(m, n)) return -(8 - off);
  if (v < 2) return -(9 - off);
  if (!valid_prec(prec) || (prec & PLU_PREC_FP64_INDICATOR)) return -(10 - off);
  if (sp && prec != PLU_PREC_FP32) return -(10 - off);   // sparse passes are float32
  if (!p) return -(13 - off);
  if (!q) return -(14 - off);
  if (!L) return -(15 - off);
  if (ldl < k) return -(16 - off);
  if (!U) return -(17 - off);
  if (ldu < n) return -(18 - off);
  PLU_TRY_HIP(hipSetDevice(h->device));
  Ws w;
  int st = ensure_ws(h, m, n, l, &w, prec, false, work, work_bytes);
  if (st == kWsTooSmall) return -20;
  if (st) return st;
  w.acol = layout == PLU_COL_MAJOR;
  w.sp = sp;
  w.no_tune = no_tune;
  trace_reset(h);
  float* V = nullptr;
  int np = 0;
  PLU_TRY_HIP(range_basis(h, w, m, n, A, lda, (int)l, v, Omega, seed, &V, &np, prec));
  // final pass: Y = A V(:, 1:k)
  PLU_TRY_HIP(run_pass(h, w, 0, m, n, A, lda, V, w.lp, k, w.ym, w.lp, nullptr, nullptr, nullptr));
  ++np;
  PLU_TRY_HIP(assemble(h, w, m, n, k, V, p, q, L, ldl, U, ldu));
  return finish_info(h, w, PLU_OK, k, np, (int)l, false, info);
}

int plu_fixed_rank(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A,
                   int64_t lda, int32_t k, int32_t p_over, int32_t v, int32_t prec,
                   const float* Omega, uint64_t seed, int32_t* p, int32_t* q, float* L,
                   int64_t ldl, float* U, int64_t ldu, void* work, size_t work_bytes,
                   plu_info* info) {
  return fixed_rank_impl(h, layout, m, n, A, lda, nullptr, 0, k, p_over, v, prec, Omega, seed, p, q,
                         L, ldl, U, ldu, work, work_bytes, info);
}

int plu_fixed_rank_static(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A,
                          int64_t lda, int32_t k, int32_t p_over, int32_t v, int32_t prec,
                          const float* Omega, uint64_t seed, int32_t* p, int32_t* q, float* L,
                          int64_t ldl, float* U, int64_t ldu, plu_info* info) {
  if (!h) return -1;
  if (!h->scratch_dev) return PLU_ERR_HIP;
  const int rc = fixed_rank_impl(h, layout, m, n, A, lda, nullptr, 0, k, p_over, v, prec, Omega,
                                 seed, p, q, L, ldl, U, ldu, h->scratch_dev, kScratchBytes, info,
                                 true);
  return rc == -20 ? PLU_ERR_TOO_LARGE : rc;
}

static int fixed_precision_impl(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A,
                                int64_t lda, const SparseMat* sp, int off, double eps, int32_t b,
                                int32_t l, int32_t v, int32_t column_exact, int32_t max_rounds,
                                int32_t prec, const float* Omega, uint64_t seed, int32_t* p,
                                int32_t* q, float* L, int64_t ldl, float* U, int64_t ldu,
                                int32_t* rank_dev, void* work, size_t work_bytes,
                                plu_info* info) {
  if (!h) return -1;
  if (!sp && !valid_layout(layout)) return -2;
  if (!sp && m <= 0) return -3;
  if (!sp && n <= 0) return -4;
  if (!sp && (!A || (reinterpret_cast<uintptr_t>(A) & 3u))) return -5;
  if (!sp && lda < (layout == PLU_COL_MAJOR ? m : n)) return -6;
  if (!(eps > 0.0)) return -(7 - off);
  if (b < 1) return -(8 - off);
  const int64_t mn = std::min(m, n);
  if (l == 0) l = (int32_t)std::min<int64_t>(50LL * b, b * ((mn - 1) / b));
  if (l <= 0 || l % b != 0 || l >= mn) return -(9 - off);
  if (v < 2) return -(10 - off);
  if (max_rounds < 1 || (int64_t)l * max_rounds >= mn) return -(12 - off);
  if (!valid_prec(prec)) return -(13 - off);
  if (sp && prec != PLU_PREC_FP32) return -(13 - off);   // sparse passes are float32
  // the float64 indicator: one round on a dense A
  if ((prec & PLU_PREC_FP64_INDICATOR) && max_rounds > 1) return PLU_ERR_NOT_IMPLEMENTED;
  if (!p) return -(16 - off);
  if (!q) return -(17 - off);
  if (!L) return -(18 - off);
  if (ldl < (int64_t)l * max_rounds) return -(19 - off);
  if (!U) return -(20 - off);
  if (ldu < n) return -(21 - off);
  PLU_TRY_HIP(hipSetDevice(h->device));
  Ws w;
  if (max_rounds > 1) {
    int st = ensure_ws(h, m, n, (int64_t)l * max_rounds, &w, prec, true, work, work_bytes);
    if (st == kWsTooSmall) return -24;
    if (st) return st;
    w.acol = layout == PLU_COL_MAJOR;
    w.sp = sp;
    trace_reset(h);
    return fixed_precision_rounds(h, w, m, n, A, lda, eps, b, l, v, column_exact, max_rounds, prec,
                                  Omega, seed, p, q, L, ldl, U, ldu, rank_dev, info);
  }
  int st = ensure_ws(h, m, n, l, &w, prec, false, work, work_bytes);
  if (st == kWsTooSmall) return -24;
  if (st) return st;
  w.acol = layout == PLU_COL_MAJOR;
  w.sp = sp;
  trace_reset(h);
  float* V = nullptr;
  int np = 0;
  PLU_TRY_HIP(range_basis(h, w, m, n, A, lda, l, v, Omega, seed, &V, &np, prec));
  // G = A V with column norms^2 (float64) fused into the reduction
  int nblk = 0;
  PLU_TRY_HIP(run_pass(h, w, 0, m, n, A, lda, V, w.lp, l, w.ym, w.lp, nullptr, w.colsq_part,
                       &nblk));
  ++np;
  if (prec & PLU_PREC_FP64_INDICATOR) {
    // the indicator from G = A V in float64, corrected to first order for
    // V^T V - I (one more pass over A, not counted among the v of Alg. 7)
    const bool g32 = fp64_ind_on_g32();
    if (!g32)
      PLU_TRY_HIP(launch_f64_gemm(w.acol ? 1 : 0, A, lda, V, w.lp, m, n, l, w.g64, w.lp,
                                  h->stream));
    PLU_TRY_HIP(launch_f64_gram_w(V, w.lp, n, l, w.w64, w.lp, h->stream));
    PLU_TRY_HIP(launch_f64_corr(g32 ? nullptr : w.g64, w.ym, w.lp, m, l, w.w64, w.lp,
                                w.ind_part, h->stream));
    PLU_TRY_HIP(launch_rank_rule(w.ind_part, f64_row_blocks(l), l, nullptr, 0, w.scal + 0, eps, b,
                                 column_exact ? 1 : 0, w.iscal + 0, w.scal + 1, w.iscal + 1,
                                 w.colnorm, h->stream));
  } else {
    // float64 squared norms of the basis columns (first-order normalization)
    PLU_TRY_HIP(launch_splitk_reduce(V, 0, 1, nullptr, w.lp, n, l, w.vsq_part, 64, h->stream));
    const int nvblk = (int)((n + 63) / 64);
    PLU_TRY_HIP(launch_rank_rule(w.colsq_part, nblk, l, w.vsq_part, nvblk, w.scal + 0, eps, b,
                                 column_exact ? 1 : 0, w.iscal + 0, w.scal + 1, w.iscal + 1,
                                 w.colnorm, h->stream));
  }
  // Alg. 9 steps 2-6 at the rank the rule left on the device (0 for a zero
  // or non-finite A: the LUs then take no step and p, q are the identity)
  PLU_TRY_HIP(assemble(h, w, m, n, l, V, p, q, L, ldl, U, ldu, nullptr, w.iscal));
  if (rank_dev)
    PLU_TRY_HIP(hipMemcpyAsync(rank_dev, w.iscal, sizeof(int32_t), hipMemcpyDeviceToDevice,
                               h->stream));
  return finish_info(h, w, PLU_OK, -1, np, l, true, info);
}

int plu_fixed_precision(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A,
                        int64_t lda, double eps, int32_t b, int32_t l, int32_t v,
                        int32_t column_exact, int32_t max_rounds, int32_t prec,
                        const float* Omega, uint64_t seed, int32_t* p, int32_t* q, float* L,
                        int64_t ldl, float* U, int64_t ldu, int32_t* rank_dev, void* work,
                        size_t work_bytes, plu_info* info) {
  return fixed_precision_impl(h, layout, m, n, A, lda, nullptr, 0, eps, b, l, v, column_exact,
                              max_rounds, prec, Omega, seed, p, q, L, ldl, U, ldu, rank_dev, work,
                              work_bytes, info);
}

int plu_single_pass(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A,
                    int64_t lda, int32_t k, const float* Omega, uint64_t seed, int32_t* p,
                    int32_t* q, float* L, int64_t ldl, float* U, int64_t ldu, plu_info* info) {
  if (!h) return -1;
  if (!valid_layout(layout)) return -2;
  if (m <= 0) return -3;
  if (n <= 0) return -4;
  if (!A || (reinterpret_cast<uintptr_t>(A) & 3u)) return -5;
  const bool col = layout == PLU_COL_MAJOR;
  if (lda < (col ? m : n)) return -6;
  if (k < 1 || k > 128 || k >= std::min(m, n)) return -7;
  if (!p) return -10;
  if (!q) return -11;
  if (!L) return -12;
  if (ldl < k) return -13;
  if (!U) return -14;
  if (ldu < n) return -15;
  PLU_TRY_HIP(hipSetDevice(h->device));
  Ws w;
  int st = ensure_ws(h, m, n, k, &w);
  if (st) return st;
  w.acol = col;
  trace_reset(h);
  hipStream_t s = h->stream;
  const int64_t lp = w.lp;
  // Alg. 10 step 1: Omega (m x k)
  if (Omega) PLU_TRY_HIP(launch_copy_pad(Omega, k, w.om, lp, m, k, k, s));
  else PLU_TRY_HIP(launch_gaussian(w.om, lp, m, k, seed, s));
  // steps 2-3: G = A^T Omega (n x k, w.zn) and H = A G (m x k, w.ym)
  if (!col) {
    // rows of A are contiguous: G is complete only after every row, so
    // these are two passes (the one-pass form needs the columns contiguous)
    PLU_TRY_HIP(run_pass(h, w, 1, m, n, A, lda, w.om, lp, k, w.zn, lp, w.scal + 0, nullptr,
                         nullptr));
    PLU_TRY_HIP(run_pass(h, w, 0, m, n, A, lda, w.zn, lp, k, w.ym, lp, nullptr, nullptr,
                         nullptr));
  } else {
    // one pass (the Remark after the derivation): column i of A is row i of
    // the storage; for a block of storage rows, G's rows = block x Omega, then
    // H -= block^T x G's rows, while the block is still in the caches (its
    // bytes are read from HBM once); H is negated at the end
    PLU_TRY_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(w.ym), (size_t)m * lp, 0u, s));
    // blocks of about 192 MB: they stay in the 256 MB last-level cache
    // between the two products (48 MB blocks measured 9.2 ms, 192 MB 6.8 ms
    // at 20000^2, k = 100: thinner blocks make thinner, slower products)
    const int64_t blk = std::max<int64_t>(128, (((int64_t)192 << 20) / (4 * m)) / 128 * 128);
    int64_t sq_off = 0;
    for (int64_t i0 = 0; i0 < n; i0 += blk) {
      const int64_t b = std::min(blk, n - i0);
      GemmArgs g;
      g.A = A + i0 * lda; g.lda = lda; g.X = w.om; g.ldx = lp;
      g.P = b; g.R = m; g.C = k;
      int max_split = (int)std::min<int64_t>(64, w.part_cap / std::max<int64_t>(b * lp, 1));
      if (max_split < 1) max_split = 1;
      const GemmPlan pl = plan_gemm(b, m, k, max_split, 1024);
      if (sq_off + (int64_t)pl.pblocks * pl.nsplit > w.sumsq_cap) return PLU_ERR_NOT_IMPLEMENTED;
      g.sumsq_part = w.sumsq_part + sq_off;   // ||A||_F^2 partials of this block
      sq_off += (int64_t)pl.pblocks * pl.nsplit;
      float* Gb = w.zn + i0 * lp;
      if (pl.nsplit > 1) {
        g.out = w.part; g.ldo = lp; g.part_stride = b * lp;
        PLU_TRY_HIP(launch_gemm(0, EPI_PART, 0, g, pl, s));
        PLU_TRY_HIP(launch_splitk_reduce(w.part, b * lp, pl.nsplit, Gb, lp, b, k, nullptr, 64, s));
      } else {
        g.out = Gb; g.ldo = lp;
        PLU_TRY_HIP(launch_gemm(0, EPI_STORE, 0, g, pl, s));
      }
      GemmArgs u;
      u.A = A + i0 * lda; u.lda = lda; u.X = Gb; u.ldx = lp; u.out = w.ym; u.ldo = lp;
      u.P = m; u.R = b; u.C = k;
      PLU_TRY_HIP(launch_gemm(1, EPI_SUB, 0, u, plan_gemm(m, b, k, 1, 1), s));
    }
    PLU_TRY_HIP(launch_sum_doubles(w.sumsq_part, sq_off, w.scal + 0, s));
    PLU_TRY_HIP(launch_negate(w.ym, lp, m, k, s));
  }
  // pinv(G^T) = Q R^{-T} with G = Q R (thin QR of a copy of G, R = Q^T G)
  const GetrfWork gw = getrf_work(h, w, 0);
  const QrWork qw = qr_work(w, w.qb, lp);
  PLU_TRY_HIP(hipMemcpy2DAsync(w.bt, lp * sizeof(float), w.zn, lp * sizeof(float),
                               k * sizeof(float), n, hipMemcpyDeviceToDevice, s));
  PLU_TRY_HIP(thin_qr_run(w.bt, lp, n, k, gw, qw, s));
  PLU_TRY_HIP(small_tn(h, w, w.qb, lp, w.zn, lp, k, n, k, w.ut2, lp));   // R (k x k)
  PLU_TRY_HIP(launch_tri_inv_t(w.ut2, lp, w.ut1, lp, k, s));              // (R^{-1})^T
  {
    GemmArgs g;
    g.A = w.qb; g.lda = lp; g.X = w.ut1; g.ldx = lp; g.out = w.zn; g.ldo = lp;
    g.P = n; g.R = k; g.C = k;
    PLU_TRY_HIP(launch_gemm(0, EPI_STORE, 0, g, plan_gemm(n, k, k, 1, 1), s));
  }
  // steps 4-7: lu(H), lu(pinv(G^T) U1^T), L = L1 U2^T, U = L2^T
  PLU_TRY_HIP(assemble(h, w, m, n, k, w.zn, p, q, L, ldl, U, ldu, w.ym));
  return finish_info(h, w, PLU_OK, k, 1, k, false, info);
}

static int randlu_impl(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A,
                       int64_t lda, const SparseMat* sp, int off, int32_t k, int32_t p_over,
                       int32_t pw, const float* Omega, uint64_t seed, int32_t* p, int32_t* q,
                       float* L, int64_t ldl, float* U, int64_t ldu, plu_info* info) {
  if (!h) return -1;
  if (!sp && !valid_layout(layout)) return -2;
  if (!sp && m <= 0) return -3;
  if (!sp && n <= 0) return -4;
  if (!sp && (!A || (reinterpret_cast<uintptr_t>(A) & 3u))) return -5;
  if (!sp && lda < (layout == PLU_COL_MAJOR ? m : n)) return -6;
  if (k < 1 || k > 128) return -(7 - off);
  if (p_over < 0) return -(8 - off);
  const int64_t l = (int64_t)k + p_over;
  if (l >= std::min(m, n)) return -(8 - off);
  if (pw < 0) return -(9 - off);
  if (!p) return -(12 - off);
  if (!q) return -(13 - off);
  if (!L) return -(14 - off);
  if (ldl < k) return -(15 - off);
  if (!U) return -(16 - off);
  if (ldu < n) return -(17 - off);
  PLU_TRY_HIP(hipSetDevice(h->device));
  Ws w;
  int st = ensure_ws(h, m, n, l, &w);
  if (st) return st;
  w.acol = layout == PLU_COL_MAJOR;
  w.sp = sp;
  trace_reset(h);
  hipStream_t s = h->stream;
  const int64_t lp = w.lp;
  const GetrfWork g0 = getrf_work(h, w, 0);
  const GetrfWork g1 = getrf_work(h, w, 1);
  const GetrfWork g2 = getrf_work(h, w, 2);
  // Alg. 4 (in place of Alg. 3 steps 1-3): Omega (n x l)
  if (Omega) PLU_TRY_HIP(launch_copy_pad(Omega, l, w.om, lp, n, l, l, s));
  else PLU_TRY_HIP(launch_gaussian(w.om, lp, n, l, seed, s));
  // Y = A Omega (the first pass also yields ||A||_F^2)
  PLU_TRY_HIP(run_pass(h, w, 0, m, n, A, lda, w.om, lp, (int)l, w.ym, lp, w.scal + 0, nullptr,
                       nullptr));
  int np = 1;
  for (int i = 1; i <= pw; ++i) {
    // L = P^T L of the previous product, then L = P^T L of lu(A^T L)
    PLU_TRY_HIP(getrf_run(w.ym, lp, m, (int)l, g0, nullptr, nullptr, 0, 0, s));
    PLU_TRY_HIP(trace_getrf(h, g0, (int)l));
    PLU_TRY_HIP(run_pass(h, w, 1, m, n, A, lda, w.ym, lp, (int)l, w.zn, lp, nullptr, nullptr,
                         nullptr));
    PLU_TRY_HIP(getrf_run(w.zn, lp, n, (int)l, g0, nullptr, nullptr, 0, 0, s));
    PLU_TRY_HIP(trace_getrf(h, g0, (int)l));
    PLU_TRY_HIP(run_pass(h, w, 0, m, n, A, lda, w.zn, lp, (int)l, w.ym, lp, nullptr, nullptr,
                         nullptr));
    np += 2;
  }
  // [L_y, U_y, P] = lu(Y): w.ym <- P^T L_y (A's row order), p <- P's order
  PLU_TRY_HIP(getrf_run(w.ym, lp, m, (int)l, g1, p, nullptr, 0, 0, s));
  PLU_TRY_HIP(trace_getrf(h, g1, (int)l));
  // Alg. 3 steps 4-5 with V = P^T L_y(:, :k): B = (V^T V)^{-1} V^T A, as
  // B^T = C R^{-1} R^{-T} with C = A^T V (the last pass) and V^T V = R^T R
  PLU_TRY_HIP(run_pass(h, w, 1, m, n, A, lda, w.ym, lp, k, w.zn, lp, nullptr, nullptr, nullptr));
  ++np;
  const QrWork qw = qr_work(w, w.qb, lp);
  PLU_TRY_HIP(gram_inverse_run(w.ym, lp, m, k, qw, s));
  {
    GemmArgs g;
    g.A = w.zn; g.lda = lp; g.X = w.rinv; g.ldx = kQB; g.out = w.bt; g.ldo = lp;
    g.P = n; g.R = k; g.C = k;
    PLU_TRY_HIP(launch_gemm(0, EPI_STORE, 0, g, plan_gemm(n, k, k, 1, 1), s));
  }
  PLU_TRY_HIP(launch_iota(w.pos, k, s));
  PLU_TRY_HIP(launch_transpose_gather(w.rinv, kQB, w.pos, k, k, w.ut1, lp, s));   // R^{-T}
  {
    GemmArgs g;
    g.A = w.bt; g.lda = lp; g.X = w.ut1; g.ldx = lp; g.out = w.zn; g.ldo = lp;
    g.P = n; g.R = k; g.C = k;
    PLU_TRY_HIP(launch_gemm(0, EPI_STORE, 0, g, plan_gemm(n, k, k, 1, 1), s));
  }
  // steps 6-8: [L2, U2, Q] = lu(B^T), L = L_y U2^T, U = L2^T
  PLU_TRY_HIP(getrf_run(w.zn, lp, n, k, g2, q, w.ut2, lp, 1, s));
  PLU_TRY_HIP(trace_getrf(h, g2, k));
  {
    GemmArgs g;
    g.A = w.ym; g.lda = lp; g.arow = p; g.X = w.ut2; g.ldx = lp; g.out = L; g.ldo = ldl;
    g.P = m; g.R = k; g.C = k;
    PLU_TRY_HIP(launch_gemm(0, EPI_STORE, 0, g, plan_gemm(m, k, k, 1, 1), s));
  }
  PLU_TRY_HIP(launch_transpose_gather(w.zn, lp, q, n, k, U, ldu, s));
  return finish_info(h, w, PLU_OK, k, np, (int)l, false, info);
}

int plu_randlu(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A, int64_t lda,
               int32_t k, int32_t p_over, int32_t pw, const float* Omega, uint64_t seed,
               int32_t* p, int32_t* q, float* L, int64_t ldl, float* U, int64_t ldu,
               plu_info* info) {
  return randlu_impl(h, layout, m, n, A, lda, nullptr, 0, k, p_over, pw, Omega, seed, p, q, L, ldl,
                     U, ldu, info);
}

static int randsvd_impl(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A,
                        int64_t lda, const SparseMat* sp, int off, int32_t k, int32_t p_over,
                        int32_t pw, const float* Omega, uint64_t seed, float* Uo, int64_t ldu,
                        float* S, float* Vo, int64_t ldv, plu_info* info) {
  if (!h) return -1;
  if (!sp && !valid_layout(layout)) return -2;
  if (!sp && m <= 0) return -3;
  if (!sp && n <= 0) return -4;
  if (!sp && (!A || (reinterpret_cast<uintptr_t>(A) & 3u))) return -5;
  if (!sp && lda < (layout == PLU_COL_MAJOR ? m : n)) return -6;
  if (k < 1) return -(7 - off);
  if (p_over < 0) return -(8 - off);
  const int64_t l = (int64_t)k + p_over;
  if (l > 128 || l >= std::min(m, n)) return -(8 - off);
  if (pw < 0) return -(9 - off);
  if (!Uo) return -(12 - off);
  if (ldu < k) return -(13 - off);
  if (!S) return -(14 - off);
  if (!Vo) return -(15 - off);
  if (ldv < k) return -(16 - off);
  PLU_TRY_HIP(hipSetDevice(h->device));
  Ws w;
  int st = ensure_ws(h, m, n, l, &w);
  if (st) return st;
  w.acol = layout == PLU_COL_MAJOR;
  w.sp = sp;
  trace_reset(h);
  hipStream_t s = h->stream;
  const int64_t lp = w.lp;
  const int c = (int)l;
  const GetrfWork gw = getrf_work(h, w, 0);
  const QrWork qw = qr_work(w, w.qb, lp);     // Q of Alg. 2 in w.qb
  const QrWork qwb = qr_work(w, w.bt, lp);    // Q_b of B^T in w.bt
  // Alg. 2: Q = qr(A Omega); p times Q = qr(A^T Q), Q = qr(A Q)
  if (Omega) PLU_TRY_HIP(launch_copy_pad(Omega, l, w.om, lp, n, l, l, s));
  else PLU_TRY_HIP(launch_gaussian(w.om, lp, n, l, seed, s));
  PLU_TRY_HIP(run_pass(h, w, 0, m, n, A, lda, w.om, lp, c, w.ym, lp, w.scal + 0, nullptr,
                       nullptr));
  PLU_TRY_HIP(thin_qr_run(w.ym, lp, m, c, gw, qw, s));
  int np = 1;
  for (int i = 1; i <= pw; ++i) {
    PLU_TRY_HIP(run_pass(h, w, 1, m, n, A, lda, w.qb, lp, c, w.zn, lp, nullptr, nullptr,
                         nullptr));
    PLU_TRY_HIP(thin_qr_run(w.zn, lp, n, c, gw, qw, s));
    PLU_TRY_HIP(run_pass(h, w, 0, m, n, A, lda, w.qb, lp, c, w.ym, lp, nullptr, nullptr,
                         nullptr));
    PLU_TRY_HIP(thin_qr_run(w.ym, lp, m, c, gw, qw, s));
    np += 2;
  }
  // Alg. 1 steps 4-6: B^T = A^T Q (n x l); B^T = Q_b R (thin QR, R = Q_b^T B^T);
  // R = U_r S V_r^T (Jacobi); U = Q V_r, V = Q_b U_r, the k leading columns
  PLU_TRY_HIP(run_pass(h, w, 1, m, n, A, lda, w.qb, lp, c, w.zn, lp, nullptr, nullptr, nullptr));
  ++np;
  PLU_TRY_HIP(hipMemcpy2DAsync(w.om, lp * sizeof(float), w.zn, lp * sizeof(float),
                               c * sizeof(float), n, hipMemcpyDeviceToDevice, s));
  PLU_TRY_HIP(thin_qr_run(w.zn, lp, n, c, gw, qwb, s));
  PLU_TRY_HIP(small_tn(h, w, w.bt, lp, w.om, lp, c, n, c, w.ut1, lp));
  PLU_TRY_HIP(launch_jacobi_svd(w.ut1, lp, c, w.ut2, lp, w.wproj, kQB, S, k, w.iscal + 2, s));
  {
    GemmArgs g;
    g.A = w.qb; g.lda = lp; g.X = w.wproj; g.ldx = kQB; g.out = Uo; g.ldo = ldu;
    g.P = m; g.R = c; g.C = k;
    PLU_TRY_HIP(launch_gemm(0, EPI_STORE, 0, g, plan_gemm(m, c, k, 1, 1), s));
  }
  {
    GemmArgs g;
    g.A = w.bt; g.lda = lp; g.X = w.ut2; g.ldx = lp; g.out = Vo; g.ldo = ldv;
    g.P = n; g.R = c; g.C = k;
    PLU_TRY_HIP(launch_gemm(0, EPI_STORE, 0, g, plan_gemm(n, c, k, 1, 1), s));
  }
  const int rs = finish_info(h, w, PLU_OK, 0, np, c, false, info);
  if (info) info->rank = k;
  return rs;
}

int plu_randsvd(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A, int64_t lda,
                int32_t k, int32_t p_over, int32_t pw, const float* Omega, uint64_t seed,
                float* Uo, int64_t ldu, float* S, float* Vo, int64_t ldv, plu_info* info) {
  return randsvd_impl(h, layout, m, n, A, lda, nullptr, 0, k, p_over, pw, Omega, seed, Uo, ldu, S,
                      Vo, ldv, info);
}

int plu_sparse_create(plu_handle h, int64_t m, int64_t n, int64_t nnz, const int64_t* rowptr,
                      const int32_t* colidx, const float* vals, plu_sparse* out) {
  if (!h) return -1;
  if (m <= 0 || m > INT32_MAX) return -2;
  if (n <= 0 || n > INT32_MAX) return -3;
  if (nnz < 0) return -4;
  if (!rowptr || (reinterpret_cast<uintptr_t>(rowptr) & 7u)) return -5;
  if (nnz > 0 && (!colidx || (reinterpret_cast<uintptr_t>(colidx) & 3u))) return -6;
  if (nnz > 0 && (!vals || (reinterpret_cast<uintptr_t>(vals) & 3u))) return -7;
  if (!out) return -8;
  *out = nullptr;
  PLU_TRY_HIP(hipSetDevice(h->device));
  plu_sparse sp = new (std::nothrow) plu_sparse_s;
  if (!sp) return PLU_ERR_OOM;
  sp->device = h->device;
  sp->mat.m = m;
  sp->mat.n = n;
  sp->mat.nnz = nnz;
  sp->mat.rowptr = rowptr;
  sp->mat.colidx = colidx;
  sp->mat.vals = vals;
  if (hipMalloc(&sp->mem, sparse_scratch_bytes(m, n, nnz) + 4096) != hipSuccess) {
    hipGetLastError();
    delete sp;
    return PLU_ERR_OOM;
  }
  int32_t bad = 0;
  if (sparse_build(sp->mat, sp->mem, &bad, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
    hipFree(sp->mem);
    delete sp;
    return PLU_ERR_HIP;
  }
  if (bad) {   // malformed compressed rows: the offending argument's index
    hipFree(sp->mem);
    delete sp;
    return (bad & 1) ? -5 : -6;
  }
  *out = sp;
  return PLU_OK;
}

int plu_sparse_destroy(plu_sparse sp) {
  if (!sp) return PLU_OK;
  if (hipSetDevice(sp->device) == hipSuccess) {
    hipDeviceSynchronize();
    hipFree(sp->mem);
  }
  delete sp;
  return PLU_OK;
}

int plu_sparse_pass(plu_handle h, plu_sparse sp, int32_t trans, const float* X, int64_t ldx,
                    int32_t l, float* out, int64_t ldo) {
  if (!h) return -1;
  if (!sp || sp->device != h->device) return -2;
  if (trans != 0 && trans != 1) return -3;
  if (!X || (reinterpret_cast<uintptr_t>(X) & 3u)) return -4;
  if (l < 1) return -6;
  if (ldx < l) return -5;
  if (!out || (reinterpret_cast<uintptr_t>(out) & 3u)) return -7;
  if (ldo < l) return -8;
  PLU_TRY_HIP(hipSetDevice(h->device));
  const SparseMat& S = sp->mat;
  PLU_TRY_HIP(trans ? launch_spmm(S.colptr, S.rowidx, S.valsT, S.n, X, ldx, l, out, ldo, h->stream)
                    : launch_spmm(S.rowptr, S.colidx, S.vals, S.m, X, ldx, l, out, ldo, h->stream));
  return PLU_OK;
}

// The sparse forms of the drivers: the dense argument list without layout,
// m, n, A and lda (so every later argument's index is 4 lower).
int plu_sparse_fixed_rank(plu_handle h, plu_sparse sp, int32_t k, int32_t p_over, int32_t v,
                          int32_t prec, const float* Omega, uint64_t seed, int32_t* p, int32_t* q,
                          float* L, int64_t ldl, float* U, int64_t ldu, plu_info* info) {
  if (!h) return -1;
  if (!sp || sp->device != h->device) return -2;
  return fixed_rank_impl(h, PLU_ROW_MAJOR, sp->mat.m, sp->mat.n, nullptr, 0, &sp->mat, 4, k, p_over,
                         v, prec, Omega, seed, p, q, L, ldl, U, ldu, nullptr, 0, info);
}

int plu_sparse_fixed_precision(plu_handle h, plu_sparse sp, double eps, int32_t b, int32_t l,
                               int32_t v, int32_t column_exact, int32_t max_rounds, int32_t prec,
                               const float* Omega, uint64_t seed, int32_t* p, int32_t* q, float* L,
                               int64_t ldl, float* U, int64_t ldu, int32_t* rank_dev,
                               plu_info* info) {
  if (!h) return -1;
  if (!sp || sp->device != h->device) return -2;
  return fixed_precision_impl(h, PLU_ROW_MAJOR, sp->mat.m, sp->mat.n, nullptr, 0, &sp->mat, 4, eps,
                              b, l, v, column_exact, max_rounds, prec, Omega, seed, p, q, L, ldl,
                              U, ldu, rank_dev, nullptr, 0, info);
}

int plu_sparse_randlu(plu_handle h, plu_sparse sp, int32_t k, int32_t p_over, int32_t pw,
                      const float* Omega, uint64_t seed, int32_t* p, int32_t* q, float* L,
                      int64_t ldl, float* U, int64_t ldu, plu_info* info) {
  if (!h) return -1;
  if (!sp || sp->device != h->device) return -2;
  return randlu_impl(h, PLU_ROW_MAJOR, sp->mat.m, sp->mat.n, nullptr, 0, &sp->mat, 4, k, p_over, pw,
                     Omega, seed, p, q, L, ldl, U, ldu, info);
}

int plu_sparse_randsvd(plu_handle h, plu_sparse sp, int32_t k, int32_t p_over, int32_t pw,
                       const float* Omega, uint64_t seed, float* Uo, int64_t ldu, float* S,
                       float* Vo, int64_t ldv, plu_info* info) {
  if (!h) return -1;
  if (!sp || sp->device != h->device) return -2;
  return randsvd_impl(h, PLU_ROW_MAJOR, sp->mat.m, sp->mat.n, nullptr, 0, &sp->mat, 4, k, p_over,
                      pw, Omega, seed, Uo, ldu, S, Vo, ldv, info);
}

int plu_rank_rule(plu_handle h, int64_t m, int32_t l, const float* G, int64_t ldg, double normA2,
                  double eps, int32_t b, int32_t column_exact, int32_t* k_out, double* E_out,
                  double* colnorm2) {
  if (!h) return -1;
  if (m <= 0) return -2;
  if (l <= 0 || l > 8192) return -3;
  if (!G) return -4;
  if (ldg < l) return -5;
  if (!(normA2 >= 0.0)) return -6;
  if (!(eps > 0.0)) return -7;
  if (b < 1) return -8;
  if (!k_out) return -10;
  PLU_TRY_HIP(hipSetDevice(h->device));
  Ws w;
  int st = ensure_ws(h, m, l + 1, l, &w);
  if (st) return st;
  PLU_TRY_HIP(hipMemcpyAsync(w.scal + 0, &normA2, sizeof(double), hipMemcpyHostToDevice,
                             h->stream));
  PLU_TRY_HIP(launch_splitk_reduce(G, 0, 1, nullptr, ldg, m, l, w.colsq_part, 64, h->stream));
  const int nblk = (int)((m + 63) / 64);
  PLU_TRY_HIP(launch_rank_rule(w.colsq_part, nblk, l, nullptr, 0, w.scal + 0, eps, b,
                               column_exact ? 1 : 0, w.iscal + 0, w.scal + 1, w.iscal + 1,
                               w.colnorm, h->stream));
  PLU_TRY_HIP(hipStreamSynchronize(h->stream));
  int32_t ks[2];
  double E;
  PLU_TRY_HIP(hipMemcpy(ks, w.iscal, sizeof(ks), hipMemcpyDeviceToHost));
  PLU_TRY_HIP(hipMemcpy(&E, w.scal + 1, sizeof(double), hipMemcpyDeviceToHost));
  if (colnorm2)
    PLU_TRY_HIP(hipMemcpy(colnorm2, w.colnorm, l * sizeof(double), hipMemcpyDeviceToHost));
  *k_out = ks[0];
  if (E_out) *E_out = E;
  return ks[1] ? PLU_OK : PLU_TOL_NOT_REACHED;
}

int plu_residual(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A,
                 int64_t lda, const int32_t* p, const int32_t* q, int32_t k, const float* L,
                 int64_t ldl, const float* U, int64_t ldu, double* rel_resid) {
  if (!h) return -1;
  if (!valid_layout(layout)) return -2;
  if (m <= 0) return -3;
  if (n <= 0) return -4;
  if (!A) return -5;
  const bool col = layout == PLU_COL_MAJOR;
  if (lda < (col ? m : n)) return -6;
  if (!p) return -7;
  if (!q) return -8;
  if (k < 1) return -9;
  if (!L) return -10;
  if (ldl < k) return -11;
  if (!U) return -12;
  if (ldu < n) return -13;
  if (!rel_resid) return -14;
  PLU_TRY_HIP(hipSetDevice(h->device));
  char* extra = nullptr;
  const GemmPlan pl = plan_gemm(m, k, n, 1, 1);
  const int64_t nparts = (int64_t)pl.pblocks * pl.cblocks;
  // L and U moved to A's own order (row p[i] of L, column q[j] of U), so
  // that the pass reads A in place: ||A - P^T L U Q^T||_F equals the
  // residual of A[p][:, q] when p and q are permutations
  const int64_t ldlp = ru(k, 4), ldup = ru(n, 4);
  const size_t bytes = (2 * nparts + 2) * sizeof(double) +
                       (size_t)(m * ldlp + (int64_t)k * ldup) * sizeof(float) + 3 * 1024;
  if (hipMalloc(reinterpret_cast<void**>(&extra), bytes) != hipSuccess) {
    hipGetLastError();
    return PLU_ERR_OOM;
  }
  Layout lay;
  lay.base = extra;
  double* rpart = lay.take<double>(nparts);
  double* spart = lay.take<double>(nparts);
  double* sums = lay.take<double>(2);
  float* Lp = lay.take<float>(m * ldlp);
  float* Up = lay.take<float>((int64_t)k * ldup);
  int rc = PLU_OK;
  do {
    // cleared first, so that entries a malformed p or q never reaches read as zero
    if (hipMemsetAsync(Lp, 0, (size_t)(m * ldlp) * sizeof(float), h->stream) != hipSuccess ||
        hipMemsetAsync(Up, 0, (size_t)((int64_t)k * ldup) * sizeof(float), h->stream) != hipSuccess ||
        launch_scatter_perm(L, ldl, Lp, ldlp, m, k, p, nullptr, h->stream) != hipSuccess ||
        launch_scatter_perm(U, ldu, Up, ldup, k, n, nullptr, q, h->stream) != hipSuccess) {
      rc = PLU_ERR_HIP;
      break;
    }
    GemmArgs g;
    g.A = Lp; g.lda = ldlp; g.X = Up; g.ldx = ldup;
    g.P = m; g.R = k; g.C = n;
    g.Aref = A; g.resid_part = rpart;
    g.aref_sq_part = spart;   // ||A||_F^2 from the entries the same pass reads
    g.ldaref = col ? 1 : lda;     // element (i, j) of A at i * ldaref + j * aref_cs
    g.aref_cs = col ? lda : 1;
    if (launch_gemm(0, EPI_RESID, 0, g, pl, h->stream) != hipSuccess) { rc = PLU_ERR_HIP; break; }
    if (launch_sum_doubles(rpart, nparts, sums + 0, h->stream) != hipSuccess) { rc = PLU_ERR_HIP; break; }
    if (launch_sum_doubles(spart, nparts, sums + 1, h->stream) != hipSuccess) { rc = PLU_ERR_HIP; break; }
    double hs[2];
    if (hipStreamSynchronize(h->stream) != hipSuccess ||
        hipMemcpy(hs, sums, sizeof(hs), hipMemcpyDeviceToHost) != hipSuccess) {
      rc = PLU_ERR_HIP;
      break;
    }
    *rel_resid = hs[1] > 0 ? std::sqrt(hs[0] / hs[1]) : 0.0;
  } while (0);
  hipStreamSynchronize(h->stream);
  hipFree(extra);
  return rc;
}

int plu_measure_peak(plu_handle h, int32_t kind, const void* buf, int64_t bytes, int32_t reps,
                     double* rate) {
  if (!h) return -1;
  if (kind < PLU_PEAK_MFMA_FP32 || kind > PLU_PEAK_HBM_READ) return -2;
  const bool hbm = kind == PLU_PEAK_HBM_READ;
  if (hbm && (!buf || (reinterpret_cast<uintptr_t>(buf) & 15u))) return -3;
  if (hbm && bytes < (int64_t)1 << 20) return -4;
  if (reps < 1) return -5;
  if (!rate) return -6;
  PLU_TRY_HIP(hipSetDevice(h->device));
  const int blocks = h->cu_count * 8;
  // about 3 ms per launch at the datasheet rates
  const int iters = kind == PLU_PEAK_MFMA_BF16 ? 8192 : 4096;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return PLU_ERR_HIP;
  }
  auto launch = [&]() {
    return hbm ? launch_peak_read(buf, bytes, blocks, h->stream)
               : launch_peak_mfma(kind, blocks, iters, h->stream);
  };
  int rc = PLU_OK;
  float best = 0.f;
  if (launch() != hipSuccess) rc = PLU_ERR_HIP;   // warm-up (clocks, caches, code)
  for (int r = 0; r < reps && rc == PLU_OK; ++r) {
    float ms = 0.f;
    if (hipEventRecord(e0, h->stream) != hipSuccess || launch() != hipSuccess ||
        hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = PLU_ERR_HIP;
      break;
    }
    if (r == 0 || ms < best) best = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != PLU_OK) return rc;
  if (hbm) {
    *rate = (double)(bytes / 16 * 16) / (best * 1e-3) / 1e9;   // GB/s
  } else {
    const double flop = (double)blocks * 4 * iters * peak_chains() * peak_flop_per_mfma(kind);
    *rate = flop / (best * 1e-3) / 1e12;   // TFLOP/s
  }
  return PLU_OK;
}

int plu_set_pivot_trace(plu_handle h, int64_t capacity) {
  if (!h) return -1;
  if (capacity < 0) return -2;
  PLU_TRY_HIP(hipSetDevice(h->device));
  PLU_TRY_HIP(hipStreamSynchronize(h->stream));
  if (h->trace_piv) (void)hipFree(h->trace_piv);
  if (h->trace_gaps) (void)hipFree(h->trace_gaps);
  h->trace_piv = nullptr;
  h->trace_gaps = nullptr;
  h->trace_cap = h->trace_n = h->trace_need = 0;
  if (capacity == 0) return PLU_OK;
  if (hipMalloc(reinterpret_cast<void**>(&h->trace_piv), capacity * sizeof(int32_t)) !=
          hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&h->trace_gaps), capacity * sizeof(float)) !=
          hipSuccess) {
    (void)hipGetLastError();
    if (h->trace_piv) (void)hipFree(h->trace_piv);
    h->trace_piv = nullptr;
    h->trace_gaps = nullptr;
    return PLU_ERR_OOM;
  }
  h->trace_cap = capacity;
  return PLU_OK;
}

int plu_pivot_trace(plu_handle h, int32_t* ipiv_out, float* gaps_out, int32_t cap,
                    int32_t* n_out) {
  if (!h) return -1;
  if (cap < 0) return -4;
  if (!n_out) return -5;
  PLU_TRY_HIP(hipSetDevice(h->device));
  PLU_TRY_HIP(hipStreamSynchronize(h->stream));
  *n_out = (int32_t)h->trace_need;
  const int64_t c = std::min<int64_t>(cap, h->trace_n);
  if (c > 0 && ipiv_out)
    PLU_TRY_HIP(hipMemcpy(ipiv_out, h->trace_piv, c * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (c > 0 && gaps_out)
    PLU_TRY_HIP(hipMemcpy(gaps_out, h->trace_gaps, c * sizeof(float), hipMemcpyDeviceToHost));
  if (h->trace_need > h->trace_n) return PLU_ERR_OOM;   // the device trace was too small
  return PLU_OK;
}

int plu_batched(plu_handle h, int32_t count, plu_request* reqs, int32_t flags) {
  if (!h) return -1;
  if (count < 0) return -2;
  if (count == 0) return PLU_OK;
  if (!reqs) return -3;
  PLU_TRY_HIP(hipSetDevice(h->device));
  bool bad = false;
  std::vector<BatchProblem> probs((size_t)count);
  size_t total = 0;
  for (int i = 0; i < count; ++i) {
    plu_request& r = reqs[i];
    std::memset(&r.info, 0, sizeof(r.info));
    r.rank = 0;
    int64_t l = 0;
    const int c = check_request(r, &l);
    r.status = c;
    if (c) {
      bad = true;
      continue;
    }
    if (r.prec & PLU_PREC_FP64_INDICATOR) {
      r.status = PLU_ERR_NOT_IMPLEMENTED;
      bad = true;
      continue;
    }
    BatchProblem& b = probs[(size_t)i];
    b.r = &r;
    b.l = l;
    // each problem rounds its own A into its own workspace on every call
    // (a batch keeps no copies between calls: PLU_PREC_A_UNCHANGED is moot)
    b.prec = r.prec & ~PLU_PREC_A_UNCHANGED;
    Layout dry;
    layout(dry, r.m, r.n, l, b.prec);
    b.bytes = ru((int64_t)(dry.off + 256), 256);
    b.off = total;
    total += b.bytes;
  }
  if (bad) return -3;
  // graph replay of an identical batch (the fixed-precision ranks stay on
  // the device, so every problem's launch sequence is known up front)
  const bool use_graph = (flags & PLU_BATCH_GRAPH) != 0;
  std::vector<unsigned char> sig;
  if (use_graph) {
    sig = batch_signature(reqs, count);
    if (h->gexec && sig == h->gsig && total <= h->batch_bytes) {
      PLU_TRY_HIP(hipGraphLaunch(h->gexec, h->stream));
      goto finish;
    }
  }
  if (total > h->batch_bytes) {
    PLU_TRY_HIP(hipStreamSynchronize(h->stream));
    drop_graph(h);   // its pointers refer to the old region
    if (h->batch_arena) (void)hipFree(h->batch_arena);
    h->batch_arena = nullptr;
    h->batch_bytes = 0;
    const size_t alloc = total + total / 8;
    if (hipMalloc(reinterpret_cast<void**>(&h->batch_arena), alloc) != hipSuccess) {
      (void)hipGetLastError();
      return PLU_ERR_OOM;
    }
    h->batch_bytes = alloc;
  }
  // the passes' splits tuned eagerly first, so that the recorded launches
  // below take the plans the single calls take (bitwise equal results in
  // either call order)
  if (!(use_graph && h->gexec && sig == h->gsig)) {
    for (BatchProblem& b : probs) {
      const plu_request& r = *b.r;
      Layout L;
      L.base = h->batch_arena + b.off;
      Ws w = layout(L, r.m, r.n, b.l, b.prec);
      w.acol = r.layout == PLU_COL_MAJOR;
      pretune_pass(h, w, 0, r.m, r.n, r.A, r.lda, w.om, w.lp, b.l, w.ym, w.lp);
      pretune_pass(h, w, 1, r.m, r.n, r.A, r.lda, w.om, w.lp, b.l, w.zn, w.lp);
      if (r.mode == 0) pretune_pass(h, w, 0, r.m, r.n, r.A, r.lda, w.om, w.lp, r.k, w.ym, w.lp);
    }
  }
  {
    std::vector<BatchProblem*> all;
    for (BatchProblem& b : probs) {
      b.hs = *h;
      b.hs.arena = h->batch_arena + b.off;
      b.hs.arena_bytes = b.bytes;
      b.hs.tag_counter = 0;   // first panel clears this problem's message slots
      b.hs.batch_arena = nullptr;
      b.hs.gexec = nullptr;
      b.hs.gstream = nullptr;
      b.hs.graph = nullptr;
      b.hs.trace_cap = 0;
      b.hs.mbuf = MergeBuffers();
      b.hs.gbuf = MergeBuffers();
      all.push_back(&b);
    }
    const bool one_stream = (flags & PLU_BATCH_ONE_STREAM) != 0;
    if (use_graph && !one_stream) {
      drop_graph(h);
      if (!h->gstream) PLU_TRY_HIP(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
      SidePlan sp;
      hipError_t pe = side_prepare(h, all, true, sp);
      if (pe != hipSuccess) return pe == hipErrorOutOfMemory ? PLU_ERR_OOM : PLU_ERR_HIP;
      PLU_TRY_HIP(hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal));
      hipError_t ce = side_launch(h, h->gstream, sp, true);
      hipGraph_t g = nullptr;
      hipError_t ee = hipStreamEndCapture(h->gstream, &g);
      if (ce != hipSuccess || ee != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        std::fprintf(stderr, "libpowerlu: batch graph capture failed: %s / %s\n",
                     hipGetErrorString(ce), hipGetErrorString(ee));
        if (ce == hipErrorOutOfMemory) return PLU_ERR_OOM;
        return ce == hipErrorStreamCaptureUnsupported || ee == hipErrorStreamCaptureUnsupported
                   ? PLU_ERR_NOT_IMPLEMENTED
                   : PLU_ERR_HIP;
      }
      h->graph = g;
      PLU_TRY_HIP(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
      h->gsig = sig;
      PLU_TRY_HIP(hipGraphLaunch(h->gexec, h->stream));
    } else if (!one_stream) {
      SidePlan sp;
      hipError_t e = side_prepare(h, all, false, sp);
      if (e == hipSuccess) e = side_launch(h, h->stream, sp, false);
      if (e != hipSuccess) return e == hipErrorOutOfMemory ? PLU_ERR_OOM : PLU_ERR_HIP;
    } else if (std::any_of(all.begin(), all.end(), rounded_form)) {
      // one stream with a rounded-form problem: every problem directly, one
      // after the other (captured as they are launched for a graph)
      hipStream_t s = h->stream;
      if (use_graph) {
        drop_graph(h);
        if (!h->gstream) PLU_TRY_HIP(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
        s = h->gstream;
        PLU_TRY_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      }
      hipError_t ce = hipSuccess;
      for (BatchProblem* b : all) {
        b->hs.stream = s;
        if ((ce = batch_phase_a(*b)) != hipSuccess) break;
      }
      if (use_graph) {
        hipGraph_t g = nullptr;
        hipError_t ee = hipStreamEndCapture(s, &g);
        if (ce != hipSuccess || ee != hipSuccess || !g) {
          if (g) (void)hipGraphDestroy(g);
          (void)hipGetLastError();
          std::fprintf(stderr, "libpowerlu: batch graph capture failed: %s / %s\n",
                       hipGetErrorString(ce), hipGetErrorString(ee));
          if (ce == hipErrorOutOfMemory) return PLU_ERR_OOM;
          return ce == hipErrorStreamCaptureUnsupported || ee == hipErrorStreamCaptureUnsupported
                     ? PLU_ERR_NOT_IMPLEMENTED
                     : PLU_ERR_HIP;
        }
        h->graph = g;
        PLU_TRY_HIP(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
        h->gsig = sig;
        PLU_TRY_HIP(hipGraphLaunch(h->gexec, h->stream));
      } else if (ce != hipSuccess) {
        return ce == hipErrorOutOfMemory ? PLU_ERR_OOM : PLU_ERR_HIP;
      }
    } else if (use_graph) {
      drop_graph(h);
      // record, size the tables outside the capture, then capture the launches
      std::vector<const Recorder*> lists;
      for (BatchProblem* b : all) {
        thread_recorder() = &b->rec;
        hipError_t e = batch_phase_a(*b);
        thread_recorder() = nullptr;
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? PLU_ERR_OOM : PLU_ERR_HIP;
        lists.push_back(&b->rec);
      }
      PLU_TRY_HIP(h->gbuf.reserve(merged_table_bytes(lists, h->cu_count)));
      if (!h->gstream) PLU_TRY_HIP(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
      h->gbuf.capturing = true;
      PLU_TRY_HIP(hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal));
      hipError_t ce = run_merged(lists, h->gstream, h->cu_count, h->gbuf, nullptr);
      hipGraph_t g = nullptr;
      hipError_t ee = hipStreamEndCapture(h->gstream, &g);
      h->gbuf.capturing = false;
      if (ce != hipSuccess || ee != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        std::fprintf(stderr, "libpowerlu: batch graph capture failed: %s / %s\n",
                     hipGetErrorString(ce), hipGetErrorString(ee));
        return ce == hipErrorStreamCaptureUnsupported || ee == hipErrorStreamCaptureUnsupported
                   ? PLU_ERR_NOT_IMPLEMENTED
                   : PLU_ERR_HIP;
      }
      h->graph = g;
      PLU_TRY_HIP(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
      h->gsig = sig;
      PLU_TRY_HIP(hipGraphLaunch(h->gexec, h->stream));
    } else {
      hipError_t e = record_and_run(h, all, batch_phase_a, h->mbuf, false, nullptr);
      if (e != hipSuccess) return e == hipErrorOutOfMemory ? PLU_ERR_OOM : PLU_ERR_HIP;
    }
  }
finish:
  PLU_TRY_HIP(hipStreamSynchronize(h->stream));
  for (int i = 0; i < count; ++i) {
    plu_request& r = reqs[i];
    // the workspace of problem i (same layout as when it was recorded)
    Layout L;
    L.base = h->batch_arena + probs[(size_t)i].off;
    int64_t l = probs[(size_t)i].l;
    const Ws w = layout(L, r.m, r.n, l, probs[(size_t)i].prec);
    if (r.mode == 0) {
      r.rank = r.k;
      r.status = finish_info(h, w, PLU_OK, r.k, r.v, (int)l, false, &r.info);
    } else {
      r.status = finish_info(h, w, PLU_OK, -1, r.v, (int)l, true, &r.info);
      r.rank = r.info.rank;
    }
  }
  return PLU_OK;
}

int plu_server_create(plu_server* out, int device, size_t hbm_budget_bytes, int32_t max_slots) {
  if (!out) return -1;
  if (max_slots < 1) return -4;
  plu_handle h = nullptr;
  int rc = plu_create(&h, device, nullptr);
  if (rc) return rc;
  plu_server S = new plu_server_s();
  S->h = h;
  S->device = device;
  S->max_slots = max_slots;
  S->t0 = std::chrono::steady_clock::now();
  if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
    plu_destroy(h);
    delete S;
    return PLU_ERR_HIP;
  }
  h->stream = S->stream;
  // copy-out runs on several threads: one would serialize the staging copies
  constexpr int kFinishers = 4;
  S->fins = std::vector<plu_server_s::Finisher>(kFinishers);
  auto drop_streams = [&]() {
    for (auto& f : S->fins)
      if (f.cs) (void)hipStreamDestroy(f.cs);
    if (S->ustream) (void)hipStreamDestroy(S->ustream);
    (void)hipStreamDestroy(S->stream);
  };
  bool ok = hipStreamCreateWithFlags(&S->ustream, hipStreamNonBlocking) == hipSuccess;
  if (!ok) S->ustream = nullptr;
  for (auto& f : S->fins)
    if (ok && hipStreamCreateWithFlags(&f.cs, hipStreamNonBlocking) != hipSuccess) {
      f.cs = nullptr;
      ok = false;
    }
  if (!ok) {
    drop_streams();
    plu_destroy(h);
    delete S;
    return PLU_ERR_HIP;
  }
  S->stage.assign(max_slots, nullptr);
  S->stage_cap.assign(max_slots, 0);
  for (int i = max_slots - 1; i >= 0; --i) S->free_slots.push_back(i);
  if (!S->pool.init(hbm_budget_bytes)) {
    drop_streams();
    plu_destroy(h);
    delete S;
    return PLU_ERR_OOM;
  }
  S->worker = std::thread(server_loop, S);
  for (int i = 0; i < kFinishers; ++i) S->fins[i].th = std::thread(server_finisher, S, i);
  *out = S;
  return PLU_OK;
}

int plu_server_submit(plu_server S, const plu_request* req, uint64_t* ticket) {
  if (!S) return -1;
  if (!req) return -2;
  if (!ticket) return -3;
  int64_t l = 0;
  const int c = check_request(*req, &l);
  if (c) return c;
  if (req->prec & PLU_PREC_FP64_INDICATOR) return PLU_ERR_NOT_IMPLEMENTED;
  auto j = std::make_unique<ServerJob>();
  j->host = *req;
  j->cap = req->mode == 0 ? req->k : l;
  j->pool_bytes = server_footprint(*req, l, j->cap, &j->ws_bytes);
  if (j->pool_bytes > S->pool.size) return PLU_ERR_OOM;
  std::lock_guard<std::mutex> lk(S->mu);
  j->ticket = S->next_ticket++;
  j->res.ticket = j->ticket;
  j->res.t_submit = now_s(S->t0);
  *ticket = j->ticket;
  S->pending.push_back(std::move(j));
  S->cv_work.notify_one();
  return PLU_OK;
}

int plu_server_poll(plu_server S, uint64_t ticket, plu_result* res) {
  if (!S) return -1;
  if (!res) return -3;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->done.find(ticket);
  if (it == S->done.end()) return ticket < S->next_ticket ? PLU_PENDING : -2;
  *res = it->second;
  return PLU_OK;
}

int plu_server_wait(plu_server S, uint64_t ticket, plu_result* res) {
  if (!S) return -1;
  if (!res) return -3;
  std::unique_lock<std::mutex> lk(S->mu);
  if (ticket == 0 || ticket >= S->next_ticket) return -2;
  S->cv_done.wait(lk, [&] { return S->done.count(ticket) > 0; });
  *res = S->done[ticket];
  return PLU_OK;
}

int plu_server_destroy(plu_server S) {
  if (!S) return -1;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->cv_work.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->cv_fin.notify_all();
  }
  for (auto& f : S->fins)
    if (f.th.joinable()) f.th.join();
  (void)hipStreamSynchronize(S->stream);
  if (const char* e = std::getenv("PLU_SERVER_STATS"); e && e[0] == '1')
    std::fprintf(stderr,
                 "libpowerlu server: %zu batches (on average %.1f problems with steps left, %.1f "
                 "admitted, %.1f pending; %zu admission stops on the budget), "
                 "%zu grouped launches carrying %zu steps; worker seconds: idle %.2f, device wait "
                 "%.2f, recording %.2f, issuing %.2f; finisher seconds copying out (all threads) %.2f\n",
                 S->batches, S->batches ? (double)S->sum_ready / S->batches : 0.0,
                 S->batches ? (double)S->sum_active / S->batches : 0.0,
                 S->batches ? (double)S->sum_pending / S->batches : 0.0, S->budget_stops,
                 S->stats.launches, S->stats.recorded, S->t_idle, S->t_devwait, S->t_record,
                 S->t_issue, S->t_copyout);
  if (const char* e = std::getenv("PLU_SERVER_STATS"); e && e[0] == '1' && S->n_done)
    std::fprintf(stderr,
                 "libpowerlu server: mean ms from admission: upload %.2f, then all steps issued "
                 "%.2f, then complete %.2f, then copied out %.2f\n",
                 1e3 * S->s_up / S->n_done, 1e3 * S->s_issue / S->n_done,
                 1e3 * S->s_compute / S->n_done, 1e3 * S->s_out / S->n_done);
  for (hipEvent_t e : S->events) (void)hipEventDestroy(e);
  if (S->pool.base) (void)hipFree(S->pool.base);
  for (unsigned char* p : S->stage)
    if (p) (void)hipHostFree(p);
  for (auto& f : S->fins) {
    if (f.ostage) (void)hipHostFree(f.ostage);
    (void)hipStreamDestroy(f.cs);
  }
  plu_destroy(S->h);
  (void)hipStreamDestroy(S->ustream);
  (void)hipStreamDestroy(S->stream);
  delete S;
  return PLU_OK;
}

}  // extern "C"
