// C ABI of libpowerlu and the drivers that sequence the kernels:
//   * fixed rank: Alg. 5 with Alg. 7 as its steps 1-2 (Sec. 3.1, 3.4);
//   * fixed precision: Alg. 9 on Alg. 8 / Alg. 11 with the Thm 4.3 indicator.
// The host only enqueues work on the handle's stream; it synchronizes only to
// fill a plu_info, to read the fixed-precision rank, or for plu_residual.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/powerlu.h"
#include "plu_internal.h"

using namespace plu;

struct plu_handle_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int cu_count = 256;
  uint64_t timeout_ticks = 0;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  uint32_t tag_counter = 0;
  size_t msg_off = 0, msg_words = 0;
};

namespace {

constexpr int kQB = 128;
constexpr int kMaxGramChunks = 256;
constexpr int kTargetWgs = 1024;  // concurrent pass workgroups: 4 per CU on 256 CUs
constexpr int kMaxSplit = 16;

inline int64_t ru4(int64_t x) { return (x + 3) & ~int64_t(3); }
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
  int64_t sumsq_cap, colsq_cap;
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

Ws layout(Layout& L, int64_t m, int64_t n, int64_t l) {
  Ws w{};
  const int64_t Mx = std::max(m, n);
  const int64_t lp = ru4(std::max<int64_t>(l, 4));
  w.lp = lp;
  w.om = L.take<float>(Mx * lp);
  w.ym = L.take<float>(m * lp);
  w.zn = L.take<float>(n * lp);
  w.qb = L.take<float>(Mx * lp);
  w.tmp = L.take<float>(Mx * kQB);
  w.bt = L.take<float>(n * lp);
  w.part_cap = std::max<int64_t>(part_need(m, n, l), 1);
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
  w.gram_part = L.take<double>((size_t)kMaxGramChunks * kQB * kQB);
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
  return w;
}

int ensure_ws(plu_handle h, int64_t m, int64_t n, int64_t l, Ws* out) {
  Layout dry;
  layout(dry, m, n, l);
  const size_t need = dry.off + 256;
  if (need > h->arena_bytes) {
    if (h->arena) {
      hipStreamSynchronize(h->stream);
      hipFree(h->arena);
      h->arena = nullptr;
      h->arena_bytes = 0;
    }
    const size_t alloc = need + need / 8;
    if (hipMalloc(reinterpret_cast<void**>(&h->arena), alloc) != hipSuccess) {
      hipGetLastError();
      return PLU_ERR_OOM;
    }
    h->arena_bytes = alloc;
    h->tag_counter = 0;   // next panel launch clears the message buffer
  }
  Layout L;
  L.base = h->arena;
  *out = layout(L, m, n, l);
  if (h->tag_counter == 0) {
    if (launch_fill_u32(reinterpret_cast<uint32_t*>(out->msg), out->msg_words * 2, 0u, h->stream) !=
        hipSuccess)
      return PLU_ERR_HIP;
  }
  // per-call status words: zero-pivot slots to "none", flags to 0
  if (launch_fill_u32(reinterpret_cast<uint32_t*>(out->status), 32, 0x7FFFFFFFu, h->stream) !=
          hipSuccess ||
      launch_fill_u32(reinterpret_cast<uint32_t*>(out->status + 32), 32, 0u, h->stream) !=
          hipSuccess)
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
  g.tag_counter = &h->tag_counter;
  g.timeout_ticks = h->timeout_ticks;
  g.max_waves = h->cu_count * 8;
  return g;
}

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
hipError_t run_pass(plu_handle h, const Ws& w, int trans, int64_t m, int64_t n, const float* A,
                    int64_t lda, const float* X, int64_t ldx, int64_t l, float* out, int64_t ldo,
                    double* normA2_dev, double* colsq, int* colsq_blocks) {
  const int64_t P = trans ? n : m, R = trans ? m : n;
  GemmPlan pl = plan_gemm(P, R, l, kMaxSplit, kTargetWgs);
  if (pl.nsplit > 1 && (int64_t)pl.nsplit * P * ldo > w.part_cap) pl = plan_gemm(P, R, l, 1, 1);
  GemmArgs g;
  g.A = A; g.lda = lda; g.X = X; g.ldx = ldx;
  g.P = P; g.R = R; g.C = l;
  if (normA2_dev) {
    if ((int64_t)pl.pblocks * pl.nsplit > w.sumsq_cap) return hipErrorInvalidValue;
    g.sumsq_part = w.sumsq_part;
  }
  hipError_t e;
  const int rb = 64;
  if (pl.nsplit > 1) {
    g.out = w.part; g.ldo = ldo; g.part_stride = P * ldo;
    if ((e = launch_gemm(trans, EPI_PART, 0, g, pl, h->stream)) != hipSuccess) return e;
    if ((e = launch_splitk_reduce(w.part, P * ldo, pl.nsplit, out, ldo, P, l, colsq, rb,
                                  h->stream)) != hipSuccess)
      return e;
  } else {
    g.out = out; g.ldo = ldo;
    if ((e = launch_gemm(trans, EPI_STORE, 0, g, pl, h->stream)) != hipSuccess) return e;
    if (colsq) {
      if ((e = launch_splitk_reduce(out, 0, 1, nullptr, ldo, P, l, colsq, rb, h->stream)) !=
          hipSuccess)
        return e;
    }
  }
  if (colsq_blocks) *colsq_blocks = (int)((P + rb - 1) / rb);
  if (normA2_dev) {
    if ((e = launch_sum_doubles(w.sumsq_part, (int64_t)pl.pblocks * pl.nsplit, normA2_dev,
                                h->stream)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

// Alg. 7.  Leaves the orthonormal n x l basis in *Vout (one of the workspace
// buffers, leading dimension w.lp); passes counted in *passes.
hipError_t range_basis(plu_handle h, const Ws& w, int64_t m, int64_t n, const float* A, int64_t lda,
                       int l, int v, const float* Omega, uint64_t seed, float** Vout,
                       int* passes) {
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
  if (v % 2 == 0) {
    if ((e = run_pass(h, w, 1, m, n, A, lda, w.om, lp, l, w.zn, lp, first ? normA2 : nullptr,
                      nullptr, nullptr)) != hipSuccess)
      return e;
    first = false;
    ++np;
    if (v > 2) {
      if ((e = getrf_run(w.zn, lp, n, l, gw, nullptr, nullptr, 0, 0, h->stream)) != hipSuccess)
        return e;
      V = w.zn;
    } else {
      if ((e = thin_qr_run(w.zn, lp, n, l, gw, qw, h->stream)) != hipSuccess) return e;
      V = w.qb;
    }
  } else {
    V = w.om;
  }
  for (int i = 1; i <= P; ++i) {
    if ((e = run_pass(h, w, 0, m, n, A, lda, V, lp, l, w.ym, lp, first ? normA2 : nullptr, nullptr,
                      nullptr)) != hipSuccess)
      return e;
    first = false;
    ++np;
    if ((e = getrf_run(w.ym, lp, m, l, gw, nullptr, nullptr, 0, 0, h->stream)) != hipSuccess)
      return e;
    if ((e = run_pass(h, w, 1, m, n, A, lda, w.ym, lp, l, w.zn, lp, nullptr, nullptr, nullptr)) !=
        hipSuccess)
      return e;
    ++np;
    if (i == P) {
      if ((e = thin_qr_run(w.zn, lp, n, l, gw, qw, h->stream)) != hipSuccess) return e;
      V = w.qb;
    } else {
      if ((e = getrf_run(w.zn, lp, n, l, gw, nullptr, nullptr, 0, 0, h->stream)) != hipSuccess)
        return e;
      V = w.zn;
    }
  }
  *Vout = V;
  *passes = np;
  return hipSuccess;
}

// Alg. 5 steps 4-8 given Y = A V(:, :k) in w.ym (leading dimension lp) and V.
hipError_t assemble(plu_handle h, const Ws& w, int64_t m, int64_t n, int k, const float* V,
                    int32_t* p, int32_t* q, float* L, int64_t ldl, float* U, int64_t ldu) {
  const int64_t lp = w.lp;
  hipError_t e;
  const GetrfWork g1 = getrf_work(h, w, 1);
  const GetrfWork g2 = getrf_work(h, w, 2);
  // [L1, U1, P] = lu(Y): ym <- P^T L1, ut1 <- U1^T
  if ((e = getrf_run(w.ym, lp, m, k, g1, p, w.ut1, lp, 1, h->stream)) != hipSuccess) return e;
  // B^T = V(:, :k) U1^T  (n x k)
  {
    GemmArgs g;
    g.A = V; g.lda = lp; g.X = w.ut1; g.ldx = lp; g.out = w.bt; g.ldo = lp;
    g.P = n; g.R = k; g.C = k;
    if ((e = launch_gemm(0, EPI_STORE, 0, g, plan_gemm(n, k, k, 1, 1), h->stream)) != hipSuccess)
      return e;
  }
  // [L2, U2, Q] = lu(B^T): bt <- Q^T L2, ut2 <- U2^T
  if ((e = getrf_run(w.bt, lp, n, k, g2, q, w.ut2, lp, 1, h->stream)) != hipSuccess) return e;
  // L = L1 U2^T with L1 = (P^T L1)[p]
  {
    GemmArgs g;
    g.A = w.ym; g.lda = lp; g.arow = p; g.X = w.ut2; g.ldx = lp; g.out = L; g.ldo = ldl;
    g.P = m; g.R = k; g.C = k;
    if ((e = launch_gemm(0, EPI_STORE, 0, g, plan_gemm(m, k, k, 1, 1), h->stream)) != hipSuccess)
      return e;
  }
  // U = L2^T with L2 = (Q^T L2)[q]
  return launch_transpose_gather(w.bt, lp, q, n, k, U, ldu, h->stream);
}

int finish_info(plu_handle h, const Ws& w, int status, int rank, int passes, int l, bool fp,
                plu_info* info) {
  if (!info) return status;
  PLU_TRY_HIP(hipStreamSynchronize(h->stream));
  int32_t st[40];
  double sc[4];
  PLU_TRY_HIP(hipMemcpy(st, w.status, sizeof(st), hipMemcpyDeviceToHost));
  PLU_TRY_HIP(hipMemcpy(sc, w.scal, sizeof(sc), hipMemcpyDeviceToHost));
  std::memset(info, 0, sizeof(*info));
  info->rank = rank;
  info->passes = passes;
  info->l = l;
  info->normA2 = sc[0];
  info->E_final = fp ? sc[1] : 0.0;
  info->tol_reached = fp ? 1 : 0;
  int zp = INT32_MAX;
  bool timeout = false;
  if (st[32] != 0) timeout = true;
  for (int wch = 1; wch <= 2; ++wch) zp = std::min(zp, st[4 * wch]);
  info->zero_pivot_step = (zp == INT32_MAX) ? -1 : zp;
  float mg = 1.f;
  if (rank > 0) {
    std::vector<float> g(2 * rank);
    PLU_TRY_HIP(hipMemcpy(g.data(), w.gaps1, rank * sizeof(float), hipMemcpyDeviceToHost));
    PLU_TRY_HIP(hipMemcpy(g.data() + rank, w.gaps2, rank * sizeof(float), hipMemcpyDeviceToHost));
    for (float x : g) mg = std::min(mg, x);
  }
  info->min_pivot_gap = mg;
  if (timeout) status = PLU_ERR_TIMEOUT;
  else if (!std::isfinite(sc[0])) status = PLU_ERR_NONFINITE;
  else if (status == PLU_OK && info->zero_pivot_step >= 0) status = PLU_WARN_ZERO_PIVOT;
  info->status = status;
  return status;
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
  // bound on any device-side wait: 5 seconds of the constant-rate wall clock
  h->timeout_ticks = (uint64_t)(clk_khz > 0 ? clk_khz : 100000) * 1000ull * 5ull;
  *out = h;
  return PLU_OK;
}

int plu_destroy(plu_handle h) {
  if (!h) return -1;
  if (h->arena) {
    hipStreamSynchronize(h->stream);
    hipFree(h->arena);
  }
  delete h;
  return PLU_OK;
}

int plu_set_stream(plu_handle h, void* hip_stream) {
  if (!h) return -1;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return PLU_OK;
}

int plu_workspace_size(plu_handle h, int64_t m, int64_t n, int32_t l, size_t* bytes) {
  if (!h) return -1;
  if (m <= 0) return -2;
  if (n <= 0) return -3;
  if (l <= 0) return -4;
  if (!bytes) return -5;
  Layout dry;
  layout(dry, m, n, l);
  *bytes = dry.off + 256;
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
  if (prec != PLU_PREC_FP32) return prec == PLU_PREC_BF16 ? PLU_ERR_NOT_IMPLEMENTED : -12;
  PLU_TRY_HIP(hipSetDevice(h->device));
  Ws w;
  int st = ensure_ws(h, m, n, l, &w);
  if (st) return st;
  const int64_t P = trans ? n : m;
  // the split-K scratch uses the output's leading dimension
  if (ru4(ldo) != ldo && plan_gemm(P, trans ? m : n, l, kMaxSplit, kTargetWgs).nsplit > 1) {
    // fall through: run_pass keeps the partials at ldo, fine for any ldo
  }
  PLU_TRY_HIP(run_pass(h, w, trans, m, n, A, lda, X, ldx, l, out, ldo, normA2_out, nullptr,
                       nullptr));
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
  PLU_TRY_HIP(getrf_run(F, ldf, M, c, g, perm, Ufac, ldu, 0, h->stream));
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

int plu_range_basis(plu_handle h, int64_t m, int64_t n, const float* A, int64_t lda, int32_t l,
                    int32_t v, int32_t prec, const float* Omega, uint64_t seed, float* V,
                    int64_t ldv) {
  if (!h) return -1;
  if (m <= 0) return -2;
  if (n <= 0) return -3;
  if (!A || (reinterpret_cast<uintptr_t>(A) & 3u)) return -4;
  if (lda < n) return -5;
  if (l <= 0 || l >= std::min(m, n)) return -6;
  if (v < 2) return -7;
  if (prec != PLU_PREC_FP32) return prec == PLU_PREC_BF16 ? PLU_ERR_NOT_IMPLEMENTED : -8;
  if (!V) return -11;
  if (ldv < l) return -12;
  PLU_TRY_HIP(hipSetDevice(h->device));
  Ws w;
  int st = ensure_ws(h, m, n, l, &w);
  if (st) return st;
  float* Vw = nullptr;
  int np = 0;
  PLU_TRY_HIP(range_basis(h, w, m, n, A, lda, l, v, Omega, seed, &Vw, &np));
  PLU_TRY_HIP(hipMemcpy2DAsync(V, ldv * sizeof(float), Vw, w.lp * sizeof(float),
                               l * sizeof(float), n, hipMemcpyDeviceToDevice, h->stream));
  return PLU_OK;
}

int plu_fixed_rank(plu_handle h, int64_t m, int64_t n, const float* A, int64_t lda, int32_t k,
                   int32_t p_over, int32_t v, int32_t prec, const float* Omega, uint64_t seed,
                   int32_t* p, int32_t* q, float* L, int64_t ldl, float* U, int64_t ldu,
                   plu_info* info) {
  if (!h) return -1;
  if (m <= 0) return -2;
  if (n <= 0) return -3;
  if (!A || (reinterpret_cast<uintptr_t>(A) & 3u)) return -4;
  if (lda < n) return -5;
  if (k < 1) return -6;
  if (p_over < 0) return -7;
  const int64_t l = (int64_t)k + p_over;
  if (l >= std::min(m, n)) return -7;
  if (v < 2) return -8;
  if (prec != PLU_PREC_FP32) return prec == PLU_PREC_BF16 ? PLU_ERR_NOT_IMPLEMENTED : -9;
  if (!p) return -12;
  if (!q) return -13;
  if (!L) return -14;
  if (ldl < k) return -15;
  if (!U) return -16;
  if (ldu < n) return -17;
  PLU_TRY_HIP(hipSetDevice(h->device));
  Ws w;
  int st = ensure_ws(h, m, n, l, &w);
  if (st) return st;
  float* V = nullptr;
  int np = 0;
  PLU_TRY_HIP(range_basis(h, w, m, n, A, lda, (int)l, v, Omega, seed, &V, &np));
  // final pass: Y = A V(:, 1:k)
  PLU_TRY_HIP(run_pass(h, w, 0, m, n, A, lda, V, w.lp, k, w.ym, w.lp, nullptr, nullptr, nullptr));
  ++np;
  PLU_TRY_HIP(assemble(h, w, m, n, k, V, p, q, L, ldl, U, ldu));
  return finish_info(h, w, PLU_OK, k, np, (int)l, false, info);
}

int plu_fixed_precision(plu_handle h, int64_t m, int64_t n, const float* A, int64_t lda,
                        double eps, int32_t b, int32_t l, int32_t v, int32_t column_exact,
                        int32_t prec, const float* Omega, uint64_t seed, int32_t* p, int32_t* q,
                        float* L, int64_t ldl, float* U, int64_t ldu, int32_t* rank_out,
                        plu_info* info) {
  if (!h) return -1;
  if (m <= 0) return -2;
  if (n <= 0) return -3;
  if (!A || (reinterpret_cast<uintptr_t>(A) & 3u)) return -4;
  if (lda < n) return -5;
  if (!(eps > 0.0)) return -6;
  if (b < 1) return -7;
  const int64_t mn = std::min(m, n);
  if (l == 0) l = (int32_t)std::min<int64_t>(50LL * b, b * ((mn - 1) / b));
  if (l <= 0 || l % b != 0 || l >= mn) return -8;
  if (v < 2) return -9;
  if (prec != PLU_PREC_FP32) return prec == PLU_PREC_BF16 ? PLU_ERR_NOT_IMPLEMENTED : -11;
  if (!p) return -14;
  if (!q) return -15;
  if (!L) return -16;
  if (ldl < l) return -17;
  if (!U) return -18;
  if (ldu < n) return -19;
  PLU_TRY_HIP(hipSetDevice(h->device));
  Ws w;
  int st = ensure_ws(h, m, n, l, &w);
  if (st) return st;
  float* V = nullptr;
  int np = 0;
  PLU_TRY_HIP(range_basis(h, w, m, n, A, lda, l, v, Omega, seed, &V, &np));
  // G = A V with column norms^2 (float64) fused into the reduction
  int nblk = 0;
  PLU_TRY_HIP(run_pass(h, w, 0, m, n, A, lda, V, w.lp, l, w.ym, w.lp, nullptr, w.colsq_part,
                       &nblk));
  ++np;
  // float64 squared norms of the basis columns (first-order normalization)
  PLU_TRY_HIP(launch_splitk_reduce(V, 0, 1, nullptr, w.lp, n, l, w.vsq_part, 64, h->stream));
  const int nvblk = (int)((n + 63) / 64);
  PLU_TRY_HIP(launch_rank_rule(w.colsq_part, nblk, l, w.vsq_part, nvblk, w.scal + 0, eps, b,
                               column_exact ? 1 : 0, w.iscal + 0, w.scal + 1, w.iscal + 1,
                               w.colnorm, h->stream));
  PLU_TRY_HIP(hipStreamSynchronize(h->stream));
  int32_t ks[2];
  double sc[2];
  PLU_TRY_HIP(hipMemcpy(ks, w.iscal, sizeof(ks), hipMemcpyDeviceToHost));
  PLU_TRY_HIP(hipMemcpy(sc, w.scal, sizeof(sc), hipMemcpyDeviceToHost));
  const int k = ks[0];
  const bool tol_ok = ks[1] != 0;
  if (!std::isfinite(sc[0])) {
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->status = PLU_ERR_NONFINITE;
      info->normA2 = sc[0];
    }
    return PLU_ERR_NONFINITE;
  }
  if (rank_out) *rank_out = k;
  int status = tol_ok ? PLU_OK : PLU_TOL_NOT_REACHED;
  if (k == 0) {
    PLU_TRY_HIP(launch_iota(p, m, h->stream));
    PLU_TRY_HIP(launch_iota(q, n, h->stream));
  } else {
    PLU_TRY_HIP(assemble(h, w, m, n, k, V, p, q, L, ldl, U, ldu));
  }
  int rs = finish_info(h, w, status, k, np, l, true, info);
  if (info) info->tol_reached = tol_ok ? 1 : 0;
  return info ? rs : status;
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

int plu_residual(plu_handle h, int64_t m, int64_t n, const float* A, int64_t lda,
                 const int32_t* p, const int32_t* q, int32_t k, const float* L, int64_t ldl,
                 const float* U, int64_t ldu, double* rel_resid) {
  if (!h) return -1;
  if (m <= 0) return -2;
  if (n <= 0) return -3;
  if (!A) return -4;
  if (lda < n) return -5;
  if (!p) return -6;
  if (!q) return -7;
  if (k < 1) return -8;
  if (!L) return -9;
  if (ldl < k) return -10;
  if (!U) return -11;
  if (ldu < n) return -12;
  if (!rel_resid) return -13;
  PLU_TRY_HIP(hipSetDevice(h->device));
  char* extra = nullptr;
  const GemmPlan pl = plan_gemm(m, k, n, 1, 1);
  const int64_t nparts = (int64_t)pl.pblocks * pl.cblocks;
  const int sq_blocks = 1024;
  const size_t bytes = (nparts + sq_blocks + 2) * sizeof(double) + 1024;
  if (hipMalloc(reinterpret_cast<void**>(&extra), bytes) != hipSuccess) {
    hipGetLastError();
    return PLU_ERR_OOM;
  }
  Layout lay;
  lay.base = extra;
  double* rpart = lay.take<double>(nparts);
  double* spart = lay.take<double>(sq_blocks);
  double* sums = lay.take<double>(2);
  int rc = PLU_OK;
  do {
    GemmArgs g;
    g.A = L; g.lda = ldl; g.X = U; g.ldx = ldu;
    g.P = m; g.R = k; g.C = n;
    g.Aref = A; g.ldaref = lda; g.pidx = p; g.qidx = q; g.resid_part = rpart;
    if (launch_gemm(0, EPI_RESID, 0, g, pl, h->stream) != hipSuccess) { rc = PLU_ERR_HIP; break; }
    if (launch_sum_doubles(rpart, nparts, sums + 0, h->stream) != hipSuccess) { rc = PLU_ERR_HIP; break; }
    if (launch_sumsq_matrix(A, lda, m, n, spart, sq_blocks, h->stream) != hipSuccess) { rc = PLU_ERR_HIP; break; }
    if (launch_sum_doubles(spart, sq_blocks, sums + 1, h->stream) != hipSuccess) { rc = PLU_ERR_HIP; break; }
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

}  // extern "C"
