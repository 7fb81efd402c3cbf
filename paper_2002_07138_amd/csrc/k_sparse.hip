// Sparse A in compressed rows (the paper's sprand inputs, Sec. 6.1, second
// experiment): the passes A X and A^T Y, and the one-time build of the
// transposed index that makes both of them row-parallel gathers.
//
//   * out = S X for S in compressed rows: one wave per row; every stored
//     entry (i, j, v) adds v X(j, :) into the row's accumulators, the lanes
//     spanning the l columns of X (a coalesced gather of one row of X per
//     entry).  No atomics: each output row is summed in storage order.
//   * A^T Y runs the same kernel on the compressed columns of A (compressed
//     rows of A^T), built once per matrix: column counts, an exclusive scan,
//     a scatter, and a sort of every column's entries by row index, so the
//     transposed storage (and every result) is independent of scheduling.
//   * ||A||_F^2 in float64 from the stored values, summed in a fixed order.
#include "plu_internal.h"

namespace plu {

namespace {

constexpr int SPMM_WAVES = 4;    // rows per workgroup, one wave each
constexpr int SPMM_CPL = 4;      // 64-column chunks a lane holds (256 columns per sweep)

struct SpmmArgs {
  const int64_t* ptr; const int32_t* idx; const float* val; int64_t rows;
  const float* X; int64_t ldx; int l; float* out; int64_t ldo;
};

__device__ void b_spmm(const SpmmArgs& a, const Grid& gr) {
  const int lane = threadIdx.x & 63;
  const int64_t i =
      (int64_t)gr.bx * SPMM_WAVES + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (i >= a.rows) return;
  const int64_t e0 = a.ptr[i], e1 = a.ptr[i + 1];
  const float* __restrict__ X = a.X;
  for (int c0 = 0; c0 < a.l; c0 += 64 * SPMM_CPL) {
    float acc[SPMM_CPL];
    bool on[SPMM_CPL];
#pragma unroll
    for (int t = 0; t < SPMM_CPL; ++t) {
      acc[t] = 0.f;
      on[t] = c0 + lane + 64 * t < a.l;
    }
    int64_t e = e0;
    for (; e + 4 <= e1; e += 4) {
      int64_t j[4];
      float v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        j[u] = a.idx[e + u];
        v[u] = a.val[e + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < SPMM_CPL; ++t)
          if (on[t]) acc[t] = fmaf(v[u], X[j[u] * a.ldx + c0 + lane + 64 * t], acc[t]);
    }
    for (; e < e1; ++e) {
      const int64_t j = a.idx[e];
      const float v = a.val[e];
#pragma unroll
      for (int t = 0; t < SPMM_CPL; ++t)
        if (on[t]) acc[t] = fmaf(v, X[j * a.ldx + c0 + lane + 64 * t], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < SPMM_CPL; ++t)
      if (on[t]) a.out[i * a.ldo + c0 + lane + 64 * t] = acc[t];
  }
}

// Structure check: ptr[0] = 0, ptr non-decreasing, ptr[rows] = nnz (bit 1 of
// *bad), every idx in [0, cols) (bit 2), set with a vector atomic.
struct ValidateArgs {
  const int64_t* ptr; const int32_t* idx; int64_t rows, cols, nnz; int32_t* bad;
};

__device__ void b_validate(const ValidateArgs& a, const Grid& gr) {
  const int64_t t = (int64_t)gr.bx * 256 + threadIdx.x;
  int wrong = 0;
  if (t <= a.rows) {
    const int64_t p = a.ptr[t];
    if (t == 0 && p != 0) wrong |= 1;
    if (t == a.rows && p != a.nnz) wrong |= 1;
    if (t < a.rows && a.ptr[t + 1] < p) wrong |= 1;
  }
  if (t < a.nnz) {
    const int32_t j = a.idx[t];
    if (j < 0 || (int64_t)j >= a.cols) wrong |= 2;
  }
  if (wrong) atomicOr(a.bad, wrong);
}

struct CountArgs { const int32_t* idx; int64_t nnz; int32_t* cnt; };

__device__ void b_count(const CountArgs& a, const Grid& gr) {
  const int64_t e = (int64_t)gr.bx * 256 + threadIdx.x;
  if (e < a.nnz) atomicAdd(&a.cnt[a.idx[e]], 1);
}

// Exclusive scan of cnt[0 .. n) into ptr[0 .. n] (ptr[n] = total), one
// workgroup: each thread sums a contiguous chunk, the chunk totals are
// scanned in LDS, then each thread writes its chunk's prefixes.
struct ScanArgs { const int32_t* cnt; int64_t n; int64_t* ptr; };

__device__ void b_scan(const ScanArgs& a, const Grid& gr) {
  (void)gr;
  constexpr int T = 1024;
  __shared__ int64_t part[T];
  const int t = threadIdx.x;
  const int64_t chunk = (a.n + T - 1) / T;
  const int64_t b0 = (int64_t)t * chunk;
  const int64_t b1 = (b0 + chunk < a.n) ? b0 + chunk : a.n;
  int64_t s = 0;
  for (int64_t j = b0; j < b1; ++j) s += a.cnt[j];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {
    const int64_t v = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;       // exclusive prefix of this chunk
  for (int64_t j = b0; j < b1; ++j) {
    a.ptr[j] = run;
    run += a.cnt[j];
  }
  if (t == T - 1) a.ptr[a.n] = part[T - 1];
}

// Entries of row i go to their columns' segments (slot order within a column
// is arbitrary here; b_colsort fixes it).
struct ScatterArgs {
  const int64_t* ptr; const int32_t* idx; const float* val; int64_t rows;
  const int64_t* cptr; int32_t* cur; int32_t* ridx; float* cval;
};

__device__ void b_scatter(const ScatterArgs& a, const Grid& gr) {
  const int lane = threadIdx.x & 63;
  const int64_t i =
      (int64_t)gr.bx * SPMM_WAVES + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (i >= a.rows) return;
  for (int64_t e = a.ptr[i] + lane; e < a.ptr[i + 1]; e += 64) {
    const int32_t j = a.idx[e];
    const int64_t pos = a.cptr[j] + atomicAdd(&a.cur[j], 1);
    a.ridx[pos] = (int32_t)i;
    a.cval[pos] = a.val[e];
  }
}

// Insertion sort of one column's entries by row index (stable; a column of
// c entries costs O(c^2), which the sprand inputs keep small).
struct ColSortArgs { const int64_t* cptr; int64_t cols; int32_t* ridx; float* cval; };

__device__ void b_colsort(const ColSortArgs& a, const Grid& gr) {
  const int64_t j = (int64_t)gr.bx * 256 + threadIdx.x;
  if (j >= a.cols) return;
  const int64_t b = a.cptr[j], e = a.cptr[j + 1];
  for (int64_t x = b + 1; x < e; ++x) {
    const int32_t r = a.ridx[x];
    const float v = a.cval[x];
    int64_t y = x - 1;
    while (y >= b && a.ridx[y] > r) {
      a.ridx[y + 1] = a.ridx[y];
      a.cval[y + 1] = a.cval[y];
      --y;
    }
    a.ridx[y + 1] = r;
    a.cval[y + 1] = v;
  }
}

// part[b] = sum of val^2 over the b-th chunk of 256 * 16 stored values.
struct SqArgs { const float* val; int64_t nnz; double* part; };

__device__ void b_sumsq_vals(const SqArgs& a, const Grid& gr) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)gr.bx * 256 * 16;
  double s = 0.0;
#pragma unroll 4
  for (int u = 0; u < 16; ++u) {
    const int64_t e = base + (int64_t)u * 256 + t;
    if (e < a.nnz) s = fma((double)a.val[e], (double)a.val[e], s);
  }
  red[t] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  if (t == 0) a.part[gr.bx] = red[0];
}

}  // namespace

hipError_t launch_spmm(const int64_t* ptr, const int32_t* idx, const float* val, int64_t rows,
                       const float* X, int64_t ldx, int l, float* out, int64_t ldo,
                       hipStream_t s) {
  if (rows <= 0 || l <= 0) return hipSuccess;
  const unsigned g = (unsigned)((rows + SPMM_WAVES - 1) / SPMM_WAVES);
  return dispatch<SpmmArgs, b_spmm, 64 * SPMM_WAVES>(
      SpmmArgs{ptr, idx, val, rows, X, ldx, l, out, ldo}, dim3(g), 0, s);
}

size_t sparse_scratch_bytes(int64_t m, int64_t n, int64_t nnz) {
  (void)m;
  const int64_t nsq = (nnz + 4095) / 4096;
  return 256 + (size_t)(n + 1) * 8 + (size_t)nnz * 8 + (size_t)n * 4 + (size_t)(nsq + 1) * 8 + 64;
}

hipError_t sparse_build(SparseMat& S, void* mem, int32_t* bad_host, hipStream_t s) {
  // carve: colptr (n + 1 int64), rowidx (nnz int32), valsT (nnz float),
  // cnt (n int32), sumsq partials, normA2, bad flag
  unsigned char* p = static_cast<unsigned char*>(mem);
  auto take = [&](size_t bytes) {
    unsigned char* r = p;
    p += (bytes + 255) / 256 * 256;
    return r;
  };
  S.colptr = reinterpret_cast<int64_t*>(take((size_t)(S.n + 1) * 8));
  S.rowidx = reinterpret_cast<int32_t*>(take((size_t)std::max<int64_t>(S.nnz, 1) * 4));
  S.valsT = reinterpret_cast<float*>(take((size_t)std::max<int64_t>(S.nnz, 1) * 4));
  int32_t* cnt = reinterpret_cast<int32_t*>(take((size_t)S.n * 4));
  const int64_t nsq = std::max<int64_t>((S.nnz + 4095) / 4096, 1);
  double* sq = reinterpret_cast<double*>(take((size_t)nsq * 8));
  S.normA2 = reinterpret_cast<double*>(take(8));
  int32_t* bad = reinterpret_cast<int32_t*>(take(4));
  hipError_t e;
  // the structure is checked before any index is used as an address
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(bad), 1, 0u, s)) != hipSuccess) return e;
  const int64_t vt = std::max(S.m + 1, S.nnz);
  if ((e = dispatch<ValidateArgs, b_validate, 256>(
           ValidateArgs{S.rowptr, S.colidx, S.m, S.n, S.nnz, bad},
           dim3((unsigned)((vt + 255) / 256)), 0, s)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(bad_host, bad, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  if (*bad_host) return hipSuccess;
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(cnt), (size_t)S.n, 0u, s)) != hipSuccess)
    return e;
  if (S.nnz > 0 &&
      (e = dispatch<CountArgs, b_count, 256>(CountArgs{S.colidx, S.nnz, cnt},
                                             dim3((unsigned)((S.nnz + 255) / 256)), 0, s)) !=
          hipSuccess)
    return e;
  if ((e = dispatch<ScanArgs, b_scan, 1024>(ScanArgs{cnt, S.n, S.colptr}, dim3(1), 0, s)) !=
      hipSuccess)
    return e;
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(cnt), (size_t)S.n, 0u, s)) != hipSuccess)
    return e;
  if ((e = dispatch<ScatterArgs, b_scatter, 64 * SPMM_WAVES>(
           ScatterArgs{S.rowptr, S.colidx, S.vals, S.m, S.colptr, cnt, S.rowidx, S.valsT},
           dim3((unsigned)((S.m + SPMM_WAVES - 1) / SPMM_WAVES)), 0, s)) != hipSuccess)
    return e;
  if ((e = dispatch<ColSortArgs, b_colsort, 256>(ColSortArgs{S.colptr, S.n, S.rowidx, S.valsT},
                                                 dim3((unsigned)((S.n + 255) / 256)), 0, s)) !=
      hipSuccess)
    return e;
  if ((e = dispatch<SqArgs, b_sumsq_vals, 256>(SqArgs{S.vals, S.nnz, sq}, dim3((unsigned)nsq), 0,
                                               s)) != hipSuccess)
    return e;
  return launch_sum_doubles(sq, nsq, S.normA2, s);
}

}  // namespace plu
