// Internal declarations shared by the libpowerlu translation units.
// Everything here is gfx950 (CDNA4) device code or its host launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "plu_launch.h"

namespace plu {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Pass GEMM (one pass over A): out = op(A) X, FP32 MFMA 16x16x4, fp32 accumulate.
//   mode 0 ("N"): out[p][c] = sum_r A[p][r] X[r][c]   (A is P x R, row-major)
//   mode 1 ("T"): out[p][c] = sum_r A[r][p] X[r][c]   (A is R x P, row-major)
// The kept dimension P is tiled by 128 (or 64) rows, the columns c by NT*16 (NT<=8),
// the reduced dimension R by 16 (direct passes) or 32 per LDS stage and split across
// workgroups (partials reduced afterwards in a fixed order).
// ---------------------------------------------------------------------------
enum Epi { EPI_STORE = 0, EPI_PART = 1, EPI_SUB = 2, EPI_RESID = 3 };

constexpr int GEMM_BP = 128;   // rows of the kept dimension per pass workgroup (2 tiles per wave)
constexpr int GEMM_BK = 32;

struct GemmArgs {
  const float* A = nullptr; int64_t lda = 0;
  const int32_t* arow = nullptr;      // mode 0 only: A row p is read from row arow[p]
  const float* X = nullptr; int64_t ldx = 0;
  const uint16_t* Ab = nullptr;       // bf16 copy of A (prec BF16), same lda
  const uint16_t* Xb = nullptr;       // bf16 copy of X (prec BF16), same ldx
  float* out = nullptr; int64_t ldo = 0;
  int64_t part_stride = 0;            // EPI_PART: elements between split partials
  int64_t P = 0, R = 0, C = 0;
  int64_t rsplit = 0; int32_t nsplit = 1;
  const int32_t* rowmask = nullptr;   // EPI_SUB: rows with rowmask[p] >= 0 are left alone
  double* sumsq_part = nullptr;       // fused ||A||_F^2: one partial per workgroup (column block 0)
  // EPI_RESID
  const float* Aref = nullptr; int64_t ldaref = 0, aref_cs = 1;   // element (i, j) at i*ldaref + j*aref_cs
  double* resid_part = nullptr;
  double* aref_sq_part = nullptr;     // nullable: ||Aref||_F^2, one partial per workgroup
  // set by launch_gemm: rows of A / X start 16-byte aligned (vector loads allowed)
  int avec = 0, xvec = 0;
  // grouped form only: direction, column tiles per block
  int mode = 0, nt = 0;
  const int32_t* run_if = nullptr;   // device flag: the launch does nothing when it reads 0
  // device column count k (nullable): output columns at or beyond
  // *kcap - kc_col_off are not computed (whole column blocks past it return
  // at once), and with kc_red_off >= 0 the reduction stops at
  // *kcap - kc_red_off.  Lets a launch sized for l columns serve a rank k
  // known only on the device.
  const int32_t* kcap = nullptr;
  int32_t kc_col_off = 0, kc_red_off = -1;
};


// Plans the split of R and launches; part must hold nsplit*P*ldo floats when
// the plan splits.  Returns the number of sumsq partials written (grid size)
// through *n_sumsq when sumsq_part is set.
struct GemmPlan {
  int pblocks, cblocks, nt, nsplit;
  int64_t rsplit;
  int bp = GEMM_BP;   // rows per workgroup: GEMM_BP, or 64 (one MFMA row tile per wave)
};
// kalign: the split length is a multiple of it (the reduction depth of one
// stage of the kernel that runs the plan).
GemmPlan plan_gemm(int64_t P, int64_t R, int64_t C, int max_split, int target_wgs,
                   int kalign = GEMM_BK, int bp = GEMM_BP);
hipError_t launch_gemm(int mode, int epi, int bf16, const GemmArgs& a, const GemmPlan& pl,
                       hipStream_t s);
hipError_t launch_splitk_reduce(const float* part, int64_t part_stride, int nsplit,
                                float* out, int64_t ldo, int64_t P, int64_t C,
                                double* colsq_part, int rows_per_block, hipStream_t s);
// The same with the partials at their own row stride pld (>= C; a multiple of
// 4 lets every column group, the last one too, be read as whole float4s).
hipError_t launch_splitk_reduce_ld(const float* part, int64_t pld, int64_t part_stride,
                                   int nsplit, float* out, int64_t ldo, int64_t P, int64_t C,
                                   double* colsq_part, int rows_per_block, hipStream_t s);
hipError_t launch_sum_doubles(const double* in, int64_t n, double* out, hipStream_t s);
hipError_t launch_sumsq_matrix(const float* A, int64_t lda, int64_t m, int64_t n,
                               double* part, int nblocks, hipStream_t s);

// ---------------------------------------------------------------------------
// Precision form of the passes (k_lowp.hip).
// ---------------------------------------------------------------------------
// bfloat16 copies of an R x C fp32 matrix: row-major (rm, ld ldr) and/or
// transposed (tr, Ct x ldt), zero-padded; ldr and ldt multiples of 64.
// Optional float64 sum-of-squares partials (count returned in *nparts).
hipError_t launch_cvt_bf16(const float* src, int64_t lds, int64_t R, int64_t C, uint16_t* rm,
                           int64_t ldr, uint16_t* tr, int64_t ldt, int64_t Ct, double* sumsq_part,
                           int64_t* nparts, hipStream_t s);
// Block-scaled FP8 E4M3 copies (blocks of 32 along the contraction index,
// E8M0 scale bytes): rm/rsc row-major R x ldr (+ R x ldr/32 scales),
// tr/tsc transposed Ct x ldt (+ Ct x ldt/32); ldr, ldt multiples of 128.
// sumsq_part (nullable): float64 partial sums of squares of src, *nparts of
// them (as launch_cvt_bf16).
hipError_t launch_cvt_fp8(const float* src, int64_t lds, int64_t R, int64_t C, uint8_t* rm,
                          uint8_t* rsc, int64_t ldr, uint8_t* tr, uint8_t* tsc, int64_t ldt,
                          int64_t Ct, double* sumsq_part, int64_t* nparts, hipStream_t s);
// out = sum_k dequant(M)[p][k] dequant(Xt)[c][k] on the scaled FP8 MFMA, A
// and the sketch staged through LDS by direct loads: workgroups of 512
// threads and 192 rows (pl.pblocks counts those, from plan_lowp), K and
// pl.rsplit multiples of 256, leading dimensions multiples of 256, pl.nt
// <= 14 (above 8 the wide kernel); epi EPI_STORE or EPI_PART.
hipError_t launch_pass_fp8(int epi, const uint8_t* M, const uint8_t* Ms, int64_t ldm,
                           const uint8_t* Xt, const uint8_t* Xsc, int64_t ldx, float* out,
                           int64_t ldo, int64_t part_stride, int64_t P, int64_t K, int64_t C,
                           const GemmPlan& pl, hipStream_t s);
// out = M Xt^T on bfloat16 MFMA (M: P x K, Xt: Ct x K), A and the sketch
// staged through LDS by direct loads: workgroups of 512 threads and 256 rows
// (pl.pblocks counts those, from plan_bf16), K and pl.rsplit multiples of
// 128, pl.nt <= 8; epi EPI_STORE or EPI_PART.
hipError_t launch_pass_bf16(int epi, const uint16_t* M, int64_t ldm, const uint16_t* Xt,
                            int64_t ldx, float* out, int64_t ldo, int64_t part_stride, int64_t P,
                            int64_t K, int64_t C, const GemmPlan& pl, hipStream_t s);

// ---------------------------------------------------------------------------
// Tall-skinny LU with partial pivoting (rows stay in place; see k_getrf.hip).
// ---------------------------------------------------------------------------
struct GetrfWork {
  int32_t* piv_step;     // M
  int32_t* pos;          // M
  int32_t* piv_row;      // >= c
  float* gaps;           // >= c
  int32_t* zstep;        // first zero-pivot step (INT_MAX if none)
  int32_t* abortf;       // timeout flag shared by every LU of a call (cleared by the caller)
  unsigned long long* msg;
  size_t msg_words;
  float* u12;            // NB x ldu12 scratch for the blocked update
  int64_t ldu12;
  uint32_t* tag_counter; // host-side counter of panel launches (owned by the handle)
  uint64_t timeout_ticks;
  int max_waves;
  const int32_t* run_if = nullptr;   // device flag: the whole LU is skipped when it reads 0
  // device column count (nullable): only the first min(c, *kcap) steps are
  // taken -- the LU of the leading *kcap columns; U (and U^T) entries
  // outside that square are written as zeros, perm is that LU's row order
  const int32_t* kcap = nullptr;
};
size_t getrf_msg_words(int64_t M);
// F: M x c (ldf).  On return F holds V = P^T L (unit lower, original row order).
// perm (nullable): F_in[perm] = L U.  Uout (nullable): U (c x c) or U^T if utrans.
hipError_t getrf_run(float* F, int64_t ldf, int64_t M, int c, const GetrfWork& w,
                     int32_t* perm, float* Uout, int64_t ldu, int utrans, hipStream_t s);

// ---------------------------------------------------------------------------
// Thin QR: LU reorthogonalization followed by block CholeskyQR2 (FP64 Gram,
// FP64 Cholesky) with block classical Gram-Schmidt between blocks.
// ---------------------------------------------------------------------------
struct QrWork {
  float* q;              // M x ldq output basis (may not alias X)
  int64_t ldq;
  float* tmp;            // M x 128
  double* gram_part;     // nchunk x 128 x 128
  int max_chunks;
  double* gram;          // 128 x 128
  float* rinv;           // 128 x 128
  double* rinv64;        // 128 x 128
  float* wproj;          // c x 128
  float* part; int64_t part_cap;   // split-K partials (floats)
  int32_t* status;       // [2] Cholesky breakdown flag, [4] "needs the LU" flag
};
hipError_t thin_qr_run(float* X, int64_t ldx, int64_t M, int c, const GetrfWork& gw,
                       const QrWork& qw, hipStream_t s);
// (X^T X)^{-1} = R^{-1} R^{-T} for an M x c X, c <= 128: the float64 Gram
// and its Cholesky factor X^T X = R^T R; R^{-1} (upper triangular, float32,
// leading dimension 128) is left in qw.rinv.
hipError_t gram_inverse_run(const float* X, int64_t ldx, int64_t M, int c, const QrWork& qw,
                            hipStream_t s);

// ---------------------------------------------------------------------------
// Misc kernels.
// ---------------------------------------------------------------------------
hipError_t launch_gaussian(float* out, int64_t ldo, int64_t rows, int64_t cols, uint64_t seed,
                           hipStream_t s);
hipError_t launch_copy_pad(const float* src, int64_t lds, float* dst, int64_t ldd,
                           int64_t rows, int64_t cols, int64_t cols_pad, hipStream_t s);
// Measured ceilings (k_peaks.hip): kind 0 / 1 / 2 = the fp32 / bfloat16 /
// scaled FP8 matrix-core loop (blocks x 4 waves, each iters x chains
// instructions), the streaming read of `bytes` from buf.
double peak_flop_per_mfma(int kind);
int peak_chains();
hipError_t launch_peak_mfma(int kind, int blocks, int iters, hipStream_t s);
hipError_t launch_peak_read(const void* buf, int64_t bytes, int blocks, hipStream_t s);
// dst[rperm[i]][cperm[j]] = src[i][j] (rows x cols; null permutation =
// identity; out-of-range indices are skipped)
hipError_t launch_scatter_perm(const float* src, int64_t lds, float* dst, int64_t ldd,
                               int64_t rows, int64_t cols, const int32_t* rperm,
                               const int32_t* cperm, hipStream_t s);
// kcap (nullable, device): rows t >= *kcap of U are not written
hipError_t launch_transpose_gather(const float* V, int64_t ldv, const int32_t* rowidx,
                                   int64_t nrows, int k, float* U, int64_t ldu, hipStream_t s,
                                   const int32_t* kcap = nullptr);
// Float64 indicator (k_f64.hip).  out (P x C, float64) = op(A) B with
// op(A)(p, r) = A[p * lda + r] (mode 0) or A[r * lda + p] (mode 1).
hipError_t launch_f64_gemm(int mode, const float* A, int64_t lda, const float* B, int64_t ldb,
                           int64_t P, int64_t R, int64_t C, double* out, int64_t ldo,
                           hipStream_t s);
// W = X^T X - I (X: R x l float32), tiles on and above the diagonal.
hipError_t launch_f64_gram_w(const float* X, int64_t ldx, int64_t R, int64_t l, double* W,
                             int64_t ldw, hipStream_t s);
// part[blk * l + j] (blk < f64_row_blocks(l)): the row block's share of
// M_jj (1 - W_jj) - 2 sum_{i<j} W_ij M_ij, M = Y^T Y (Y float64, or Y32
// float32 when Y is null).
hipError_t launch_f64_corr(const double* Y, const float* Y32, int64_t ldy, int64_t R, int64_t l,
                           const double* W, int64_t ldw, double* part, hipStream_t s);
int f64_row_blocks(int64_t l);

hipError_t launch_rank_rule(const double* colsq_part, int nblk, int l, const double* vsq_part,
                            int nvblk, const double* normA2, double eps, int b, int col_mode,
                            int32_t* kout, double* Eout, int32_t* tol, double* colnorm,
                            hipStream_t s, const double* E0 = nullptr);
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);
hipError_t launch_iota(int32_t* p, int64_t n, hipStream_t s);
// p[r][c] = -p[r][c] over a rows x cols block (leading dimension ld)
hipError_t launch_negate(float* p, int64_t ld, int64_t rows, int64_t cols, hipStream_t s);
// ---------------------------------------------------------------------------
// Sparse A (compressed rows, with the compressed columns built once).
// ---------------------------------------------------------------------------
struct SparseMat {
  int64_t m = 0, n = 0, nnz = 0;
  const int64_t* rowptr = nullptr;   // m + 1 (caller's)
  const int32_t* colidx = nullptr;   // nnz (caller's)
  const float* vals = nullptr;       // nnz (caller's)
  int64_t* colptr = nullptr;         // n + 1 (built)
  int32_t* rowidx = nullptr;         // nnz, rows ascending within a column (built)
  float* valsT = nullptr;            // nnz (built)
  double* normA2 = nullptr;          // ||A||_F^2 (built)
};
// Bytes of device memory sparse_build needs for an m x n matrix with nnz
// stored entries.
size_t sparse_scratch_bytes(int64_t m, int64_t n, int64_t nnz);
// Checks the compressed rows of S (when malformed, sets *bad_host -- bit 1 for
// the row pointers, bit 2 for the column indices -- and returns hipSuccess;
// synchronizes on s), then builds the compressed columns and ||A||_F^2 in
// mem (sparse_scratch_bytes long).
hipError_t sparse_build(SparseMat& S, void* mem, int32_t* bad_host, hipStream_t s);
// out (rows x l, ldo) = S X for S given by (ptr, idx, val) in compressed
// rows and X with at least max(idx) + 1 rows (ldx).
hipError_t launch_spmm(const int64_t* ptr, const int32_t* idx, const float* val, int64_t rows,
                       const float* X, int64_t ldx, int l, float* out, int64_t ldo, hipStream_t s);

// R = U_r diag(S) V_r^T for a square l x l R, l <= 128 (one-sided Jacobi in
// one workgroup): Ur, Vr l x l with columns in non-increasing order of the
// singular values, the kout largest of which go to S; sweeps_out nullable.
hipError_t launch_jacobi_svd(const float* R, int64_t ldr, int l, float* Ur, int64_t ldur,
                             float* Vr, int64_t ldvr, float* S, int kout, int32_t* sweeps_out,
                             hipStream_t s);
// X = (R^{-1})^T for an upper triangular k x k R, k <= 128 (one workgroup)
hipError_t launch_tri_inv_t(const float* R, int64_t ldr, float* X, int64_t ldx, int k,
                            hipStream_t s);

}  // namespace plu
