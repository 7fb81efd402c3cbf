/*
 * powerlu.h -- C ABI of libpowerlu, an MI355X (gfx950) implementation of
 * PowerLU and PowerLU_FP: randomized LU low-rank approximation with any number
 * of passes v >= 2 over the input matrix (B. Zhang, M. Mascagni,
 * "Pass-Efficient Randomized LU Algorithms for Computing Low-Rank Matrix
 * Approximation", arXiv:2002.07138).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Matrices are float32, row-major, with an explicit leading dimension
 *    (elements between the starts of consecutive rows).  Leading dimensions
 *    must be >= the row length and, for the fast paths, multiples of 4;
 *    device pointers must be 16-byte aligned.
 *  - Pointers named in an entry point's comment as "device" point to memory on
 *    the handle's device (hipMalloc / torch CUDA tensors); "host" pointers are
 *    ordinary host memory.  The caller owns all of them; the library never
 *    frees caller memory and never writes to the input matrix A.
 *  - Every call is asynchronous on the handle's stream unless it takes a
 *    non-NULL plu_info*, in which case it synchronizes that stream and fills
 *    the struct before returning.
 *  - Permutations are 0-based int32 vectors: p (length m) and q (length n)
 *    such that A[p[i], q[j]] ~= sum_t L[i, t] * U[t, j]  (the paper's
 *    P A Q ~= L U, eq. powerlufinal in Sec. 3.1, written in index form).
 *  - L (m x k) is lower trapezoidal with diag(L) = diag(U2); U (k x n) is unit
 *    upper trapezoidal with |u_ij| <= 1 (U = L2^T, Alg. 5 step 8).
 *  - Return value: 0 on success; -i when argument i (1-based) is invalid;
 *    a positive PLU_* code otherwise.
 *  - Workspace: plu_fixed_rank and plu_fixed_precision take an optional
 *    caller workspace (work, work_bytes: device memory, any alignment, at
 *    least plu_workspace_size bytes; owned by the caller, contents on entry
 *    irrelevant, clobbered by the call; one call at a time may use it).
 *    With work = NULL -- and for every other call -- the library keeps a
 *    workspace on the handle and grows it on demand (PLU_ERR_OOM if that
 *    fails).
 *  - Graph capture: a call whose workspace already exists (a caller
 *    workspace, or an earlier call of the same shape on the handle) makes no
 *    allocation and no synchronization when info is NULL, so it can be
 *    captured into a HIP graph on the handle's stream (plu_fixed_rank, and
 *    plu_fixed_precision with max_rounds = 1).  Captured calls run the
 *    default split of the passes unless an eager call of the same shape has
 *    already tuned it in the process; each replay recomputes from the
 *    current contents of the captured buffers.
 */
#ifndef POWERLU_H
#define POWERLU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PLU_OK = 0,
  PLU_WARN_ZERO_PIVOT = 1,     /* an LU step met an exactly zero pivot column (LAPACK getrf INFO > 0) */
  PLU_TOL_NOT_REACHED = 2,     /* fixed precision: eps not met with l columns; rank-l result returned */
  PLU_ERR_NONFINITE = 3,       /* A holds NaN or Inf */
  PLU_ERR_OOM = 4,             /* device workspace allocation failed */
  PLU_ERR_HIP = 5,             /* a HIP runtime call failed */
  PLU_ERR_NOT_IMPLEMENTED = 6,
  PLU_ERR_TIMEOUT = 7,         /* a device-side wait in the cooperative LU panel exceeded its bound */
  PLU_PENDING = 8,             /* server: request not finished yet */
  PLU_ERR_TOO_LARGE = 9        /* plu_fixed_rank_static: the problem's workspace exceeds its
                                  static scratch */
};

typedef enum {
  PLU_PREC_FP32 = 0,       /* passes on the fp32 matrix cores */
  PLU_PREC_BF16 = 1,       /* pass operands rounded to bfloat16 (round to nearest even) */
  PLU_PREC_FP8_E4M3 = 2,   /* pass operands rounded to FP8 E4M3 (OCP e4m3fn) with one
                              power-of-two (E8M0) scale per 32 consecutive entries along
                              the contraction index: the smallest 2^e, e >= -127, with
                              max|x| / 2^e <= 448 */
  PLU_PREC_FORMAT_MASK = 15,
  PLU_PREC_REFINE_LAST = 16, /* flag, OR-ed with BF16 or FP8_E4M3: the last of the v-1
                              passes of Alg. 7 (the one whose result the final QR
                              orthonormalizes) also runs on the fp32 A, re-projecting the
                              rounded iterate; for v = 2 nothing is then rounded */
  PLU_PREC_REFINE_TWO = 32, /* flag, OR-ed with BF16 or FP8_E4M3 (instead of REFINE_LAST):
                              the last two of the v-1 passes of Alg. 7 -- the A X and
                              A^T Y of its final loop iteration -- run on the fp32 A, one
                              full fp32 power step on the basis the rounded passes
                              found; for v <= 3 nothing is then rounded.  The E4M3 form
                              needs it to stay within 1.05x of the exact residual when
                              the rounding error of A exceeds sigma_{k+1} */
  PLU_PREC_A_UNCHANGED = 64 /* flag, OR-ed with BF16 or FP8_E4M3: A (same pointer, shape,
                              leading dimension and storage order) has not changed since
                              the last call on this handle that rounded it to this format
                              on the handle's own workspace: the rounded copies still kept
                              there are reused instead of made again (4 m n bytes read,
                              4 m n or 2 m n written).  The caller guarantees A is
                              unchanged; without a matching copy the flag does nothing.
                              Any call on the handle in another format or shape
                              invalidates the copies. */,
  PLU_PREC_FP64_INDICATOR = 128 /* flag, fixed precision only (any format; dense A, one
                              round): the stopping indicator of Thm 4.3 from G = A V
                              with float64 products and sums, first-order corrected for
                              the basis' deviation from orthonormality (V^T V - I in
                              float64), instead of the float32 column energies of G.  The
                              float32 indicator resolves E to about 1e-8 ||A||_F^2, so
                              tolerances eps below about 3e-4 need this form; it costs
                              one more pass over A in float64 and two l x l float64
                              Gram products. */
} plu_prec;

/* Storage order of the input matrix A (the paper's A is m x n, Def. 1.1).
 * Row-major: element (i, j) at A[i * lda + j], lda >= n.  Column-major:
 * element (i, j) at A[i + j * lda], lda >= m.  Only A takes a layout; every
 * output (p, q, L, U) is row-major.  Both orders run the same kernels: a
 * column-major A is the row-major storage of A^T, so A X and A^T Y swap
 * directions. */
typedef enum {
  PLU_ROW_MAJOR = 0,
  PLU_COL_MAJOR = 1
} plu_layout;

/* What plu_measure_peak measures. */
typedef enum {
  PLU_PEAK_MFMA_FP32 = 0,
  PLU_PEAK_MFMA_BF16 = 1,
  PLU_PEAK_MFMA_FP8 = 2,
  PLU_PEAK_HBM_READ = 3
} plu_peak_kind;

typedef struct plu_handle_s* plu_handle;

/* Filled on request after the stream has synchronized. */
typedef struct {
  int32_t status;            /* same code the call returned */
  int32_t rank;              /* k used for L and U */
  int32_t passes;            /* passes over A actually made (= v) */
  int32_t zero_pivot_step;   /* first zero pivot over the final two LU steps, -1 if none */
  int32_t tol_reached;       /* fixed precision: 1 if E <= eps^2 ||A||_F^2 */
  int32_t l;                 /* sketch width used */
  double normA2;             /* ||A||_F^2, float64 accumulation */
  double E_final;            /* fixed precision: indicator E_k (Thm 4.3) */
  float min_pivot_gap;       /* min over the final two LU steps of (|top1|-|top2|)/|top1| */
  float pad_;
} plu_info;

/* Handle bound to one device and one stream (hip_stream NULL = null stream).
 * Not thread-safe: one host thread per handle. */
int plu_create(plu_handle* h, int device, void* hip_stream);
int plu_destroy(plu_handle h);
int plu_set_stream(plu_handle h, void* hip_stream);
/* Bytes of device workspace a fixed-rank call (l = k + p_over, max_rounds
 * = 1) or fixed-precision call (l its sketch width, with its max_rounds) of
 * this shape and pass precision needs, as a caller workspace or on the
 * handle (the bfloat16 form adds two rounded copies of A, 4 m n bytes; the
 * E4M3 form 2 m n bytes and scales).                                      */
int plu_workspace_size(plu_handle h, int64_t m, int64_t n, int32_t l, int32_t max_rounds,
                       int32_t prec, size_t* bytes);
const char* plu_status_string(int status);

/* ---- Fixed-rank problem (Def. 1.1, Sec. 1) solved by PowerLU: Alg. 5 with
 * its steps 1-2 replaced by Alg. 7 (Sec. 3.4).
 *   layout storage order of A (plu_layout); lda >= n (row-major) or >= m.
 *   A      device, m x n, lda.
 *   k      target rank, 1 <= k;  p_over >= 0 oversampling (the paper's q);
 *          l = k + p_over must satisfy l < min(m, n) (Alg. 7 REQUIRE).
 *   v      passes over A, v >= 2.
 *   prec   arithmetic of the v-1 passes inside Alg. 7: FP32 (MFMA fp32),
 *          BF16 or FP8_E4M3 (A and the iterate rounded to that format, see
 *          plu_prec; exact products on the matrix cores with fp32
 *          accumulation), optionally | PLU_PREC_REFINE_LAST or | PLU_PREC_REFINE_TWO.  The final pass
 *          Y = A V(:,1:k) always runs in FP32 on the fp32 A: it is the
 *          refinement pass of the precision form.
 *          The rounded copies of A cost 4 m n (BF16) or 2 m n (FP8) bytes
 *          of workspace; they are made on every call unless prec carries
 *          PLU_PREC_A_UNCHANGED and the handle still holds them.
 *   Omega  device, nullable.  (v even ? m : n) x l Gaussian test matrix with
 *          leading dimension l.  NULL draws it on the device from `seed` with
 *          the Philox4x32-10 layout of plu_gaussian.
 *   p, q   device int32 outputs, lengths m and n.
 *   L, U   device outputs: L m x k (ldl >= k), U k x n (ldu >= n).
 *   work, work_bytes  nullable caller workspace (see the conventions);
 *          -20 when work_bytes is too small.
 *   info   host, nullable (non-NULL synchronizes).                        */
int plu_fixed_rank(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A,
                   int64_t lda, int32_t k, int32_t p_over, int32_t v, int32_t prec,
                   const float* Omega, uint64_t seed,
                   int32_t* p, int32_t* q, float* L, int64_t ldl, float* U, int64_t ldu,
                   void* work, size_t work_bytes, plu_info* info);

/* ---- plu_fixed_rank without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture that brings no
 * workspace, tight serving loops, harnesses that forbid allocation).  Same
 * arguments, kernels and results as plu_fixed_rank with work = NULL, but the
 * workspace is a static array of 64 MiB in the library's device code object
 * -- one per device, present from the library's load on that device until
 * the process ends -- so the call makes no hipMalloc / hipFree (nor any host
 * heap allocation) and runs the default split of the passes (no tuning).
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (the call clears what must start at zero): calls that
 * overlap on one device -- from two threads, or on two streams -- race.
 * Returns PLU_ERR_TOO_LARGE when plu_workspace_size(m, n, k + p_over, 1,
 * prec) exceeds 64 MiB (for example 8192 x 8192 with l = 64 fits; 20000 x
 * 20000 does not), and PLU_ERR_HIP if the array's device address could not
 * be obtained when the handle was created.                                */
int plu_fixed_rank_static(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A,
                          int64_t lda, int32_t k, int32_t p_over, int32_t v, int32_t prec,
                          const float* Omega, uint64_t seed, int32_t* p, int32_t* q, float* L,
                          int64_t ldl, float* U, int64_t ldu, plu_info* info);

/* ---- Fixed-precision problem (Sec. 1, last paragraph of Def. 1.1's
 * discussion) solved by PowerLU_FP: Alg. 9 on top of Alg. 8 (block rule) or
 * Alg. 11 (column rule, column_exact = 1), with the error indicator of
 * Thm 4.3 accumulated in float64 and the stopping test E <= eps^2 ||A||_F^2.
 *   layout, A, lda, prec, Omega, seed, p, q   as for plu_fixed_rank.
 *   eps    > 0 relative Frobenius tolerance.
 *   b      block size >= 1; l (sketch width) must be a multiple of b and
 *          < min(m, n); l = 0 selects min(50 b, b * floor((min(m,n)-1)/b)).
 *   max_rounds >= 1, with l * max_rounds < min(m, n).  1 is Alg. 9 as
 *          printed.  Above 1, a round whose l columns miss the tolerance is
 *          followed by another (the restart of the Remark after Alg. 8):
 *          a fresh Gaussian matrix, drawn on the device from seed + r for
 *          round r (0-based; round 0 uses Omega when given), and Alg. 7 on
 *          the remainder A - A V V^T of the columns kept so far; the
 *          indicator continues over all columns.  One synchronization per
 *          round.  Needs l * max_rounds columns of L and rows of U.
 *   L, U   device outputs with room for l * max_rounds columns / rows:
 *          L m x (l max_rounds) (ldl >= l max_rounds), U (l max_rounds) x n
 *          (ldu >= n); the leading rank columns / rows hold the factors,
 *          the rest is unspecified.
 *   rank_dev device int32*, nullable: receives the rank k.  With
 *          max_rounds = 1 the rank never leaves the device: the rule of
 *          Alg. 8 / Alg. 11 runs in a kernel, and the assembly's launches,
 *          sized for l columns, stop at the rank they read there, so the
 *          call is asynchronous when info is NULL (and capturable).  k = 0
 *          (a zero matrix, or a non-finite A: then info reports
 *          PLU_ERR_NONFINITE) leaves p and q the identity.
 *   work, work_bytes  nullable caller workspace; -24 when too small.
 *   info   host, nullable: synchronizes and reports the rank, the status
 *          and whether eps was reached.
 * If eps is not met within l * max_rounds columns, that factorization is
 * returned (status PLU_TOL_NOT_REACHED in info, and as the return value
 * when max_rounds > 1 or info is given).  A zero matrix gives rank 0.
 * With the pivot trace on, each final LU of a max_rounds = 1 call records l
 * entries, of which the first rank are its steps.                         */
int plu_fixed_precision(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A,
                        int64_t lda, double eps, int32_t b, int32_t l, int32_t v,
                        int32_t column_exact, int32_t max_rounds, int32_t prec,
                        const float* Omega, uint64_t seed, int32_t* p, int32_t* q, float* L,
                        int64_t ldl, float* U, int64_t ldu, int32_t* rank_dev, void* work,
                        size_t work_bytes, plu_info* info);

/* ---- Single-pass randomized LU (Alg. 10, Sec. 5): G = A^T Omega and
 * H = A G from one pass over A, [L1, U1, P] = lu(H), [L2, U2, Q] =
 * lu(pinv(G^T) U1^T), L = L1 U2^T, U = L2^T.  The one-pass schedule needs
 * the columns of A contiguous (layout PLU_COL_MAJOR, as the paper states):
 * blocks of columns are read from HBM once, multiplied into G and, while
 * still cached, into H.  With PLU_ROW_MAJOR the same result takes two
 * passes.  pinv(G^T) = Q R^{-T} from a thin QR G = Q R.
 *   k      1 <= k <= 128, k < min(m, n); no oversampling (as in Alg. 10).
 *   Omega  device, nullable: m x k with leading dimension k (NULL: drawn
 *          from seed as in plu_gaussian).
 *   A, lda, p, q, L, ldl, U, ldu, info   as for plu_fixed_rank.           */
int plu_single_pass(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A,
                    int64_t lda, int32_t k, const float* Omega, uint64_t seed, int32_t* p,
                    int32_t* q, float* L, int64_t ldl, float* U, int64_t ldu, plu_info* info);

/* ---- RandLU (Alg. 3 with its steps 1-3 replaced by the LU power iteration
 * of Alg. 4, Sec. 2.2): the comparison algorithm the paper measures PowerLU
 * against.  P Y = L_y U_y for Y = A (A^T A)^pw Omega with an LU
 * reorthogonalization after every product; L_y = L_y(:, 1:k);
 * B = L_y^+ P A with L_y^+ = (L_y^T L_y)^{-1} L_y^T (the Remark after
 * Alg. 4; the Gram matrix and its Cholesky factor in float64);
 * [L2, U2, Q] = lu(B^T) (B Q = L_b U_b with L_b = U2^T, U_b = L2^T);
 * L = L_y U2^T, U = L2^T.  2 pw + 2 passes over A.
 *   k       1 <= k <= 128.
 *   p_over  oversampling >= 0; l = k + p_over < min(m, n).
 *   pw      power exponent p >= 0 of Alg. 3 / Alg. 4.
 *   Omega   device, nullable: n x l with leading dimension l (NULL: drawn
 *           from seed as in plu_gaussian).
 *   layout, A, lda, p, q, L, ldl, U, ldu, info   as for plu_fixed_rank
 *           (A[p][:, q] ~ L U; L is lower trapezoidal in the row order p,
 *           U unit upper trapezoidal).
 * Errors: -(argument index) for invalid arguments; PLU_ERR_OOM,
 * PLU_ERR_HIP, PLU_ERR_TIMEOUT as for plu_fixed_rank.                      */
int plu_randlu(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A, int64_t lda,
               int32_t k, int32_t p_over, int32_t pw, const float* Omega, uint64_t seed,
               int32_t* p, int32_t* q, float* L, int64_t ldl, float* U, int64_t ldu,
               plu_info* info);

/* ---- RandSVD (Alg. 1 with the QR power iteration of Alg. 2, Sec. 2): the
 * other comparison algorithm.  Q = qr(A Omega), then pw times Q = qr(A^T Q),
 * Q = qr(A Q); B = Q^T A (l x n); B = U_hat S V^T; U = Q U_hat.  The SVD of
 * B is taken as B^T = Q_b R (thin QR) and R = U_r S V_r^T by one-sided
 * Jacobi in one workgroup (U_hat = V_r, V = Q_b U_r).  The k leading
 * singular triplets are returned.  2 pw + 2 passes over A.
 *   k, p_over  l = k + p_over <= 128, l < min(m, n).
 *   pw         power exponent p >= 0 of Alg. 1 / Alg. 2.
 *   Omega      device, nullable: n x l (leading dimension l).
 *   U          device m x k (ldu >= k), orthonormal columns.
 *   S          device k float32, non-increasing.
 *   V          device n x k (ldv >= k), orthonormal columns.
 *   info       as for plu_fixed_rank (rank = k; no pivot fields).
 * Errors: -(argument index) for invalid arguments; PLU_ERR_OOM, PLU_ERR_HIP,
 * PLU_ERR_TIMEOUT.                                                          */
int plu_randsvd(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A, int64_t lda,
                int32_t k, int32_t p_over, int32_t pw, const float* Omega, uint64_t seed,
                float* U, int64_t ldu, float* S, float* V, int64_t ldv, plu_info* info);

/* ---- Sparse A (the sprand inputs of Sec. 6.1's second experiment).  A
 * matrix in compressed rows is bound to the handle's device once; the
 * drivers then run their passes A X and A^T Y as row-parallel gathers over
 * the compressed rows and over compressed columns built on the device (with
 * each column's entries in ascending row order, so results do not depend on
 * scheduling).  The rest of every algorithm (LU, QR, assembly, indicator) is
 * the dense path's.
 *   plu_sparse_create: m, n in [1, 2^31); nnz >= 0 stored entries;
 *     rowptr device int64 (m + 1), rowptr[0] = 0, non-decreasing,
 *     rowptr[m] = nnz; colidx device int32 (nnz), each in [0, n); vals
 *     device float32 (nnz).  Entries need not be sorted within a row;
 *     repeated (i, j) entries act as their sum (in an unspecified order).
 *     The arrays are borrowed: they must stay valid and unchanged until
 *     plu_sparse_destroy.  The object owns about 8 (n + nnz) more bytes of
 *     device memory (compressed columns, ||A||_F^2).  The structure is
 *     checked on the device first; a violation returns -5 (rowptr) or -6
 *     (colidx) and no object.  Synchronizes the handle's stream.
 *   plu_sparse_destroy: waits for the device, frees the object (NULL is a
 *     no-op).
 *   plu_sparse_pass: out = A X (trans 0; X n x l, out m x l) or A^T X
 *     (trans 1; X m x l, out n x l), row-major, float32, on the handle's
 *     stream.
 *   plu_sparse_fixed_rank, plu_sparse_fixed_precision, plu_sparse_randlu,
 *   plu_sparse_randsvd: as plu_fixed_rank, plu_fixed_precision, plu_randlu
 *     and plu_randsvd with (layout, m, n, A, lda) replaced by sp and without
 *     the caller workspace (they use the handle's); m and n are the
 *     matrix's; prec must be PLU_PREC_FP32.  Argument errors are -(index in
 *     this signature): the dense index minus 4 for every argument after sp.
 */
typedef struct plu_sparse_s* plu_sparse;
int plu_sparse_create(plu_handle h, int64_t m, int64_t n, int64_t nnz, const int64_t* rowptr,
                      const int32_t* colidx, const float* vals, plu_sparse* out);
int plu_sparse_destroy(plu_sparse sp);
int plu_sparse_pass(plu_handle h, plu_sparse sp, int32_t trans, const float* X, int64_t ldx,
                    int32_t l, float* out, int64_t ldo);
int plu_sparse_fixed_rank(plu_handle h, plu_sparse sp, int32_t k, int32_t p_over, int32_t v,
                          int32_t prec, const float* Omega, uint64_t seed, int32_t* p, int32_t* q,
                          float* L, int64_t ldl, float* U, int64_t ldu, plu_info* info);
int plu_sparse_fixed_precision(plu_handle h, plu_sparse sp, double eps, int32_t b, int32_t l,
                               int32_t v, int32_t column_exact, int32_t max_rounds, int32_t prec,
                               const float* Omega, uint64_t seed, int32_t* p, int32_t* q, float* L,
                               int64_t ldl, float* U, int64_t ldu, int32_t* rank_dev,
                               plu_info* info);
int plu_sparse_randlu(plu_handle h, plu_sparse sp, int32_t k, int32_t p_over, int32_t pw,
                      const float* Omega, uint64_t seed, int32_t* p, int32_t* q, float* L,
                      int64_t ldl, float* U, int64_t ldu, plu_info* info);
int plu_sparse_randsvd(plu_handle h, plu_sparse sp, int32_t k, int32_t p_over, int32_t pw,
                       const float* Omega, uint64_t seed, float* U, int64_t ldu, float* S,
                       float* V, int64_t ldv, plu_info* info);

/* ---- Relative residual ||A[p][:, q] - L U||_F / ||A||_F (eq. "error",
 * Sec. 6.2), recomputing L U tile by tile with float64 accumulation.
 *   all matrix/vector pointers device; rel_resid host; layout of A as in
 *   plu_fixed_rank (L and U row-major).  p and q must be permutations of
 *   0..m-1 and 0..n-1 (as the factorizations return them): the call moves
 *   row i of L to row p[i] and column j of U to column q[j] in a workspace
 *   of its own, then reads A once, in place, summing ||A - L' U'||_F^2 and
 *   ||A||_F^2 together.  Indices out of range are skipped (those rows or
 *   columns of L U count as zero).  Allocates its workspace; synchronizes. */
int plu_residual(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A,
                 int64_t lda,
                 const int32_t* p, const int32_t* q, int32_t k,
                 const float* L, int64_t ldl, const float* U, int64_t ldu,
                 double* rel_resid);

/* ---- Batched problems: many fixed-rank and fixed-precision problems of
 * uneven shapes solved together on the handle's stream.  Every problem runs
 * exactly the steps of plu_fixed_rank / plu_fixed_precision; launches of the
 * same kernel by different problems are merged into one grouped launch (the
 * problems own consecutive ranges of its workgroups), so the passes of all
 * problems share one persistent grouped GEMM launch and their LU panels one
 * cooperative batched launch.  Each problem's result is bit-identical to the
 * single-problem call with the same arguments.
 *   A, Omega, p, q, L, U   device pointers as in the single calls.
 *   prec                   any form of the single calls except
 *                          PLU_PREC_FP64_INDICATOR (status
 *                          PLU_ERR_NOT_IMPLEMENTED).  A rounded form makes
 *                          the problem's copies of A in its own workspace
 *                          on every call (PLU_PREC_A_UNCHANGED is ignored).
 * Outputs (host, in each request): rank, status and info; the call
 * synchronizes once, at the end (the fixed-precision ranks stay on the
 * device until then, as in plu_fixed_precision).
 * Execution: the problems run side by side on up to four streams of the
 * handle, forked from its stream and joined back into it (the longest
 * problem first, each to the least loaded stream), so that one problem's
 * latency-bound steps (the LU panels, the thin QR) overlap other problems'
 * passes over A.  A stream with one problem launches its kernels as the
 * single call does; a stream with several merges their launch sequences into
 * grouped launches, unless one of them is in a rounded form: that stream runs
 * its problems one after the other as single calls.  Results are bitwise
 * those of the single calls either way.
 * flags: PLU_BATCH_GRAPH captures the batch's launches (fixed-rank and
 * fixed-precision problems alike, every stream) into a HIP graph kept by the
 * handle and replays it when the next call has the same requests (same
 * shapes and pointers).  PLU_BATCH_ONE_STREAM keeps every problem on the
 * handle's stream, in one merged launch sequence (one after the other when
 * some problem is in a rounded form).
 * Returns PLU_OK, or -3 when some request is invalid (its status then holds
 * -i for its i-th field, counted from 1 in declaration order).             */
/* ---- Measured ceilings for the rooflines of the pass kernels (the
 * datasheet peaks are the reference; these are what this GPU sustains).
 *   kind  PLU_PEAK_MFMA_FP32 / _BF16 / _FP8: back-to-back matrix-core
 *         instructions of the kinds the passes issue
 *         (v_mfma_f32_16x16x4f32, v_mfma_f32_16x16x32_bf16, the scaled
 *         v_mfma_scale_f32_16x16x128_f8f6f4), 8 independent accumulators
 *         per wave, 8 workgroups of 4 waves per CU, hashed operands;
 *         *rate in TFLOP/s (dense, 2 m n k per instruction).
 *         PLU_PEAK_HBM_READ: a streaming read of `bytes` (at least 1 MiB)
 *         from the device buffer buf (16-byte aligned; contents ignored),
 *         16-byte non-temporal loads; *rate in GB/s.
 *   reps  timed launches after one warm-up; *rate is the best of them.
 * Runs on the handle's stream and synchronizes.  Returns PLU_OK, a negative
 * argument index, or PLU_ERR_HIP.                                          */
int plu_measure_peak(plu_handle h, int32_t kind, const void* buf, int64_t bytes, int32_t reps,
                     double* rate);

/* ---- Pivot trace: the pivot rows and relative pivot gaps of every GETRF of
 * the last plu_fixed_rank / plu_fixed_precision / plu_range_basis /
 * plu_getrf call on the handle, in the order the paper's algorithm makes
 * them: the LU reorthogonalizations of Alg. 7 (l steps each, lu(.) of
 * Alg. 6/7), then lu(Y) and lu(B^T) of Alg. 5 steps 4 and 6 (k steps each).
 * The LU inside the thin QR is an implementation detail and not traced.
 * Entry j of a GETRF: the input row chosen as pivot at step j, and
 * (|top1| - |top2|) / |top1| over the candidates of that step.
 *   plu_set_pivot_trace  capacity > 0: record up to that many entries per
 *                        call (device memory, owned by the handle); 0 stops
 *                        recording and frees it.  Off by default.
 *   plu_pivot_trace      synchronizes; *n_out = entries the last call made;
 *                        copies min(cap, recorded) of them into the host
 *                        arrays (either may be NULL).  PLU_ERR_OOM when the
 *                        call made more entries than the capacity held.    */
int plu_set_pivot_trace(plu_handle h, int64_t capacity);
int plu_pivot_trace(plu_handle h, int32_t* ipiv_out, float* gaps_out, int32_t cap,
                    int32_t* n_out);

typedef struct {
  int32_t mode;            /* 0: fixed rank, 1: fixed precision */
  int32_t column_exact;    /* fixed precision: Alg. 11 column rule */
  int64_t m, n, lda;
  const float* A;
  int32_t k, p_over;       /* fixed rank */
  int32_t v;               /* passes over A */
  int32_t b, l;            /* fixed precision (l = 0: the default sketch width) */
  double eps;              /* fixed precision */
  int32_t prec;
  const float* Omega;      /* nullable */
  uint64_t seed;
  int32_t* p;
  int32_t* q;
  float* L;
  int64_t ldl;
  float* U;
  int64_t ldu;
  int32_t layout;          /* plu_layout of A */
  int32_t rank;            /* out */
  int32_t status;          /* out: PLU_* status of this problem */
  plu_info info;           /* out */
} plu_request;

#define PLU_BATCH_GRAPH 1
#define PLU_BATCH_ONE_STREAM 2

int plu_batched(plu_handle h, int32_t count, plu_request* reqs, int32_t flags);

/* ---- Serving: a request loop on its own stream and worker thread.
 * Requests are admitted in arrival order while the device memory they need
 * (the copy of A, the outputs and the workspace) fits in the HBM budget and
 * a slot is free; admitted requests are batched continuously: every loop
 * iteration first admits what arrived, then advances all admitted problems
 * through a bounded number of grouped launches (the merged launch sequence
 * of plu_batched), so a request that arrives while others run joins them at
 * the next iteration.  A request in a rounded precision form is not merged:
 * all its launches go out on its lane at its first issue (its kernels are
 * launched directly).  Results are bit-identical to the single calls.
 *   plu_server_create   hbm_budget_bytes: device memory the server may use;
 *                       max_slots: problems admitted at once (>= 1).
 *   plu_server_submit   req: as for plu_batched, but A, p, q, L, U are HOST
 *                       pointers (pinned memory recommended); they must stay
 *                       valid until the request completes.  The server
 *                       copies A in and the results out (p, q, the leading
 *                       rank columns of L with leading dimension ldl and
 *                       rows of U with ldu).  Never blocks.  Returns -i for
 *                       an invalid field i, PLU_ERR_OOM when the request
 *                       alone exceeds the budget, PLU_ERR_NOT_IMPLEMENTED
 *                       for PLU_PREC_FP64_INDICATOR.
 *   plu_server_poll     PLU_PENDING, or PLU_OK with *res filled.
 *   plu_server_wait     blocks until the ticket completes.
 *   plu_server_destroy  finishes all submitted work, then frees.
 * Times in plu_result are seconds since plu_server_create.                */
typedef struct plu_server_s* plu_server;
typedef struct {
  uint64_t ticket;
  int32_t status;          /* PLU_* status of the problem */
  int32_t rank;
  double t_submit, t_admit, t_done;
  plu_info info;
} plu_result;

int plu_server_create(plu_server* s, int device, size_t hbm_budget_bytes, int32_t max_slots);
int plu_server_submit(plu_server s, const plu_request* req, uint64_t* ticket);
int plu_server_poll(plu_server s, uint64_t ticket, plu_result* res);
int plu_server_wait(plu_server s, uint64_t ticket, plu_result* res);
int plu_server_destroy(plu_server s);

/* ================= Building blocks (one call per step of the path) ======= */

/* Gaussian test matrix (Sec. 1; Alg. 7): out (device,
 * rows x cols, ldo) filled with N(0,1) values.  Element e = i*cols + j is
 * word e%4 of Philox4x32-10 block e/4 (Salmon et al., SC'11) with counter
 * (e/4 mod 2^32, e/4 div 2^32, 0, 0) and key (seed mod 2^32, seed div 2^32);
 * words map to (0,1] as u = ((x >> 8) + 1) 2^-24 and pairs (w0,w1), (w2,w3)
 * become (r cos t, r sin t) with r = sqrt(-2 ln u_a), t = 2 pi u_b.       */
int plu_gaussian(plu_handle h, int64_t rows, int64_t cols, uint64_t seed,
                 float* out, int64_t ldo);

/* One pass over A (the matrix products of Alg. 7 and Alg. 5 step 3):
 * trans = 0: out (m x l) = A X with X n x l;  trans = 1: out (n x l) = A^T X
 * with X m x l.  All device.  normA2_out: device double*, nullable; receives
 * ||A||_F^2 accumulated in float64 while A streams through (Alg. 8).
 * prec: PLU_PREC_FP32, PLU_PREC_BF16 or PLU_PREC_FP8_E4M3 (operands rounded
 * to that format), optionally | PLU_PREC_A_UNCHANGED (the rounded copies of
 * A from an earlier call are reused: the call is then the pass alone).    */
int plu_pass(plu_handle h, int32_t trans, int64_t m, int64_t n, const float* A, int64_t lda,
             int32_t l, const float* X, int64_t ldx, float* out, int64_t ldo,
             int32_t prec, double* normA2_out);

/* Rounded copy of an operand of the precision form of the passes (the
 * rounding the v-1 passes of Alg. 7 apply to A and to the iterate when prec
 * is not FP32).  src: device fp32 rows x cols (lds).
 *   fmt        PLU_PREC_BF16: uint16 bfloat16 codes (NaN kept quiet);
 *              PLU_PREC_FP8_E4M3: uint8 E4M3 codes plus one E8M0 scale byte
 *              (e + 127) per block of 32 consecutive entries of a dst row;
 *              code = round(x / 2^e) to nearest even.
 *   transpose  0: dst is rows x ldd, dst[i][j] = code(src[i][j]);
 *              1: dst is cols x ldd, dst[j][i] = code(src[i][j]) (blocks of
 *              32 then run along the columns of src).
 *   dst        device codes; ldd a multiple of 64 (BF16) or 128 (FP8), at
 *              least the row length; entries past the row length are set to
 *              zero (the padded layout the passes read).
 *   scales     device uint8, (transpose ? cols : rows) x ldd/32, FP8 only
 *              (ignored for BF16, may be NULL); blocks wholly in the padding
 *              get scale byte 0.                                           */
int plu_quantize(plu_handle h, int32_t fmt, int64_t rows, int64_t cols, const float* src,
                 int64_t lds, int32_t transpose, void* dst, int64_t ldd, void* scales);

/* LU with partial pivoting of a tall M x c matrix (M >= c), the paper's
 * lu(.) (Sec. 2 notation): pivots are the first maximum |value| in LAPACK's
 * current row order.  F (device, in/out, ldf) is replaced by V = P^T L, the
 * unit lower trapezoidal factor placed back in F's own row order (the
 * two-output form [V, ~] = lu(X) of Alg. 6/7).  perm (device int32, length
 * M, nullable) receives the row order: F_in[perm] = L U.  Ufac (device,
 * c x c, ldu, nullable) receives U (upper triangular, zeros below).
 * info (host, nullable): zero_pivot_step and min_pivot_gap.               */
int plu_getrf(plu_handle h, int64_t M, int32_t c, float* F, int64_t ldf,
              int32_t* perm, float* Ufac, int64_t ldu, plu_info* info);

/* Thin QR basis (the paper's [V, ~] = qr(X) in Alg. 6 and Alg. 7): X
 * (device, M x c, ldx, M > c) is replaced by an orthonormal Q with
 * Range(Q(:,1:j)) = Range(X(:,1:j)) for every j (column signs are
 * unspecified).                                                           */
int plu_thin_qr(plu_handle h, int64_t M, int32_t c, float* X, int64_t ldx);

/* Alg. 7 alone: V (device, n x l, ldv) = orthonormal basis after v-1 passes.
 * layout, A, lda, Omega as in plu_fixed_rank (Omega nullable -> drawn from
 * seed).                                                                  */
int plu_range_basis(plu_handle h, int32_t layout, int64_t m, int64_t n, const float* A,
                    int64_t lda, int32_t l, int32_t v, int32_t prec, const float* Omega,
                    uint64_t seed, float* V, int64_t ldv);

/* Thm 4.3 indicator and the Alg. 8 / Alg. 11 rule on G = A V (device,
 * m x l, ldg): column norms^2 in float64, E_j = normA2 - sum_{i<=j}, k = the
 * first column (column_exact) or block end (else) with E_j <= eps^2 normA2.
 * k_out, E_out (host) receive k and E_k; colnorm2 (host, length l,
 * nullable) the column norms.  Returns PLU_TOL_NOT_REACHED when no column
 * qualifies (k = l).  Synchronizes.                                       */
int plu_rank_rule(plu_handle h, int64_t m, int32_t l, const float* G, int64_t ldg,
                  double normA2, double eps, int32_t b, int32_t column_exact,
                  int32_t* k_out, double* E_out, double* colnorm2);

#ifdef __cplusplus
}
#endif

#endif /* POWERLU_H */
