// Precision form of the passes over A: reduced-precision copies of A and of
// the sketch, and the pass kernels on the bfloat16 and scaled FP8 matrix
// cores.
//
// The v - 1 passes of Alg. 7 (Sec. 3.4) run on rounded operands with fp32
// accumulation; the final product with A (Alg. 5 step 3, Alg. 9 step 2) stays
// on the fp32 path and is the refinement pass.
//
// Both operands of a pass are read with the contraction index contiguous:
// A is kept twice, row-major (for A X) and transposed (for A^T Y), and the
// sketch X (K x l) is stored transposed (l x K).  Every copy is zero-padded
// along the contraction index to whole stages of the pass kernel (128
// entries for bfloat16, 256 for FP8), and the sketch to whole column tiles,
// so the pass kernels have no bounds checks along K.
#include "plu_internal.h"

#include <algorithm>

namespace plu {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// bfloat16 of an fp32 value: round to nearest, ties to even, on the 16
// discarded bits; NaN is kept quiet.
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return ((u >> 16) | 0x40u) & 0xFFFFu;
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

__device__ __forceinline__ double wg_sum_double(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// src: R x C fp32 (ld lds).  Writes, for the tiles of 64 x 64 this workgroup
// owns,
//   rm (nullable): R x ldr bf16, rm[i][j] = bf16(src[i][j]) for j < C, 0 for C <= j < ldr;
//   tr (nullable): Ct x ldt bf16, tr[j][i] = bf16(src[i][j]) for i < R, j < C, 0 elsewhere.
// blockIdx.y: band of 64 rows of the tile grid (covering max(R, ldt) rows);
// blockIdx.x: first column tile, then strided by gridDim.x (covering
// max(ldr, Ct) columns).  Optional float64 sum of squares of src, one
// partial per workgroup.
__global__ __launch_bounds__(256) void k_cvt_bf16(const float* __restrict__ src, int64_t lds,
                                                  int64_t R, int64_t C, uint16_t* rm, int64_t ldr,
                                                  uint16_t* tr, int64_t ldt, int64_t Ct,
                                                  int64_t ncol_tiles, double* sumsq_part) {
  __shared__ uint16_t T[64][64 + 4];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * 64;
  const int tr_row = tid >> 4, tc4 = (tid & 15) * 4;   // 16 threads x 4 columns per row
  const bool svec = ((reinterpret_cast<uintptr_t>(src) & 15u) == 0) && ((lds & 3) == 0);
  double ss = 0.0;
  for (int64_t tj = blockIdx.x; tj < ncol_tiles; tj += gridDim.x) {
    const int64_t j0 = tj * 64;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int rr = it * 16 + tr_row;
      const int64_t i = i0 + rr, j = j0 + tc4;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (i < R) {
        const float* s = src + i * lds + j;
        if (svec && j + 3 < C) {
          const f32x4 q = *reinterpret_cast<const f32x4*>(s);
          v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (j + e < C) v[e] = s[e];
        }
      }
      uint32_t b[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (sumsq_part) {
          const double d = v[e];
          ss = fma(d, d, ss);
        }
        b[e] = bf16_bits(v[e]);
        T[tc4 + e][rr] = (uint16_t)b[e];
      }
      if (rm && i < R && j < ldr) {
        uint2 w;
        w.x = b[0] | (b[1] << 16);
        w.y = b[2] | (b[3] << 16);
        *reinterpret_cast<uint2*>(rm + i * ldr + j) = w;
      }
    }
    __syncthreads();
    if (tr) {
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int cc = it * 16 + tr_row;
        const int64_t j = j0 + cc, i = i0 + tc4;
        if (j < Ct && i < ldt) {
          uint2 w;
          w.x = (uint32_t)T[cc][tc4 + 0] | ((uint32_t)T[cc][tc4 + 1] << 16);
          w.y = (uint32_t)T[cc][tc4 + 2] | ((uint32_t)T[cc][tc4 + 3] << 16);
          *reinterpret_cast<uint2*>(tr + j * ldt + i) = w;
        }
      }
    }
    __syncthreads();
  }
  if (sumsq_part) {
    const double t = wg_sum_double(ss, red);
    if (tid == 0) sumsq_part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
  }
}

// One pass on the bfloat16 matrix cores: out[p][c] = sum_k M[p][k] Xt[c][k],
//   M: P x K bf16 (ld ldm, 16-byte aligned rows, zero beyond the logical K),
//   Xt: Ct x K bf16 (ld ldx), K a multiple of 128, Ct >= gridDim.y * NT * 16,
// with A and the sketch staged through LDS by direct loads (global_load_lds,
// 16 bytes per lane, nothing held in registers).  A pass over A is bound by
// HBM, and HBM delivers far less for short runs per row: a plain streaming
// kernel reads 3.3 TB/s in runs of 128 bytes per row and 5.4-5.9 TB/s in
// runs of 256-2048 bytes (measured).  So a stage here spans 128 entries of K
// (256 bytes of each row), and every load instruction moves 4 whole rows of
// a stage.
// The 16-byte chunks are placed in LDS by an XOR of chunk and row index so
// that the MFMA operand reads stay free of bank conflicts.
//   Workgroup: 512 threads, 256 rows of P x NT*16 columns (NT <= 8).  The
//   sketch block of a stage is re-read from L2 by every workgroup: 256 rows
//   keep that traffic at NT * 16 / 256 of A's (measured: with 128 rows the
//   sketch traffic alone cost a fifth of the pass).  LDS: A in two 64 KB
//   buffers (loaded up to two stages ahead, non-temporal, from HBM), the
//   sketch in one of 32 KB.
//   Each wave loads 32 rows of A (8 instructions) and up to 4 of the
//   sketch's 4 NT blocks per stage, A last, and waits with vmcnt(8): loads
//   complete in order, so at that point only its A loads of the next stage
//   may still be outstanding.  The MFMA work of a stage is split over the
//   waves along the contraction (2 x 32 entries each, for 64 rows), which
//   keeps the LDS reads at 1.5 bytes per byte of A; the two partial sums of
//   each row block are added once at the end.
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));

// LDS byte offset of a __shared__ object (its address in the local space).
__device__ __forceinline__ uint32_t lds_off(const void* p) {
  return static_cast<uint32_t>(reinterpret_cast<uintptr_t>(
      (const __attribute__((address_space(3))) void*)p));
}

// The MFMA operands of a wave's step of a stage, read from LDS in one block
// that waits for its own reads: A's fragments of 4 row tiles at a + 4 KB t
// and the sketch's fragments of NX column tiles at x + 4 KB j.  The compiler
// does not see these reads, so it adds no wait for the loads to LDS still in
// flight (it cannot tell that they write other buffers); the kernel orders
// them itself.
template <int NX>
__device__ __forceinline__ void lds_operands(uint32_t a, uint32_t x, u32x4v (&ao)[4],
                                             u32x4v (&xo)[8]) {
  if constexpr (NX == 8) {
    asm volatile(
        "ds_read_b128 %0, %12\n\t"
        "ds_read_b128 %1, %12 offset:4096\n\t"
        "ds_read_b128 %2, %12 offset:8192\n\t"
        "ds_read_b128 %3, %12 offset:12288\n\t"
        "ds_read_b128 %4, %13\n\t"
        "ds_read_b128 %5, %13 offset:4096\n\t"
        "ds_read_b128 %6, %13 offset:8192\n\t"
        "ds_read_b128 %7, %13 offset:12288\n\t"
        "ds_read_b128 %8, %13 offset:16384\n\t"
        "ds_read_b128 %9, %13 offset:20480\n\t"
        "ds_read_b128 %10, %13 offset:24576\n\t"
        "ds_read_b128 %11, %13 offset:28672\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(ao[0]), "=&v"(ao[1]), "=&v"(ao[2]), "=&v"(ao[3]), "=&v"(xo[0]), "=&v"(xo[1]),
          "=&v"(xo[2]), "=&v"(xo[3]), "=&v"(xo[4]), "=&v"(xo[5]), "=&v"(xo[6]), "=&v"(xo[7])
        : "v"(a), "v"(x)
        : "memory");
  } else {
    static_assert(NX == 4, "4 or 8 sketch fragments");
    asm volatile(
        "ds_read_b128 %0, %8\n\t"
        "ds_read_b128 %1, %8 offset:4096\n\t"
        "ds_read_b128 %2, %8 offset:8192\n\t"
        "ds_read_b128 %3, %8 offset:12288\n\t"
        "ds_read_b128 %4, %9\n\t"
        "ds_read_b128 %5, %9 offset:4096\n\t"
        "ds_read_b128 %6, %9 offset:8192\n\t"
        "ds_read_b128 %7, %9 offset:12288\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(ao[0]), "=&v"(ao[1]), "=&v"(ao[2]), "=&v"(ao[3]), "=&v"(xo[0]), "=&v"(xo[1]),
          "=&v"(xo[2]), "=&v"(xo[3])
        : "v"(a), "v"(x)
        : "memory");
  }
}

template <int NT, int EPI>
__global__ __launch_bounds__(512, 1) void k_pass_bf16(const uint16_t* __restrict__ M,
                                                          int64_t ldm,
                                                          const uint16_t* __restrict__ Xt,
                                                          int64_t ldx, float* out, int64_t ldo,
                                                          int64_t part_stride, int64_t P,
                                                          int64_t K, int64_t C, int64_t ksplit,
                                                          int nsplit) {
  static_assert(NT >= 1 && NT <= 8, "at most 8 column tiles");
  constexpr int KS = 128;
  constexpr int BLK = 512;                      // uint16 per 1 KB block (4 rows of a stage)
  __shared__ __attribute__((aligned(16))) uint16_t As[2][64 * BLK];
  __shared__ __attribute__((aligned(16))) uint16_t Xs[32 * BLK];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, r = lane & 15, g4 = lane >> 4;
  const int nwg = gridDim.x;
  const int xcd = blockIdx.x & 7, idx = blockIdx.x >> 3;
  const int per = nwg >> 3, rem = nwg & 7;
  const int lid = (xcd < rem) ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
  const int npb = nwg / nsplit;
  const int split = lid / npb;
  const int64_t p0 = (int64_t)(lid % npb) * 256;
  const int64_t c0 = (int64_t)blockIdx.y * (NT * 16);
  const int64_t kb = (int64_t)split * ksplit;
  const int64_t ke = (kb + ksplit < K) ? kb + ksplit : K;
  const int nst = kb < ke ? (int)((ke - kb) / KS) : 0;

  // A load t (0..7) of wave w moves 4 rows of its 32, 256 bytes (the whole
  // stage) of each: lane l writes the 16 bytes at 16 l of 1 KB block 8 w + t,
  // i.e. row rho = 4 (t % 4) + l / 16 of 16-row tile 2 w + t / 4, slot
  // l % 16, and fetches into it the 16-byte chunk (l % 16) ^ rho of that
  // row.  Chunk c of row rho thus sits at slot c ^ rho: the MFMA reads below
  // (16 rows, one chunk each) fall in 16 distinct bank groups.  Rows past P
  // read row P - 1 (valid memory whose products are never stored).
  const uint16_t* aa[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int rho = 4 * (t & 3) + g4;
    const int64_t ra = p0 + wave * 32 + 16 * (t >> 2) + rho;
    aa[t] = M + (ra < P ? ra : P - 1) * ldm + kb + ((r ^ rho) * 8);
  }
  // sketch block q = 4 wave + i holds columns 4 q .. 4 q + 3 of the column
  // block, same arrangement (column tile q / 4, rows 4 (q % 4) + l / 16);
  // blocks past the 4 NT real ones are not loaded
  const uint16_t* xs[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = wave * 4 + i;
    const int rho = 4 * (q & 3) + g4;
    xs[i] = Xt + (c0 + 4 * (q < 4 * NT ? q : 0) + g4) * ldx + kb + ((r ^ rho) * 8);
  }
  // wave w computes, for rows 64 (w / 2) .. + 64 (4 row tiles) and all NT
  // column tiles, the 32-deep steps h = 2 (w % 2) and 2 (w % 2) + 1 of every
  // stage; the two partial products of a row quarter are added at the end.
  // Its fragment of step h of a 16-row tile: row r, chunk 4 h + g4, at byte
  // r * 256 + ((4 h + g4) ^ r) * 16 of the tile's 4 KB.
  const int quarter = wave >> 1, hk = wave & 1;
  uint32_t off[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int h = 2 * hk + u;
    off[u] = (uint32_t)(r * 256 + (((4 * h + g4) ^ r) * 16));
  }

  f32x4 acc[4][NT];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // each issue moves the next stage of this wave's blocks and advances its
  // source pointers by a stage; A is streamed once, so its loads are
  // non-temporal (they should not push the sketch, re-read by every
  // workgroup, out of L2)
  auto issue_a = [&](uint16_t* Ab) __attribute__((always_inline)) {
    uint16_t* ad = Ab + (wave * 8) * BLK;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      __builtin_amdgcn_global_load_lds(aa[t], ad + t * BLK, 16, 0, 2);
      aa[t] += KS;
    }
  };
  auto issue_x = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (wave * 4 + i < 4 * NT) {
        __builtin_amdgcn_global_load_lds(xs[i], Xs + (wave * 4 + i) * BLK, 16, 0, 0);
        xs[i] += KS;
      }
  };
  constexpr int NX = NT <= 4 ? 4 : 8;
  auto compute = [&](const uint16_t* Ab) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      u32x4v ao[4], xo[8];
      lds_operands<NX>(lds_off(Ab) + (uint32_t)(quarter * 16384) + off[u], lds_off(Xs) + off[u],
                       ao, xo);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bf16x8 f = __builtin_bit_cast(bf16x8, ao[t]);
#pragma unroll
        for (int j = 0; j < NT; ++j)
          acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              f, __builtin_bit_cast(bf16x8, xo[j]), acc[t][j], 0, 0, 0);
      }
      // the fragments past NT were read too (the block reads NX); their
      // values are not needed
#pragma unroll
      for (int j = NT; j < NX; ++j) asm volatile("" ::"v"(xo[j]));
    }
  };
  // stage s: wait for its loads (A of stage s + 1 may stay in flight: the
  // last 8 loads of this wave), a plain barrier (not __syncthreads(), whose
  // fence would wait for every load to LDS in flight) that publishes the
  // other waves' blocks, multiply, a barrier (every wave is done with the
  // sketch and with A of stage s), then the sketch of stage s + 1 and A of
  // stage s + 2 into those buffers.  The multiplication is short next to a
  // stage of HBM traffic, so A's loads stay 1-2 stages ahead.
  if (nst > 0) {
    issue_a(As[0]);
    issue_x();
  }
  if (nst > 1) issue_a(As[1]);
  for (int s = 0; s < nst; ++s) {
    if (s + 1 < nst) __builtin_amdgcn_s_waitcnt(0x0F78);   // vmcnt(8)
    else __builtin_amdgcn_s_waitcnt(0x0F70);               // vmcnt(0)
    __builtin_amdgcn_s_barrier();
    compute(As[s & 1]);
    __builtin_amdgcn_s_barrier();
    if (s + 1 < nst) issue_x();
    if (s + 2 < nst) issue_a(As[s & 1]);
  }

  // the two partial products of each row quarter, added through LDS (the
  // stage buffers are free: every wave is past its last step's barrier and
  // no load is outstanding).  Lane-contiguous layout: entry (t, j, e) of a
  // lane at ((t NT + j) 4 + e) 64 + lane, quarter q's at 28 KB q.
  float* const red = reinterpret_cast<float*>(As[0]) + quarter * (4 * 8 * 4 * 64);
  if (hk == 1) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) red[((t * NT + j) * 4 + e) * 64 + lane] = acc[t][j][e];
  }
  __syncthreads();
  if (hk == 1) return;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[t][j][e] += red[((t * NT + j) * 4 + e) * 64 + lane];

  // acc[t][j][e] is out[p][c], p = p0 + 64 quarter + 16 t + 4 g4 + e,
  // c = c0 + 16 j + r
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t p = p0 + quarter * 64 + t * 16 + g4 * 4 + e;
      if (p >= P) continue;
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const int64_t c = c0 + j * 16 + r;
        if (c >= C) continue;
        if (EPI == EPI_PART)
          out[(int64_t)split * part_stride + p * ldo + c] = acc[t][j][e];
        else
          out[p * ldo + c] = acc[t][j][e];
      }
    }
}

// ---------------------------------------------------------------------------
// Block-scaled FP8 E4M3 (OCP "e4m3fn": bias 7, 3 mantissa bits, largest
// finite 448, subnormal spacing 2^-9).  Each block of 32 consecutive entries
// along the contraction index shares a power-of-two scale 2^e (an E8M0 byte
// e + 127), e the smallest integer with max|x| / 2^e <= 448, at least -127.
// ---------------------------------------------------------------------------
typedef int i32x8 __attribute__((ext_vector_type(8)));

// e for a block whose largest magnitude is amax (>= 0, finite): with
// amax = f 2^E, f in [1, 2), 448 = 1.75 2^8, e = E - 8 when f <= 1.75 and
// E - 7 otherwise.
__device__ __forceinline__ int mx_exponent(float amax) {
  const uint32_t u = __float_as_uint(amax);
  const int eb = (int)(u >> 23);
  if (eb == 0) return -127;
  const int e = eb - 127 - 8 + (((u & 0x7FFFFFu) > 0x600000u) ? 1 : 0);
  return e < -127 ? -127 : e;
}

// E4M3 code of y, |y| <= 448, round to nearest even.
__device__ __forceinline__ uint32_t e4m3_code(float y) {
  const uint32_t s = (__float_as_uint(y) >> 24) & 0x80u;
  const float a = fabsf(y);
  uint32_t c;
  if (a < 0.015625f) {
    // below 2^-6: multiples of 2^-9 (8 * 2^-9 = 2^-6 is the code of the
    // smallest normal, so rounding up into it needs no special case)
    c = (uint32_t)rintf(a * 512.0f);
  } else {
    const uint32_t ua = __float_as_uint(a);
    const uint32_t E = (ua >> 23) - 120u;                    // biased exponent: 127 - 7
    const uint32_t m = ua & 0x7FFFFFu;
    const uint32_t m3 = (m + 0x7FFFFu + ((m >> 20) & 1u)) >> 20;   // 0..8, carry into E
    c = (E << 3) + m3;
  }
  return s | c;
}

// Largest magnitude over the 8 lanes l with equal l >> 3 (a 32-entry block
// held as 4 entries per lane).
__device__ __forceinline__ float max8(float v) {
  v = fmaxf(v, __shfl_xor(v, 1, 64));
  v = fmaxf(v, __shfl_xor(v, 2, 64));
  v = fmaxf(v, __shfl_xor(v, 4, 64));
  return v;
}

// 4 codes of v[0..3] under the block exponent e, packed little-endian.
__device__ __forceinline__ uint32_t pack4_e4m3(const float* v, int e) {
  uint32_t w = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) w |= e4m3_code(ldexpf(v[q], -e)) << (8 * q);
  return w;
}

// src: R x C fp32 (ld lds).  Writes, for the 64 x 64 tiles this workgroup
// owns (same tiling as k_cvt_bf16),
//   rm/rsc (nullable): R x ldr codes and R x ldr/32 scales, blocks of 32
//     along each row (j), zero codes and scale byte 0 past C;
//   tr/tsc (nullable): Ct x ldt codes and Ct x ldt/32 scales of src^T,
//     blocks of 32 along i, zero past R and for rows j >= C;
// and optionally the float64 sum of squares of src, one partial per
// workgroup (as k_cvt_bf16).
__global__ __launch_bounds__(256) void k_cvt_fp8(const float* __restrict__ src, int64_t lds,
                                                 int64_t R, int64_t C, uint8_t* rm, uint8_t* rsc,
                                                 int64_t ldr, uint8_t* tr, uint8_t* tsc,
                                                 int64_t ldt, int64_t Ct, int64_t ncol_tiles,
                                                 double* sumsq_part) {
  __shared__ float T[64][64 + 1];
  __shared__ double red[4];
  double ss = 0.0;
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * 64;
  const int tr_row = tid >> 4, tc4 = (tid & 15) * 4;
  const bool svec = ((reinterpret_cast<uintptr_t>(src) & 15u) == 0) && ((lds & 3) == 0);
  for (int64_t tj = blockIdx.x; tj < ncol_tiles; tj += gridDim.x) {
    const int64_t j0 = tj * 64;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int rr = it * 16 + tr_row;
      const int64_t i = i0 + rr, j = j0 + tc4;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (i < R) {
        const float* sp = src + i * lds + j;
        if (svec && j + 3 < C) {
          const f32x4 q = *reinterpret_cast<const f32x4*>(sp);
          v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (j + e < C) v[e] = sp[e];
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        T[tc4 + e][rr] = v[e];
        if (sumsq_part) {
          const double d = v[e];
          ss = fma(d, d, ss);
        }
      }
      if (rm) {
        float am = fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])));
        am = max8(am);
        const int e = mx_exponent(am);
        if (i < R && j < ldr) {
          *reinterpret_cast<uint32_t*>(rm + i * ldr + j) = pack4_e4m3(v, e);
          if ((tid & 7) == 0) rsc[i * (ldr / 32) + j / 32] = (uint8_t)(e + 127);
        }
      }
    }
    __syncthreads();
    if (tr) {
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int cc = it * 16 + tr_row;
        const int64_t j = j0 + cc, i = i0 + tc4;
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = T[cc][tc4 + e];
        float am = fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])));
        am = max8(am);
        const int e = mx_exponent(am);
        if (j < Ct && i < ldt) {
          *reinterpret_cast<uint32_t*>(tr + j * ldt + i) = pack4_e4m3(v, e);
          if ((tid & 7) == 0) tsc[j * (ldt / 32) + i / 32] = (uint8_t)(e + 127);
        }
      }
    }
    __syncthreads();
  }
  if (sumsq_part) {
    const double t = wg_sum_double(ss, red);
    if (tid == 0) sumsq_part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
  }
}

// One pass on the FP8 matrix cores with per-block scales:
// out[p][c] = sum_k (M[p][k] 2^sM[p][k/32]) (Xt[c][k] 2^sX[c][k/32]).
//   M: P x K codes (ld ldm, K a multiple of 256), Ms: P x K/32 scale bytes
//   (ld ldm / 32, 4-byte aligned rows); Xt: Ct x K codes (ld ldx), Xsc:
//   Ct x K/32 (ld ldx / 32).
// v_mfma_scale_f32_16x16x128_f8f6f4 (layout measured on gfx950): lane
// (r, g) supplies row r's codes k0 + 16 g + [0, 16) in its first 16 bytes and
// k0 + 64 + 16 g + [0, 16) in its last 16, and the scale of block
// k0/32 + g; the hardware applies the scale of lane group b to the 32
// entries k0 + 32 b + [0, 32), which lane groups 2(b mod 2) and 2(b mod 2)+1
// hold.  Both operands use this layout.
// Same design as the bfloat16 pass: a stage is 256 entries of K (256 bytes
// of each row), every load moves whole rows of a stage into LDS with the
// chunks XOR-swizzled, A non-temporal in two buffers, the sketch in one.
// The scale bytes of a stage (8 per row) come along by 4-byte direct loads.
// LDS holds 192 rows of A per buffer (2 x 48 KB + 2 x 1.5 KB of scales, the
// sketch 32 KB + 1 KB): 256 rows would not leave room for the scales.  The
// two 128-deep MFMA steps of a stage are split over the waves (wave w: 3 row
// tiles of rows 48 (w / 2) .., step w % 2); the two partial sums of each row
// block are added once at the end.
// 3 row tiles of A: both 16-byte halves of each fragment, the first at
// a1 + 4 KB t, the second at a2 + 4 KB t.
__device__ __forceinline__ void lds_read2x3(uint32_t a1, uint32_t a2, u32x4v (&o)[6]) {
  asm volatile(
      "ds_read_b128 %0, %6\n\t"
      "ds_read_b128 %1, %7\n\t"
      "ds_read_b128 %2, %6 offset:4096\n\t"
      "ds_read_b128 %3, %7 offset:4096\n\t"
      "ds_read_b128 %4, %6 offset:8192\n\t"
      "ds_read_b128 %5, %7 offset:8192\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3]), "=&v"(o[4]), "=&v"(o[5])
      : "v"(a1), "v"(a2)
      : "memory");
}

// 4 column tiles of the sketch: both 16-byte halves of each fragment, the
// first at x1 + 4 KB j, the second at x2 + 4 KB j.
__device__ __forceinline__ void lds_read2x4(uint32_t x1, uint32_t x2, u32x4v (&o)[8]) {
  asm volatile(
      "ds_read_b128 %0, %8\n\t"
      "ds_read_b128 %1, %9\n\t"
      "ds_read_b128 %2, %8 offset:4096\n\t"
      "ds_read_b128 %3, %9 offset:4096\n\t"
      "ds_read_b128 %4, %8 offset:8192\n\t"
      "ds_read_b128 %5, %9 offset:8192\n\t"
      "ds_read_b128 %6, %8 offset:12288\n\t"
      "ds_read_b128 %7, %9 offset:12288\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3]), "=&v"(o[4]), "=&v"(o[5]),
        "=&v"(o[6]), "=&v"(o[7])
      : "v"(x1), "v"(x2)
      : "memory");
}

// Scale bytes: 3 of A at sa + 128 t, 8 of the sketch at sx + 128 j.
__device__ __forceinline__ void lds_scales(uint32_t sa, uint32_t sx, uint32_t (&ao)[3],
                                           uint32_t (&xo)[8]) {
  asm volatile(
      "ds_read_u8 %0, %11\n\t"
      "ds_read_u8 %1, %11 offset:128\n\t"
      "ds_read_u8 %2, %11 offset:256\n\t"
      "ds_read_u8 %3, %12\n\t"
      "ds_read_u8 %4, %12 offset:128\n\t"
      "ds_read_u8 %5, %12 offset:256\n\t"
      "ds_read_u8 %6, %12 offset:384\n\t"
      "ds_read_u8 %7, %12 offset:512\n\t"
      "ds_read_u8 %8, %12 offset:640\n\t"
      "ds_read_u8 %9, %12 offset:768\n\t"
      "ds_read_u8 %10, %12 offset:896\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(ao[0]), "=&v"(ao[1]), "=&v"(ao[2]), "=&v"(xo[0]), "=&v"(xo[1]), "=&v"(xo[2]),
        "=&v"(xo[3]), "=&v"(xo[4]), "=&v"(xo[5]), "=&v"(xo[6]), "=&v"(xo[7])
      : "v"(sa), "v"(sx)
      : "memory");
}

__device__ __forceinline__ i32x8 cat8(const u32x4v& lo, const u32x4v& hi) {
  return __builtin_bit_cast(i32x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}

template <int NT, int EPI>
__global__ __launch_bounds__(512, 1) void k_pass_fp8(const uint8_t* __restrict__ M,
                                                     const uint8_t* __restrict__ Ms, int64_t ldm,
                                                     const uint8_t* __restrict__ Xt,
                                                     const uint8_t* __restrict__ Xsc, int64_t ldx,
                                                     float* out, int64_t ldo, int64_t part_stride,
                                                     int64_t P, int64_t K, int64_t C,
                                                     int64_t ksplit, int nsplit) {
  static_assert(NT >= 1 && NT <= 8, "at most 8 column tiles");
  constexpr int KS = 256;
  constexpr int ROWS = 192;
  __shared__ __attribute__((aligned(16))) uint8_t As[2][ROWS * 256];
  __shared__ __attribute__((aligned(16))) uint8_t Ass[2][ROWS * 8];
  __shared__ __attribute__((aligned(16))) uint8_t Xs[128 * 256];
  __shared__ __attribute__((aligned(16))) uint8_t Xss[128 * 8];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, r = lane & 15, g4 = lane >> 4;
  const int nwg = gridDim.x;
  const int xcd = blockIdx.x & 7, idx = blockIdx.x >> 3;
  const int per = nwg >> 3, rem = nwg & 7;
  const int lid = (xcd < rem) ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
  const int npb = nwg / nsplit;
  const int split = lid / npb;
  const int64_t p0 = (int64_t)(lid % npb) * ROWS;
  const int64_t c0 = (int64_t)blockIdx.y * (NT * 16);
  const int64_t kb = (int64_t)split * ksplit;
  const int64_t ke = (kb + ksplit < K) ? kb + ksplit : K;
  const int nst = kb < ke ? (int)((ke - kb) / KS) : 0;
  const int64_t lds_ = ldm / 32, ldxs = ldx / 32;

  // A codes: load t (0..5) of wave w moves rows 24 w + 4 t + l / 16 (16-row
  // tile (24 w + 4 t) / 16), lane l into slot l % 16 of its row with chunk
  // (l % 16) ^ rho, rho the row's index in its tile.  Rows past P read row
  // P - 1 (valid memory whose products are never stored).
  const uint8_t* aa[6];
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    const int row = wave * 24 + 4 * t + g4;
    const int rho = row & 15;
    const int64_t ra = p0 + row;
    aa[t] = M + (ra < P ? ra : P - 1) * ldm + kb + ((r ^ rho) * 16);
  }
  // A scales: waves 0..5 move 32 rows each, lane l the 4 bytes (l & 1) of
  // row 32 w + l / 2 (8 bytes per row and stage)
  const uint8_t* as_;
  {
    const int64_t ra = p0 + (wave < 6 ? wave : 0) * 32 + (lane >> 1);
    as_ = Ms + (ra < P ? ra : P - 1) * lds_ + kb / 32 + (lane & 1) * 4;
  }
  // sketch codes: block q = 4 w + i (columns 4 q .. 4 q + 3 of the column
  // block), as for A; blocks past the 4 NT real ones are not loaded
  const uint8_t* xs[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = wave * 4 + i;
    const int rho = 4 * (q & 3) + g4;
    xs[i] = Xt + (c0 + 4 * (q < 4 * NT ? q : 0) + g4) * ldx + kb + ((r ^ rho) * 16);
  }
  // sketch scales: waves 0..3 move 32 columns each (those past 16 NT read
  // column 0 again, into slots never used)
  const uint8_t* xss;
  {
    const int col = (wave < 4 ? wave : 0) * 32 + (lane >> 1);
    xss = Xsc + (c0 + (col < 16 * NT ? col : 0)) * ldxs + kb / 32 + (lane & 1) * 4;
  }

  // wave w: rows 48 grp .. + 48 (3 row tiles), MFMA step u of each stage
  const int grp = wave >> 1, u = wave & 1;
  const uint32_t off1 = (uint32_t)(r * 256 + (((8 * u + g4) ^ r) * 16));
  const uint32_t off2 = (uint32_t)(r * 256 + (((8 * u + 4 + g4) ^ r) * 16));
  const uint32_t soff = (uint32_t)(r * 8 + 4 * u + g4);

  f32x4 acc[3][NT];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  auto issue_a = [&](int b) __attribute__((always_inline)) {
    uint8_t* ad = As[b] + wave * 6 * 1024;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      __builtin_amdgcn_global_load_lds(aa[t], ad + t * 1024, 16, 0, 2);
      aa[t] += KS;
    }
  };
  // sketch and scales of a stage; the A scales ride here too (issued before
  // the sketch's codes, so a wait for those covers them)
  auto issue_x = [&](int b_scales) __attribute__((always_inline)) {
    if (wave < 6) __builtin_amdgcn_global_load_lds(as_, Ass[b_scales] + wave * 256, 4, 0, 0);
    as_ += KS / 32;
    if (wave < 4) __builtin_amdgcn_global_load_lds(xss, Xss + wave * 256, 4, 0, 0);
    xss += KS / 32;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (wave * 4 + i < 4 * NT) {
        __builtin_amdgcn_global_load_lds(xs[i], Xs + (wave * 4 + i) * 1024, 16, 0, 0);
        xs[i] += KS;
      }
  };
  auto compute = [&](int b) __attribute__((always_inline)) {
    uint32_t sa[3], sx[8];
    lds_scales(lds_off(Ass[b]) + (uint32_t)(grp * 48 * 8) + soff, lds_off(Xss) + soff, sa, sx);
    u32x4v ao[6];
    const uint32_t abase = lds_off(As[b]) + (uint32_t)(grp * 3 * 4096);
    lds_read2x3(abase + off1, abase + off2, ao);
    i32x8 fa[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) fa[t] = cat8(ao[2 * t], ao[2 * t + 1]);
    const uint32_t xbase = lds_off(Xs);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if (half * 4 >= NT) break;
      u32x4v xo[8];
      lds_read2x4(xbase + (uint32_t)(half * 16384) + off1, xbase + (uint32_t)(half * 16384) + off2,
                  xo);
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int j = half * 4 + jj;
        if (j < NT) {
          const i32x8 fb = cat8(xo[2 * jj], xo[2 * jj + 1]);
#pragma unroll
          for (int t = 0; t < 3; ++t)
            acc[t][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                fa[t], fb, acc[t][j], 0, 0, 0, (int)sa[t], 0, (int)sx[j]);
        } else {
          asm volatile("" ::"v"(xo[2 * jj]), "v"(xo[2 * jj + 1]));
        }
      }
    }
#pragma unroll
    for (int j = NT; j < 8; ++j) asm volatile("" ::"v"(sx[j]));
  };
  // stage s: wait for its loads (A of stage s + 1 may stay in flight: the
  // last 6 loads of this wave), barrier, multiply, barrier, then the scales
  // and sketch of stage s + 1 and A of stage s + 2.  The A scales of stage
  // s + 1 go with the sketch of stage s + 1 into the scale buffer of stage
  // s - 1 (free: its multiplication is past the last barrier).
  if (nst > 0) {
    issue_x(0);
    issue_a(0);
  }
  if (nst > 1) issue_a(1);
  for (int s = 0; s < nst; ++s) {
    if (s + 1 < nst) __builtin_amdgcn_s_waitcnt(0x0F76);   // vmcnt(6)
    else __builtin_amdgcn_s_waitcnt(0x0F70);               // vmcnt(0)
    __builtin_amdgcn_s_barrier();
    compute(s & 1);
    __builtin_amdgcn_s_barrier();
    if (s + 1 < nst) issue_x((s + 1) & 1);
    if (s + 2 < nst) issue_a(s & 1);
  }

  // the two partial products of each row block, added through LDS (every
  // wave is past its last barrier and no load is outstanding).  Entry
  // (t, j, e) of a lane at ((t NT + j) 4 + e) 64 + lane, group g's at 24 KB g.
  float* const red = reinterpret_cast<float*>(As[0]) + grp * (3 * 8 * 4 * 64);
  if (u == 1) {
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) red[((t * NT + j) * 4 + e) * 64 + lane] = acc[t][j][e];
  }
  __syncthreads();
  if (u == 1) return;
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[t][j][e] += red[((t * NT + j) * 4 + e) * 64 + lane];

  // acc[t][j][e] is out[p][c], p = p0 + 48 grp + 16 t + 4 g4 + e, c = c0 + 16 j + r
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t p = p0 + grp * 48 + t * 16 + g4 * 4 + e;
      if (p >= P) continue;
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const int64_t c = c0 + j * 16 + r;
        if (c >= C) continue;
        if (EPI == EPI_PART)
          out[(int64_t)split * part_stride + p * ldo + c] = acc[t][j][e];
        else
          out[p * ldo + c] = acc[t][j][e];
      }
    }
}

// The wide forms of both passes (NT > 8 column tiles, sketches of more than
// 128 columns): one workgroup holds all column tiles, so A is streamed once
// (two column blocks would read it twice).  192 rows per workgroup (the
// sketch stage takes up to 64 KB of LDS); wave w takes rows 48 (w / 2) ..
// + 48 (3 row tiles) and the column tiles NTH (w % 2) .. + NTH (NTH =
// ceil(NT / 2)) over the whole stage, so no partial sums are exchanged.
// Loads, swizzle and stage schedule as in the narrow kernels.

// 3 A fragments at a + 4 KB t and 8 sketch fragments at x + 2 KB j (the
// sketch half-stage layout: 16 columns of 128 bytes per tile).
__device__ __forceinline__ void lds_read_3_8h(uint32_t a, uint32_t x, u32x4v (&ao)[3],
                                              u32x4v (&xo)[8]) {
  asm volatile(
      "ds_read_b128 %0, %11\n\t"
      "ds_read_b128 %1, %11 offset:4096\n\t"
      "ds_read_b128 %2, %11 offset:8192\n\t"
      "ds_read_b128 %3, %12\n\t"
      "ds_read_b128 %4, %12 offset:2048\n\t"
      "ds_read_b128 %5, %12 offset:4096\n\t"
      "ds_read_b128 %6, %12 offset:6144\n\t"
      "ds_read_b128 %7, %12 offset:8192\n\t"
      "ds_read_b128 %8, %12 offset:10240\n\t"
      "ds_read_b128 %9, %12 offset:12288\n\t"
      "ds_read_b128 %10, %12 offset:14336\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(ao[0]), "=&v"(ao[1]), "=&v"(ao[2]), "=&v"(xo[0]), "=&v"(xo[1]), "=&v"(xo[2]),
        "=&v"(xo[3]), "=&v"(xo[4]), "=&v"(xo[5]), "=&v"(xo[6]), "=&v"(xo[7])
      : "v"(a), "v"(x)
      : "memory");
}

// The sketch stage is kept in two half-stages (64 entries of K each, 32 KB
// for 16 column tiles), reloaded separately: the next stage's first half
// streams in while the second half is multiplied, and its second half while
// the next stage's first half is, so the L2 latency of the sketch overlaps
// the matrix-core work.  A half-stage column is 128 bytes; chunk c (0..7) of
// column q sits at slot c ^ ((q / 2) mod 8), which keeps the operand reads
// of 16 columns in 16 distinct bank groups.
template <int NT, int EPI>
__global__ __launch_bounds__(512, 1) void k_pass_bf16_wide(const uint16_t* __restrict__ M,
                                                           int64_t ldm,
                                                           const uint16_t* __restrict__ Xt,
                                                           int64_t ldx, float* out, int64_t ldo,
                                                           int64_t part_stride, int64_t P,
                                                           int64_t K, int64_t C, int64_t ksplit,
                                                           int nsplit) {
  static_assert(NT > 8 && NT <= 16, "9 to 16 column tiles");
  constexpr int KS = 128, ROWS = 192, NTH = (NT + 1) / 2;
  constexpr int BLK = 512;                      // uint16 per 1 KB block
  __shared__ __attribute__((aligned(16))) uint16_t As[2][48 * BLK];
  __shared__ __attribute__((aligned(16))) uint16_t Xh[2][32 * BLK];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, r = lane & 15, g4 = lane >> 4;
  const int nwg = gridDim.x;
  const int xcd = blockIdx.x & 7, idx = blockIdx.x >> 3;
  const int per = nwg >> 3, rem = nwg & 7;
  const int lid = (xcd < rem) ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
  const int npb = nwg / nsplit;
  const int split = lid / npb;
  const int64_t p0 = (int64_t)(lid % npb) * ROWS;
  const int64_t c0 = (int64_t)blockIdx.y * (NT * 16);
  const int64_t kb = (int64_t)split * ksplit;
  const int64_t ke = (kb + ksplit < K) ? kb + ksplit : K;
  const int nst = kb < ke ? (int)((ke - kb) / KS) : 0;

  // A: load t (0..5) of wave w moves rows 24 w + 4 t + l / 16 into block
  // 6 w + t (256 bytes per row, chunk (l % 16) ^ (row mod 16) at slot l % 16)
  const uint16_t* aa[6];
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    const int row = wave * 24 + 4 * t + g4;
    const int rho = row & 15;
    const int64_t ra = p0 + row;
    aa[t] = M + (ra < P ? ra : P - 1) * ldm + kb + ((r ^ rho) * 8);
  }
  // sketch half-stage: block b = 4 w + i (0..31) holds columns 8 b .. 8 b + 7,
  // lane l column 8 b + l / 8 at slot l % 8; columns past 16 NT load column
  // 0 (into slots never read), so every wave issues 4 loads per half
  const uint16_t* xs[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int col = 8 * (4 * wave + i) + (lane >> 3);
    const int slot = lane & 7;
    const int chunk = slot ^ ((col >> 1) & 7);
    xs[i] = Xt + (c0 + (col < 16 * NT ? col : 0)) * ldx + kb + chunk * 8;
  }
  const int grp = wave >> 1, half = wave & 1;
  uint32_t off[4], xoff[2];
#pragma unroll
  for (int h = 0; h < 4; ++h) off[h] = (uint32_t)(r * 256 + (((4 * h + g4) ^ r) * 16));
#pragma unroll
  for (int h = 0; h < 2; ++h) xoff[h] = (uint32_t)(r * 128 + (((4 * h + g4) ^ ((r >> 1) & 7)) * 16));

  f32x4 acc[3][NTH];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int j = 0; j < NTH; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  auto issue_a = [&](int b) __attribute__((always_inline)) {
    uint16_t* ad = As[b] + (wave * 6) * BLK;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      __builtin_amdgcn_global_load_lds(aa[t], ad + t * BLK, 16, 0, 2);
      aa[t] += KS;
    }
  };
  // half-stage hx (0, 1) of the next sketch stage; the pointers advance a
  // stage after the second half
  auto issue_x = [&](int hx) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      __builtin_amdgcn_global_load_lds(xs[i] + hx * 64, Xh[hx] + (wave * 4 + i) * BLK, 16, 0, 0);
    if (hx == 1) {
#pragma unroll
      for (int i = 0; i < 4; ++i) xs[i] += KS;
    }
  };
  // the two 32-deep steps of half-stage hx
  auto compute = [&](int b, int hx) __attribute__((always_inline)) {
    const uint32_t abase = lds_off(As[b]) + (uint32_t)(grp * 3 * 4096);
    const uint32_t xbase = lds_off(Xh[hx]) + (uint32_t)(half * NTH * 2048);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      u32x4v ao[3], xo[8];
      lds_read_3_8h(abase + off[2 * hx + h], xbase + xoff[h], ao, xo);
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const bf16x8 f = __builtin_bit_cast(bf16x8, ao[t]);
#pragma unroll
        for (int j = 0; j < NTH; ++j)
          acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              f, __builtin_bit_cast(bf16x8, xo[j]), acc[t][j], 0, 0, 0);
      }
#pragma unroll
      for (int j = NTH; j < 8; ++j) asm volatile("" ::"v"(xo[j]));
    }
  };
  // issue order per wave: ... [X(s) half 1, A(s+1)] [X(s+1) half 0]
  // [X(s+1) half 1, A(s+2)] ...; loads complete in order, so at the top of
  // stage s (A(s) and X(s) half 0 needed) X(s) half 1 and A(s + 1) may be
  // outstanding, and before its second half only A(s + 1)
  if (nst > 0) {
    issue_a(0);
    issue_x(0);
    issue_x(1);
  }
  if (nst > 1) issue_a(1);
  for (int s = 0; s < nst; ++s) {
    if (s + 1 < nst) __builtin_amdgcn_s_waitcnt(0x0F7A);   // vmcnt(10)
    else __builtin_amdgcn_s_waitcnt(0x0F74);               // vmcnt(4)
    __builtin_amdgcn_s_barrier();
    compute(s & 1, 0);
    if (s + 1 < nst) __builtin_amdgcn_s_waitcnt(0x0F76);   // vmcnt(6)
    else __builtin_amdgcn_s_waitcnt(0x0F70);               // vmcnt(0)
    __builtin_amdgcn_s_barrier();
    if (s + 1 < nst) issue_x(0);
    compute(s & 1, 1);
    __builtin_amdgcn_s_barrier();
    if (s + 1 < nst) issue_x(1);
    if (s + 2 < nst) issue_a(s & 1);
  }

  // acc[t][j][e] is out[p][c], p = p0 + 48 grp + 16 t + 4 g4 + e,
  // c = c0 + 16 (NTH half + j) + r
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t p = p0 + grp * 48 + t * 16 + g4 * 4 + e;
      if (p >= P) continue;
#pragma unroll
      for (int j = 0; j < NTH; ++j) {
        const int64_t c = c0 + (half * NTH + j) * 16 + r;
        if (half * NTH + j >= NT || c >= C) continue;
        if (EPI == EPI_PART)
          out[(int64_t)split * part_stride + p * ldo + c] = acc[t][j][e];
        else
          out[p * ldo + c] = acc[t][j][e];
      }
    }
}

// Scale bytes: 3 of A at sa + 128 t, 7 of the sketch at sx + 128 j.
__device__ __forceinline__ void lds_scales_3_7(uint32_t sa, uint32_t sx, uint32_t (&ao)[3],
                                               uint32_t (&xo)[7]) {
  asm volatile(
      "ds_read_u8 %0, %10\n\t"
      "ds_read_u8 %1, %10 offset:128\n\t"
      "ds_read_u8 %2, %10 offset:256\n\t"
      "ds_read_u8 %3, %11\n\t"
      "ds_read_u8 %4, %11 offset:128\n\t"
      "ds_read_u8 %5, %11 offset:256\n\t"
      "ds_read_u8 %6, %11 offset:384\n\t"
      "ds_read_u8 %7, %11 offset:512\n\t"
      "ds_read_u8 %8, %11 offset:640\n\t"
      "ds_read_u8 %9, %11 offset:768\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(ao[0]), "=&v"(ao[1]), "=&v"(ao[2]), "=&v"(xo[0]), "=&v"(xo[1]), "=&v"(xo[2]),
        "=&v"(xo[3]), "=&v"(xo[4]), "=&v"(xo[5]), "=&v"(xo[6])
      : "v"(sa), "v"(sx)
      : "memory");
}

template <int NT, int EPI>
__global__ __launch_bounds__(512, 1) void k_pass_fp8_wide(const uint8_t* __restrict__ M,
                                                          const uint8_t* __restrict__ Ms,
                                                          int64_t ldm,
                                                          const uint8_t* __restrict__ Xt,
                                                          const uint8_t* __restrict__ Xsc,
                                                          int64_t ldx, float* out, int64_t ldo,
                                                          int64_t part_stride, int64_t P,
                                                          int64_t K, int64_t C, int64_t ksplit,
                                                          int nsplit) {
  static_assert(NT > 8 && NT <= 14, "9 to 14 column tiles");
  constexpr int KS = 256, ROWS = 192, NTH = (NT + 1) / 2;
  __shared__ __attribute__((aligned(16))) uint8_t As[2][ROWS * 256];
  __shared__ __attribute__((aligned(16))) uint8_t Ass[2][ROWS * 8];
  __shared__ __attribute__((aligned(16))) uint8_t Xs[14 * 4096];
  __shared__ __attribute__((aligned(16))) uint8_t Xss[14 * 16 * 8];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, r = lane & 15, g4 = lane >> 4;
  const int nwg = gridDim.x;
  const int xcd = blockIdx.x & 7, idx = blockIdx.x >> 3;
  const int per = nwg >> 3, rem = nwg & 7;
  const int lid = (xcd < rem) ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
  const int npb = nwg / nsplit;
  const int split = lid / npb;
  const int64_t p0 = (int64_t)(lid % npb) * ROWS;
  const int64_t c0 = (int64_t)blockIdx.y * (NT * 16);
  const int64_t kb = (int64_t)split * ksplit;
  const int64_t ke = (kb + ksplit < K) ? kb + ksplit : K;
  const int nst = kb < ke ? (int)((ke - kb) / KS) : 0;
  const int64_t lds_ = ldm / 32, ldxs = ldx / 32;

  const uint8_t* aa[6];
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    const int row = wave * 24 + 4 * t + g4;
    const int rho = row & 15;
    const int64_t ra = p0 + row;
    aa[t] = M + (ra < P ? ra : P - 1) * ldm + kb + ((r ^ rho) * 16);
  }
  const uint8_t* as_;
  {
    const int64_t ra = p0 + (wave < 6 ? wave : 0) * 32 + (lane >> 1);
    as_ = Ms + (ra < P ? ra : P - 1) * lds_ + kb / 32 + (lane & 1) * 4;
  }
  // sketch: block q = 8 w + i (q < 4 NT), columns 4 q + l / 16; blocks i
  // and i + 4 differ by 16 columns, same chunk order
  const uint8_t* xs[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int rho = 4 * i + g4;
    xs[i] = Xt + (c0 + 4 * (wave * 8 + i) + g4) * ldx + kb + ((r ^ rho) * 16);
  }
  const int64_t x16 = 16 * ldx;
  // sketch scales: waves 0..6 move 32 columns each (16 NT columns in all;
  // those past it read column 0 again, into slots never used)
  const uint8_t* xss;
  {
    const int col = (wave < 7 ? wave : 0) * 32 + (lane >> 1);
    xss = Xsc + (c0 + (col < 16 * NT ? col : 0)) * ldxs + kb / 32 + (lane & 1) * 4;
  }

  const int grp = wave >> 1, half = wave & 1;
  uint32_t off1[2], off2[2], soff[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    off1[u] = (uint32_t)(r * 256 + (((8 * u + g4) ^ r) * 16));
    off2[u] = (uint32_t)(r * 256 + (((8 * u + 4 + g4) ^ r) * 16));
    soff[u] = (uint32_t)(r * 8 + 4 * u + g4);
  }

  f32x4 acc[3][NTH];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int j = 0; j < NTH; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  auto issue_a = [&](int b) __attribute__((always_inline)) {
    uint8_t* ad = As[b] + wave * 6 * 1024;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      __builtin_amdgcn_global_load_lds(aa[t], ad + t * 1024, 16, 0, 2);
      aa[t] += KS;
    }
  };
  auto issue_x = [&](int b_scales) __attribute__((always_inline)) {
    if (wave < 6) __builtin_amdgcn_global_load_lds(as_, Ass[b_scales] + wave * 256, 4, 0, 0);
    as_ += KS / 32;
    if (wave < 7) __builtin_amdgcn_global_load_lds(xss, Xss + wave * 256, 4, 0, 0);
    xss += KS / 32;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (wave * 8 + i < 4 * NT)
        __builtin_amdgcn_global_load_lds(xs[i & 3] + (i >= 4 ? x16 : 0),
                                         Xs + (wave * 8 + i) * 1024, 16, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) xs[i] += KS;
  };
  auto compute = [&](int b) __attribute__((always_inline)) {
    const uint32_t abase = lds_off(As[b]) + (uint32_t)(grp * 3 * 4096);
    const uint32_t xbase = lds_off(Xs) + (uint32_t)(half * NTH * 4096);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      uint32_t sa[3], sx[7];
      lds_scales_3_7(lds_off(Ass[b]) + (uint32_t)(grp * 48 * 8) + soff[u],
                     lds_off(Xss) + (uint32_t)(half * NTH * 128) + soff[u], sa, sx);
      u32x4v ao[6];
      lds_read2x3(abase + off1[u], abase + off2[u], ao);
      i32x8 fa[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) fa[t] = cat8(ao[2 * t], ao[2 * t + 1]);
      // the sketch's 7 tiles in two phases (4, then 3)
      // (for odd NT the second half's last tile is past the sketch: LDS
      // inside the buffer, multiplied but never stored)
      auto mma = [&](int j, const u32x4v& lo, const u32x4v& hi) __attribute__((always_inline)) {
        const i32x8 fb = cat8(lo, hi);
        if (j < NTH) {
#pragma unroll
          for (int t = 0; t < 3; ++t)
            acc[t][j < NTH ? j : 0] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                fa[t], fb, acc[t][j < NTH ? j : 0], 0, 0, 0, (int)sa[t], 0, (int)sx[j]);
        } else {
          asm volatile("" ::"v"(fb), "v"(sx[j]));
        }
      };
      {
        u32x4v x4[8];
        lds_read2x4(xbase + off1[u], xbase + off2[u], x4);
#pragma unroll
        for (int j = 0; j < 4; ++j) mma(j, x4[2 * j], x4[2 * j + 1]);
      }
      {
        u32x4v x3[6];
        lds_read2x3(xbase + 16384 + off1[u], xbase + 16384 + off2[u], x3);
#pragma unroll
        for (int j = 4; j < 7; ++j) mma(j, x3[2 * (j - 4)], x3[2 * (j - 4) + 1]);
      }
      // the first step's MFMAs stay ahead of the second step's reads; those
      // of the second may move past the stage's barrier and overlap the
      // next loads (all of them there would keep both steps' operands live)
      if (u == 0) {
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
          for (int j = 0; j < NTH; ++j) asm volatile("" : "+v"(acc[t][j]));
      }
    }
  };
  if (nst > 0) {
    issue_x(0);
    issue_a(0);
  }
  if (nst > 1) issue_a(1);
  for (int s = 0; s < nst; ++s) {
    if (s + 1 < nst) __builtin_amdgcn_s_waitcnt(0x0F76);   // vmcnt(6)
    else __builtin_amdgcn_s_waitcnt(0x0F70);               // vmcnt(0)
    __builtin_amdgcn_s_barrier();
    compute(s & 1);
    __builtin_amdgcn_s_barrier();
    if (s + 1 < nst) issue_x((s + 1) & 1);
    if (s + 2 < nst) issue_a(s & 1);
  }

#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t p = p0 + grp * 48 + t * 16 + g4 * 4 + e;
      if (p >= P) continue;
#pragma unroll
      for (int j = 0; j < NTH; ++j) {
        const int64_t c = c0 + (half * NTH + j) * 16 + r;
        if (half * NTH + j >= NT || c >= C) continue;
        if (EPI == EPI_PART)
          out[(int64_t)split * part_stride + p * ldo + c] = acc[t][j][e];
        else
          out[p * ldo + c] = acc[t][j][e];
      }
    }
}

template <int EPI>
hipError_t launch_fp8_nt(int nt, dim3 grid, const uint8_t* M, const uint8_t* Ms, int64_t ldm,
                         const uint8_t* Xt, const uint8_t* Xsc, int64_t ldx, float* out,
                         int64_t ldo, int64_t ps, int64_t P, int64_t K, int64_t C, int64_t ks,
                         int ns, hipStream_t s) {
  switch (nt) {
#define PLU_F8_CASE(N)                                                                     \
  case N:                                                                                  \
    hipLaunchKernelGGL((k_pass_fp8<N, EPI>), grid, dim3(512), 0, s, M, Ms, ldm, Xt, Xsc, \
                       ldx, out, ldo, ps, P, K, C, ks, ns);                                \
    break;
    PLU_F8_CASE(1) PLU_F8_CASE(2) PLU_F8_CASE(3) PLU_F8_CASE(4)
    PLU_F8_CASE(5) PLU_F8_CASE(6) PLU_F8_CASE(7) PLU_F8_CASE(8)
#undef PLU_F8_CASE
#define PLU_F8W_CASE(N)                                                                         \
  case N:                                                                                       \
    hipLaunchKernelGGL((k_pass_fp8_wide<N, EPI>), grid, dim3(512), 0, s, M, Ms, ldm, Xt, Xsc, \
                       ldx, out, ldo, ps, P, K, C, ks, ns);                                     \
    break;
    PLU_F8W_CASE(9) PLU_F8W_CASE(10) PLU_F8W_CASE(11) PLU_F8W_CASE(12) PLU_F8W_CASE(13)
    PLU_F8W_CASE(14)
#undef PLU_F8W_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int EPI>
hipError_t launch_bf16_nt(int nt, dim3 grid, const uint16_t* M, int64_t ldm,
                              const uint16_t* Xt, int64_t ldx, float* out, int64_t ldo, int64_t ps,
                              int64_t P, int64_t K, int64_t C, int64_t ks, int ns, hipStream_t s) {
  switch (nt) {
#define PLU_BF_CASE(N)                                                                       \
  case N:                                                                                     \
    hipLaunchKernelGGL((k_pass_bf16<N, EPI>), grid, dim3(512), 0, s, M, ldm, Xt, ldx, out, \
                       ldo, ps, P, K, C, ks, ns);                                             \
    break;
    PLU_BF_CASE(1) PLU_BF_CASE(2) PLU_BF_CASE(3) PLU_BF_CASE(4)
    PLU_BF_CASE(5) PLU_BF_CASE(6) PLU_BF_CASE(7) PLU_BF_CASE(8)
#undef PLU_BF_CASE
#define PLU_BFW_CASE(N)                                                                         \
  case N:                                                                                       \
    hipLaunchKernelGGL((k_pass_bf16_wide<N, EPI>), grid, dim3(512), 0, s, M, ldm, Xt, ldx, out, \
                       ldo, ps, P, K, C, ks, ns);                                               \
    break;
    PLU_BFW_CASE(9) PLU_BFW_CASE(10) PLU_BFW_CASE(11) PLU_BFW_CASE(12) PLU_BFW_CASE(13)
    PLU_BFW_CASE(14) PLU_BFW_CASE(15) PLU_BFW_CASE(16)
#undef PLU_BFW_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pass_bf16(int epi, const uint16_t* M, int64_t ldm, const uint16_t* Xt,
                                int64_t ldx, float* out, int64_t ldo, int64_t part_stride,
                                int64_t P, int64_t K, int64_t C, const GemmPlan& pl,
                                hipStream_t s) {
  // pl: nt <= 8 column tiles per column block with pblocks of 256 rows, or
  // 9..16 (one column block) with pblocks of 192 rows; rsplit and K
  // multiples of 128; the sketch must have gridDim.y * nt * 16 rows
  if (K % 128 != 0 || pl.rsplit % 128 != 0 || (ldm & 7) || (ldx & 7) || pl.nt > 16 || P <= 0 ||
      (reinterpret_cast<uintptr_t>(M) & 15u) || (reinterpret_cast<uintptr_t>(Xt) & 15u) ||
      (int64_t)pl.pblocks * (pl.nt > 8 ? 192 : 256) < P)
    return hipErrorInvalidValue;
  dim3 grid(pl.pblocks * pl.nsplit, pl.cblocks);
  if (epi == EPI_PART)
    return launch_bf16_nt<EPI_PART>(pl.nt, grid, M, ldm, Xt, ldx, out, ldo, part_stride, P,
                                        K, C, pl.rsplit, pl.nsplit, s);
  if (epi == EPI_STORE)
    return launch_bf16_nt<EPI_STORE>(pl.nt, grid, M, ldm, Xt, ldx, out, ldo, 0, P, K, C,
                                         pl.rsplit, pl.nsplit, s);
  return hipErrorInvalidValue;
}

hipError_t launch_cvt_bf16(const float* src, int64_t lds, int64_t R, int64_t C, uint16_t* rm,
                           int64_t ldr, uint16_t* tr, int64_t ldt, int64_t Ct, double* sumsq_part,
                           int64_t* nparts, hipStream_t s) {
  if ((rm && (ldr % 64 != 0 || ldr < C)) || (tr && (ldt % 64 != 0 || ldt < R || Ct < C)))
    return hipErrorInvalidValue;
  const int64_t rows = std::max<int64_t>(R, tr ? ldt : 0);
  const int64_t cols = std::max<int64_t>(rm ? ldr : 0, tr ? Ct : 0);
  const int64_t bands = (rows + 63) / 64, ctiles = (cols + 63) / 64;
  const int groups = (int)std::min<int64_t>(ctiles, 8);
  if (nparts) *nparts = bands * groups;
  hipLaunchKernelGGL(k_cvt_bf16, dim3((unsigned)groups, (unsigned)bands), dim3(256), 0, s, src,
                     lds, R, C, rm, ldr, tr, ldt, Ct, ctiles, sumsq_part);
  return hipGetLastError();
}

hipError_t launch_cvt_fp8(const float* src, int64_t lds, int64_t R, int64_t C, uint8_t* rm,
                          uint8_t* rsc, int64_t ldr, uint8_t* tr, uint8_t* tsc, int64_t ldt,
                          int64_t Ct, double* sumsq_part, int64_t* nparts, hipStream_t s) {
  if ((rm && (ldr % 128 != 0 || ldr < C || !rsc)) ||
      (tr && (ldt % 128 != 0 || ldt < R || Ct < C || !tsc)))
    return hipErrorInvalidValue;
  const int64_t rows = std::max<int64_t>(R, tr ? ldt : 0);
  const int64_t cols = std::max<int64_t>(rm ? ldr : 0, tr ? Ct : 0);
  const int64_t bands = (rows + 63) / 64, ctiles = (cols + 63) / 64;
  const int groups = (int)std::min<int64_t>(ctiles, 8);
  if (nparts) *nparts = bands * groups;
  hipLaunchKernelGGL(k_cvt_fp8, dim3((unsigned)groups, (unsigned)bands), dim3(256), 0, s, src,
                     lds, R, C, rm, rsc, ldr, tr, tsc, ldt, Ct, ctiles, sumsq_part);
  return hipGetLastError();
}

hipError_t launch_pass_fp8(int epi, const uint8_t* M, const uint8_t* Ms, int64_t ldm,
                           const uint8_t* Xt, const uint8_t* Xsc, int64_t ldx, float* out,
                           int64_t ldo, int64_t part_stride, int64_t P, int64_t K, int64_t C,
                           const GemmPlan& pl, hipStream_t s) {
  // pl: pblocks of 192 rows, nt <= 14 (above 8: the wide kernel, one column
  // block), rsplit and K multiples of 256, the leading dimensions multiples
  // of 256 (4-byte aligned scale rows)
  if (K % 256 != 0 || pl.rsplit % 256 != 0 || (ldm % 256) || (ldx % 256) || pl.nt > 14 ||
      P <= 0 || (int64_t)pl.pblocks * 192 < P || (reinterpret_cast<uintptr_t>(M) & 15u) ||
      (reinterpret_cast<uintptr_t>(Xt) & 15u) || (reinterpret_cast<uintptr_t>(Ms) & 3u) ||
      (reinterpret_cast<uintptr_t>(Xsc) & 3u))
    return hipErrorInvalidValue;
  dim3 grid(pl.pblocks * pl.nsplit, pl.cblocks);
  if (epi == EPI_PART)
    return launch_fp8_nt<EPI_PART>(pl.nt, grid, M, Ms, ldm, Xt, Xsc, ldx, out, ldo, part_stride,
                                   P, K, C, pl.rsplit, pl.nsplit, s);
  if (epi == EPI_STORE)
    return launch_fp8_nt<EPI_STORE>(pl.nt, grid, M, Ms, ldm, Xt, Xsc, ldx, out, ldo, 0, P, K, C,
                                    pl.rsplit, pl.nsplit, s);
  return hipErrorInvalidValue;
}

}  // namespace plu
