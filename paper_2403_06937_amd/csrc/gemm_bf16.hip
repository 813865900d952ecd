// Split-BF16 complex matrix products on gfx950 BF16 MFMA (v_mfma_f32_16x16x32_bf16).
//
// Operands are four bfloat16 planes (Re hi, Re lo, Im hi, Im lo), each stored
// with K contiguous: rows of A are its M rows, rows of B are its N columns.
// The planes are interleaved by 32-deep K slices (Planes4), so the K tile of
// one row is 256 contiguous bytes: a load covers whole cache lines.
// For one 16 x 16 output block and a 32-deep K slice the kernel issues
//   Re += Ar_h Br_h + Ar_h Br_l + Ar_l Br_h - Ai_h Bi_h - Ai_h Bi_l - Ai_l Bi_h
//   Im += Ar_h Bi_h + Ar_h Bi_l + Ar_l Bi_h + Ai_h Br_h + Ai_h Br_l + Ai_l Br_h
// (lo*lo dropped), twelve MFMAs, accumulating in FP32 from zero.  The minus
// sign is a sign-bit flip of the Ai fragments in registers.
//
// Lane layout of v_mfma_f32_16x16x32_bf16: lane l supplies A[l%16][8(l/16) .. +7]
// and B[8(l/16) .. +7][l%16] (eight consecutive K values, one 16-byte LDS
// read) and holds D[4(l/16)+r][l%16], r = 0..3.
//
// Tiling: 128 x 128 outputs per workgroup, K tile 32, all eight planes
// double-buffered in LDS (128 KB).  Default shape: 512 threads = 2 x 4 waves
// of 64 x 32 outputs (4 x 2 blocks), two waves per SIMD, run as two ping-pong
// groups: while one wave of a SIMD issues the products of a K tile from
// fragments it already holds, the other reads its fragments, stores its share
// of the next tile (staged in registers) and loads the one after, with two
// workgroup barriers per K tile.  Measured at N = 12288 (mean of a full and a
// triangle launch, one box): 18.6 ms, against 20.4 ms with both waves of a
// SIMD in lockstep (reads, then products, one barrier per K tile).  Earlier
// lockstep measurements: the planes stored one after another instead of
// interleaved 24.8 ms against 21.2 ms, the store at the end of the loading
// iteration 25.2 ms; 4 waves of 64 x 64: 29.5 ms.
// A variant with one wave per SIMD (128 x 32 outputs each, accumulators in
// AGPRs) that reads its B fragments straight from global memory ran at 31 ms.
// 16-byte chunks are XOR-swizzled by row and the planes padded so that
// neither the fragment reads nor the staged stores conflict on LDS banks
// (SQ_LDS_BANK_CONFLICT: 0; with unpadded planes the stores conflicted, 29 %
// of the LDS cycles).  Tile order: a full product on a tile grid that is a
// multiple of 16 x 16 walks 16-row bands shared by all XCDs (band_coords);
// otherwise, as in the FP64 kernel, XCD-contiguous ranges walked in groups of
// 8 tile rows; a Hermitian result walks the upper tile triangle only.
//
// The epilogue forms alpha * acc + beta * Cin in FP32 and writes any of: the
// FP32 result, and the hi/lo planes of the result (row-major or transposed)
// for the next product.
#include "gemm_bf16.h"
#include "profile.h"

#include <atomic>
#include <cstdlib>

namespace tcm {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef uint32_t u2 __attribute__((ext_vector_type(2)));

// Global-memory accesses through address-space-1 pointers of scalar or vector
// type: the grouped kernel reads its operand pointers from a descriptor array,
// where the compiler could not otherwise tell them from LDS and would issue
// flat accesses (which the LDS barrier's lgkmcnt wait would also wait for).
typedef float f2v __attribute__((ext_vector_type(2), aligned(4)));
__device__ __forceinline__ u4 gld_u4(const void* p) {
  typedef __attribute__((address_space(1))) const u4 G;
  return *(G*)p;
}
__device__ __forceinline__ c64 gld_c64(const c64* p) {
  typedef __attribute__((address_space(1))) const f2v G;
  const f2v v = *(G*)p;
  return c64{v.x, v.y};
}
__device__ __forceinline__ void gst_c64(c64* p, float re, float im) {
  typedef __attribute__((address_space(1))) f2v G;
  *(G*)p = f2v{re, im};
}
__device__ __forceinline__ void gst_u2(uint16_t* p, u2 v) {
  typedef u2 u2a __attribute__((aligned(4)));
  typedef __attribute__((address_space(1))) u2a G;
  *(G*)p = v;
}
__device__ __forceinline__ void gst_u16(uint16_t* p, uint16_t v) {
  typedef __attribute__((address_space(1))) uint16_t G;
  *(G*)p = v;
}
__device__ __forceinline__ void gst_u4(void* p, u4 v) {
  typedef __attribute__((address_space(1))) u4 G;
  *(G*)p = v;
}

__device__ __forceinline__ uint16_t rne_bf16(float x) {
  const uint32_t b = __float_as_uint(x);
  if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu) != 0)
    return uint16_t((b >> 16) | 0x40u);
  const uint32_t upper = b >> 16, rem = b & 0xFFFFu;
  const uint32_t up = (rem > 0x8000u) || (rem == 0x8000u && (upper & 1u));
  return uint16_t(upper + up);
}
// hi = RNE_bf16(x), lo = RNE_bf16(x - hi) by the hardware conversion
// (v_cvt_pk_bf16_f32, round to nearest even), which gives rne_bf16's bits for
// every non-NaN binary32 input (checked exhaustively on gfx950 over all 2^32
// patterns; a NaN stays a NaN); x - hi is exact in binary32.  One instruction
// per conversion instead of rne_bf16's integer sequence, which made the split
// of the result a fifth of the epilogue's instructions.
__device__ __forceinline__ uint16_t cvt_bf16(float x) {
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(x));
}
__device__ __forceinline__ void split2(float x, uint16_t& h, uint16_t& l) {
  h = cvt_bf16(x);
  l = cvt_bf16(x - __uint_as_float(uint32_t(h) << 16));
}

__device__ __forceinline__ f4 mma(const u4& a, const u4& b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a),
                                                 __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

// LDS bank conflicts of 16-byte accesses (measured with SQ_LDS_BANK_CONFLICT
// on gfx950): lanes are served 8 at a time over 32 banks of 4 bytes, so 8
// lanes are conflict-free when their 16-byte addresses are distinct modulo 8.
// A plane holds 128 rows of four 16-byte chunks; the chunk of row r is XORed
// with (r >> 1) & 3, which spreads the 8 consecutive rows of a fragment read
// over the 8 positions, and each plane is padded by four chunks, so that a
// store's 8 lanes (two planes of one row) land on distinct positions too.
__device__ __forceinline__ int swz(int r) { return (r >> 1) & 3; }
constexpr int LDS_PLANE = SPLIT_BM * 4 + 4;     // 16-byte chunks per padded plane

// Plane operands are in the interleaved layout of Planes4; lda, ldb and ldp
// are their padded K extents (the row stride is four times that).
struct SplitParams {
  const uint16_t* A; int64_t lda;
  const uint16_t* B; int64_t ldb;
  int64_t M, N, Kp;
  float ar, ai, br, bi;
  const c64* Cin; int64_t ldcin; int cin_trans;
  c64* Cf; int64_t ldcf;
  uint16_t* P; int64_t ldp; int p_trans;
  int herm;   // Hermitian result (M == N): upper tile triangle, mirrored stores
  int tiles_m, tiles_n;
};

constexpr int GROUP_M = 8;

// Consecutive workgroup ids go round the 8 XCDs; give each XCD a contiguous
// run of the tile order so that its tiles share operand rows in its L2.
__device__ __forceinline__ int xcd_linear(int pid, int total) {
  const int q = total / 8, r = total % 8;
  const int xcd = pid % 8, local = pid / 8;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + local;
}

// Tile lists of grouped launches are sorted by decreasing K, so consecutive
// ids have similar work.  Within each run of 256 ids (one tile per CU), XCD x
// (id mod 8) takes the 32 consecutive list entries 32 x .. 32 x + 31, so that
// its concurrent tiles are neighbours of one product that share operand
// panels in its L2, while every XCD still gets an equal share of each run.
// Ids past the last whole run keep their place.
__device__ __forceinline__ int round_xcd(int pid, int total) {
  const int whole = total - total % 256;
  if (pid >= whole) return pid;
  return (pid / 256) * 256 + (pid % 8) * 32 + (pid % 256) / 8;
}

// Tile lin of the upper block triangle (tm <= tn) of a T x T tile grid:
// GROUP_M tile rows at a time, column by column within a group.
__device__ __forceinline__ void tri_coords(int lin, int T, int& tm, int& tn) {
  int first = 0;
  for (;;) {
    const int gs = min(T - first, GROUP_M);
    const int tri = gs * (gs - 1) / 2;              // the group's leading triangle
    const int cnt = gs * (T - first) - tri;
    if (lin < cnt) {
      if (lin < tri) {
        int c = 0;
        while ((c + 1) * (c + 2) / 2 <= lin) ++c;
        tn = first + c;
        tm = first + lin - c * (c + 1) / 2;
      } else {
        const int q = lin - tri;
        tn = first + gs - 1 + q / gs;
        tm = first + q % gs;
      }
      return;
    }
    lin -= cnt;
    first += gs;
  }
}

// Tile order of a full product whose tile grid is a multiple of 16 x 16:
// all 8 XCDs (workgroup id mod 8) work in the same 16-row band at a time, so
// its A panels are fetched once into the memory-side cache for all of them.
// XCD x takes rows 8 (x / 4) .. + 7 of the band and its own quarter of the
// columns, walked 4 columns at a time, so that its 32 concurrent tiles are
// 8 x 4 neighbours sliding along the band (the same L2 reuse as the
// contiguous ranges below).  Measured at N = 12288: full product 23.27 ms
// against 23.62 ms for the contiguous per-XCD ranges.
__device__ __forceinline__ bool band_coords(int pid, int tiles_m, int tiles_n, int& tm, int& tn) {
  if (tiles_m % 16 != 0 || tiles_n % 16 != 0) return false;
  const int x = pid % 8, local = pid / 8;
  const int strip = tiles_n / 4;                       // columns per XCD and band
  const int band = local / (2 * tiles_n), w = local % (2 * tiles_n);
  const int step = w / 32, t = w % 32;
  tm = 16 * band + 8 * (x / 4) + t % 8;
  tn = strip * (x % 4) + 4 * step + t / 8;
  return true;
}

__device__ __forceinline__ void tile_coords(int pid, int tiles_m, int tiles_n, int& tm, int& tn) {
  if (band_coords(pid, tiles_m, tiles_n, tm, tn)) return;
  const int lin = xcd_linear(pid, tiles_m * tiles_n);
  const int per_group = GROUP_M * tiles_n;
  const int group = lin / per_group;
  const int first_m = group * GROUP_M;
  const int gsize = min(tiles_m - first_m, GROUP_M);
  const int in_group = lin % per_group;
  tm = first_m + in_group % gsize;
  tn = in_group / gsize;
}

// beta's operand for one wave's WM x WN blocks of 16 x 16 outputs, loaded all
// at once before any of it is used: every lane loads from an address clamped
// into the matrix (the value is discarded outside it), so the loads need no
// branch and the wave waits for them once instead of once per element.
template <int WM, int WN>
__device__ __forceinline__ void load_cin(const SplitParams& p, int64_t r0, int64_t c0,
                                         c64 (&cin)[WM][WN][4]) {
  const int lr = threadIdx.x & 15, lc = (threadIdx.x >> 4) & 3;
  const int64_t sr = p.cin_trans ? 1 : p.ldcin, sc = p.cin_trans ? p.ldcin : 1;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = min(r0 + i * 16 + 4 * lc + r, p.M - 1);
        const int64_t col = min(c0 + j * 16 + lr, p.N - 1);
        cin[i][j][r] = gld_c64(p.Cin + row * sr + col * sc);
      }
}

// Epilogue of one wave's WM x WN blocks of 16 x 16 outputs whose first output
// is (r0, c0): alpha * acc + beta * Cin in FP32, then any of the FP32 result
// and its hi/lo planes (row-major or transposed).  mirror: the tile lies above
// the diagonal of a Hermitian result, so element (col, row) = conj(row, col)
// is stored as well.
template <int WM, int WN>
__device__ __forceinline__ void split_epilogue(const SplitParams& p, const f4 (&acc_re)[WM][WN],
                                               const f4 (&acc_im)[WM][WN], int64_t r0,
                                               int64_t c0, bool mirror) {
  const bool use_beta = p.Cin != nullptr && (p.br != 0.f || p.bi != 0.f);
  const int lr = threadIdx.x & 15, lc = (threadIdx.x >> 4) & 3;
  c64 cin[WM][WN][4];
  if (use_beta) load_cin<WM, WN>(p, r0, c0, cin);
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const int64_t row0 = r0 + i * 16 + 4 * lc;
      const int64_t col = c0 + j * 16 + lr;
      float vr[4], vi[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + r;
        const float xr = acc_re[i][j][r], xi = acc_im[i][j][r];
        float yr = p.ar * xr - p.ai * xi;
        float yi = p.ar * xi + p.ai * xr;
        const bool inb = row < p.M && col < p.N;
        if (use_beta) {
          const c64 c = cin[i][j][r];
          yr += p.br * c.re - p.bi * c.im;
          yi += p.br * c.im + p.bi * c.re;
        }
        if (!inb) { yr = 0.f; yi = 0.f; }
        vr[r] = yr;
        vi[r] = yi;
        if (p.Cf && inb) {
          gst_c64(p.Cf + row * p.ldcf + col, yr, yi);
          if (mirror) gst_c64(p.Cf + col * p.ldcf + row, yr, -yi);
        }
      }
      if (p.P) {
        uint16_t h[4][4];   // [plane][r]
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          split2(vr[r], h[PL_RH][r], h[PL_RL][r]);
          split2(vi[r], h[PL_IH][r], h[PL_IL][r]);
        }
        // the split of -x is the negated split of x (RNE is symmetric), so the
        // mirrored element's imaginary planes are the sign-flipped h[PL_I*]
        const uint16_t neg[4] = {0, 0, 0x8000u, 0x8000u};
        if (p.p_trans || mirror) {
          const uint16_t f = p.p_trans ? 0 : 0x8000u;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const uint32_t m = (PL_IH == q || PL_IL == q) ? f : 0;
            const u2 v = u2{(uint32_t(h[q][0]) | (uint32_t(h[q][1]) << 16)) ^ (m | (m << 16)),
                            (uint32_t(h[q][2]) | (uint32_t(h[q][3]) << 16)) ^ (m | (m << 16))};
            gst_u2(p.P + plane_offset(p.ldp, col, row0, q), v);
          }
        }
        if (!p.p_trans || mirror) {
          const bool flip = p.p_trans;   // here this is the mirrored element
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              gst_u16(p.P + plane_offset(p.ldp, row0 + r, col, q),
                      uint16_t(h[q][r] ^ (flip ? neg[q] : 0)));
        }
      }
    }
}

// Epilogue of the default shape (a wave owns 64 x 32 outputs, 4 x 2 blocks):
// the same results as split_epilogue, with the bf16 planes and the mirrored
// FP32 result staged through this wave's 16 KB of LDS, so that each of those
// global stores is 16 bytes of a contiguous run (a plane row's 256 or 512
// bytes, a mirrored row's 512 bytes) instead of scattered two- and eight-byte
// stores, which took a fifth of the product's time.  The caller guarantees
// that no wave of the workgroup still reads the K loop's LDS buffers.
// Staging layouts (16-byte chunks XOR-swizzled so that the 8 lanes served
// together hit distinct banks on the reads):
//   row-major planes: 64 rows x 16 chunks (4 planes x 32 K values),
//                     chunk ^ 2 ((row >> 2) & 3)
//   transposed planes: 32 plane rows x 32 chunks (2 K slices x 4 planes x 32),
//                     chunk ^ (row & 7)
//   mirrored FP32:    32 rows x 32 chunks (64 complex values), chunk ^ (row & 7)
static_assert(PL_IH == 2 && PL_IL == 3, "imaginary planes are the upper two of each K slice");
static_assert(2 * 4 * LDS_PLANE >= 4 * 1024, "each of the 8 waves stages through 16 KB of sA or sB");
__device__ __forceinline__ void split_epilogue_staged(const SplitParams& p, f4 (&acc_re)[4][2],
                                                      f4 (&acc_im)[4][2], int64_t r0, int64_t c0,
                                                      bool mirror, u4* __restrict__ stage) {
  constexpr int WM = 4, WN = 2;
  const bool use_beta = p.Cin != nullptr && (p.br != 0.f || p.bi != 0.f);
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lc = lane >> 4;
  const u4 sgn4 = u4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};

  // alpha acc + beta Cin, kept in acc; the FP32 result row-major from registers
  c64 cin[WM][WN][4];
  if (use_beta) load_cin<WM, WN>(p, r0, c0, cin);
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const int64_t row0 = r0 + i * 16 + 4 * lc;
      const int64_t col = c0 + j * 16 + lr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + r;
        const float xr = acc_re[i][j][r], xi = acc_im[i][j][r];
        float yr = p.ar * xr - p.ai * xi;
        float yi = p.ar * xi + p.ai * xr;
        const bool inb = row < p.M && col < p.N;
        if (use_beta) {
          const c64 c = cin[i][j][r];
          yr += p.br * c.re - p.bi * c.im;
          yi += p.br * c.im + p.bi * c.re;
        }
        if (!inb) { yr = 0.f; yi = 0.f; }
        acc_re[i][j][r] = yr;
        acc_im[i][j][r] = yi;
        if (p.Cf && inb) gst_c64(p.Cf + row * p.ldcf + col, yr, yi);
      }
    }

  // mirrored FP32 result: Cf[col][row] = conj(y) for every element in bounds
  if (mirror && p.Cf) {
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int mrow = 16 * j + lr;          // local mirrored row = local column
        const int ch = 8 * i + 2 * lc;         // chunk of the 4 values of rows 4 lc .. + 3
        const int sw = mrow & 7;
        const f4& yr = acc_re[i][j];
        const f4& yi = acc_im[i][j];
        stage[mrow * 32 + (ch ^ sw)] =
            u4{__float_as_uint(yr[0]), __float_as_uint(-yi[0]), __float_as_uint(yr[1]),
               __float_as_uint(-yi[1])};
        stage[mrow * 32 + ((ch + 1) ^ sw)] =
            u4{__float_as_uint(yr[2]), __float_as_uint(-yi[2]), __float_as_uint(yr[3]),
               __float_as_uint(-yi[3])};
      }
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int t = lane + 64 * s;
      const int mrow = t >> 5, ch = t & 31;
      const u4 v = stage[mrow * 32 + (ch ^ (mrow & 7))];
      const int64_t grow = c0 + mrow, gcol = r0 + 2 * ch;
      if (grow < p.N && gcol < p.M) {
        c64* dst = p.Cf + grow * p.ldcf + gcol;
        if (gcol + 1 < p.M && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
          gst_u4(dst, v);
        } else {
          gst_c64(dst, __uint_as_float(v.x), __uint_as_float(v.y));
          if (gcol + 1 < p.M) gst_c64(dst + 1, __uint_as_float(v.z), __uint_as_float(v.w));
        }
      }
    }
  }

  if (!p.P) return;
  // hi/lo planes of every value, four consecutive rows packed per plane
  u2 hb[WM][WN][4];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      uint16_t h[4][4];   // [plane][r]
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        split2(acc_re[i][j][r], h[PL_RH][r], h[PL_RL][r]);
        split2(acc_im[i][j][r], h[PL_IH][r], h[PL_IL][r]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        hb[i][j][q] = u2{uint32_t(h[q][0]) | (uint32_t(h[q][1]) << 16),
                         uint32_t(h[q][2]) | (uint32_t(h[q][3]) << 16)};
    }

  // row-major planes (plane row = result row, K = result column): the result
  // itself, or with p_trans the mirrored element (imaginary planes negated)
  if (!p.p_trans || mirror) {
    uint16_t* st16 = reinterpret_cast<uint16_t*>(stage);
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * i + 4 * lc + r, col = 16 * j + lr;
            const int ch = (q * 4 + (col >> 3)) ^ (2 * ((row >> 2) & 3));
            const uint32_t w = r < 2 ? hb[i][j][q].x : hb[i][j][q].y;
            st16[row * 128 + ch * 8 + (col & 7)] = uint16_t(r & 1 ? w >> 16 : w);
          }
    const bool flip = p.p_trans;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int t = lane + 64 * s;
      const int row = t >> 4, ch = t & 15;
      u4 v = stage[row * 16 + (ch ^ (2 * ((row >> 2) & 3)))];
      if (flip && (ch >> 2) >= PL_IH) v ^= sgn4;
      gst_u4(p.P + plane_offset(p.ldp, r0 + row, c0, 0) + ch * 8, v);
    }
  }
  // transposed planes (plane row = result column, K = result row): the
  // result with p_trans, or else the mirrored element (imaginary negated)
  if (p.p_trans || mirror) {
    u2* st2 = reinterpret_cast<u2*>(stage);
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int prow = 16 * j + lr;
          const int k = 16 * i + 4 * lc;
          const int byte = (k >> 5) * 256 + q * 64 + (k & 31) * 2;
          const int ch = (byte >> 4) ^ (prow & 7);
          st2[prow * 64 + ch * 2 + ((byte >> 3) & 1)] = hb[i][j][q];
        }
    const bool flip = !p.p_trans;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int t = lane + 64 * s;
      const int prow = t >> 5, ch = t & 31;
      u4 v = stage[prow * 32 + (ch ^ (prow & 7))];
      if (flip && ((ch & 15) >> 2) >= PL_IH) v ^= sgn4;
      gst_u4(p.P + plane_offset(p.ldp, c0 + prow, r0, 0) + ch * 8, v);
    }
  }
}

// Publishes this wave's LDS writes to the workgroup: waits for them, then a
// barrier.  Outstanding global loads are not waited for (__syncthreads would
// wait for those too).  The wait and the barrier are builtins, not inline
// asm, so that the compiler's wait-count tracking sees the LDS counter
// drained here and later waits can be partial; the empty asm statements with
// a memory clobber keep LDS accesses from moving across, and the scheduling
// fences keep the machine scheduler from doing so.
constexpr unsigned WAIT_LGKM0 = 0xC07F;   // s_waitcnt vmcnt(63) expcnt(7) lgkmcnt(0)
__device__ __forceinline__ void sync_lds() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_waitcnt(WAIT_LGKM0);
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("" ::: "memory");
}

// WGM x WGN waves, each owning WM x WN blocks of 16 x 16 outputs of a
// 128 x 128 tile.  Both operands pass through LDS, [buf][plane][row][chunk]
// with 16-byte chunks (4 per 32-deep row), double-buffered (128 KB).  The next
// K tile is staged in registers: at the start of iteration t, tile t + 1 goes
// from the registers into the LDS buffer freed by the last barrier and the
// registers are refilled with tile t + 2 before the products, so a load has a
// whole iteration to arrive and the barrier waits for no global load.
typedef u4 SplitLds[2][4][LDS_PLANE];
#define LDS_AT(buf, q, row, chunk) [buf][q][(row) * 4 + (chunk)]

// PARTIAL: no epilogue; the raw FP32 accumulators go to partial
// (float4 k of thread t at element 4 (k NT + t), k over the wave's blocks,
// real then imaginary) and the epilogue is left to a later kernel that adds
// the partial sums of the K ranges.
template <int WGM, int WGN, int WM, int WN, bool PP, bool PARTIAL = false>
__device__ __forceinline__ void split_tile(const SplitParams& p, int tm, int tn, SplitLds& sA,
                                           SplitLds& sB, float* __restrict__ partial = nullptr) {
  constexpr int NT = 64 * WGM * WGN;
  static_assert(16 * WM * WGM == SPLIT_BM && 16 * WN * WGN == SPLIT_BN, "128 x 128 tile");
  static_assert(SPLIT_BM == SPLIT_BN, "square tile");
  static_assert(NT == 256 || NT == 512, "staging pattern");
  // a tile of one operand is 128 rows x 256 bytes (four planes of 32 bf16):
  // 2048 chunks; thread t moves chunk t % 16 of rows t / 16 + h NT / 16
  constexpr int RPT = 2048 / NT;        // chunks per thread and operand

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int64_t m0 = int64_t(tm) * SPLIT_BM, n0 = int64_t(tn) * SPLIT_BN;

  // Each K tile of a row is 256 contiguous bytes, so a wave's load covers
  // whole 128-byte lines.  Chunk c of a row slice holds plane c / 4, K chunk
  // c % 4; it lands in LDS at [plane][row][(c % 4) ^ swz(row)].
  const int64_t rsa = 4 * p.lda, rsb = 4 * p.ldb;     // row strides
  const int srow = tid >> 4, sc = tid & 15;
  const int sq = sc >> 2, sw = (sc & 3) ^ swz(srow);  // swz(srow + 16 h) == swz(srow)
  static_assert(NT / 16 % 4 == 0, "the staged rows of one thread share their swizzle");
  // workgroup-uniform bases and one 32-bit per-lane byte offset per operand
  // (rows below 128 of at most 2^23 bf16), so each load is a uniform base plus
  // a lane offset
  const uint16_t* __restrict__ baseA = p.A + m0 * rsa;
  const uint16_t* __restrict__ baseB = p.B + n0 * rsb;
  const uint32_t offA = uint32_t((srow * rsa + sc * 8) * 2);
  const uint32_t offB = uint32_t((srow * rsb + sc * 8) * 2);
  auto load = [&](u4 (&st)[2 * RPT], int64_t kt) {
    const int64_t k0 = kt * 4 * SPLIT_BK;
#pragma unroll
    for (int h = 0; h < RPT; ++h) {
      const char* ga = reinterpret_cast<const char*>(baseA + h * (NT / 16) * rsa + k0);
      const char* gb = reinterpret_cast<const char*>(baseB + h * (NT / 16) * rsb + k0);
      st[h] = gld_u4(ga + offA);
      st[RPT + h] = gld_u4(gb + offB);
    }
  };
  auto store = [&](const u4 (&st)[2 * RPT], int buf) {
#pragma unroll
    for (int h = 0; h < RPT; ++h) {
      sA LDS_AT(buf, sq, srow + (NT / 16) * h, sw) = st[h];
      sB LDS_AT(buf, sq, srow + (NT / 16) * h, sw) = st[RPT + h];
    }
  };

  f4 acc_re[WM][WN], acc_im[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      acc_re[i][j] = f4{0, 0, 0, 0};
      acc_im[i][j] = f4{0, 0, 0, 0};
    }

  const int64_t ktiles = p.Kp / SPLIT_BK;
  const int lr = lane & 15, lc = lane >> 4;
  const u4 sgn = u4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  u4 st[2 * RPT];
  auto read_a = [&](u4 (&a)[4], int buf, int i) {
    const int row = (wm * WM + i) * 16 + lr;
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = sA LDS_AT(buf, q, row, lc ^ swz(row));
  };
  auto read_b = [&](u4 (&b)[WN][4], int buf) {
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const int row = (wn * WN + j) * 16 + lr;
#pragma unroll
      for (int q = 0; q < 4; ++q) b[j][q] = sB LDS_AT(buf, q, row, lc ^ swz(row));
    }
  };
  // the twelve products of block row i with every block column of the wave
  auto mma_row = [&](const u4 (&a)[4], const u4 (&b)[WN][4], int i) {
    const u4 nih = a[PL_IH] ^ sgn, nil = a[PL_IL] ^ sgn;
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      f4 re = acc_re[i][j], im = acc_im[i][j];
      re = mma(a[PL_RH], b[j][PL_RH], re);
      im = mma(a[PL_RH], b[j][PL_IH], im);
      re = mma(a[PL_RH], b[j][PL_RL], re);
      im = mma(a[PL_RH], b[j][PL_IL], im);
      re = mma(a[PL_RL], b[j][PL_RH], re);
      im = mma(a[PL_RL], b[j][PL_IH], im);
      re = mma(nih, b[j][PL_IH], re);
      im = mma(a[PL_IH], b[j][PL_RH], im);
      re = mma(nih, b[j][PL_IL], re);
      im = mma(a[PL_IH], b[j][PL_RL], im);
      re = mma(nil, b[j][PL_IH], re);
      im = mma(a[PL_IL], b[j][PL_RH], im);
      acc_re[i][j] = re;
      acc_im[i][j] = im;
    }
  };

  if constexpr (PP) {
    // Ping-pong: waves w and w + 4 share a SIMD, so the workgroup splits into
    // two groups of four, one wave of each on every SIMD.  A group alternates
    // a memory phase (the fragments of K tile x from LDS into registers, its
    // share of tile x + 1 from registers into LDS, its share of tile x + 2
    // from global memory into registers) with a compute phase (the products of
    // tile x from the registers, no memory access), and the second group runs
    // one phase behind the first, separated by workgroup barriers: while one
    // wave of a SIMD issues products back to back, the other moves data.
    //
    // Barriers: both groups pass the prologue barrier, then group 0 runs
    // M(0) | C(0) | M(1) | ... | C(K-1) with a barrier after every phase, and
    // group 1 passes one extra barrier first and none after its last C(K-1),
    // so both pass 2K + 1 barriers.  Tile x + 1 overwrites the buffer of tile
    // x - 1, whose last reader (group 1, M(x-1)) finished two barriers before
    // group 0's M(x) and one before group 1's M(x); tile x is complete in LDS
    // one barrier before its first reader.
    static_assert(WGM * WGN == 8 && WGN == 4, "two groups of four waves");
    const int grp = __builtin_amdgcn_readfirstlane(wave) >> 2;   // wave-uniform
    u4 fa[WM][4], fb[WN][4];
    auto memory = [&](int64_t x) {
      const int buf = int(x & 1);
      read_b(fb, buf);
#pragma unroll
      for (int i = 0; i < WM; ++i) read_a(fa[i], buf, i);
      if (x + 1 < ktiles) store(st, int((x + 1) & 1));
      if (x + 2 < ktiles) load(st, x + 2);
    };
    if (ktiles > 0) {
      load(st, 0);
      store(st, 0);
      if (ktiles > 1) load(st, 1);
    }
    sync_lds();
    if (ktiles > 0 && grp == 1) sync_lds();
    for (int64_t x = 0; x < ktiles; ++x) {
      memory(x);
      sync_lds();
#pragma unroll
      for (int i = 0; i < WM; ++i) mma_row(fa[i], fb, i);
      if (grp == 0 || x + 1 < ktiles) sync_lds();
    }
  } else {
    // One K tile from LDS buffer buf.  The fragment reads of the first block
    // row go out first, so that the products start as soon as they arrive;
    // the staged tile's LDS stores and the next global loads follow the first
    // row's products, and each later row's reads are issued one row ahead.
    // The scheduling fences keep the compiler from hoisting every read (and
    // the stores) to the top, where the wave would wait for all of them
    // before its first product.  At most 12 LDS operations are outstanding
    // when a product waits, so the waits stay partial.
    static_assert(WM % 2 == 0, "rows are read two ahead in pairs");
    auto step = [&](int buf, bool do_store, int store_buf, bool do_load, int64_t load_kt) {
      u4 b[WN][4], a0[4], a1[4];
      read_a(a0, buf, 0);
      read_b(b, buf);
      __builtin_amdgcn_sched_barrier(0);
      read_a(a1, buf, 1);
      mma_row(a0, b, 0);
      __builtin_amdgcn_sched_barrier(0);
      if (do_store) store(st, store_buf);
      if (do_load) load(st, load_kt);
      __builtin_amdgcn_sched_barrier(0);
  #pragma unroll
      for (int i = 1; i < WM; i += 2) {
        if (i + 1 < WM) read_a(a0, buf, i + 1);
        mma_row(a1, b, i);
        __builtin_amdgcn_sched_barrier(0);
        if (i + 2 < WM) read_a(a1, buf, i + 2);
        if (i + 1 < WM) mma_row(a0, b, i + 1);
        __builtin_amdgcn_sched_barrier(0);
      }
    };

    // LDS buffer t % 2 holds tile t.  The last two tiles are peeled so that
    // the steady-state body has no branches around its stores and loads.
    if (ktiles > 0) {
      load(st, 0);
      store(st, 0);
      if (ktiles > 1) load(st, 1);
    }
    sync_lds();
    int64_t kt = 0;
    for (; kt + 2 < ktiles; ++kt) {
      step(int(kt & 1), true, int((kt + 1) & 1), true, kt + 2);
      sync_lds();
    }
    if (kt + 1 < ktiles) {
      step(int(kt & 1), true, int((kt + 1) & 1), false, 0);
      sync_lds();
      ++kt;
    }
    if (kt < ktiles) step(int(kt & 1), false, 0, false, 0);
  }

  if constexpr (PARTIAL) {
    int k = 0;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        gst_u4(partial + 4 * ((k++) * NT + tid), __builtin_bit_cast(u4, acc_re[i][j]));
        gst_u4(partial + 4 * ((k++) * NT + tid), __builtin_bit_cast(u4, acc_im[i][j]));
      }
    return;
  }

  if constexpr (WM == 4 && WN == 2) {
    // the lockstep loop ends without a barrier: its last fragment reads may
    // still be in flight in other waves
    if constexpr (!PP) sync_lds();
    u4* stage = (wave < 4 ? &sA[0][0][0] : &sB[0][0][0]) + (wave & 3) * 1024;
    split_epilogue_staged(p, acc_re, acc_im, m0 + wm * WM * 16, n0 + wn * WN * 16,
                          p.herm && tm != tn, stage);
  } else {
    split_epilogue<WM, WN>(p, acc_re, acc_im, m0 + wm * WM * 16, n0 + wn * WN * 16,
                           p.herm && tm != tn);
  }
}

template <int WGM, int WGN, int WM, int WN, bool PP>
__global__ void __launch_bounds__(64 * WGM * WGN, 1) split_gemm_kernel(const SplitParams p) {
  __shared__ SplitLds sA, sB;
  int tm, tn;
  if (p.herm)
    tri_coords(xcd_linear(blockIdx.x, p.tiles_m * (p.tiles_m + 1) / 2), p.tiles_m, tm, tn);
  else
    tile_coords(blockIdx.x, p.tiles_m, p.tiles_n, tm, tn);
  split_tile<WGM, WGN, WM, WN, PP>(p, tm, tn, sA, sB);
}

// A product's last round, split over K.  The Hermitian product's 4656 tiles
// at N = 12288 fill 18 rounds of 256 CUs and leave 48 for a 19th that would
// hold most CUs idle for a whole tile (at N = 5120 the full product leaves 64
// after 6 rounds; below N = 2048 a whole product has fewer tiles than half
// the CUs).  Instead those tiles are cut into S K ranges (one workgroup each,
// S x tail <= 256): split_tail_kernel writes each range's FP32 accumulators
// to a slot of acc, and split_tail_finish_kernel adds a tile's S slots in
// order (deterministic) and runs the usual epilogue, mirror included.
// Positions base .. base + tail - 1 of the launch's tile order are the tiles
// the main launch (grid base, none when base is 0) leaves out.
__device__ __forceinline__ void launch_tile(const SplitParams& p, int pid, int& tm, int& tn) {
  if (p.herm)
    tri_coords(xcd_linear(pid, p.tiles_m * (p.tiles_m + 1) / 2), p.tiles_m, tm, tn);
  else
    tile_coords(pid, p.tiles_m, p.tiles_n, tm, tn);
}

constexpr int TAIL_SLOTS = 256;                        // slots of acc
constexpr int TILE_ACC = SPLIT_BM * SPLIT_BN * 2;      // floats per slot (128 KB)

__global__ void __launch_bounds__(512, 1)
split_tail_kernel(const SplitParams p, int base, int S, int kc, float* __restrict__ acc) {
  __shared__ SplitLds sA, sB;
  const int i = blockIdx.x / S, r = blockIdx.x % S;
  int tm, tn;
  launch_tile(p, base + i, tm, tn);
  const int64_t ktiles = p.Kp / SPLIT_BK;
  const int64_t k0 = int64_t(r) * kc;
  SplitParams q = p;
  q.A = p.A + k0 * 4 * SPLIT_BK;        // K tile k0 of every row (row stride 4 lda unchanged)
  q.B = p.B + k0 * 4 * SPLIT_BK;
  q.Kp = min(int64_t(kc), ktiles - k0) * SPLIT_BK;
  split_tile<2, 4, 4, 2, true, true>(q, tm, tn, sA, sB, acc + size_t(blockIdx.x) * TILE_ACC);
}

__global__ void __launch_bounds__(512, 1)
split_tail_finish_kernel(const SplitParams p, int base, int S, const float* __restrict__ acc) {
  __shared__ SplitLds sA, sB;
  constexpr int NT = 512, WM = 4, WN = 2, WGN = 4;
  const int i = blockIdx.x;
  int tm, tn;
  launch_tile(p, base + i, tm, tn);
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  f4 acc_re[WM][WN], acc_im[WM][WN];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b) {
      acc_re[a][b] = f4{0, 0, 0, 0};
      acc_im[a][b] = f4{0, 0, 0, 0};
    }
  for (int r = 0; r < S; ++r) {          // K ranges in order
    const float* src = acc + size_t(i * S + r) * TILE_ACC;
    int k = 0;
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
      for (int b = 0; b < WN; ++b) {
        acc_re[a][b] += __builtin_bit_cast(f4, gld_u4(src + 4 * ((k++) * NT + tid)));
        acc_im[a][b] += __builtin_bit_cast(f4, gld_u4(src + 4 * ((k++) * NT + tid)));
      }
  }
  const int64_t m0 = int64_t(tm) * SPLIT_BM, n0 = int64_t(tn) * SPLIT_BN;
  u4* stage = (wave < 4 ? &sA[0][0][0] : &sB[0][0][0]) + (wave & 3) * 1024;
  split_epilogue_staged(p, acc_re, acc_im, m0 + wm * WM * 16, n0 + wn * WN * 16,
                        p.herm && tm != tn, stage);
}

// Many split products in one launch, one workgroup per tile of the
// concatenated tile list (item i's tiles start at tile_begin; no Hermitian
// items): the excitation-sector blocks of one step.
struct SplitItem {
  SplitParams p;
  int tile_begin;
};

template <int WGM, int WGN, int WM, int WN, bool PP>
__global__ void __launch_bounds__(64 * WGM * WGN, 1)
split_grouped_kernel(const SplitItem* __restrict__ items, int count) {
  __shared__ SplitLds sA, sB;
  const int t = round_xcd(blockIdx.x, gridDim.x);
  int lo = 0, hi = count - 1;              // last item with tile_begin <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
  }
  const SplitParams p = items[lo].p;
  const int local = t - items[lo].tile_begin;
  const int per_group = GROUP_M * p.tiles_n;
  const int first_m = (local / per_group) * GROUP_M;
  const int gsize = min(p.tiles_m - first_m, GROUP_M);
  const int in_group = local % per_group;
  split_tile<WGM, WGN, WM, WN, PP>(p, first_m + in_group % gsize, in_group / gsize, sA, sB);
}

// out(r, c) for r < Rp, c < Cp from src (R x C valid, element (r, c) at
// src[r*ld + c], or src[c*ld + r] when trans), conjugated if conj, zero outside.
constexpr int ST = 32;
__global__ void split_matrix_kernel(const c64* __restrict__ src, int64_t ld, int64_t R, int64_t C,
                                    int trans, int conj, uint16_t* __restrict__ P, int64_t ldp) {
  __shared__ float2 tile[ST][ST + 1];
  const int tx = threadIdx.x % ST, ty = threadIdx.x / ST;   // 32 x 8
  const int64_t r0 = int64_t(blockIdx.y) * ST, c0 = int64_t(blockIdx.x) * ST;
  for (int y = ty; y < ST; y += 8) {
    float2 v = make_float2(0.f, 0.f);
    if (trans) {
      // tile[y][x] = out(r0 + x, c0 + y) = src[(c0 + y) * ld + r0 + x]
      const int64_t r = r0 + tx, c = c0 + y;
      if (r < R && c < C) { const c64 s = src[c * ld + r]; v = make_float2(s.re, s.im); }
    } else {
      const int64_t r = r0 + y, c = c0 + tx;
      if (r < R && c < C) { const c64 s = src[r * ld + c]; v = make_float2(s.re, s.im); }
    }
    tile[y][tx] = v;
  }
  __syncthreads();
  for (int y = ty; y < ST; y += 8) {
    const float2 v = trans ? tile[tx][y] : tile[y][tx];
    const int64_t r = r0 + y, c = c0 + tx;
    uint16_t rh, rl, ih, il;
    split2(v.x, rh, rl);
    split2(conj ? -v.y : v.y, ih, il);
    P[plane_offset(ldp, r, c, PL_RH)] = rh;
    P[plane_offset(ldp, r, c, PL_RL)] = rl;
    P[plane_offset(ldp, r, c, PL_IH)] = ih;
    P[plane_offset(ldp, r, c, PL_IL)] = il;
  }
}

Planes4 take_planes(Arena& ar, int64_t rows, int64_t ld) {
  Planes4 p;
  p.rows = rows;
  p.ld = ld;
  p.base = static_cast<uint16_t*>(ar.take(size_t(4) * size_t(rows) * size_t(ld) * 2));
  return p;
}

int split_into(const c64* src, int64_t ld, int64_t R, int64_t C, bool trans, bool conj,
               const Planes4& P, hipStream_t s) {
  // fills all P.rows x P.ld entries (padding becomes zero)
  dim3 grid(unsigned(P.ld / ST), unsigned(P.rows / ST));
  hipLaunchKernelGGL(split_matrix_kernel, grid, dim3(256), 0, s, src, ld, R, C, int(trans),
                     int(conj), P.base, P.ld);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

// Kernel shape: 0 = 8 waves of 64 x 32 outputs in two ping-pong groups
// (default), 1 = 4 waves of 64 x 64, 2 = 8 waves of 64 x 32 in lockstep.
// TC_SPLIT_VARIANT selects one for timing.
int split_variant() {
  static const int v = [] {
    const char* e = getenv("TC_SPLIT_VARIANT");
    return e ? atoi(e) : 0;
  }();
  return v;
}

// Compute units of the current device (queried once per device).
int device_cu_count(int* cus) {
  static std::atomic<int> cache[64];
  int dev = 0;
  TC_TRY_HIP(hipGetDevice(&dev));
  if (dev >= 0 && dev < 64 && cache[dev].load() > 0) {
    *cus = cache[dev].load();
    return TC_OK;
  }
  int n = 0;
  TC_TRY_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
  if (n <= 0) {
    set_error("the device reports no compute units");
    return TC_ERR_HIP;
  }
  if (dev >= 0 && dev < 64) cache[dev].store(n);
  *cus = n;
  return TC_OK;
}

int run_split(const Planes4& A, const Planes4& B, int64_t M, int64_t N, int64_t Kp, float ar,
              float ai, float br, float bi, const c64* Cin, int64_t ldcin, bool cin_trans, c64* Cf,
              int64_t ldcf, const Planes4* P, bool p_trans, bool herm, hipStream_t s,
              float* tail_acc = nullptr, int tail_slots = 0) {
  SplitParams q;
  q.A = A.base; q.lda = A.ld;
  q.B = B.base; q.ldb = B.ld;
  q.M = M; q.N = N; q.Kp = Kp;
  q.ar = ar; q.ai = ai; q.br = br; q.bi = bi;
  q.Cin = Cin; q.ldcin = ldcin; q.cin_trans = cin_trans;
  q.Cf = Cf; q.ldcf = ldcf;
  q.P = P ? P->base : nullptr; q.ldp = P ? P->ld : 0;
  q.p_trans = p_trans;
  q.herm = herm;
  q.tiles_m = int((M + SPLIT_BM - 1) / SPLIT_BM);
  q.tiles_n = int((N + SPLIT_BN - 1) / SPLIT_BN);
  if (herm && M != N) {
    set_error("split product: a Hermitian result must be square");
    return TC_ERR_INVALID_ARGUMENT;
  }
  const int64_t tiles = herm ? int64_t(q.tiles_m) * (q.tiles_m + 1) / 2
                             : int64_t(q.tiles_m) * q.tiles_n;
  if (tiles == 0) return TC_OK;
  // the padded planes must cover every tile row / column and the K extent
  if (A.rows < int64_t(q.tiles_m) * SPLIT_BM || B.rows < int64_t(q.tiles_n) * SPLIT_BN ||
      A.ld < Kp || B.ld < Kp || Kp % SPLIT_BK != 0 ||
      (P && (P->rows < (p_trans ? int64_t(q.tiles_n) * SPLIT_BN : int64_t(q.tiles_m) * SPLIT_BM) ||
             P->ld < (p_trans ? int64_t(q.tiles_m) * SPLIT_BM : int64_t(q.tiles_n) * SPLIT_BN) ||
             (herm && (P->rows < int64_t(q.tiles_m) * SPLIT_BM ||
                       P->ld < int64_t(q.tiles_m) * SPLIT_BM))))) {
    set_error("split product: plane buffers do not cover the padded tiles");
    return TC_ERR_INVALID_ARGUMENT;
  }
  ProfileScope prof(TC_KERNEL_SPLIT_BF16, s);
  if (tail_acc && tail_slots > 0 && split_variant() == 0) {
    // a last round that would leave at least half of the CUs idle (the whole
    // product, when it has that few tiles): its tiles go split over K, one
    // workgroup and one slot of partial sums per K range of at least 4 K slices
    int cus = 0;
    TC_RETURN_IF(device_cu_count(&cus));
    const int64_t full = tiles / cus, tail = tiles % cus, kt = Kp / SPLIT_BK;
    const int64_t slots = std::min<int64_t>(tail_slots, TAIL_SLOTS);
    int S = int(std::min<int64_t>(std::min<int64_t>(cus, slots) / std::max<int64_t>(tail, 1),
                                  std::min<int64_t>(8, kt / 4)));
    if (tail > 0 && tail * 2 <= cus && S >= 2) {
      const int64_t kc = (kt + S - 1) / S;
      S = int((kt + kc - 1) / kc);         // every K range non-empty
      const int base = int(full * cus);
      if (base > 0) {
        hipLaunchKernelGGL((split_gemm_kernel<2, 4, 4, 2, true>), dim3(unsigned(base)),
                           dim3(512), 0, s, q);
        TC_TRY_HIP(hipGetLastError());
      }
      hipLaunchKernelGGL(split_tail_kernel, dim3(unsigned(tail * S)), dim3(512), 0, s, q, base, S,
                         int(kc), tail_acc);
      TC_TRY_HIP(hipGetLastError());
      hipLaunchKernelGGL(split_tail_finish_kernel, dim3(unsigned(tail)), dim3(512), 0, s, q, base,
                         S, static_cast<const float*>(tail_acc));
      TC_TRY_HIP(hipGetLastError());
      return TC_OK;
    }
  }
  const dim3 grid{unsigned(tiles), 1u, 1u};
  if (split_variant() == 1)
    hipLaunchKernelGGL((split_gemm_kernel<2, 2, 4, 4, false>), grid, dim3(256), 0, s, q);
  else if (split_variant() == 2)
    hipLaunchKernelGGL((split_gemm_kernel<2, 4, 4, 2, false>), grid, dim3(512), 0, s, q);
  else
    hipLaunchKernelGGL((split_gemm_kernel<2, 4, 4, 2, true>), grid, dim3(512), 0, s, q);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

}  // namespace

Planes4 split_take_planes(Arena& ar, int64_t rows, int64_t ld) { return take_planes(ar, rows, ld); }

int split_matrix(const c64* src, int64_t ld, int64_t R, int64_t C, bool trans, bool conj,
                 const Planes4& P, hipStream_t s) {
  return split_into(src, ld, R, C, trans, conj, P, s);
}

size_t split_grouped_bytes(int count) { return size_t(count) * sizeof(SplitItem); }

int split_grouped_build(const std::vector<SplitProduct>& ps, void* items_dev, SplitGrouped* g,
                        hipStream_t s) {
  std::vector<SplitItem> items;
  int64_t t = 0;
  for (const SplitProduct& d : ps) {
    if (d.M % SPLIT_BM != 0 || d.N % SPLIT_BN != 0 || d.Kp % SPLIT_BK != 0 || d.Kp <= 0 ||
        d.M <= 0 || d.N <= 0) {
      set_error("grouped split products take whole 128 x 128 tiles and a K extent of 32s");
      return TC_ERR_INVALID_ARGUMENT;
    }
    SplitItem it;
    SplitParams& q = it.p;
    q.A = d.A; q.lda = d.lda;
    q.B = d.B; q.ldb = d.ldb;
    q.M = d.M; q.N = d.N; q.Kp = d.Kp;
    q.ar = d.ar; q.ai = d.ai; q.br = d.br; q.bi = d.bi;
    q.Cin = d.Cin; q.ldcin = d.ldcin; q.cin_trans = 0;
    q.Cf = d.Cf; q.ldcf = d.ldcf;
    q.P = d.P; q.ldp = d.ldp; q.p_trans = d.p_trans ? 1 : 0;
    q.herm = 0;
    q.tiles_m = int(d.M / SPLIT_BM);
    q.tiles_n = int(d.N / SPLIT_BN);
    it.tile_begin = int(t);
    t += int64_t(q.tiles_m) * q.tiles_n;
    items.push_back(it);
  }
  if (t > (int64_t(1) << 30)) { set_error("too many tiles in one group"); return TC_ERR_UNSUPPORTED; }
  g->count = int(items.size());
  g->total_tiles = int(t);
  g->items_dev = items_dev;
  if (!items.empty()) {
    TC_TRY_HIP(hipMemcpyAsync(items_dev, items.data(), items.size() * sizeof(SplitItem),
                              hipMemcpyHostToDevice, s));
    TC_TRY_HIP(hipStreamSynchronize(s));   // items is host memory of this call
  }
  return TC_OK;
}

int split_grouped_run(const SplitGrouped& g, hipStream_t s) {
  if (g.count == 0 || g.total_tiles == 0) return TC_OK;
  ProfileScope prof(TC_KERNEL_SPLIT_BF16, s);
  if (split_variant() == 2)
    hipLaunchKernelGGL((split_grouped_kernel<2, 4, 4, 2, false>), dim3(unsigned(g.total_tiles)),
                       dim3(512), 0, s, static_cast<const SplitItem*>(g.items_dev), g.count);
  else
    hipLaunchKernelGGL((split_grouped_kernel<2, 4, 4, 2, true>), dim3(unsigned(g.total_tiles)),
                       dim3(512), 0, s, static_cast<const SplitItem*>(g.items_dev), g.count);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

void split_plan(Arena& ar, int64_t N, SplitPlanes* p) {
  const int64_t Np = round_up(N, SPLIT_BM);   // SPLIT_BM = SPLIT_BN, multiple of SPLIT_BK
  p->N = N;
  p->Np = Np;
  p->opA = take_planes(ar, Np, Np);
  p->opB = take_planes(ar, Np, Np);
  p->X = take_planes(ar, Np, Np);
  p->Rt = take_planes(ar, Np, Np);
}

int split_operand(const c64* op, int64_t ld, int64_t N, const SplitPlanes& p, hipStream_t s) {
  TC_RETURN_IF(split_into(op, ld, N, N, false, false, p.opA, s));
  TC_RETURN_IF(split_into(op, ld, N, N, true, true, p.opB, s));
  // X planes: their padding must be zero before the first product writes them
  TC_TRY_HIP(hipMemsetAsync(p.X.base, 0, size_t(4) * p.X.rows * p.X.ld * 2, s));
  return TC_OK;
}

int split_state(const c64* rho, int64_t ld, int64_t N, const SplitPlanes& p, hipStream_t s) {
  return split_into(rho, ld, N, N, true, false, p.Rt, s);
}

int step_split(c64* rho, int64_t ldr, c64* X, int64_t ldx, int64_t N, bool rotating, bool herm,
               const SplitPlanes& p, hipStream_t s) {
  // X = op rho (+ rho): A = split(op), B = split(rho^T); planes of X row-major
  TC_RETURN_IF(run_split(p.opA, p.Rt, N, N, p.Np, 1.f, 0.f, rotating ? 1.f : 0.f, 0.f,
                         rotating ? rho : nullptr, ldr, false, rotating ? X : nullptr, ldx,
                         &p.X, false, false, s, p.tail_acc, p.tail_slots));
  // rho' = X conj(op) (+ X): A = split(X), B = split(conj(op)^T); FP32 rho and
  // transposed planes of rho for the next step.  rho' is Hermitian, so with
  // herm only its upper tile triangle is multiplied.
  TC_RETURN_IF(run_split(p.X, p.opB, N, N, p.Np, 1.f, 0.f, rotating ? 1.f : 0.f, 0.f,
                         rotating ? X : nullptr, ldx, false, rho, ldr, &p.Rt, true, herm, s,
                         p.tail_acc, p.tail_slots));
  return TC_OK;
}

void split_gemm_plan(Arena& ar, int64_t M, int64_t N, int64_t K, SplitGemmPlan* p) {
  const int64_t Mp = round_up(std::max<int64_t>(M, 1), SPLIT_BM);
  const int64_t Np = round_up(std::max<int64_t>(N, 1), SPLIT_BN);
  const int64_t Kp = round_up(std::max<int64_t>(K, 1), SPLIT_BK);
  Planes4 a = take_planes(ar, Mp, Kp);
  Planes4 b = take_planes(ar, Np, Kp);
  if (p) { p->A = a; p->B = b; }
}

int split_gemm(const GemmDesc& d, const SplitGemmPlan& p, hipStream_t s) {
  // A planes: element (m, k) of op(A); B planes: row n holds column n of op(B)
  const c64* A = static_cast<const c64*>(d.A);
  const c64* B = static_cast<const c64*>(d.B);
  if (d.K > 0) {
    // op(A)(m, k) = A[k*lda + m] when a_kmaj: a transposed read
    TC_RETURN_IF(split_into(A, d.lda, d.M, d.K, d.a_kmaj, d.conj_a, p.A, s));
    // B plane row n, column k = op(B)(k, n) = B[k*ldb + n] when b_kmaj: transposed read
    TC_RETURN_IF(split_into(B, d.ldb, d.N, d.K, d.b_kmaj, d.conj_b, p.B, s));
  } else {
    TC_TRY_HIP(hipMemsetAsync(p.A.base, 0, size_t(4) * p.A.rows * p.A.ld * 2, s));
    TC_TRY_HIP(hipMemsetAsync(p.B.base, 0, size_t(4) * p.B.rows * p.B.ld * 2, s));
  }
  return run_split(p.A, p.B, d.M, d.N, p.A.ld, float(d.alpha_re), float(d.alpha_im),
                   float(d.beta_re), float(d.beta_im), static_cast<const c64*>(d.Cin), d.ldcin,
                   d.cin_trans, static_cast<c64*>(d.C), d.ldc, nullptr, false, d.herm, s);
}

}  // namespace tcm
