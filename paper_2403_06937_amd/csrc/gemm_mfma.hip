// MFMA matrix products in FP64 and FP32 for gfx950 (CDNA4).
//
// One templated kernel covers the complex products of the time step
// (rho <- U rho U^dag, two complex N x N x N products per step) and the real
// and complex products used to form U.  Design:
//   * 256 threads = 4 wavefronts of 64 lanes; the wave grid is WGM x WGN and
//     each wave owns WM x WN blocks of 16 x 16 outputs.
//   * v_mfma_f64_16x16x4_f64 / v_mfma_f32_16x16x4_f32: lane l supplies
//     A[l%16][l/16] and B[l/16][l%16] of a 16x4 / 4x16 slice.  Output r of
//     lane l is D[4*(l/16)+r][l%16] for FP32 but D[l/16+4r][l%16] for FP64
//     (measured on gfx950).  A complex block needs four real
//     products: Re += Ar*Br - Ai*Bi, Im += Ar*Bi + Ai*Br.  For FP64 the minus
//     sign is the instruction's own A-negation modifier.
//   * Tiles of A and B are staged through LDS "K-major" (sA[k][m], sB[k][n]) so
//     a wave's 16 lanes read 16 consecutive elements; two LDS buffers, one
//     barrier per K-tile, global loads for tile t+1 in flight while tile t
//     is multiplied.
//   * Complex elements stay interleaved (re, im): one 16-byte LDS read gives a
//     lane both parts of its FP64 operand.
//   * Workgroups are renumbered so each XCD (workgroup id mod 8) owns a
//     contiguous range of tiles, walked in groups of GROUP_M tile rows, so
//     tiles that share A rows / B columns share that XCD's L2.
#include "gemm_mfma.h"
#include "profile.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>

namespace tcm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct acc_t;
template <> struct acc_t<double> { typedef d4 type; };
template <> struct acc_t<float> { typedef f4 type; };

__device__ __forceinline__ d4 mma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// -a * b + c via the FP64 MFMA negation modifier (neg:[1,0,0]).
__device__ __forceinline__ d4 mma_nega(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 1);
}
__device__ __forceinline__ f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mma_nega(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(-a, b, c, 0, 0, 0);
}

template <typename T, bool CPLX> struct elem;
template <typename T> struct elem<T, true> {
  typedef cplx<T> type;
  static __device__ __forceinline__ type zero() { return type{T(0), T(0)}; }
  static __device__ __forceinline__ type cj(type x, bool c) { if (c) x.im = -x.im; return x; }
};
template <typename T> struct elem<T, false> {
  typedef T type;
  static __device__ __forceinline__ type zero() { return T(0); }
  static __device__ __forceinline__ type cj(type x, bool) { return x; }
};

struct Params {
  int64_t M, N, K;
  const void* A; int64_t lda;
  const void* B; int64_t ldb;
  void* C; int64_t ldc;
  const void* Cin; int64_t ldcin;
  double alpha_re, alpha_im, beta_re, beta_im, gamma;
  int conj_a, conj_b, c_trans, cin_trans;
  int herm;
  int tiles_m, tiles_n;
};

constexpr int GROUP_M = 8;

// Default tile variant per element type for the step / exponential layout,
// chosen by timing every variant at N = 12288 on gfx950:
//   complex FP64: 128x128 tiles, 8 waves, K tile 16 (240 ms per full
//                 product before the staged tile was stored early, 231 ms
//                 after; 64x64: 285 ms; 128x128 with K tile 8: 294 ms;
//                 128x64: 438 ms; LDS row padding of 0, 16 or 32 bytes: no
//                 difference)
//   real FP64:    128x128 tiles, 8 waves (U formation 1.07 s; 128x64: 1.42 s)
//   complex FP32: 128x128 tiles, 8 waves (112 ms; 128x64: 118 ms)
template <typename T, bool CPLX> struct DefaultVariant { static constexpr int value = 1; };
template <> struct DefaultVariant<double, true> { static constexpr int value = 6; };

// Consecutive workgroup ids go round the 8 XCDs; give each XCD a contiguous
// run of the tile order so that its tiles share operand rows in its L2.
__device__ __forceinline__ int xcd_linear(int pid, int total) {
  const int q = total / 8, r = total % 8;
  const int xcd = pid % 8, local = pid / 8;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + local;
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

// Publishes this wave's LDS writes to the workgroup: waits for them, then a
// barrier.  Outstanding global loads are not waited for (__syncthreads would
// wait for those too); the memory clobber keeps the compiler from moving LDS
// accesses across it.
__device__ __forceinline__ void sync_lds() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Tile coordinates of this workgroup (XCD-contiguous, grouped ordering).
__device__ __forceinline__ void tile_coords(int pid, int tiles_m, int tiles_n, int& tm, int& tn) {
  const int lin = xcd_linear(pid, tiles_m * tiles_n);
  const int per_group = GROUP_M * tiles_n;
  const int group = lin / per_group;
  const int first_m = group * GROUP_M;
  const int gsize = min(tiles_m - first_m, GROUP_M);
  const int in_group = lin % per_group;
  tm = first_m + in_group % gsize;
  tn = in_group / gsize;
}

// Global-memory element access.  The persistent kernel reads its operand
// pointers from the descriptor array rather than from kernel arguments, so
// the compiler cannot infer their address space and would issue flat
// accesses (which also count against lgkmcnt, so the LDS barrier would wait
// for them).  Loads and stores through address-space-1 pointers of scalar or
// vector type (a struct copy would drop the address space) are global.
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
  typedef __attribute__((address_space(1))) const T gT;
  return *(gT*)p;
}
template <typename T>
__device__ __forceinline__ cplx<T> gload(const cplx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2), aligned(sizeof(T))));
  typedef __attribute__((address_space(1))) const v2 gv2;
  const v2 v = *(gv2*)p;
  return cplx<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void gstore(T* p, T x) {
  typedef __attribute__((address_space(1))) T gT;
  *(gT*)p = x;
}
template <typename T>
__device__ __forceinline__ void gstore(cplx<T>* p, cplx<T> x) {
  typedef T v2 __attribute__((ext_vector_type(2), aligned(sizeof(T))));
  typedef __attribute__((address_space(1))) v2 gv2;
  *(gv2*)p = v2{x.re, x.im};
}

// LDS of one tile: two buffers of the A and B K tiles (K-major rows padded by
// PADB bytes).  Declared by the kernels, so a kernel that instantiates the
// tile for both the checked and the exact case still holds one copy.
template <typename T, bool CPLX, int BM, int BN, int BKT, int PADB>
struct TileLds {
  typedef typename elem<T, CPLX>::type E;
  static constexpr int PADE = PADB / int(sizeof(E));
  static constexpr int LDA_S = BM + PADE;
  static constexpr int LDB_S = BN + PADE;
  static constexpr int elems = 2 * BKT * (LDA_S + LDB_S);
};

// One BM x BN output tile (tm, tn) of the product described by p.  Shared by
// the one-product kernel and the persistent grouped kernel; the caller must
// separate two calls in one workgroup by a barrier (the LDS is reused).
// Modes of gemm_tile: the whole tile; PARTIAL: the K loop only, the raw
// accumulators stored to part (16-byte chunk c of thread t at chunk c NT + t,
// over the blocks' real then imaginary accumulators); FINISH: no K loop, the
// accumulators are the in-order sum of nparts such slots from part, then the
// epilogue.
enum TileMode { TILE_FULL = 0, TILE_PARTIAL = 1, TILE_FINISH = 2 };

template <typename T, bool CPLX, bool AK, bool BK, bool CHECKED,
          int BM, int BN, int BKT, int WM, int WN, int PADB, int MODE = TILE_FULL>
__device__ __forceinline__ void gemm_tile(const Params& p, int tm, int tn, bool mirror,
                                          typename elem<T, CPLX>::type* lds,
                                          void* part = nullptr, int nparts = 0) {
  typedef typename elem<T, CPLX>::type E;
  typedef typename acc_t<T>::type A4;
  constexpr int WGN = BN / (16 * WN);
  constexpr int WGM = BM / (16 * WM);
  constexpr int NT = 64 * WGM * WGN;          // threads per workgroup
  static_assert(BKT % 4 == 0, "K tile is a multiple of the MFMA depth");
  constexpr int PADE = PADB / int(sizeof(E));   // LDS row padding in elements
  constexpr int LDA_S = BM + PADE;
  constexpr int LDB_S = BN + PADE;
  constexpr int A_PT = BKT * BM / NT;          // staged elements per thread
  constexpr int B_PT = BKT * BN / NT;
  static_assert(BKT * BM % NT == 0 && BKT * BN % NT == 0, "tile split");
  // a thread's staged elements share one row (K-major) or one column of the tile
  static_assert(AK ? NT % BM == 0 : NT % BKT == 0, "A staging pattern");
  static_assert(BK ? NT % BN == 0 : NT % BKT == 0, "B staging pattern");

  typedef E ARow[BKT][LDA_S];
  typedef E BRow[BKT][LDB_S];
  ARow* sA = reinterpret_cast<ARow*>(lds);
  BRow* sB = reinterpret_cast<BRow*>(lds + 2 * BKT * LDA_S);

  // kernel arguments into registers once
  const int64_t M = p.M, N = p.N, K = p.K;
  const int64_t lda = p.lda, ldb = p.ldb;
  const bool cja = p.conj_a != 0, cjb = p.conj_b != 0;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int64_t m0 = int64_t(tm) * BM, n0 = int64_t(tn) * BN;

  // Staging pattern: element j of this thread sits at (ka + j*dka, ma + j*dma)
  // of the A tile and (kb + j*dkb, nb + j*dnb) of the B tile.
  const int ka = AK ? tid / BM : tid % BKT;
  const int ma = AK ? tid % BM : tid / BKT;
  constexpr int dka = AK ? NT / BM : 0;
  constexpr int dma = AK ? 0 : NT / BKT;
  const int kb = BK ? tid / BN : tid % BKT;
  const int nb = BK ? tid % BN : tid / BKT;
  constexpr int dkb = BK ? NT / BN : 0;
  constexpr int dnb = BK ? 0 : NT / BKT;
  // global offsets of element 0 at k0 = 0, strides per j and per K tile
  const E* __restrict__ pa = static_cast<const E*>(p.A) +
      (AK ? int64_t(ka) * lda + (m0 + ma) : (m0 + ma) * lda + ka);
  const E* __restrict__ pb = static_cast<const E*>(p.B) +
      (BK ? int64_t(kb) * ldb + (n0 + nb) : (n0 + nb) * ldb + kb);
  const int64_t sja = AK ? int64_t(dka) * lda : int64_t(dma) * lda;
  const int64_t sjb = BK ? int64_t(dkb) * ldb : int64_t(dnb) * ldb;
  const int64_t ska = AK ? int64_t(BKT) * lda : BKT;
  const int64_t skb = BK ? int64_t(BKT) * ldb : BKT;

  A4 acc_re[WM][WN], acc_im[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      acc_re[i][j] = A4{0, 0, 0, 0};
      acc_im[i][j] = A4{0, 0, 0, 0};
    }

  E ra[A_PT], rb[B_PT];
  const int64_t ktiles = (K + BKT - 1) / BKT;

  // Ragged tiles (CHECKED): every lane loads from an address clamped into the
  // operand and zeroes the value if its (row, k) lies outside, so the loads
  // stay unconditional (no exec-mask branches around them).  The loads land in
  // ra / rb untouched; the conjugation and the zeroing are applied when the
  // registers go to LDS, a K tile later, so that nothing waits for a global
  // load in the iteration that issues it.
  const E* __restrict__ A0 = static_cast<const E*>(p.A);
  const E* __restrict__ B0 = static_cast<const E*>(p.B);
  auto load_tiles = [&](int64_t kt) {
    const E* qa = pa + kt * ska;
    const E* qb = pb + kt * skb;
    const int64_t k0 = kt * BKT;
#pragma unroll
    for (int j = 0; j < A_PT; ++j) {
      if constexpr (CHECKED) {
        const int64_t m = m0 + ma + j * dma, k = k0 + ka + j * dka;
        const int64_t mc = m < M ? m : M - 1, kc = k < K ? k : K - 1;
        ra[j] = gload(A0 + (AK ? kc * lda + mc : mc * lda + kc));
      } else {
        ra[j] = gload(qa + j * sja);
      }
    }
#pragma unroll
    for (int j = 0; j < B_PT; ++j) {
      if constexpr (CHECKED) {
        const int64_t nn = n0 + nb + j * dnb, k = k0 + kb + j * dkb;
        const int64_t nc = nn < N ? nn : N - 1, kc = k < K ? k : K - 1;
        rb[j] = gload(B0 + (BK ? kc * ldb + nc : nc * ldb + kc));
      } else {
        rb[j] = gload(qb + j * sjb);
      }
    }
  };
  // registers of K tile kt into LDS buffer buf
  auto store_tiles = [&](int buf, int64_t kt) {
    const int64_t k0 = kt * BKT;
#pragma unroll
    for (int j = 0; j < A_PT; ++j) {
      E v = elem<T, CPLX>::cj(ra[j], cja);
      if constexpr (CHECKED) {
        if (!(m0 + ma + j * dma < M && k0 + ka + j * dka < K)) v = elem<T, CPLX>::zero();
      }
      sA[buf][ka + j * dka][ma + j * dma] = v;
    }
#pragma unroll
    for (int j = 0; j < B_PT; ++j) {
      E v = elem<T, CPLX>::cj(rb[j], cjb);
      if constexpr (CHECKED) {
        if (!(n0 + nb + j * dnb < N && k0 + kb + j * dkb < K)) v = elem<T, CPLX>::zero();
      }
      sB[buf][kb + j * dkb][nb + j * dnb] = v;
    }
  };

  const int lrow = lane >> 4;   // k offset within the 4-deep slice
  const int lcol = lane & 15;   // m / n offset within the 16-wide block
  // the accumulators as 16-byte chunks, in a fixed order over the blocks
  struct Chunks { u4 c[sizeof(A4) / 16]; };
  constexpr int NCH = int(sizeof(A4) / 16);
  if constexpr (MODE == TILE_FINISH) {
    // one row of blocks at a time, the slots in order inside it, so that only
    // that row's partial sums are live next to the accumulators
    constexpr int PER_ROW = (CPLX ? 2 : 1) * WN * NCH;          // chunks per row of blocks
    const size_t slot = size_t((CPLX ? 2 : 1) * WM * WN * NCH) * NT;
#pragma unroll
    for (int i = 0; i < WM; ++i) {
#pragma unroll 1
      for (int r = 0; r < nparts; ++r) {
        const u4* src = static_cast<const u4*>(part) + size_t(r) * slot + size_t(i) * PER_ROW * NT;
        int c = 0;
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          Chunks a, b;
#pragma unroll
          for (int h = 0; h < NCH; ++h) a.c[h] = gload(src + size_t(c + h) * NT + tid);
          c += NCH;
          acc_re[i][j] += __builtin_bit_cast(A4, a);
          if constexpr (CPLX) {
#pragma unroll
            for (int h = 0; h < NCH; ++h) b.c[h] = gload(src + size_t(c + h) * NT + tid);
            c += NCH;
            acc_im[i][j] += __builtin_bit_cast(A4, b);
          }
        }
      }
    }
  } else {
    // LDS buffer t % 2 holds K tile t.  The registers carry tile t + 1 into the
    // other buffer at the start of iteration t (free since the last barrier)
    // and are refilled with tile t + 2 before the products, so a load has a
    // whole iteration to arrive and the barrier waits for no global load.
    // Past the last K tile the load and the store repeat the last tile (in
    // bounds, into a buffer no wave reads again) instead of being skipped: with
    // no branch around them the loaded registers need no copies at a merge,
    // which would wait for the loads right after issuing them.
    const int64_t klast = ktiles - 1;
    if (ktiles > 0) {
      load_tiles(0);
      store_tiles(0, 0);
      load_tiles(klast < 1 ? klast : 1);
    }
    sync_lds();

    for (int64_t kt = 0; kt < ktiles; ++kt) {
      const int buf = int(kt & 1);
      // the first 4-deep slice's fragments are read before the staged tile
      // goes to the other buffer, so their latency overlaps the stores
      E a0[WM], b0[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) a0[i] = sA[buf][lrow][(wm * WM + i) * 16 + lcol];
#pragma unroll
      for (int j = 0; j < WN; ++j) b0[j] = sB[buf][lrow][(wn * WN + j) * 16 + lcol];
      store_tiles(buf ^ 1, kt + 1 < klast ? kt + 1 : klast);
      load_tiles(kt + 2 < klast ? kt + 2 : klast);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k4 = 0; k4 < BKT / 4; ++k4) {
        E a[WM], b[WN];
        if (k4 == 0) {
#pragma unroll
          for (int i = 0; i < WM; ++i) a[i] = a0[i];
#pragma unroll
          for (int j = 0; j < WN; ++j) b[j] = b0[j];
        } else {
#pragma unroll
          for (int i = 0; i < WM; ++i) a[i] = sA[buf][k4 * 4 + lrow][(wm * WM + i) * 16 + lcol];
#pragma unroll
          for (int j = 0; j < WN; ++j) b[j] = sB[buf][k4 * 4 + lrow][(wn * WN + j) * 16 + lcol];
        }
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) {
            if constexpr (CPLX) {
              acc_re[i][j] = mma(a[i].re, b[j].re, acc_re[i][j]);
              acc_re[i][j] = mma_nega(a[i].im, b[j].im, acc_re[i][j]);
              acc_im[i][j] = mma(a[i].re, b[j].im, acc_im[i][j]);
              acc_im[i][j] = mma(a[i].im, b[j].re, acc_im[i][j]);
            } else {
              acc_re[i][j] = mma(a[i], b[j], acc_re[i][j]);
            }
          }
      }
      sync_lds();
    }
  }
  if constexpr (MODE == TILE_PARTIAL) {
    u4* dst = static_cast<u4*>(part);
    int c = 0;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const Chunks a = __builtin_bit_cast(Chunks, acc_re[i][j]);
#pragma unroll
        for (int h = 0; h < NCH; ++h) gstore(dst + size_t(c + h) * NT + tid, a.c[h]);
        c += NCH;
        if constexpr (CPLX) {
          const Chunks b = __builtin_bit_cast(Chunks, acc_im[i][j]);
#pragma unroll
          for (int h = 0; h < NCH; ++h) gstore(dst + size_t(c + h) * NT + tid, b.c[h]);
          c += NCH;
        }
      }
    return;
  }

  // Epilogue: C = alpha * acc + beta * Cin + gamma * [m == n]
  E* __restrict__ Cg = static_cast<E*>(p.C);
  const E* __restrict__ Cin = static_cast<const E*>(p.Cin);
  const int64_t ldc = p.ldc, ldcin = p.ldcin;
  const bool ctr = p.c_trans != 0, citr = p.cin_trans != 0;
  const T ar = T(p.alpha_re), ai = T(p.alpha_im), br = T(p.beta_re), bi = T(p.beta_im);
  const T gam = T(p.gamma);
  const bool use_beta = (Cin != nullptr) && (p.beta_re != 0.0 || p.beta_im != 0.0);
  // FP64 MFMA output r of lane l is row l/16 + 4r; FP32 is row 4(l/16) + r
  auto out_row = [&](int i, int r) -> int64_t {
    return m0 + (wm * WM + i) * 16 + (sizeof(T) == 8 ? lrow + 4 * r : 4 * lrow + r);
  };
#pragma unroll
  for (int i = 0; i < WM; ++i) {
    // beta's operand for this row of blocks, loaded before any of it is used
    // (addresses clamped into the matrix, so no branch): one wait per row of
    // blocks instead of one per element
    E cin[WN][4];
    if (use_beta) {
      const int64_t sr = citr ? 1 : ldcin, sc = citr ? ldcin : 1;
#pragma unroll
      for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int64_t row = out_row(i, r), col = n0 + (wn * WN + j) * 16 + lcol;
          if constexpr (CHECKED) {
            row = row < M ? row : M - 1;
            col = col < N ? col : N - 1;
          }
          cin[j][r] = gload(Cin + row * sr + col * sc);
        }
    }
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = out_row(i, r);
        const int64_t col = n0 + (wn * WN + j) * 16 + lcol;
        if (CHECKED && (row >= M || col >= N)) continue;
        const int64_t caddr = ctr ? col * ldc + row : row * ldc + col;
        E out;
        if constexpr (CPLX) {
          const T xr = acc_re[i][j][r], xi = acc_im[i][j][r];
          out.re = ar * xr - ai * xi;
          out.im = ar * xi + ai * xr;
          if (use_beta) {
            const E y = cin[j][r];
            out.re += br * y.re - bi * y.im;
            out.im += br * y.im + bi * y.re;
          }
          if (row == col) out.re += gam;
        } else {
          out = ar * acc_re[i][j][r];
          if (use_beta) out += br * cin[j][r];
          if (row == col) out += gam;
        }
        gstore(Cg + caddr, out);
        if (mirror) {
          if constexpr (CPLX) out.im = -out.im;
          gstore(Cg + (ctr ? row * ldc + col : col * ldc + row), out);
        }
      }
  }
}

template <typename T, bool CPLX, bool AK, bool BK, bool CHECKED,
          int BM, int BN, int BKT, int WM, int WN, int PADB>
__global__ void __launch_bounds__(64 * (BM / (16 * WM)) * (BN / (16 * WN)), 1)
gemm_kernel(const Params p) {
  typedef TileLds<T, CPLX, BM, BN, BKT, PADB> L;
  __shared__ typename L::E lds[L::elems];
  int tm, tn;
  if (p.herm)
    tri_coords(xcd_linear(blockIdx.x, p.tiles_m * (p.tiles_m + 1) / 2), p.tiles_m, tm, tn);
  else
    tile_coords(blockIdx.x, p.tiles_m, p.tiles_n, tm, tn);
  gemm_tile<T, CPLX, AK, BK, CHECKED, BM, BN, BKT, WM, WN, PADB>(p, tm, tn, p.herm && tm != tn,
                                                                 lds);
}

// A product's last round split over K, as for the split-BF16 product: the
// main launch runs the full rounds of one tile per CU (none for a product
// with fewer tiles than half the CUs), gemm_tail_kernel runs
// the remaining tiles' S K ranges (kc K tiles each) and stores their
// accumulators to one slot each of part, and gemm_tail_finish_kernel adds
// each tile's S slots in order and runs the epilogue (mirror included for a
// Hermitian product).  Positions base .. base + tail - 1 of the launch's tile
// order are the tiles the main launch (grid base) leaves out.
__device__ __forceinline__ void launch_tile(const Params& p, int pid, int& tm, int& tn) {
  if (p.herm)
    tri_coords(xcd_linear(pid, p.tiles_m * (p.tiles_m + 1) / 2), p.tiles_m, tm, tn);
  else
    tile_coords(pid, p.tiles_m, p.tiles_n, tm, tn);
}

template <typename T, bool CPLX, bool AK, bool BK, int BM, int BN, int BKT, int WM, int WN,
          int PADB>
__global__ void __launch_bounds__(64 * (BM / (16 * WM)) * (BN / (16 * WN)), 1)
gemm_tail_kernel(const Params p, int base, int S, int kc, void* part, size_t slot_bytes) {
  typedef TileLds<T, CPLX, BM, BN, BKT, PADB> L;
  typedef typename L::E E;
  __shared__ E lds[L::elems];
  const int i = blockIdx.x / S, r = blockIdx.x % S;
  int tm, tn;
  launch_tile(p, base + i, tm, tn);
  const int64_t k0 = int64_t(r) * kc * BKT;
  Params q = p;
  q.A = static_cast<const E*>(p.A) + (AK ? k0 * p.lda : k0);
  q.B = static_cast<const E*>(p.B) + (BK ? k0 * p.ldb : k0);
  q.K = min(int64_t(kc) * BKT, p.K - k0);
  gemm_tile<T, CPLX, AK, BK, false, BM, BN, BKT, WM, WN, PADB, TILE_PARTIAL>(
      q, tm, tn, false, lds, static_cast<char*>(part) + size_t(blockIdx.x) * slot_bytes);
}

template <typename T, bool CPLX, bool AK, bool BK, int BM, int BN, int BKT, int WM, int WN,
          int PADB>
__global__ void __launch_bounds__(64 * (BM / (16 * WM)) * (BN / (16 * WN)), 1)
gemm_tail_finish_kernel(const Params p, int base, int S, const void* part, size_t slot_bytes) {
  typedef TileLds<T, CPLX, BM, BN, BKT, PADB> L;
  __shared__ typename L::E lds[L::elems];
  int tm, tn;
  launch_tile(p, base + int(blockIdx.x), tm, tn);
  gemm_tile<T, CPLX, AK, BK, false, BM, BN, BKT, WM, WN, PADB, TILE_FINISH>(
      p, tm, tn, p.herm && tm != tn, lds,
      const_cast<char*>(static_cast<const char*>(part)) + size_t(blockIdx.x) * S * slot_bytes, S);
}

// Persistent grouped products: items[0 .. count) each describe one product
// and the first index of its tiles in the concatenated tile list
// (tile_begin ascending).  The grid is sized to the workgroups the device
// keeps resident; workgroup w takes tiles w, w + gridDim.x, ... until the
// list ends, so every workgroup exits after a bounded number of tiles.
struct GroupItem {
  Params p;
  int tile_begin;
  int exact;        // M, N multiples of the tile and K of the K tile
};

// Tile ranges per XCD: the workgroups with id % 8 == x (one XCD) walk the
// tiles [bound[x], bound[x + 1]) of the concatenated list, so the tiles that
// run together on an XCD are neighbours that share operand panels in its L2.
// The host cuts the list where the estimated work (K tiles per tile) reaches
// each XCD's share of the workgroups.
struct XcdSplit { int bound[9]; };

// ALL_EXACT: every product of the launch is a multiple of the tile in M, N
// and of the K tile in K, so only the unchecked tile is instantiated (fewer
// registers than a kernel that holds both).
template <typename T, bool CPLX, bool AK, bool BK, int BM, int BN, int BKT, int WM, int WN,
          int PADB, bool ALL_EXACT>
__global__ void __launch_bounds__(64 * (BM / (16 * WM)) * (BN / (16 * WN)), 1)
grouped_gemm_kernel(const GroupItem* __restrict__ items, int count, XcdSplit xs) {
  typedef TileLds<T, CPLX, BM, BN, BKT, PADB> L;
  __shared__ typename L::E lds[L::elems];
  const int x = blockIdx.x % 8;
  const int nx = (int(gridDim.x) - x + 7) / 8;      // workgroups of XCD x
  const int end = xs.bound[x + 1];
  for (int t = xs.bound[x] + int(blockIdx.x) / 8; t < end; t += nx) {
    int lo = 0, hi = count - 1;          // last item with tile_begin <= t
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
    }
    const Params p = items[lo].p;
    const int local = t - items[lo].tile_begin;
    int tm, tn;
    if (p.herm) {
      tri_coords(local, p.tiles_m, tm, tn);
    } else {                              // GROUP_M tile rows at a time, column by column
      const int per_group = GROUP_M * p.tiles_n;
      const int first_m = (local / per_group) * GROUP_M;
      const int gsize = min(p.tiles_m - first_m, GROUP_M);
      const int in_group = local % per_group;
      tm = first_m + in_group % gsize;
      tn = in_group / gsize;
    }
    const bool mirror = p.herm && tm != tn;
    if (ALL_EXACT || items[lo].exact)
      gemm_tile<T, CPLX, AK, BK, false, BM, BN, BKT, WM, WN, PADB>(p, tm, tn, mirror, lds);
    else
      gemm_tile<T, CPLX, AK, BK, true, BM, BN, BKT, WM, WN, PADB>(p, tm, tn, mirror, lds);
    __syncthreads();
  }
}

// One workgroup per tile of the concatenated list (every product a multiple
// of the tile; a Hermitian product walks its upper tile triangle and mirrors):
// no loop state across tiles, so the register count is that of the
// one-product kernel, and the hardware hands out tiles as CUs free up.
template <typename T, bool CPLX, bool AK, bool BK, int BM, int BN, int BKT, int WM, int WN,
          int PADB>
__global__ void __launch_bounds__(64 * (BM / (16 * WM)) * (BN / (16 * WN)), 1)
grouped_tile_kernel(const GroupItem* __restrict__ items, int count) {
  typedef TileLds<T, CPLX, BM, BN, BKT, PADB> L;
  __shared__ typename L::E lds[L::elems];
  const int t = blockIdx.x;
  int lo = 0, hi = count - 1;            // last item with tile_begin <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
  }
  const Params p = items[lo].p;
  const int local = t - items[lo].tile_begin;
  int tm, tn;
  if (p.herm) {
    tri_coords(local, p.tiles_m, tm, tn);
  } else {
    const int per_group = GROUP_M * p.tiles_n;
    const int first_m = (local / per_group) * GROUP_M;
    const int gsize = min(p.tiles_m - first_m, GROUP_M);
    const int in_group = local % per_group;
    tm = first_m + in_group % gsize;
    tn = in_group / gsize;
  }
  gemm_tile<T, CPLX, AK, BK, false, BM, BN, BKT, WM, WN, PADB>(p, tm, tn, p.herm && tm != tn,
                                                               lds);
}

// Tile shapes (BM, BN, BKT, WM, WN); the wave count is (BM/16WM)(BN/16WN).
struct ShapeDesc { int BM, BN, BKT, WM, WN; };

template <int BM_, int BN_, int BKT_, int WM_, int WN_, int PADB_ = 16> struct Shp {
  static constexpr int BM = BM_, BN = BN_, BKT = BKT_, WM = WM_, WN = WN_, PADB = PADB_;
  static constexpr int NT = 64 * (BM / (16 * WM)) * (BN / (16 * WN));
};

// Variant lists per element type; variant 0 is the default for every layout,
// the others serve the step and exponential layout (A row-major, B row-major).
template <typename T, bool CPLX> struct Variants;
template <> struct Variants<double, true> {
  typedef Shp<128, 64, 8, 4, 2> V0;
  typedef Shp<128, 128, 8, 4, 2> V1;
  typedef Shp<64, 64, 16, 2, 2> V2;
  typedef Shp<128, 128, 8, 2, 4> V3;
  typedef Shp<64, 64, 16, 2, 2, 0> V4;
  typedef Shp<64, 64, 16, 2, 2, 32> V5;
  typedef Shp<128, 128, 16, 4, 2> V6;
};
template <> struct Variants<double, false> {
  typedef Shp<128, 64, 16, 4, 2> V0;
  typedef Shp<128, 128, 16, 4, 2> V1;
  typedef Shp<64, 64, 16, 2, 2> V2;
  typedef Shp<128, 128, 16, 2, 4> V3;
  typedef Shp<64, 64, 16, 2, 2, 0> V4;
  typedef Shp<64, 64, 16, 2, 2, 32> V5;
  typedef Shp<128, 128, 16, 4, 2, 0> V6;
};
template <> struct Variants<float, true> {
  typedef Shp<128, 64, 16, 4, 2> V0;
  typedef Shp<128, 128, 16, 4, 2> V1;
  typedef Shp<64, 64, 16, 2, 2> V2;
  typedef Shp<128, 128, 16, 2, 4> V3;
  typedef Shp<64, 64, 16, 2, 2, 0> V4;
  typedef Shp<64, 64, 16, 2, 2, 32> V5;
  typedef Shp<128, 128, 16, 4, 2, 0> V6;
};
template <> struct Variants<float, false> {
  typedef Shp<128, 64, 16, 4, 2> V0;
  typedef Shp<128, 128, 16, 4, 2> V1;
  typedef Shp<64, 64, 16, 2, 2> V2;
  typedef Shp<128, 128, 16, 2, 4> V3;
  typedef Shp<64, 64, 16, 2, 2, 0> V4;
  typedef Shp<64, 64, 16, 2, 2, 32> V5;
  typedef Shp<128, 128, 16, 4, 2, 0> V6;
};

int device_cus();

template <typename T, bool CPLX, bool AK, bool BK, typename S>
int launch_shape(const GemmDesc& d, hipStream_t s) {
  Params p;
  p.M = d.M; p.N = d.N; p.K = d.K;
  p.A = d.A; p.lda = d.lda; p.B = d.B; p.ldb = d.ldb;
  p.C = d.C; p.ldc = d.ldc; p.Cin = d.Cin; p.ldcin = d.ldcin;
  p.alpha_re = d.alpha_re; p.alpha_im = d.alpha_im;
  p.beta_re = d.beta_re; p.beta_im = d.beta_im; p.gamma = d.gamma;
  p.conj_a = d.conj_a; p.conj_b = d.conj_b; p.c_trans = d.c_trans; p.cin_trans = d.cin_trans;
  // the triangle needs square tiles; other shapes compute every tile
  p.herm = d.herm && S::BM == S::BN && d.M == d.N;
  p.tiles_m = int((d.M + S::BM - 1) / S::BM);
  p.tiles_n = int((d.N + S::BN - 1) / S::BN);
  const int64_t tiles = p.herm ? int64_t(p.tiles_m) * (p.tiles_m + 1) / 2
                               : int64_t(p.tiles_m) * p.tiles_n;
  if (tiles <= 0) return TC_OK;
  if (tiles > (int64_t(1) << 31) - 1) { set_error("product too large"); return TC_ERR_UNSUPPORTED; }
  const bool exact = d.M % S::BM == 0 && d.N % S::BN == 0 && d.K % S::BKT == 0 && d.K > 0;
  const dim3 grid{unsigned(tiles), 1u, 1u}, block{unsigned(S::NT), 1u, 1u};
  ProfileScope prof(sizeof(T) == 8 ? TC_KERNEL_GEMM_F64 : TC_KERNEL_GEMM_F32, s);
  if (exact && d.tail_ws) {
    // a last round that would leave at least half of the CUs idle (the whole
    // product, when it has that few tiles): its tiles go split over K, one
    // workgroup and one slot of partial sums per K range of at least 4 K tiles
    const int cus = device_cus();
    const int64_t full = tiles / cus, tail = tiles % cus, kt = d.K / S::BKT;
    const size_t slot = size_t(S::BM) * S::BN * (CPLX ? 2 : 1) * sizeof(T);
    const int64_t slots = int64_t(d.tail_ws_bytes / slot);
    int R = int(std::min<int64_t>(std::min<int64_t>(cus, slots) / std::max<int64_t>(tail, 1),
                                  std::min<int64_t>(8, kt / 4)));
    if (tail > 0 && tail * 2 <= cus && R >= 2) {
      const int64_t kc = (kt + R - 1) / R;
      R = int((kt + kc - 1) / kc);         // every K range non-empty
      const int base = int(full * cus);
      if (base > 0) {
        hipLaunchKernelGGL((gemm_kernel<T, CPLX, AK, BK, false, S::BM, S::BN, S::BKT, S::WM,
                                        S::WN, S::PADB>),
                           dim3(unsigned(base)), block, 0, s, p);
        TC_TRY_HIP(hipGetLastError());
      }
      hipLaunchKernelGGL((gemm_tail_kernel<T, CPLX, AK, BK, S::BM, S::BN, S::BKT, S::WM, S::WN,
                                           S::PADB>),
                         dim3(unsigned(tail * R)), block, 0, s, p, base, R, int(kc), d.tail_ws,
                         slot);
      TC_TRY_HIP(hipGetLastError());
      hipLaunchKernelGGL((gemm_tail_finish_kernel<T, CPLX, AK, BK, S::BM, S::BN, S::BKT, S::WM,
                                                  S::WN, S::PADB>),
                         dim3(unsigned(tail)), block, 0, s, p, base, R,
                         static_cast<const void*>(d.tail_ws), slot);
      TC_TRY_HIP(hipGetLastError());
      return TC_OK;
    }
  }
  if (exact)
    hipLaunchKernelGGL((gemm_kernel<T, CPLX, AK, BK, false, S::BM, S::BN, S::BKT, S::WM, S::WN, S::PADB>),
                       grid, block, 0, s, p);
  else
    hipLaunchKernelGGL((gemm_kernel<T, CPLX, AK, BK, true, S::BM, S::BN, S::BKT, S::WM, S::WN, S::PADB>),
                       grid, block, 0, s, p);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int variant_for(int default_variant) {
  static const int env = [] {
    const char* v = getenv("TC_GEMM_VARIANT");
    return v ? atoi(v) : -1;
  }();
  return env >= 0 ? env : default_variant;
}

template <typename T, bool CPLX>
int launch2(const GemmDesc& d, hipStream_t s) {
  typedef Variants<T, CPLX> V;
  if (!d.a_kmaj && d.b_kmaj) {
    // A product of at most 16 tiles of 128 x 128 (N <= 512 when square)
    // takes 64 x 64 tiles (variant 2 in every element type): four times the
    // workgroups before the K split of its one partial round, so each
    // workgroup's share of the work is smaller, and a quarter of the padded
    // work when the product is smaller than one 128 x 128 tile.  (At N = 768
    // the K-split 128 x 128 tiles give the shorter critical path.)
    const int env = variant_for(-1);
    const int64_t t128 = ((d.M + 127) / 128) * ((d.N + 127) / 128);
    const int v = env >= 0 ? env : (t128 <= 16 ? 2 : DefaultVariant<T, CPLX>::value);
    switch (v) {
      case 1: return launch_shape<T, CPLX, false, true, typename V::V1>(d, s);
      case 2: return launch_shape<T, CPLX, false, true, typename V::V2>(d, s);
      case 3: return launch_shape<T, CPLX, false, true, typename V::V3>(d, s);
      case 4: return launch_shape<T, CPLX, false, true, typename V::V4>(d, s);
      case 5: return launch_shape<T, CPLX, false, true, typename V::V5>(d, s);
      case 6: return launch_shape<T, CPLX, false, true, typename V::V6>(d, s);
      default: return launch_shape<T, CPLX, false, true, typename V::V0>(d, s);
    }
  }
  if (d.a_kmaj && d.b_kmaj) return launch_shape<T, CPLX, true, true, typename V::V0>(d, s);
  if (d.a_kmaj && !d.b_kmaj) return launch_shape<T, CPLX, true, false, typename V::V0>(d, s);
  return launch_shape<T, CPLX, false, false, typename V::V0>(d, s);
}

template <typename S>
Params make_params(const GemmDesc& d) {
  Params p;
  p.M = d.M; p.N = d.N; p.K = d.K;
  p.A = d.A; p.lda = d.lda; p.B = d.B; p.ldb = d.ldb;
  p.C = d.C; p.ldc = d.ldc; p.Cin = d.Cin; p.ldcin = d.ldcin;
  p.alpha_re = d.alpha_re; p.alpha_im = d.alpha_im;
  p.beta_re = d.beta_re; p.beta_im = d.beta_im; p.gamma = d.gamma;
  p.conj_a = d.conj_a; p.conj_b = d.conj_b; p.c_trans = d.c_trans; p.cin_trans = d.cin_trans;
  p.herm = d.herm && S::BM == S::BN && d.M == d.N;
  p.tiles_m = int((d.M + S::BM - 1) / S::BM);
  p.tiles_n = int((d.N + S::BN - 1) / S::BN);
  return p;
}

template <typename S>
int build_items(const std::vector<GemmDesc>& ds, std::vector<GroupItem>& items, int* total) {
  int64_t t = 0;
  items.clear();
  for (const GemmDesc& d : ds) {
    if (d.a_kmaj || !d.b_kmaj || !d.complex) {
      set_error("grouped products take A and B row-major, complex");
      return TC_ERR_UNSUPPORTED;
    }
    GroupItem it;
    it.p = make_params<S>(d);
    it.tile_begin = int(t);
    it.exact = d.M % S::BM == 0 && d.N % S::BN == 0 && d.K % S::BKT == 0 && d.K > 0;
    t += it.p.herm ? int64_t(it.p.tiles_m) * (it.p.tiles_m + 1) / 2
                   : int64_t(it.p.tiles_m) * it.p.tiles_n;
    items.push_back(it);
  }
  if (t > (int64_t(1) << 30)) { set_error("too many tiles in one group"); return TC_ERR_UNSUPPORTED; }
  *total = int(t);
  return TC_OK;
}

int device_cus() {
  static int cus = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
    return n > 0 ? n : 256;
  }();
  return cus;
}

}  // namespace

// Cuts the concatenated tile list into 8 ranges whose work is proportional to
// each XCD's workgroup count (workgroup w runs on XCD w % 8); a tile's work is
// its K tiles plus one for its epilogue.
void xcd_split(const std::vector<int64_t>& begins, const std::vector<int64_t>& tiles,
               const std::vector<int64_t>& ks, int64_t total_tiles, int grid, int bkt,
               int bound[9]) {
  double total_work = 0.0;
  for (size_t i = 0; i < tiles.size(); ++i)
    total_work += double(tiles[i]) * double((ks[i] + bkt - 1) / bkt + 1);
  bound[0] = 0;
  size_t item = 0;
  int64_t t = 0;                 // first tile not yet assigned
  double done = 0.0;             // work of tiles [0, t)
  int wg_before = 0;
  for (int x = 0; x < 8; ++x) {
    wg_before += (grid - x + 7) / 8;
    const double target = total_work * double(wg_before) / double(grid);
    while (item < tiles.size()) {
      const int64_t last = begins[item] + tiles[item];
      const double w = double((ks[item] + bkt - 1) / bkt + 1);
      if (t >= last) { ++item; continue; }
      const int64_t need = int64_t(std::ceil((target - done) / w - 1e-9));
      if (need <= 0) break;
      const int64_t take = std::min<int64_t>(need, last - t);
      t += take;
      done += double(take) * w;
      if (t < last) break;
    }
    // the last XCD that has workgroups takes whatever rounding left over
    bound[x + 1] = x >= std::min(grid, 8) - 1 ? int(total_tiles)
                                              : int(std::min<int64_t>(t, total_tiles));
  }
}

namespace {

template <typename T, typename S, bool ALL_EXACT>
int grouped_launch_t(const GroupedProducts& g, hipStream_t s) {
  auto kern = grouped_gemm_kernel<T, true, false, true, S::BM, S::BN, S::BKT, S::WM, S::WN,
                                  S::PADB, ALL_EXACT>;
  static int per_cu = -1;
  if (per_cu < 0) {
    int nb = 0;
    TC_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, S::NT, 0));
    per_cu = nb > 0 ? nb : 1;
  }
  const int64_t resident = int64_t(device_cus()) * per_cu;
  const int grid = int(std::min<int64_t>(g.total_tiles, resident));
  if (grid <= 0) return TC_OK;
  XcdSplit xs;
  xcd_split(g.begins, g.tiles, g.ks, g.total_tiles, grid, S::BKT, xs.bound);
  ProfileScope prof(sizeof(T) == 8 ? TC_KERNEL_GEMM_F64 : TC_KERNEL_GEMM_F32, s);
  hipLaunchKernelGGL(kern, dim3(unsigned(grid)), dim3(unsigned(S::NT)), 0, s,
                     static_cast<const GroupItem*>(g.items_dev), g.count, xs);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

}  // namespace

size_t grouped_bytes(int count) { return size_t(count) * sizeof(GroupItem); }

int grouped_build(const std::vector<GemmDesc>& ds, bool f64, int variant, void* items_dev,
                  GroupedProducts* g, hipStream_t s) {
  std::vector<GroupItem> items;
  int total = 0;
  if (variant != 1 && variant != 2) { set_error("grouped tile variant must be 1 or 2"); return TC_ERR_INVALID_ARGUMENT; }
  typedef Variants<double, true> VD;
  typedef Variants<float, true> VF;
  int rc;
  if (f64)
    rc = variant == 1 ? build_items<VD::V6>(ds, items, &total) : build_items<VD::V2>(ds, items, &total);
  else
    rc = variant == 1 ? build_items<VF::V1>(ds, items, &total) : build_items<VF::V2>(ds, items, &total);
  TC_RETURN_IF(rc);
  g->variant = variant;
  g->f64 = f64;
  g->count = int(items.size());
  g->total_tiles = total;
  g->items_dev = items_dev;
  g->all_exact = true;
  for (const GroupItem& it : items) g->all_exact = g->all_exact && it.exact;
  g->begins.clear(); g->tiles.clear(); g->ks.clear();
  for (size_t i = 0; i < items.size(); ++i) {
    const int64_t next = i + 1 < items.size() ? items[i + 1].tile_begin : total;
    g->begins.push_back(items[i].tile_begin);
    g->tiles.push_back(next - items[i].tile_begin);
    g->ks.push_back(items[i].p.K);
  }
  if (!items.empty()) {
    // one synchronous upload per call; the descriptors are reused by every step
    TC_TRY_HIP(hipMemcpyAsync(items_dev, items.data(), items.size() * sizeof(GroupItem),
                              hipMemcpyHostToDevice, s));
    TC_TRY_HIP(hipStreamSynchronize(s));
  }
  return TC_OK;
}

template <typename T, typename S>
int grouped_launch_tiles(const GroupedProducts& g, hipStream_t s) {
  auto kern = grouped_tile_kernel<T, true, false, true, S::BM, S::BN, S::BKT, S::WM, S::WN,
                                  S::PADB>;
  ProfileScope prof(sizeof(T) == 8 ? TC_KERNEL_GEMM_F64 : TC_KERNEL_GEMM_F32, s);
  hipLaunchKernelGGL(kern, dim3(unsigned(g.total_tiles)), dim3(unsigned(S::NT)), 0, s,
                     static_cast<const GroupItem*>(g.items_dev), g.count);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

template <typename T, typename S>
int grouped_launch_any(const GroupedProducts& g, hipStream_t s) {
  if (g.all_exact && !g.persistent) return grouped_launch_tiles<T, S>(g, s);
  return g.all_exact ? grouped_launch_t<T, S, true>(g, s) : grouped_launch_t<T, S, false>(g, s);
}

int grouped_run(const GroupedProducts& g, hipStream_t s) {
  if (g.count == 0 || g.total_tiles == 0) return TC_OK;
  if (g.f64)
    return g.variant == 1 ? grouped_launch_any<double, Variants<double, true>::V6>(g, s)
                          : grouped_launch_any<double, Variants<double, true>::V2>(g, s);
  return g.variant == 1 ? grouped_launch_any<float, Variants<float, true>::V1>(g, s)
                        : grouped_launch_any<float, Variants<float, true>::V2>(g, s);
}

int gemm_f64(const GemmDesc& d, hipStream_t s) {
  if (d.M == 0 || d.N == 0) return TC_OK;
  return d.complex ? launch2<double, true>(d, s) : launch2<double, false>(d, s);
}

int gemm_f32(const GemmDesc& d, hipStream_t s) {
  if (d.M == 0 || d.N == 0) return TC_OK;
  return d.complex ? launch2<float, true>(d, s) : launch2<float, false>(d, s);
}

}  // namespace tcm
