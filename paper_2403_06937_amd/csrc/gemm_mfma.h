// Dense MFMA matrix products for FP64 and FP32 (complex and real).
#pragma once
#include <vector>

#include "common.h"

namespace tcm {

// C = alpha * op(A) op(B) + beta * Cin + gamma * I   (M x N, inner dimension K)
//
// Operand storage (element type: cplx<T> if complex else T):
//   a_kmaj: element (m, k) of op(A) at A[k * lda + m]  ("K-major"),
//           else at A[m * lda + k]                      (row-major).
//   b_kmaj: element (k, n) of op(B) at B[k * ldb + n]   (row-major),
//           else at B[n * ldb + k]                      ("N-major", i.e. B^T stored).
//   conj_a / conj_b conjugate the operand while it is staged.
//   c_trans: element (m, n) of the result goes to C[n * ldc + m] instead of
//            C[m * ldc + n].
//   cin_trans: element (m, n) of Cin is read from Cin[n * ldcin + m] instead of
//            Cin[m * ldcin + n].  Cin may alias C only with the same layout.
struct GemmDesc {
  int64_t M = 0, N = 0, K = 0;
  const void* A = nullptr; int64_t lda = 0; bool a_kmaj = false; bool conj_a = false;
  const void* B = nullptr; int64_t ldb = 0; bool b_kmaj = true;  bool conj_b = false;
  void* C = nullptr; int64_t ldc = 0; bool c_trans = false;
  const void* Cin = nullptr; int64_t ldcin = 0; bool cin_trans = false;
  double alpha_re = 1.0, alpha_im = 0.0;
  double beta_re = 0.0, beta_im = 0.0;
  double gamma = 0.0;       // added to the real part of the diagonal (m == n)
  bool complex = true;
  // The caller guarantees that C is Hermitian (symmetric when real), M == N:
  // only the tiles on and above the tile diagonal are computed, and each
  // off-diagonal tile also stores its conjugate transpose.
  bool herm = false;
  // optional device buffer for a product's last round split over K (partial
  // sums of its tiles); nullptr: one pass per tile
  void* tail_ws = nullptr; size_t tail_ws_bytes = 0;
};

int gemm_f64(const GemmDesc& d, hipStream_t s);   // elements double / cplx<double>
int gemm_f32(const GemmDesc& d, hipStream_t s);   // elements float / cplx<float>

// Grouped complex products (A and B row-major, the layout of the time step):
// every product of the group shares one tile shape and one persistent launch.
//   variant 1: 128 x 128 tiles, 8 waves (K tile 16 for FP64, as the one-product
//              FP64 default);  variant 2: 64 x 64 tiles, 4 waves.
struct GroupedProducts {
  int variant = 1;
  bool f64 = false;
  int count = 0;
  int total_tiles = 0;
  bool all_exact = false;      // every product a multiple of the tile (unchecked kernel)
  bool persistent = true;      // false (all_exact only): one workgroup per tile
  void* items_dev = nullptr;   // device copy of the descriptors (grouped_bytes(count))
  // host copy of each product's first tile, tile count and K (the launch
  // splits the tile list over the XCDs by work)
  std::vector<int64_t> begins, tiles, ks;
};
size_t grouped_bytes(int count);
// Builds the descriptors of ds and uploads them to items_dev (synchronises s).
int grouped_build(const std::vector<GemmDesc>& ds, bool f64, int variant, void* items_dev,
                  GroupedProducts* g, hipStream_t s);
int grouped_run(const GroupedProducts& g, hipStream_t s);
// Tile ranges [bound[x], bound[x + 1]) of the 8 XCDs for a persistent launch
// of grid workgroups (K tile bkt).
void xcd_split(const std::vector<int64_t>& begins, const std::vector<int64_t>& tiles,
               const std::vector<int64_t>& ks, int64_t total_tiles, int grid, int bkt,
               int bound[9]);

// Tile variant for an N x N x N complex product, from the autotuner's table
// (or its defaults when no tuning ran and no cache file is set).
int tile_variant_for(int64_t N, bool f64);

}  // namespace tcm
