// Split-BF16 complex products: every real operand x is carried as two bfloat16
// values hi = rne(x), lo = rne(x - hi); a real product a*b is formed as
// hi_a hi_b + hi_a lo_b + lo_a hi_b on BF16 MFMA with FP32 accumulation.
#pragma once
#include <vector>

#include "common.h"
#include "gemm_mfma.h"

namespace tcm {

// Plane order inside a 4-plane operand.
enum { PL_RH = 0, PL_RL = 1, PL_IH = 2, PL_IL = 3 };

// Tile of the split product kernel; padded plane dimensions are multiples of it.
constexpr int SPLIT_BM = 128, SPLIT_BN = 128, SPLIT_BK = 32;

inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// A 4-plane operand of rows x ld bf16 per plane (K-contiguous rows, ld a
// multiple of SPLIT_BK), the planes interleaved by 32-deep K slices: element k
// of row r of plane q sits at base + plane_offset(ld, r, k, q), so the four
// planes of one row's K slice are 256 contiguous bytes (two cache lines).
struct Planes4 {
  uint16_t* base = nullptr;
  int64_t ld = 0, rows = 0;
};
__host__ __device__ inline int64_t plane_offset(int64_t ld, int64_t r, int64_t k, int q) {
  return r * 4 * ld + (k / SPLIT_BK) * (4 * SPLIT_BK) + q * SPLIT_BK + k % SPLIT_BK;
}

// Planes used by the split-BF16 time step of one N x N instance (padded to Np).
struct SplitPlanes {
  int64_t N = 0, Np = 0;
  Planes4 opA;   // split(op)            rows m, K-contiguous: A operand of X = op rho
  Planes4 opB;   // split(conj(op)^T)    rows n: B operand of rho' = X conj(op)
  Planes4 X;     // split(X)             rows m: A operand of the second product
  Planes4 Rt;    // split(rho^T)         rows n: B operand of the first product
  float* tail_acc = nullptr;   // partial sums of a product's last round split
  int tail_slots = 0;          // over K: slots of 128 x 128 complex FP32 (or none)
};

void split_plan(Arena& ar, int64_t N, SplitPlanes* p);
// opA / opB from the c64 operand (U or D); clears the padding.
int split_operand(const c64* op, int64_t ld, int64_t N, const SplitPlanes& p, hipStream_t s);
// Rt from the c64 master state (after preparation and after each renormalisation).
int split_state(const c64* rho, int64_t ld, int64_t N, const SplitPlanes& p, hipStream_t s);
// One step rho <- op rho op^dag (lab) or rho <- (I + D) rho (I + D)^dag (rotating).
// herm: rho is Hermitian, so the second product forms its upper tile triangle
// and mirrors it.
int step_split(c64* rho, int64_t ldr, c64* X, int64_t ldx, int64_t N, bool rotating, bool herm,
               const SplitPlanes& p, hipStream_t s);

// Planes of rows x ld bf16 (ld a multiple of SPLIT_BK) carved from a workspace.
Planes4 split_take_planes(Arena& ar, int64_t rows, int64_t ld);
// All P.rows x P.ld entries of P from the c64 matrix src (R x C valid, element
// (r, c) at src[r*ld + c], or src[c*ld + r] when trans), conjugated if conj,
// zero outside.
int split_matrix(const c64* src, int64_t ld, int64_t R, int64_t C, bool trans, bool conj,
                 const Planes4& P, hipStream_t s);

// Split products of whole 128 x 128 tiles launched together, one workgroup
// per tile (the excitation-sector blocks of a step).  A and B point at the
// product's first row and K offset inside 4-plane operands (K offsets are
// multiples of SPLIT_BK); the result goes to any of the FP32 Cf and the hi/lo
// planes P (row-major, or transposed when p_trans), as in step_split.
struct SplitProduct {
  const uint16_t* A = nullptr; int64_t lda = 0;   // lda, ldb, ldp: padded K extents of the planes
  const uint16_t* B = nullptr; int64_t ldb = 0;
  int64_t M = 0, N = 0, Kp = 0;
  float ar = 1.f, ai = 0.f, br = 0.f, bi = 0.f;   // alpha, beta
  const c64* Cin = nullptr; int64_t ldcin = 0;
  c64* Cf = nullptr; int64_t ldcf = 0;
  uint16_t* P = nullptr; int64_t ldp = 0; bool p_trans = false;
};
struct SplitGrouped {
  int count = 0;
  int total_tiles = 0;
  void* items_dev = nullptr;
};
size_t split_grouped_bytes(int count);
// Uploads the descriptors (synchronises s).
int split_grouped_build(const std::vector<SplitProduct>& ps, void* items_dev, SplitGrouped* g,
                        hipStream_t s);
int split_grouped_run(const SplitGrouped& g, hipStream_t s);

// General split product on c64 operands (kernel-level entry point).
struct SplitGemmPlan {
  Planes4 A, B;
};
void split_gemm_plan(Arena& ar, int64_t M, int64_t N, int64_t K, SplitGemmPlan* p);
int split_gemm(const GemmDesc& d, const SplitGemmPlan& p, hipStream_t s);

}  // namespace tcm
