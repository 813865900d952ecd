// Split-BF16 complex products: every real operand x is carried as two bfloat16
// values hi = rne(x), lo = rne(x - hi); a real product a*b is formed as
// hi_a hi_b + hi_a lo_b + lo_a hi_b on BF16 MFMA with FP32 accumulation.
#pragma once
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

// General split product on c64 operands (kernel-level entry point).
struct SplitGemmPlan {
  Planes4 A, B;
};
void split_gemm_plan(Arena& ar, int64_t M, int64_t N, int64_t K, SplitGemmPlan* p);
int split_gemm(const GemmDesc& d, const SplitGemmPlan& p, hipStream_t s);

}  // namespace tcm
