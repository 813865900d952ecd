// tc_evolve_backward: adjoint gradient of the final atomic excitation with
// respect to the couplings g_i and detunings delta_i.
//
// L = Tr(O rho_S), rho_s = U rho_{s-1} U^dag, U = exp(A), A = -i H dt.
// Define O_S = O and O_{s-1} = U^dag O_s U.  Then
//   dL = 2 Re Tr(dU M),   M = sum_{s=1}^{S} rho_{s-1} U^dag O_s,
// dU = L(A, dA) is the Frechet derivative of exp, and the trace pairing
// Tr(L(A, E) M) = Tr(E L(A, M)) gives, with G = L(A, M),
//   dL/dtheta = 2 Re Tr(dA/dtheta G),  dA/dtheta = -i dt dH/dtheta.
// Backward pass per step: Y = U^dag O_s, M += rho_{s-1} Y, O_{s-1} = Y U;
// rho_{s-1} is recomputed segment by segment from the forward checkpoints.
// G is the upper-right block of exp([[A, M], [0, A]]) (block-triangular
// exponential), formed by shifting A by its spectral centre, scaling by 2^-s,
// a degree-18 block Taylor series and s block squarings, all in FP64.
//
// The sweep runs in the rotating frame rho~ = e^{i w_c N t} rho e^{-i w_c N t}
// (N = total excitation number, which commutes with H and O): U~ =
// e^{i w_c N dt} U = exp(-i H' dt) with H' = H - w_c N, and dH'/dtheta =
// dH/dtheta, so the same formulas hold with U~, A~ = -i H' dt and rotating-
// frame states; L = Tr(O rho~_S) because O commutes with N.  Every product is
// written with U~ = I + D (Y = O + D^dag O, O' = Y + Y D, rho' = X + X conj(D)
// with X = rho + D rho), so in FP32 only the small D is rounded.
#include <cmath>
#include <string>
#include <vector>
#include <algorithm>

#include "common.h"
#include "gemm_mfma.h"
#include "kernels.h"

namespace tcm {
namespace {

constexpr int FRECHET_DEGREE = 18;   // ||B|| <= 1/2: first omitted term < 2e-23 relative

// Slots for the partial sums of a product's last round split over K (FP64
// tiles of 128 x 128 complex elements; an FP32 product fits twice as many).
struct TailWs {
  void* p = nullptr;
  size_t bytes = 0;
};

struct BwdLayout {
  bool f64 = true;          // product precision of the backward sweep
  size_t eb = 16;           // element bytes of the sweep
  int64_t seg = 0;          // states per segment buffer
  void* D = nullptr;        // U~ - I in the sweep precision
  void* segbuf = nullptr;   // [seg][N][N] states rho_{s0} .. rho_{s0+seg-1}
  void* X = nullptr;        // forward step temporary / rho_S
  void* O = nullptr;
  void* Y = nullptr;
  void* T = nullptr;        // rho Y (FP32 sweep only)
  c128* M = nullptr;
  c128* Bs = nullptr;
  c128 *P0 = nullptr, *P1 = nullptr, *Q0 = nullptr, *Q1 = nullptr;
  double* scratch = nullptr;
  TailWs tail;
};

void bwd_layout(Arena& ar, int64_t N, const tc_evolve_opts& o, BwdLayout* L) {
  const size_t NN = size_t(N) * size_t(N);
  L->f64 = o.gemm_mode == TC_GEMM_F64;
  L->eb = L->f64 ? 16 : 8;
  L->seg = o.checkpoint_every;
  L->D = ar.take(NN * L->eb);
  L->segbuf = ar.take(size_t(L->seg) * NN * L->eb);
  L->X = ar.take(NN * L->eb);
  L->O = ar.take(NN * L->eb);
  L->Y = ar.take(NN * L->eb);
  if (!L->f64) L->T = ar.take(NN * 8);
  L->M = static_cast<c128*>(ar.take(NN * 16));
  L->Bs = static_cast<c128*>(ar.take(NN * 16));
  L->P0 = static_cast<c128*>(ar.take(NN * 16));
  L->P1 = static_cast<c128*>(ar.take(NN * 16));
  L->Q0 = static_cast<c128*>(ar.take(NN * 16));
  L->Q1 = static_cast<c128*>(ar.take(NN * 16));
  L->scratch = static_cast<double*>(ar.take(8 * sizeof(double)));
  // 8 slots per tile of the N x N product, at most 256, from 2 tile rows on
  const int64_t t = (N + 127) / 128;
  if (t >= 2) {
    L->tail.bytes = size_t(std::min<int64_t>(256, 8 * t * t)) * 128 * 128 * 16;
    L->tail.p = ar.take(L->tail.bytes);
  }
}

// General complex product in the sweep precision: C = alpha op(A) op(B) + beta C.
int cgemm(const TailWs& tw, bool f64, int64_t N, const void* A, int64_t lda, bool a_kmaj,
          bool conj_a, const void* B, int64_t ldb, bool b_kmaj, bool conj_b, void* C, int64_t ldc,
          double alpha_re, double beta_re, hipStream_t s) {
  GemmDesc d;
  d.tail_ws = tw.p; d.tail_ws_bytes = tw.bytes;
  d.M = d.N = d.K = N;
  d.A = A; d.lda = lda; d.a_kmaj = a_kmaj; d.conj_a = conj_a;
  d.B = B; d.ldb = ldb; d.b_kmaj = b_kmaj; d.conj_b = conj_b;
  d.C = C; d.ldc = ldc;
  d.alpha_re = alpha_re;
  if (beta_re != 0.0) { d.Cin = C; d.ldcin = ldc; d.beta_re = beta_re; }
  return f64 ? gemm_f64(d, s) : gemm_f32(d, s);
}

// C = op(A) op(B) + Cin in the sweep precision (Cin must not alias C); herm:
// C is Hermitian, so only its upper tile triangle is multiplied and mirrored.
int cgemm_in(const TailWs& tw, bool f64, int64_t N, const void* A, int64_t lda, bool a_kmaj,
             bool conj_a, const void* B, int64_t ldb, bool b_kmaj, bool conj_b, void* C,
             int64_t ldc, const void* Cin, hipStream_t s, bool herm = false) {
  GemmDesc d;
  d.tail_ws = tw.p; d.tail_ws_bytes = tw.bytes;
  d.herm = herm;
  d.M = d.N = d.K = N;
  d.A = A; d.lda = lda; d.a_kmaj = a_kmaj; d.conj_a = conj_a;
  d.B = B; d.ldb = ldb; d.b_kmaj = b_kmaj; d.conj_b = conj_b;
  d.C = C; d.ldc = ldc;
  d.Cin = Cin; d.ldcin = N; d.beta_re = 1.0;
  return f64 ? gemm_f64(d, s) : gemm_f32(d, s);
}

// FP64 complex product with complex alpha and a real diagonal shift gamma.
int zgemm64(const TailWs& tw, int64_t N, const c128* A, const c128* B, c128* C, double ar,
            double beta, const c128* Cin, double gamma, hipStream_t s) {
  GemmDesc d;
  d.tail_ws = tw.p; d.tail_ws_bytes = tw.bytes;
  d.M = d.N = d.K = N;
  d.A = A; d.lda = N; d.a_kmaj = false;
  d.B = B; d.ldb = N; d.b_kmaj = true;
  d.C = C; d.ldc = N;
  d.alpha_re = ar;
  if (beta != 0.0) { d.Cin = Cin; d.ldcin = N; d.beta_re = beta; }
  d.gamma = gamma;
  return gemm_f64(d, s);
}

char* state_at(const BwdLayout& L, int64_t N, int64_t k) {
  return static_cast<char*>(L.segbuf) + size_t(k) * size_t(N) * size_t(N) * L.eb;
}

// ------------------------------------------------------------ by sectors
// O and every d(H)/d(theta) conserve the excitation number, and so do H and
// U: with O = (+)_k O_k, L = sum_k Tr(O_k U_k^S rho0_kk U_k^dag^S) depends on
// the diagonal blocks rho0_kk only, and the adjoint splits into one
// independent sweep per sector on d_k x d_k blocks (M_k, G_k = L(A_k, M_k)).
// Blocks are padded to multiples of 64 (zeros) and stored one after another;
// every product of a sweep step is one grouped launch over the blocks.
struct SecBwd {
  int nb = 0;
  int64_t Np = 0, total = 0;           // padded positions, elements of one block set
  std::vector<int64_t> d, dim, spo, boff;
  int64_t* dboff = nullptr; int64_t* dspo = nullptr; int64_t* ddim = nullptr;
  int32_t* perm = nullptr;             // [Np] basis state of a position, -1 = padding
  int32_t* inv = nullptr;              // [N] position of a basis state
  void* D = nullptr;                   // blocks of U~ - I (sweep precision)
  void* seg = nullptr;                 // C block sets: rho_{s0} .. rho_{s0+C-1}
  void *X = nullptr, *O = nullptr, *Y = nullptr, *T = nullptr, *diag = nullptr;
  c128 *M = nullptr, *Bs = nullptr, *P0 = nullptr, *P1 = nullptr, *Q0 = nullptr, *Q1 = nullptr;
  c128* G = nullptr;                   // N x N, G scattered for the gradient traces
  char* items = nullptr;               // descriptors of every grouped product
  int ngroups = 0;
  BlockTable table() const { return BlockTable{dboff, dspo, ddim, perm, nb}; }
};

// forward 2C, backward C + 2, Horner 3 x FRECHET_DEGREE, squarings 6
int sec_groups(int64_t C) { return int(3 * C + 2 + 3 * FRECHET_DEGREE + 6); }

void sec_layout(Arena& ar, const ModelArgs& a, int64_t N, const tc_evolve_opts& o, SecBwd* L) {
  const bool f64 = o.gemm_mode == TC_GEMM_F64;
  const size_t eb = f64 ? 16 : 8;
  const int n = a.n, c = a.c, nb = n + c + 1;
  std::vector<int64_t> binom(n + 1, 0);
  binom[0] = 1;
  for (int i = 1; i <= n; ++i)
    for (int j = i; j >= 1; --j) binom[j] += binom[j - 1];
  L->nb = nb;
  L->d.assign(nb, 0); L->dim.assign(nb, 0); L->spo.assign(nb, 0); L->boff.assign(nb + 1, 0);
  int64_t pos = 0;
  for (int k = 0; k < nb; ++k) {
    for (int mm = std::max(0, k - n); mm <= std::min(k, c); ++mm) L->d[k] += binom[k - mm];
    L->dim[k] = (L->d[k] + 63) / 64 * 64;
    L->spo[k] = pos;
    pos += L->dim[k];
    L->boff[k + 1] = L->boff[k] + L->dim[k] * L->dim[k];
  }
  L->Np = pos;
  L->total = L->boff[nb];
  const size_t T = size_t(L->total);
  L->dboff = static_cast<int64_t*>(ar.take(size_t(nb + 1) * 8));
  L->dspo = static_cast<int64_t*>(ar.take(size_t(nb) * 8));
  L->ddim = static_cast<int64_t*>(ar.take(size_t(nb) * 8));
  L->perm = static_cast<int32_t*>(ar.take(size_t(pos) * 4));
  L->inv = static_cast<int32_t*>(ar.take(size_t(N) * 4));
  L->D = ar.take(T * eb);
  L->seg = ar.take(size_t(o.checkpoint_every) * T * eb);
  L->X = ar.take(T * eb);
  L->O = ar.take(T * eb);
  L->Y = ar.take(T * eb);
  if (!f64) L->T = ar.take(T * 8);
  L->diag = ar.take(size_t(pos) * eb);
  L->M = static_cast<c128*>(ar.take(T * 16));
  L->Bs = static_cast<c128*>(ar.take(T * 16));
  L->P0 = static_cast<c128*>(ar.take(T * 16));
  L->P1 = static_cast<c128*>(ar.take(T * 16));
  L->Q0 = static_cast<c128*>(ar.take(T * 16));
  L->Q1 = static_cast<c128*>(ar.take(T * 16));
  L->G = static_cast<c128*>(ar.take(size_t(N) * size_t(N) * 16));
  L->ngroups = sec_groups(o.checkpoint_every);
  L->items = static_cast<char*>(ar.take(size_t(L->ngroups) * grouped_bytes(nb)));
}

int backward_by_sectors(const ModelArgs& a, const double* H, int64_t ldh, const c128* U,
                        int64_t ldu, int64_t N, const tc_evolve_opts& oo, const void* checkpoints,
                        double lam_lo, double lam_hi, double* loss_out, double* grad_g,
                        double* grad_delta, Arena& ar, hipStream_t s) {
  SecBwd L;
  sec_layout(ar, a, N, oo, &L);
  const bool f64 = oo.gemm_mode == TC_GEMM_F64;
  const size_t eb = f64 ? 16 : 8;
  const int nb = L.nb, n = a.n;
  const int64_t S = oo.steps, C = oo.checkpoint_every, Np = L.Np;
  // index maps of the padded sorted order and the block table
  {
    std::vector<int32_t> perm(Np, -1), inv(N);
    std::vector<int64_t> next(L.spo);
    const uint64_t mask = (uint64_t(1) << n) - 1;
    for (int64_t st = 0; st < N; ++st) {
      const int k = int(st >> n) + __builtin_popcountll(uint64_t(st) & mask);
      const int64_t p = next[k]++;
      perm[p] = int32_t(st);
      inv[st] = int32_t(p);
    }
    TC_TRY_HIP(hipMemcpyAsync(L.perm, perm.data(), size_t(Np) * 4, hipMemcpyHostToDevice, s));
    TC_TRY_HIP(hipMemcpyAsync(L.inv, inv.data(), size_t(N) * 4, hipMemcpyHostToDevice, s));
    TC_TRY_HIP(hipMemcpyAsync(L.dboff, L.boff.data(), size_t(nb + 1) * 8, hipMemcpyHostToDevice, s));
    TC_TRY_HIP(hipMemcpyAsync(L.dspo, L.spo.data(), size_t(nb) * 8, hipMemcpyHostToDevice, s));
    TC_TRY_HIP(hipMemcpyAsync(L.ddim, L.dim.data(), size_t(nb) * 8, hipMemcpyHostToDevice, s));
    TC_TRY_HIP(hipStreamSynchronize(s));   // host vectors of this scope
  }
  const BlockTable tb = L.table();
  auto blk = [&](void* base, int k, size_t esz) {
    return static_cast<void*>(static_cast<char*>(base) + size_t(L.boff[k]) * esz);
  };
  auto slot = [&](int64_t k) {
    return static_cast<void*>(static_cast<char*>(L.seg) + size_t(k) * size_t(L.total) * eb);
  };
  // D_k = e^{i w_c k dt} U_k - I
  for (int k = 0; k < nb; ++k) {
    const double ph = a.omega_c * double(k) * oo.dt;
    if (f64)
      TC_RETURN_IF(launch_gather_c128_c128(U, ldu, L.perm, L.spo[k], L.spo[k], L.dim[k], L.dim[k],
                                           std::cos(ph), std::sin(ph), true,
                                           static_cast<c128*>(blk(L.D, k, 16)), L.dim[k], s));
    else
      TC_RETURN_IF(launch_gather_c128_c64(U, ldu, L.perm, L.spo[k], L.spo[k], L.dim[k], L.dim[k],
                                          std::cos(ph), std::sin(ph), true,
                                          static_cast<c64*>(blk(L.D, k, 8)), L.dim[k], s));
  }
  // grouped block products: C_k = alpha op(A_k) op(B_k) + beta Cin_k + gamma I
  char* items = L.items;
  auto group = [&](const void* A, bool ca, const void* B, bool cb, void* Cm, const void* Cin,
                   double alpha, double beta, double gamma, bool herm, bool g64,
                   GroupedProducts* g) -> int {
    const size_t e = g64 ? 16 : 8;
    std::vector<GemmDesc> ds;
    for (int k = 0; k < nb; ++k) {
      GemmDesc dd;
      dd.M = dd.N = dd.K = L.dim[k];
      dd.A = blk(const_cast<void*>(A), k, e); dd.lda = L.dim[k]; dd.a_kmaj = false; dd.conj_a = ca;
      dd.B = blk(const_cast<void*>(B), k, e); dd.ldb = L.dim[k]; dd.b_kmaj = true; dd.conj_b = cb;
      dd.C = blk(Cm, k, e); dd.ldc = L.dim[k];
      dd.alpha_re = alpha;
      if (beta != 0.0) {
        dd.Cin = blk(const_cast<void*>(Cin), k, e); dd.ldcin = L.dim[k]; dd.beta_re = beta;
      }
      dd.gamma = gamma;
      dd.herm = herm;
      ds.push_back(dd);
    }
    if (items + grouped_bytes(nb) > L.items + size_t(L.ngroups) * grouped_bytes(nb)) {
      set_error("sector adjoint: descriptor buffer exhausted");
      return TC_ERR_INVALID_ARGUMENT;
    }
    TC_RETURN_IF(grouped_build(ds, g64, 2, items, g, s));
    items += grouped_bytes(nb);
    g->persistent = false;
    return TC_OK;
  };
  // forward step from slot k - 1 into slot k (k = 1 .. C - 1) or into Y (k = C):
  // X = src + D src, dst = X + X conj(D)
  std::vector<GroupedProducts> f1(C + 1), f2(C + 1), gm(C);
  for (int64_t k = 1; k <= C; ++k) {
    void* src = slot(k - 1);
    void* dst = k < C ? slot(k) : L.Y;
    TC_RETURN_IF(group(L.D, false, src, false, L.X, src, 1.0, 1.0, 0.0, false, f64, &f1[k]));
    TC_RETURN_IF(group(L.X, false, L.D, true, dst, L.X, 1.0, 1.0, 0.0, true, f64, &f2[k]));
  }
  // backward step: Y = O + conj(D) O (D symmetric, so conj(D) = D^dag); M += rho Y;
  // O = Y + Y D (Hermitian)
  GroupedProducts gy, go;
  TC_RETURN_IF(group(L.D, true, L.O, false, L.Y, L.O, 1.0, 1.0, 0.0, false, f64, &gy));
  for (int64_t k = 0; k < C; ++k) {
    if (f64) TC_RETURN_IF(group(slot(k), false, L.Y, false, L.M, L.M, 1.0, 1.0, 0.0, false, true, &gm[k]));
    else TC_RETURN_IF(group(slot(k), false, L.Y, false, L.T, nullptr, 1.0, 0.0, 0.0, false, false, &gm[k]));
  }
  TC_RETURN_IF(group(L.Y, false, L.D, false, L.O, L.Y, 1.0, 1.0, 0.0, true, f64, &go));
  // Frechet derivative (FP64): Horner on [[P, Q], [0, P]] (step k scales by
  // 1/k, so each step has its own descriptors) and squarings, P / Q buffers
  // alternating between the two copies
  c128* Pb[2] = {L.P0, L.P1};
  c128* Qb[2] = {L.Q0, L.Q1};
  std::vector<GroupedProducts> hq1(FRECHET_DEGREE + 1), hq2(FRECHET_DEGREE + 1),
      hp(FRECHET_DEGREE + 1);
  int par = 0;
  for (int k = FRECHET_DEGREE; k >= 1; --k, par ^= 1) {
    c128 *P = Pb[par], *Pn = Pb[par ^ 1], *Q = Qb[par], *Qn = Qb[par ^ 1];
    const double inv = 1.0 / double(k);
    TC_RETURN_IF(group(L.Bs, false, Q, false, Qn, nullptr, inv, 0.0, 0.0, false, true, &hq1[k]));
    TC_RETURN_IF(group(L.M, false, P, false, Qn, Qn, inv, 1.0, 0.0, false, true, &hq2[k]));
    TC_RETURN_IF(group(L.Bs, false, P, false, Pn, nullptr, inv, 0.0, 1.0, false, true, &hp[k]));
  }
  const int par_after_horner = par;
  GroupedProducts sq1[2], sq2[2], sp[2];
  for (int pp = 0; pp < 2; ++pp) {
    c128 *P = Pb[pp], *Pn = Pb[pp ^ 1], *Q = Qb[pp], *Qn = Qb[pp ^ 1];
    TC_RETURN_IF(group(P, false, Q, false, Qn, nullptr, 1.0, 0.0, 0.0, false, true, &sq1[pp]));
    TC_RETURN_IF(group(Q, false, P, false, Qn, Qn, 1.0, 1.0, 0.0, false, true, &sq2[pp]));
    TC_RETURN_IF(group(P, false, P, false, Pn, nullptr, 1.0, 0.0, 0.0, false, true, &sp[pp]));
  }

  auto load_checkpoint = [&](int64_t k, void* dst) -> int {
    const size_t ceb = oo.rho_dtype == TC_C128 ? 16 : 8;
    const char* src = static_cast<const char*>(checkpoints) + size_t(k) * size_t(N) * size_t(N) * ceb;
    // within a diagonal block the frame phase is 1: lab and rotating agree
    for (int b = 0; b < nb; ++b) {
      const int64_t o = L.spo[b], D = L.dim[b];
      if (ceb == 16 && f64)
        TC_RETURN_IF(launch_gather_c128_c128(reinterpret_cast<const c128*>(src), N, L.perm, o, o, D,
                                             D, 1.0, 0.0, false,
                                             static_cast<c128*>(blk(dst, b, 16)), D, s));
      else if (ceb == 16)
        TC_RETURN_IF(launch_gather_c128_c64(reinterpret_cast<const c128*>(src), N, L.perm, o, o, D,
                                            D, 1.0, 0.0, false,
                                            static_cast<c64*>(blk(dst, b, 8)), D, s));
      else if (f64)
        TC_RETURN_IF(launch_gather_c64_c128(reinterpret_cast<const c64*>(src), N, L.perm, o, o, D,
                                            D, 1.0, 0.0, false,
                                            static_cast<c128*>(blk(dst, b, 16)), D, s));
      else
        TC_RETURN_IF(launch_gather_c64_c64(reinterpret_cast<const c64*>(src), N, L.perm, o, o, D,
                                           D, 1.0, 0.0, false,
                                           static_cast<c64*>(blk(dst, b, 8)), D, s));
    }
    return TC_OK;
  };
  auto loss_of = [&](const void* blocks) -> int {
    if (!loss_out) return TC_OK;
    if (f64) {
      TC_RETURN_IF(launch_block_diag_c128(tb, static_cast<const c128*>(blocks), Np,
                                          static_cast<c128*>(L.diag), s));
      // the readout with leading dimension 0 reads element q of the diagonal
      return launch_readout_c128(a, static_cast<const c128*>(L.diag), 0, loss_out, nullptr, s,
                                 L.inv);
    }
    TC_RETURN_IF(launch_block_diag_c64(tb, static_cast<const c64*>(blocks), Np,
                                       static_cast<c64*>(L.diag), s));
    return launch_readout_c64(a, static_cast<const c64*>(L.diag), 0, loss_out, nullptr, s, L.inv);
  };

  // O_S = O, M = 0
  if (f64) TC_RETURN_IF(launch_block_fill_c128(tb, L.total, 1, n, static_cast<c128*>(L.O), s));
  else TC_RETURN_IF(launch_block_fill_c64(tb, L.total, 1, n, static_cast<c64*>(L.O), s));
  TC_TRY_HIP(hipMemsetAsync(L.M, 0, size_t(L.total) * 16, s));
  const int64_t nseg = S > 0 ? (S + C - 1) / C : 0;
  if (S == 0) {
    TC_RETURN_IF(load_checkpoint(0, slot(0)));
    TC_RETURN_IF(loss_of(slot(0)));
  }
  for (int64_t sg = nseg - 1; sg >= 0; --sg) {
    const int64_t s0 = sg * C, s1 = std::min(S, s0 + C);
    TC_RETURN_IF(load_checkpoint(sg, slot(0)));
    for (int64_t k = 1; k < s1 - s0; ++k) {
      TC_RETURN_IF(grouped_run(f1[k], s));
      TC_RETURN_IF(grouped_run(f2[k], s));
    }
    if (sg == nseg - 1) {
      // rho_S into Y (the descriptors of the step into "slot C" write Y),
      // from the last state of the segment
      const int64_t last = s1 - s0;             // 1 .. C
      if (last == C) {
        TC_RETURN_IF(grouped_run(f1[C], s));
        TC_RETURN_IF(grouped_run(f2[C], s));
      } else {
        // a short last segment: its final state is slot(last - 1); step it
        // into slot(last) (free) and read the loss there
        TC_RETURN_IF(grouped_run(f1[last], s));
        TC_RETURN_IF(grouped_run(f2[last], s));
      }
      TC_RETURN_IF(loss_of(last == C ? L.Y : slot(last)));
    }
    for (int64_t st = s1; st > s0; --st) {
      TC_RETURN_IF(grouped_run(gy, s));
      TC_RETURN_IF(grouped_run(gm[st - 1 - s0], s));
      if (!f64)
        TC_RETURN_IF(launch_accumulate_vec_c64(static_cast<const c64*>(L.T), L.M, L.total, s));
      TC_RETURN_IF(grouped_run(go, s));
    }
  }

  // G_k = L(A~_k, M_k), A~_k = -i (H_k - w_c k) dt, with the shift mu and the
  // scaling 2^-q of the whole spectrum
  const double dt = oo.dt;
  const double mu = 0.5 * (lam_lo + lam_hi);
  int q = 0;
  double r = 0.5 * (lam_hi - lam_lo) * std::fabs(dt);
  while (r > 0.5) { r *= 0.5; ++q; }
  const double sc = std::ldexp(1.0, -q);
  TC_RETURN_IF(launch_block_minus_i_shift(tb, L.total, H, ldh, a.omega_c, mu, dt * sc, L.Bs, s));
  TC_RETURN_IF(launch_scale_vec_c128(L.M, L.total, sc, s));
  TC_RETURN_IF(launch_block_fill_c128(tb, L.total, 0, n, Pb[0], s));
  TC_TRY_HIP(hipMemsetAsync(Qb[0], 0, size_t(L.total) * 16, s));
  for (int k = FRECHET_DEGREE; k >= 1; --k) {
    TC_RETURN_IF(grouped_run(hq1[k], s));           // Qn = B Q / k
    TC_RETURN_IF(grouped_run(hq2[k], s));           // Qn += M P / k
    TC_RETURN_IF(grouped_run(hp[k], s));            // Pn = I + B P / k
  }
  par = par_after_horner;
  for (int k = 0; k < q; ++k, par ^= 1) {
    TC_RETURN_IF(grouped_run(sq1[par], s));         // Qn = P Q
    TC_RETURN_IF(grouped_run(sq2[par], s));         // Qn += Q P
    TC_RETURN_IF(grouped_run(sp[par], s));          // Pn = P P
  }
  TC_TRY_HIP(hipMemsetAsync(L.G, 0, size_t(N) * size_t(N) * 16, s));
  TC_RETURN_IF(launch_block_scatter(tb, L.total, Qb[par], L.G, N, s));
  const double ph = -mu * dt;
  return launch_grad_trace(a, L.G, N, std::cos(ph), std::sin(ph), dt, grad_g, grad_delta, s);
}

}  // namespace
}  // namespace tcm

using namespace tcm;

extern "C" {

int tc_evolve_backward_workspace_size(const tc_model* m, int64_t N, const tc_evolve_opts* o,
                                      size_t* bytes) {
  clear_error();
  TC_CHECK_ARG(bytes != nullptr && o != nullptr, "NULL argument");
  ModelArgs a;
  TC_RETURN_IF(make_model_args(m, &a));
  TC_CHECK_ARG(N == a.N, "N != (c+1) 2^n");
  if (a.kappa != 0.0 || a.gamma != 0.0) {
    set_error("tc_evolve_backward: the adjoint covers the unitary step only (kappa = gamma = 0)");
    return TC_ERR_UNSUPPORTED;
  }
  TC_CHECK_ARG(o->steps >= 0, "steps < 0");
  TC_CHECK_ARG(o->checkpoint_every >= 1, "checkpoint_every must be >= 1");
  TC_CHECK_ARG(o->gemm_mode == TC_GEMM_F64 || o->gemm_mode == TC_GEMM_F32 ||
               o->gemm_mode == TC_GEMM_SPLIT_BF16, "unknown gemm_mode");
  TC_CHECK_ARG(o->rho_dtype == TC_C64 || o->rho_dtype == TC_C128, "unknown rho_dtype");
  TC_CHECK_ARG(o->sectors == 0 || o->sectors == 1, "sectors must be 0 or 1");
  tc_evolve_opts oo = *o;
  if (oo.gemm_mode == TC_GEMM_SPLIT_BF16) oo.gemm_mode = TC_GEMM_F32;
  Arena ar(nullptr, 0);
  if (oo.sectors) {
    SecBwd L;
    sec_layout(ar, a, N, oo, &L);
  } else {
    BwdLayout L;
    bwd_layout(ar, N, oo, &L);
  }
  *bytes = ar.used;
  return TC_OK;
}

int tc_evolve_backward(const tc_model* m, const double* H, int64_t ldh, const tc_c128* U,
                       int64_t ldu, int64_t N, const tc_evolve_opts* o, const void* checkpoints,
                       int32_t observable, double* loss_out, double* grad_g, double* grad_delta,
                       void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  size_t need = 0;
  TC_RETURN_IF(tc_evolve_backward_workspace_size(m, N, o, &need));
  TC_CHECK_ARG(observable == TC_OBS_EXCITED_TOTAL, "unknown observable");
  TC_CHECK_ARG(H != nullptr && U != nullptr && checkpoints != nullptr, "H / U / checkpoints NULL");
  TC_CHECK_ARG(grad_g != nullptr && grad_delta != nullptr, "gradient outputs NULL");
  TC_CHECK_ARG(ldh >= N && ldu >= N, "leading dimension < N");
  TC_CHECK_ARG(std::isfinite(o->dt), "dt not finite");
  TC_CHECK_ARG(ws != nullptr, "workspace is NULL");
  if (ws_bytes < need) {
    set_error("workspace too small for tc_evolve_backward: need " + std::to_string(need));
    return TC_ERR_WORKSPACE;
  }
  ModelArgs a;
  TC_RETURN_IF(make_model_args(m, &a));
  // Gershgorin interval of H' = H - w_c N_exc: centre sum_i (w_a,i - w_c) l_i,
  // radius of the couplings leaving the state
  double lam_lo = INFINITY, lam_hi = -INFINITY;
  {
    const int64_t per = int64_t(1) << a.n;
    for (int64_t st = 0; st < a.N; ++st) {
      const int64_t mm = st / per, l = st % per;
      double centre = 0.0, radius = 0.0;
      for (int i = 0; i < a.n; ++i) {
        if ((l >> (a.n - 1 - i)) & 1) {
          centre += a.omega_a[i] - a.omega_c;
          if (mm < a.c) radius += std::fabs(a.g[i]) * std::sqrt(double(mm + 1));
        } else if (mm > 0) {
          radius += std::fabs(a.g[i]) * std::sqrt(double(mm));
        }
      }
      lam_lo = std::min(lam_lo, centre - radius);
      lam_hi = std::max(lam_hi, centre + radius);
    }
  }
  tc_evolve_opts oo = *o;
  if (oo.gemm_mode == TC_GEMM_SPLIT_BF16) oo.gemm_mode = TC_GEMM_F32;

  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);
  if (oo.sectors)
    return backward_by_sectors(a, H, ldh, reinterpret_cast<const c128*>(U), ldu, N, oo,
                               checkpoints, lam_lo, lam_hi, loss_out, grad_g, grad_delta, ar, s);
  BwdLayout L;
  bwd_layout(ar, N, oo, &L);
  const bool f64 = L.f64;
  const size_t NN = size_t(N) * size_t(N);
  const int64_t S = oo.steps, C = oo.checkpoint_every;

  // D = U~ - I in the sweep precision
  if (f64) TC_RETURN_IF(launch_rotating_d(a, reinterpret_cast<const c128*>(U), ldu, oo.dt,
                                          static_cast<c128*>(L.D), N, s));
  else TC_RETURN_IF(launch_rotating_d_c64(a, reinterpret_cast<const c128*>(U), ldu, oo.dt,
                                          static_cast<c64*>(L.D), N, s));
  // forward step into dst: X = src + D src, dst = X + X conj(D)
  auto fstep = [&](const void* src, void* dst) -> int {
    GemmDesc g1;
    g1.M = g1.N = g1.K = N;
    g1.A = L.D; g1.lda = N; g1.a_kmaj = false;
    g1.B = src; g1.ldb = N; g1.b_kmaj = true;
    g1.C = L.X; g1.ldc = N; g1.Cin = src; g1.ldcin = N; g1.beta_re = 1.0;
    GemmDesc g2;
    g2.M = g2.N = g2.K = N;
    g2.A = L.X; g2.lda = N; g2.a_kmaj = false;
    g2.B = L.D; g2.ldb = N; g2.b_kmaj = true; g2.conj_b = true;
    g2.C = dst; g2.ldc = N; g2.Cin = L.X; g2.ldcin = N; g2.beta_re = 1.0;
    g2.herm = true;   // the state after the step is Hermitian
    g1.tail_ws = g2.tail_ws = L.tail.p;
    g1.tail_ws_bytes = g2.tail_ws_bytes = L.tail.bytes;
    TC_RETURN_IF(f64 ? gemm_f64(g1, s) : gemm_f32(g1, s));
    return f64 ? gemm_f64(g2, s) : gemm_f32(g2, s);
  };
  auto load_checkpoint = [&](int64_t k, void* dst) -> int {
    const size_t ceb = oo.rho_dtype == TC_C128 ? 16 : 8;
    const char* src = static_cast<const char*>(checkpoints) + size_t(k) * NN * ceb;
    if (ceb == L.eb) {
      TC_TRY_HIP(hipMemcpyAsync(dst, src, NN * ceb, hipMemcpyDeviceToDevice, s));
    } else if (f64) {
      TC_RETURN_IF(launch_copy_c64_to_c128(reinterpret_cast<const c64*>(src), N,
                                           static_cast<c128*>(dst), N, N, N, s));
    } else {
      TC_RETURN_IF(launch_copy_c128_to_c64(reinterpret_cast<const c128*>(src), N,
                                           static_cast<c64*>(dst), N, N, N, s));
    }
    // lab frame at t = k C dt  ->  rotating frame
    const double t = double(k) * double(oo.checkpoint_every) * oo.dt;
    if (t != 0.0) {
      if (f64) TC_RETURN_IF(launch_frame_phase_c128(a, static_cast<c128*>(dst), N, -t, s));
      else TC_RETURN_IF(launch_frame_phase_c64(a, static_cast<c64*>(dst), N, -t, s));
    }
    return TC_OK;
  };

  // O_S = O, M = 0
  if (f64) TC_RETURN_IF(launch_excitation_op_c128(a, static_cast<c128*>(L.O), N, s));
  else TC_RETURN_IF(launch_excitation_op_c64(a, static_cast<c64*>(L.O), N, s));
  TC_TRY_HIP(hipMemsetAsync(L.M, 0, NN * 16, s));

  const int64_t nseg = S > 0 ? (S + C - 1) / C : 0;
  if (S == 0) {
    TC_RETURN_IF(load_checkpoint(0, L.X));
  }
  for (int64_t seg = nseg - 1; seg >= 0; --seg) {
    const int64_t s0 = seg * C, s1 = std::min(S, s0 + C);
    // recompute rho_{s0} .. rho_{s1-1}
    TC_RETURN_IF(load_checkpoint(seg, state_at(L, N, 0)));
    for (int64_t k = 1; k < s1 - s0; ++k)
      TC_RETURN_IF(fstep(state_at(L, N, k - 1), state_at(L, N, k)));
    if (seg == nseg - 1) {
      // rho_S for the loss (X is free afterwards; fstep uses it as scratch, so
      // form rho_S into Y and keep it only for the readout)
      TC_RETURN_IF(fstep(state_at(L, N, s1 - s0 - 1), L.Y));
      if (loss_out) {
        if (f64) TC_RETURN_IF(launch_readout_c128(a, static_cast<const c128*>(L.Y), N, loss_out, nullptr, s));
        else TC_RETURN_IF(launch_readout_c64(a, static_cast<const c64*>(L.Y), N, loss_out, nullptr, s));
      }
    }
    for (int64_t st = s1; st > s0; --st) {
      const void* rho_prev = state_at(L, N, st - 1 - s0);
      // Y = U~^dag O_s = O_s + D^dag O_s  (op(A) = conj(D)^T)
      TC_RETURN_IF(cgemm_in(L.tail, f64, N, L.D, N, true, true, L.O, N, true, false, L.Y, N, L.O, s));
      // M += rho_{s-1} Y
      if (f64) {
        TC_RETURN_IF(cgemm(L.tail, true, N, rho_prev, N, false, false, L.Y, N, true, false, L.M, N, 1.0, 1.0, s));
      } else {
        TC_RETURN_IF(cgemm(L.tail, false, N, rho_prev, N, false, false, L.Y, N, true, false, L.T, N, 1.0, 0.0, s));
        TC_RETURN_IF(launch_accumulate_c64(static_cast<const c64*>(L.T), N, L.M, N, N, s));
      }
      // O_{s-1} = Y U~ = Y + Y D, Hermitian (= U~^dag O_s U~)
      TC_RETURN_IF(cgemm_in(L.tail, f64, N, L.Y, N, false, false, L.D, N, true, false, L.O, N, L.Y, s,
                            true));
    }
  }
  if (S == 0 && loss_out) {
    if (f64) TC_RETURN_IF(launch_readout_c128(a, static_cast<const c128*>(L.X), N, loss_out, nullptr, s));
    else TC_RETURN_IF(launch_readout_c64(a, static_cast<const c64*>(L.X), N, loss_out, nullptr, s));
  }

  // G = L(A~, M), A~ = -i H' dt = -i mu dt I + B with B = -i (H' - mu I) dt:
  // L(A, M) = e^{-i mu dt} L(B, M); scale B and M by 2^-q, block Taylor, q squarings.
  const double dt = oo.dt;
  const double mu = 0.5 * (lam_lo + lam_hi);
  int q = 0;
  double r = 0.5 * (lam_hi - lam_lo) * std::fabs(dt);
  while (r > 0.5) { r *= 0.5; ++q; }
  const double sc = std::ldexp(1.0, -q);
  TC_RETURN_IF(launch_minus_i_shifted(a, H, ldh, mu, dt * sc, L.Bs, N, s));
  TC_RETURN_IF(launch_scale_c128(L.M, N, sc, N, s));
  // Horner: T_K = I; T_{k-1} = I + X T_k / k on [[P, Q], [0, P]]
  c128 *P = L.P0, *Pn = L.P1, *Q = L.Q0, *Qn = L.Q1;
  TC_RETURN_IF(launch_identity_c128(P, N, N, s));
  TC_TRY_HIP(hipMemsetAsync(Q, 0, NN * 16, s));
  for (int k = FRECHET_DEGREE; k >= 1; --k) {
    const double inv = 1.0 / double(k);
    TC_RETURN_IF(zgemm64(L.tail, N, L.Bs, Q, Qn, inv, 0.0, nullptr, 0.0, s));     // Qn = B Q / k
    TC_RETURN_IF(zgemm64(L.tail, N, L.M, P, Qn, inv, 1.0, Qn, 0.0, s));           // Qn += M P / k
    TC_RETURN_IF(zgemm64(L.tail, N, L.Bs, P, Pn, inv, 0.0, nullptr, 1.0, s));     // Pn = I + B P / k
    std::swap(P, Pn);
    std::swap(Q, Qn);
  }
  for (int k = 0; k < q; ++k) {
    TC_RETURN_IF(zgemm64(L.tail, N, P, Q, Qn, 1.0, 0.0, nullptr, 0.0, s));        // Qn = P Q
    TC_RETURN_IF(zgemm64(L.tail, N, Q, P, Qn, 1.0, 1.0, Qn, 0.0, s));             // Qn += Q P
    TC_RETURN_IF(zgemm64(L.tail, N, P, P, Pn, 1.0, 0.0, nullptr, 0.0, s));        // Pn = P P
    std::swap(P, Pn);
    std::swap(Q, Qn);
  }
  const double ph = -mu * dt;
  return launch_grad_trace(a, Q, N, std::cos(ph), std::sin(ph), dt, grad_g, grad_delta, s);
}

}  // extern "C"
