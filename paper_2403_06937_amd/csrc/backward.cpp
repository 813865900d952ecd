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
}

// General complex product in the sweep precision: C = alpha op(A) op(B) + beta C.
int cgemm(bool f64, int64_t N, const void* A, int64_t lda, bool a_kmaj, bool conj_a, const void* B,
          int64_t ldb, bool b_kmaj, bool conj_b, void* C, int64_t ldc, double alpha_re,
          double beta_re, hipStream_t s) {
  GemmDesc d;
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
int cgemm_in(bool f64, int64_t N, const void* A, int64_t lda, bool a_kmaj, bool conj_a,
             const void* B, int64_t ldb, bool b_kmaj, bool conj_b, void* C, int64_t ldc,
             const void* Cin, hipStream_t s, bool herm = false) {
  GemmDesc d;
  d.herm = herm;
  d.M = d.N = d.K = N;
  d.A = A; d.lda = lda; d.a_kmaj = a_kmaj; d.conj_a = conj_a;
  d.B = B; d.ldb = ldb; d.b_kmaj = b_kmaj; d.conj_b = conj_b;
  d.C = C; d.ldc = ldc;
  d.Cin = Cin; d.ldcin = N; d.beta_re = 1.0;
  return f64 ? gemm_f64(d, s) : gemm_f32(d, s);
}

// FP64 complex product with complex alpha and a real diagonal shift gamma.
int zgemm64(int64_t N, const c128* A, const c128* B, c128* C, double ar, double beta,
            const c128* Cin, double gamma, hipStream_t s) {
  GemmDesc d;
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
  tc_evolve_opts oo = *o;
  if (oo.gemm_mode == TC_GEMM_SPLIT_BF16) oo.gemm_mode = TC_GEMM_F32;
  Arena ar(nullptr, 0);
  BwdLayout L;
  bwd_layout(ar, N, oo, &L);
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
      TC_RETURN_IF(cgemm_in(f64, N, L.D, N, true, true, L.O, N, true, false, L.Y, N, L.O, s));
      // M += rho_{s-1} Y
      if (f64) {
        TC_RETURN_IF(cgemm(true, N, rho_prev, N, false, false, L.Y, N, true, false, L.M, N, 1.0, 1.0, s));
      } else {
        TC_RETURN_IF(cgemm(false, N, rho_prev, N, false, false, L.Y, N, true, false, L.T, N, 1.0, 0.0, s));
        TC_RETURN_IF(launch_accumulate_c64(static_cast<const c64*>(L.T), N, L.M, N, N, s));
      }
      // O_{s-1} = Y U~ = Y + Y D, Hermitian (= U~^dag O_s U~)
      TC_RETURN_IF(cgemm_in(f64, N, L.Y, N, false, false, L.D, N, true, false, L.O, N, L.Y, s,
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
    TC_RETURN_IF(zgemm64(N, L.Bs, Q, Qn, inv, 0.0, nullptr, 0.0, s));     // Qn = B Q / k
    TC_RETURN_IF(zgemm64(N, L.M, P, Qn, inv, 1.0, Qn, 0.0, s));           // Qn += M P / k
    TC_RETURN_IF(zgemm64(N, L.Bs, P, Pn, inv, 0.0, nullptr, 1.0, s));     // Pn = I + B P / k
    std::swap(P, Pn);
    std::swap(Q, Qn);
  }
  for (int k = 0; k < q; ++k) {
    TC_RETURN_IF(zgemm64(N, P, Q, Qn, 1.0, 0.0, nullptr, 0.0, s));        // Qn = P Q
    TC_RETURN_IF(zgemm64(N, Q, P, Qn, 1.0, 1.0, Qn, 0.0, s));             // Qn += Q P
    TC_RETURN_IF(zgemm64(N, P, P, Pn, 1.0, 0.0, nullptr, 0.0, s));        // Pn = P P
    std::swap(P, Pn);
    std::swap(Q, Qn);
  }
  const double ph = -mu * dt;
  return launch_grad_trace(a, Q, N, std::cos(ph), std::sin(ph), dt, grad_g, grad_delta, s);
}

}  // extern "C"
