// extern "C" entry points of libtcm: argument validation, workspace layout
// and the host-side sequencing of the kernels.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>
#include <algorithm>

#include "common.h"
#include "gemm_mfma.h"
#include "kernels.h"

namespace tcm {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

int make_model_args(const tc_model* m, ModelArgs* out) {
  TC_CHECK_ARG(m != nullptr, "model is NULL");
  TC_CHECK_ARG(m->n_atoms >= 1 && m->n_atoms <= TC_MAX_ATOMS, "n_atoms out of range [1, 24]");
  TC_CHECK_ARG(m->photon_cutoff >= 0, "photon_cutoff < 0");
  TC_CHECK_ARG(m->omega_a != nullptr && m->g != nullptr, "omega_a / g is NULL");
  int64_t N = 0;
  TC_RETURN_IF(tc_dim(m->n_atoms, m->photon_cutoff, &N));
  out->n = m->n_atoms;
  out->c = m->photon_cutoff;
  out->N = N;
  out->omega_c = m->omega_c;
  TC_CHECK_ARG(std::isfinite(m->omega_c), "omega_c not finite");
  TC_CHECK_ARG(std::isfinite(m->kappa) && m->kappa >= 0.0, "kappa must be finite and >= 0");
  TC_CHECK_ARG(std::isfinite(m->gamma) && m->gamma >= 0.0, "gamma must be finite and >= 0");
  out->kappa = m->kappa;
  out->gamma = m->gamma;
  for (int i = 0; i < TC_MAX_ATOMS; ++i) {
    out->omega_a[i] = i < m->n_atoms ? m->omega_a[i] : 0.0;
    out->g[i] = i < m->n_atoms ? m->g[i] : 0.0;
    if (i < m->n_atoms) {
      TC_CHECK_ARG(std::isfinite(m->omega_a[i]) && std::isfinite(m->g[i]),
                   "omega_a / g not finite");
    }
  }
  return TC_OK;
}

// ----------------------------------------------------------------- expm
namespace {

// Real FP64 product C = alpha A B + gamma I (all N x N row-major, ld N).
int rgemm(const double* A, const double* B, double* C, int64_t N, double alpha, double gamma,
          hipStream_t s) {
  GemmDesc d;
  d.M = d.N = d.K = N;
  d.A = A; d.lda = N; d.a_kmaj = false;
  d.B = B; d.ldb = N; d.b_kmaj = true;
  d.C = C; d.ldc = N;
  d.alpha_re = alpha; d.gamma = gamma;
  d.complex = false;
  return gemm_f64(d, s);
}

struct ExpmLayout {
  double *B, *X, *P0, *P1, *Q0, *Q1;
  c128* T;   // complex ping-pong for squaring (aliases P0..P1 storage)
};

void expm_layout(Arena& ar, int64_t N, ExpmLayout* L) {
  const size_t rb = size_t(N) * size_t(N) * sizeof(double);
  L->B = static_cast<double*>(ar.take(rb));
  L->X = static_cast<double*>(ar.take(rb));
  L->P0 = static_cast<double*>(ar.take(2 * rb));  // 2 rb: also holds a complex N x N
  L->P1 = L->P0 ? L->P0 + size_t(N) * size_t(N) : nullptr;
  L->Q0 = static_cast<double*>(ar.take(rb));
  L->Q1 = static_cast<double*>(ar.take(rb));
  L->T = reinterpret_cast<c128*>(L->P0);
}

// Horner: out = sum_{k=0}^{deg} coef[k] X^k  (uses ping-pong a/b; returns the buffer holding it)
int horner(const double* X, const std::vector<double>& coef, double* a, double* b, int64_t N,
           hipStream_t s, double** result) {
  const int deg = int(coef.size()) - 1;
  // P = coef[deg] X + coef[deg-1] I  (first step without a product)
  if (deg == 0) {
    TC_RETURN_IF(launch_axpb_identity(X, N, 0.0, coef[0], a, N, N, s));
    *result = a;
    return TC_OK;
  }
  TC_RETURN_IF(launch_axpb_identity(X, N, coef[deg], coef[deg - 1], a, N, N, s));
  double* cur = a;
  double* nxt = b;
  for (int k = deg - 2; k >= 0; --k) {
    TC_RETURN_IF(rgemm(cur, X, nxt, N, 1.0, coef[k], s));
    std::swap(cur, nxt);
  }
  *result = cur;
  return TC_OK;
}

}  // namespace
}  // namespace tcm

using namespace tcm;

extern "C" {

int tc_version(void) { return TC_VERSION; }

const char* tc_last_error(void) { return g_last_error.c_str(); }

int tc_dim(int32_t n, int32_t c, int64_t* N) {
  clear_error();
  TC_CHECK_ARG(N != nullptr, "N is NULL");
  TC_CHECK_ARG(n >= 1 && n <= TC_MAX_ATOMS, "n_atoms out of range [1, 24]");
  TC_CHECK_ARG(c >= 0 && c < (1 << 20), "photon_cutoff out of range");
  const int64_t v = int64_t(c + 1) << n;
  TC_CHECK_ARG(v <= (int64_t(1) << 27), "dimension (c+1) 2^n exceeds 2^27");
  *N = v;
  return TC_OK;
}

int tc_spectral_bounds(const tc_model* m, double* lam_lo, double* lam_hi) {
  clear_error();
  TC_CHECK_ARG(lam_lo != nullptr && lam_hi != nullptr, "output is NULL");
  ModelArgs a;
  TC_RETURN_IF(make_model_args(m, &a));
  const int n = a.n;
  const int64_t per = int64_t(1) << n;
  double lo = INFINITY, hi = -INFINITY;
  for (int64_t s = 0; s < a.N; ++s) {
    const int64_t mm = s / per;
    const int64_t l = s % per;
    double centre = a.omega_c * double(mm), radius = 0.0;
    for (int i = 0; i < n; ++i) {
      const bool ex = (l >> (n - 1 - i)) & 1;
      if (ex) {
        centre += a.omega_a[i];
        if (mm < a.c) radius += std::fabs(a.g[i]) * std::sqrt(double(mm + 1));
      } else if (mm > 0) {
        radius += std::fabs(a.g[i]) * std::sqrt(double(mm));
      }
    }
    lo = std::min(lo, centre - radius);
    hi = std::max(hi, centre + radius);
  }
  *lam_lo = lo;
  *lam_hi = hi;
  return TC_OK;
}

int tc_sector_dim(const tc_model* m, int32_t k, int64_t* d) {
  clear_error();
  ModelArgs a;
  TC_RETURN_IF(make_model_args(m, &a));
  TC_CHECK_ARG(d != nullptr, "d is NULL");
  TC_CHECK_ARG(k >= 0 && k <= a.n + a.c, "sector k outside [0, n + c]");
  int64_t cnt = 0;
  for (int mm = std::max(0, k - a.n); mm <= std::min(k, a.c); ++mm) {
    const int p = k - mm;
    int64_t v = 1;
    for (int q = 1; q <= p; ++q) v = v * (a.n - p + q) / q;   // C(n, p)
    cnt += v;
  }
  *d = cnt;
  return TC_OK;
}

int tc_sector_states(const tc_model* m, int32_t k, int64_t* states) {
  clear_error();
  int64_t d = 0;
  TC_RETURN_IF(tc_sector_dim(m, k, &d));
  TC_CHECK_ARG(states != nullptr || d == 0, "states is NULL");
  const int n = m->n_atoms;
  const int64_t N = int64_t(m->photon_cutoff + 1) << n;
  const uint64_t mask = (uint64_t(1) << n) - 1;
  int64_t i = 0;
  for (int64_t s = 0; s < N; ++s)
    if (int(s >> n) + __builtin_popcountll(uint64_t(s) & mask) == k) states[i++] = s;
  return TC_OK;
}

int tc_sector_spectral_bounds(const tc_model* m, int32_t k, double* lam_lo, double* lam_hi) {
  clear_error();
  TC_CHECK_ARG(lam_lo != nullptr && lam_hi != nullptr, "output is NULL");
  int64_t d = 0;
  TC_RETURN_IF(tc_sector_dim(m, k, &d));
  ModelArgs a;
  TC_RETURN_IF(make_model_args(m, &a));
  const int n = a.n;
  const uint64_t mask = (uint64_t(1) << n) - 1;
  double lo = INFINITY, hi = -INFINITY;
  // a sector state couples only to states of its own sector, so the row
  // radii of the full H are those of the block
  for (int64_t s = 0; s < a.N; ++s) {
    const int64_t mm = s >> n;
    const uint64_t l = uint64_t(s) & mask;
    if (int(mm) + __builtin_popcountll(l) != k) continue;
    double centre = a.omega_c * double(mm), radius = 0.0;
    for (int i = 0; i < n; ++i) {
      const bool ex = (l >> (n - 1 - i)) & 1;
      if (ex) {
        centre += a.omega_a[i];
        if (mm < a.c) radius += std::fabs(a.g[i]) * std::sqrt(double(mm + 1));
      } else if (mm > 0) {
        radius += std::fabs(a.g[i]) * std::sqrt(double(mm));
      }
    }
    lo = std::min(lo, centre - radius);
    hi = std::max(hi, centre + radius);
  }
  *lam_lo = lo;
  *lam_hi = hi;
  return TC_OK;
}

int tc_build_sector_hamiltonian(const tc_model* m, int32_t k, double* H, int64_t ldh,
                                void* stream) {
  clear_error();
  int64_t d = 0;
  TC_RETURN_IF(tc_sector_dim(m, k, &d));
  ModelArgs a;
  TC_RETURN_IF(make_model_args(m, &a));
  TC_CHECK_ARG(H != nullptr, "H is NULL");
  TC_CHECK_ARG(ldh >= d, "ldh < d_k");
  return launch_ham_sector(a, k, d, H, ldh, as_stream(stream));
}

int tc_build_hamiltonian(const tc_model* m, double* H, int64_t ldh, void* stream) {
  clear_error();
  ModelArgs a;
  TC_RETURN_IF(make_model_args(m, &a));
  TC_CHECK_ARG(H != nullptr, "H is NULL");
  TC_CHECK_ARG(ldh >= a.N, "ldh < N");
  return launch_ham_fill(a, H, ldh, as_stream(stream));
}

int tc_expm_workspace_size(int64_t N, int32_t method, size_t* bytes) {
  clear_error();
  TC_CHECK_ARG(bytes != nullptr, "bytes is NULL");
  TC_CHECK_ARG(N >= 0, "N < 0");
  TC_CHECK_ARG(method == TC_EXPM_SS_TAYLOR || method == TC_EXPM_TAYLOR10, "unknown expm method");
  Arena ar(nullptr, 0);
  ExpmLayout L;
  expm_layout(ar, N, &L);
  *bytes = ar.used;
  return TC_OK;
}

int tc_expm(const double* H, int64_t N, int64_t ldh, double dt, double lam_lo, double lam_hi,
            int32_t method, tc_c128* U, int64_t ldu, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  TC_CHECK_ARG(N >= 0, "N < 0");
  TC_CHECK_ARG(H != nullptr && U != nullptr, "H / U is NULL");
  TC_CHECK_ARG(ldh >= N && ldu >= N, "leading dimension < N");
  TC_CHECK_ARG(std::isfinite(dt), "dt not finite");
  TC_CHECK_ARG(method == TC_EXPM_SS_TAYLOR || method == TC_EXPM_TAYLOR10, "unknown expm method");
  if (method == TC_EXPM_SS_TAYLOR)
    TC_CHECK_ARG(std::isfinite(lam_lo) && std::isfinite(lam_hi) && lam_lo <= lam_hi,
                 "spectral bounds must be finite with lo <= hi");
  size_t need = 0;
  TC_RETURN_IF(tc_expm_workspace_size(N, method, &need));
  TC_CHECK_ARG(ws != nullptr || need == 0, "workspace is NULL");
  if (ws_bytes < need) {
    set_error("workspace too small for tc_expm");
    return TC_ERR_WORKSPACE;
  }
  if (N == 0) return TC_OK;
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);
  ExpmLayout L;
  expm_layout(ar, N, &L);

  double mu = 0.0, scale = dt;
  int sq = 0;
  int kc, ks;   // polynomial degrees in X = B^2 of cos and sin / B
  if (method == TC_EXPM_SS_TAYLOR) {
    mu = 0.5 * (lam_lo + lam_hi);
    double r = 0.5 * (lam_hi - lam_lo) * std::fabs(dt);
    while (r > 0.5) { r *= 0.5; ++sq; }
    scale = dt * std::ldexp(1.0, -sq);
    kc = 9;   // cos: degree 18 in B, first omitted term <= 0.5^20/20! < 1e-24
    ks = 9;   // sin: degree 19 in B
  } else {
    kc = 5;   // Eq. (10) truncated at k = 10: even part degree 10, odd part degree 9
    ks = 4;
  }
  // B = (H - mu I) * scale  (copy into the dense N x N workspace, ld N)
  {
    // the helper reads with ld = ldh and writes with ld = N
    TC_RETURN_IF(launch_axpb_identity(H, ldh, scale, -mu * scale, L.B, N, N, s));
  }
  TC_RETURN_IF(rgemm(L.B, L.B, L.X, N, 1.0, 0.0, s));                  // X = B^2
  std::vector<double> cc(kc + 1), cs(ks + 1);
  {
    double f = 1.0;   // (2k)!
    for (int k = 0; k <= kc; ++k) {
      if (k > 0) f *= double(2 * k - 1) * double(2 * k);
      cc[k] = (k % 2 ? -1.0 : 1.0) / f;
    }
    f = 1.0;          // (2k+1)!
    for (int k = 0; k <= ks; ++k) {
      if (k > 0) f *= double(2 * k) * double(2 * k + 1);
      cs[k] = (k % 2 ? -1.0 : 1.0) / f;
    }
  }
  double* cosB = nullptr;
  double* sinpoly = nullptr;
  TC_RETURN_IF(horner(L.X, cc, L.Q0, L.Q1, N, s, &cosB));
  // sin poly goes to the ping-pong pair not holding cos: use P0/P1 (real halves)
  TC_RETURN_IF(horner(L.X, cs, L.P0, L.P1, N, s, &sinpoly));
  double* sinB = (cosB == L.Q0) ? L.Q1 : L.Q0;
  TC_RETURN_IF(rgemm(L.B, sinpoly, sinB, N, 1.0, 0.0, s));             // sin B = B p(B^2)
  // U0 = e^{-i mu scale} (cos B - i sin B)
  const double ph = -mu * scale;
  if (sq == 0) {
    TC_RETURN_IF(launch_assemble_cs(cosB, sinB, N, std::cos(ph), std::sin(ph),
                                    reinterpret_cast<c128*>(U), ldu, N, s));
  } else {
    // squarings ping-pong between T (workspace, ld N) and U (ldu); the last lands in U
    c128* bufs[2] = {L.T, reinterpret_cast<c128*>(U)};
    int64_t lds[2] = {N, ldu};
    int cur = (sq % 2 == 0) ? 1 : 0;  // start so that after sq squarings we are in U
    // T aliases P0/P1, which held the sin polynomial; it is consumed already.
    TC_RETURN_IF(launch_assemble_cs(cosB, sinB, N, std::cos(ph), std::sin(ph), bufs[cur],
                                    lds[cur], N, s));
    for (int q = 0; q < sq; ++q) {
      const int nxt = cur ^ 1;
      GemmDesc d;
      d.M = d.N = d.K = N;
      d.A = bufs[cur]; d.lda = lds[cur]; d.a_kmaj = false;
      d.B = bufs[cur]; d.ldb = lds[cur]; d.b_kmaj = true;
      d.C = bufs[nxt]; d.ldc = lds[nxt];
      TC_RETURN_IF(gemm_f64(d, s));
      cur = nxt;
    }
  }
  TC_RETURN_IF(launch_symmetrize(reinterpret_cast<c128*>(U), ldu, N, s));
  return TC_OK;
}

}  // extern "C"
