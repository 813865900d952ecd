// Host launchers of the HBM-bound and latency-bound kernels of libtcm.
#pragma once
#include "common.h"

namespace tcm {

// a1: dense Eq. (4) into H (N x N, ldh).
int launch_ham_fill(const ModelArgs& m, double* H, int64_t ldh, hipStream_t s);

// out = a * X + b * I  (real N x N).
int launch_axpb_identity(const double* X, int64_t ldx, double a, double b,
                         double* out, int64_t ldo, int64_t N, hipStream_t s);

// U = ph * (Cm - i Sm) (complex from two real N x N), ph = (ph_re, ph_im).
int launch_assemble_cs(const double* Cm, const double* Sm, int64_t ld, double ph_re,
                       double ph_im, c128* U, int64_t ldu, int64_t N, hipStream_t s);

// U <- (U + U^T) / 2 in place (complex, square).
int launch_symmetrize(c128* U, int64_t ldu, int64_t N, hipStream_t s);

// Copies with type conversion; ld in elements.
int launch_copy_c128_to_c64(const c128* src, int64_t lds, c64* dst, int64_t ldd,
                            int64_t rows, int64_t cols, hipStream_t s);
int launch_copy_c64_to_c128(const c64* src, int64_t lds, c128* dst, int64_t ldd,
                            int64_t rows, int64_t cols, hipStream_t s);

// Rotating frame: U~[i][j] = e^{+i w_c k_i dt} U[i][j] minus the identity (D = U~ - I)
// written as c128 (row phase with the excitation number k_i of row i).
int launch_rotating_d(const ModelArgs& m, const c128* U, int64_t ldu, double dt,
                      c128* D, int64_t ldd, hipStream_t s);
int launch_rotating_d_c64(const ModelArgs& m, const c128* U, int64_t ldu, double dt,
                          c64* D, int64_t ldd, hipStream_t s);

// Element phase rho[i][j] *= e^{-i w_c (k_i - k_j) t} (t = elapsed time), for the
// FP64 master (c128) or the FP32 master (c64).
int launch_frame_phase_c128(const ModelArgs& m, c128* rho, int64_t ld, double t, hipStream_t s);
int launch_frame_phase_c64(const ModelArgs& m, c64* rho, int64_t ld, double t, hipStream_t s);

// Dissipation over dt, exp(dt L) for the Lindblad term of the model (in
// place; no-op when kappa = gamma = 0): one amplitude-damping channel per atom,
// two atoms per pass, then the cavity channel.  Commutes with the rotating
// frame's phase, so it applies in either frame.
int launch_dissipation_c128(const ModelArgs& m, c128* rho, int64_t ld, double dt, hipStream_t s);
int launch_dissipation_c64(const ModelArgs& m, c64* rho, int64_t ld, double dt, hipStream_t s);

// Per-step readout of the diagonal: *pop = sum_s |l(s)| Re rho_ss; if
// pdist != NULL, pdist[m] = sum_{photon(s) = m} Re rho_ss (m = 0..c); if
// pstate != NULL, pstate[m] = P({m>) of Eq. (13), the sum over the states with
// m photons and n - m excited atoms (m = 0..min(n, c)).  With a map, basis
// state s is row and column map[s] of rho (sector-sorted order).
int launch_readout_c128(const ModelArgs& m, const c128* rho, int64_t ld, double* pop,
                        double* pdist, hipStream_t s, const int32_t* map = nullptr,
                        double* pstate = nullptr);
int launch_readout_c64(const ModelArgs& m, const c64* rho, int64_t ld, double* pop,
                       double* pdist, hipStream_t s, const int32_t* map = nullptr,
                       double* pstate = nullptr);

// Readout of many instances in one launch (one workgroup each): record index
// r = *counter; pop[r], pdist[r*(c+1) + m] and pstate[r*(min(n,c)+1) + m] as
// above.  advance_counter adds 1.
struct ReadoutItem {
  const void* rho;
  int64_t ld;
  int n, c;
  double* pop;      // may be NULL
  double* pdist;    // may be NULL
  const int32_t* map;   // NULL, or the position of each basis state in rho (sector order)
  double* pstate;   // may be NULL
};
// advance: also move the record index on (count must be 1)
int launch_grouped_readout(const ReadoutItem* items_dev, int count, bool c128_storage,
                           int* counter, hipStream_t s, bool advance = false);
int launch_advance_counter(int* counter, hipStream_t s);

// Hermitise and divide by Re Tr rho, in FP64.  scratch: device double[2]
// (trace, non-finite flag).  For c64 storage the arithmetic is FP64 too.
int launch_renorm_c128(c128* rho, int64_t ld, int64_t N, double* scratch, hipStream_t s);
int launch_renorm_c64(c64* rho, int64_t ld, int64_t N, double* scratch, hipStream_t s);

// tc_observables: partials buffer of observables_partials_count(N) doubles.
size_t observables_partials_count(int64_t N);
int launch_observables(const ModelArgs& m, const void* rho, int dtype, int64_t ld,
                       double* partials, double* scalars, double* atom_pop,
                       double* photon_dist, double* exc_dist, double* photon_state,
                       double* dicke, hipStream_t s);

// ---- adjoint helpers
// O = diag(sum_i s_i^+ s_i^-) written densely (zeros off the diagonal).
int launch_excitation_op_c128(const ModelArgs& m, c128* O, int64_t ld, hipStream_t s);
int launch_excitation_op_c64(const ModelArgs& m, c64* O, int64_t ld, hipStream_t s);
// M += T (complex64 into complex128).
int launch_accumulate_c64(const c64* T, int64_t ldt, c128* M, int64_t ldm, int64_t N,
                          hipStream_t s);
// out = -i (H - w_c N_exc - mu I) * scale  (complex128 from real FP64): the
// rotating-frame generator H' = H - w_c N_exc, shifted by mu.
int launch_minus_i_shifted(const ModelArgs& m, const double* H, int64_t ldh, double mu,
                           double scale, c128* out, int64_t ldo, hipStream_t s);
// X *= a (complex128, in place).
int launch_scale_c128(c128* X, int64_t ld, double a, int64_t N, hipStream_t s);
// X = I (complex128).
int launch_identity_c128(c128* X, int64_t ld, int64_t N, hipStream_t s);
// Parameter gradients from G (scaled by the complex factor ph):
//   grad_g[i]     = 2 dt Im( ph sum_{s,t} sqrt(m+1) (G_st + G_ts) )   over the (s, t)
//                   pairs coupled by g_i (s = (m, l) with l_i = 1, t = (m+1, l - e_i))
//   grad_delta[i] = 2 dt Im( ph sum_{s: l_i = 1} G_ss )
int launch_grad_trace(const ModelArgs& m, const c128* G, int64_t ld, double ph_re, double ph_im,
                      double dt, double* grad_g, double* grad_delta, hipStream_t s);

// ---- excitation-sector stepping (sectors.hip)
// dst[i][j] = ph * src[map[ro + i]][map[co + j]] - sub_identity * [ro + i == co + j]
// for i < rows, j < cols, with type conversion (ph = (ph_re, ph_im)); 0 where
// either map entry is negative (a padding position).
int launch_gather_c128_c128(const c128* src, int64_t lds, const int32_t* map, int64_t ro,
                            int64_t co, int64_t rows, int64_t cols, double ph_re, double ph_im,
                            bool sub_identity, c128* dst, int64_t ldd, hipStream_t s);
int launch_gather_c128_c64(const c128* src, int64_t lds, const int32_t* map, int64_t ro,
                           int64_t co, int64_t rows, int64_t cols, double ph_re, double ph_im,
                           bool sub_identity, c64* dst, int64_t ldd, hipStream_t s);
int launch_gather_c64_c64(const c64* src, int64_t lds, const int32_t* map, int64_t ro,
                          int64_t co, int64_t rows, int64_t cols, double ph_re, double ph_im,
                          bool sub_identity, c64* dst, int64_t ldd, hipStream_t s);
int launch_gather_c64_c128(const c64* src, int64_t lds, const int32_t* map, int64_t ro,
                           int64_t co, int64_t rows, int64_t cols, double ph_re, double ph_im,
                           bool sub_identity, c128* dst, int64_t ldd, hipStream_t s);
// In the sector-sorted order (position i in sector sec[i], sec non-decreasing):
// rho[i][j] = conj(rho[j][i]) wherever sec[i] > sec[j], i.e. the lower block
// triangle is rebuilt from the upper one.
int launch_mirror_lower_c128(c128* rho, int64_t ld, int64_t N, const int32_t* sec,
                             hipStream_t s);
int launch_mirror_lower_c64(c64* rho, int64_t ld, int64_t N, const int32_t* sec, hipStream_t s);

// ---- one excitation sector (sectors.hip)
// H_k[i][j] = H[s_i][s_j] (Eq. (4)) over the d states s_0 < s_1 < ... of sector k.
int launch_ham_sector(const ModelArgs& m, int k, int64_t d, double* H, int64_t ldh,
                      hipStream_t s);
// out = ph * U - I (N x N, ph = (ph_re, ph_im)).
int launch_phase_minus_identity_c128(const c128* U, int64_t ldu, double ph_re, double ph_im,
                                     c128* out, int64_t ldo, int64_t N, hipStream_t s);
int launch_phase_minus_identity_c64(const c128* U, int64_t ldu, double ph_re, double ph_im,
                                    c64* out, int64_t ldo, int64_t N, hipStream_t s);

// ---- block-diagonal storage of padded sectors (sectors.hip)
// Block k (k < nb) is dim[k] x dim[k], row-major, at element offset boff[k]
// (boff[nb] = total elements); its rows are the padded sorted positions
// spo[k] .. spo[k] + dim[k] - 1, and position p holds basis state perm[p]
// (-1 for padding).  All arrays are device memory.
struct BlockTable {
  const int64_t* boff;
  const int64_t* spo;
  const int64_t* dim;
  const int32_t* perm;
  int nb;
};
// what = 0: identity blocks; 1: diag(sum_i s_i^+ s_i^-) over the block's states
int launch_block_fill_c128(const BlockTable& t, int64_t total, int what, int n, c128* out,
                           hipStream_t s);
int launch_block_fill_c64(const BlockTable& t, int64_t total, int what, int n, c64* out,
                          hipStream_t s);
// out = -i scale (H_k - (w_c k + mu) I) for every block (0 at padding)
int launch_block_minus_i_shift(const BlockTable& t, int64_t total, const double* H, int64_t ldh,
                               double omega_c, double mu, double scale, c128* out, hipStream_t s);
// full[s_i][s_j] = G_k[i][j] over the blocks' states
int launch_block_scatter(const BlockTable& t, int64_t total, const c128* G, c128* full, int64_t ld,
                         hipStream_t s);
// diag[p] = diagonal element of position p (p < Np)
int launch_block_diag_c128(const BlockTable& t, const c128* blocks, int64_t Np, c128* diag,
                           hipStream_t s);
int launch_block_diag_c64(const BlockTable& t, const c64* blocks, int64_t Np, c64* diag,
                          hipStream_t s);
int launch_scale_vec_c128(c128* x, int64_t count, double a, hipStream_t s);
int launch_accumulate_vec_c64(const c64* t, c128* m, int64_t count, hipStream_t s);

// ---- LDS-resident stepping of one small instance (resident.hip)
// All steps in one launch of one workgroup, op, rho and X held in LDS:
// X = op R (+ R if rot), R' = X op^dag (+ X if rot) per step, renormalisation
// in FP64 every renorm_every steps (scratch[0] = last trace, scratch[1] = 1
// once a trace is non-finite or non-positive), records of the diagonal
// every record_every steps (record 0 = the initial state), rho written back at
// the end.  The master storage is c128 (N <= 48) or c64 (N <= 64).
constexpr int RESIDENT_MAX_N_C128 = 48;
constexpr int RESIDENT_MAX_N_C64 = 64;
struct ResidentArgs {
  const void* op; int64_t ldop;   // U (lab) or D = U~ - I (rotating), master precision
  void* rho; int64_t ldr;         // master state, in/out
  int rot;
  int64_t steps;
  int renorm_every, record_every;
  double* pop;                    // [steps/record_every + 1] or NULL
  double* pdist;                  // [..][c + 1] or NULL
  double* pstate;                 // [..][min(n, c) + 1] or NULL
  double* scratch;                // [2]
};
int launch_resident_c128(const ModelArgs& m, const ResidentArgs& a, hipStream_t s);
int launch_resident_c64(const ModelArgs& m, const ResidentArgs& a, hipStream_t s);

// bfloat16 hi/lo split of binary32 values.
int launch_split_bf16(const float* x, int64_t count, uint16_t* hi, uint16_t* lo, hipStream_t s);

}  // namespace tcm
