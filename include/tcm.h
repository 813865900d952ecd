/*
 * tcm.h -- C ABI of the Tavis-Cummings density-matrix stepper for MI355X (gfx950).
 *
 * The library evolves the density matrix of n two-level atoms coupled to one
 * cavity mode,  rho(t + dt) = U rho(t) U^dag  with  U = exp(-i H dt)  formed
 * once (Miao & Ozhigov, arXiv 2403.06937, Sec. III.A, Eq. (6)), so every time
 * step is two dense complex matrix-matrix products.  H is the Tavis-Cummings
 * Hamiltonian of Sec. II, Eq. (4), with hbar = 1, a single bosonic cavity mode
 * truncated at photon number c, per-atom frequencies w_a,i = 1 + delta_i and
 * real couplings g_i.
 *
 * Basis order: photon-major Kronecker order |m>|l_1 ... l_n>, atom 1 the most
 * significant bit, l_i = 1 for an excited atom; index s = m 2^n + sum_i l_i 2^(n-i),
 * dimension N = (c + 1) 2^n.
 *
 * Conventions shared by every call
 *   - Matrices are row-major with a leading dimension (ld >= N, in elements).
 *   - Complex matrices are interleaved (re, im) pairs: tc_c128 (2 x double) or
 *     tc_c64 (2 x float), the layout of torch.complex128 / torch.complex64.
 *   - Pointers documented "device" must be device memory of the current HIP
 *     device; "host" pointers are read during the call only.  The caller owns
 *     all memory.  The library never allocates or frees caller memory; scratch
 *     comes from a caller-provided workspace sized by the *_workspace_size
 *     query of the same call.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is enqueued on it asynchronously; a call returns as soon as
 *     its work is enqueued, unless documented otherwise.
 *   - Every argument is validated before any device work is enqueued.  On
 *     failure the return value is a TC_ERR_* code, no device work has been
 *     enqueued for argument errors, outputs are unspecified for device errors,
 *     and tc_last_error() returns a message for the calling thread (valid
 *     until that thread's next library call).  No C++ exception crosses this
 *     interface.
 */
#ifndef TCM_H
#define TCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TC_VERSION 120

/* Status codes. */
#define TC_OK                     0
#define TC_ERR_INVALID_ARGUMENT   1
#define TC_ERR_UNSUPPORTED        2
#define TC_ERR_WORKSPACE          3
#define TC_ERR_HIP                4
#define TC_ERR_NONFINITE          5

typedef struct { double re, im; } tc_c128;
typedef struct { float re, im; } tc_c64;

/* Storage type of rho at the interface. */
#define TC_C64   1
#define TC_C128  2

/* Arithmetic of the per-step products. */
#define TC_GEMM_F64          0   /* complex FP64 on FP64 MFMA                          */
#define TC_GEMM_F32          1   /* complex FP32 on FP32 MFMA                          */
#define TC_GEMM_SPLIT_BF16   2   /* each real operand split hi+lo in bfloat16; products
                                    hi*hi + hi*lo + lo*hi on BF16 MFMA, FP32 accumulate */

/* Method of tc_expm. */
#define TC_EXPM_SS_TAYLOR  0     /* shift, scale, Taylor (cos/sin) and squaring, FP64  */
#define TC_EXPM_TAYLOR10   1     /* Sec. III.B, Eq. (10): sum_{k=0}^{10} (-i H dt)^k/k!,
                                    no shift, no scaling                              */

/* Frame in which the products run (the result is always the lab frame). */
#define TC_FRAME_LAB       0
#define TC_FRAME_ROTATING  1     /* rho~ = e^{+i w_c N t} rho e^{-i w_c N t}, where N is the
                                    total excitation number; steps use U~ = I + D with
                                    U~ = e^{+i w_c N dt} U, so the rounded operand is D  */

/* Observable of tc_evolve_backward. */
#define TC_OBS_EXCITED_TOTAL 0   /* L = sum_i <s_i^+ s_i^-> at the final step          */

/* Model of Eq. (4), with the Lindblad term of Eq. (5), which the paper sets
 * to zero, read as cavity leakage and atomic emission at zero temperature:
 *   L(rho) = kappa D[a] rho + gamma sum_i D[s_i^-] rho,
 *   D[A] rho = A rho A^dag - (A^dag A rho + rho A^dag A) / 2.
 * With kappa = gamma = 0 (the paper's case) every step is Eq. (6).  Otherwise
 * tc_evolve follows each unitary step by exp(dt L), applied exactly as one
 * amplitude-damping channel per atom (p = 1 - e^{-gamma dt}) and one for the
 * cavity (eta = e^{-kappa dt}); the splitting is first order in dt. */
typedef struct {
  int32_t n_atoms;          /* n >= 1                                               */
  int32_t photon_cutoff;    /* c >= 0: photon numbers 0..c, a^dag|c> = 0            */
  double  omega_c;          /* cavity frequency                                     */
  const double* omega_a;    /* host [n]: atomic frequencies 1 + delta_i             */
  const double* g;          /* host [n]: real couplings g_i                         */
  double  kappa;            /* cavity leakage rate >= 0 (read by tc_evolve only)     */
  double  gamma;            /* atomic emission rate >= 0 (read by tc_evolve only)    */
} tc_model;

/* ---------------------------------------------------------------- helpers */

int         tc_version(void);
const char* tc_last_error(void);

/* N = (c + 1) 2^n.  TC_ERR_INVALID_ARGUMENT if n < 1, c < 0 or N > 2^31 / 16. */
int tc_dim(int32_t n_atoms, int32_t photon_cutoff, int64_t* N);

/* Host-only.  Gershgorin interval [lo, hi] containing the spectrum of H
 * (Eq. (4)): centre H_ss, radius sum_i g_i sqrt(m+1) over the couplings that
 * leave |m, l> (O(N n) work). */
int tc_spectral_bounds(const tc_model* m, double* lam_lo, double* lam_hi);

/* ------------------------------------------- one excitation sector */

/* H of Eq. (4) conserves the excitation number k = m + |l| (photons plus
 * excited atoms), so it is block diagonal over the sectors k = 0 .. n + c, and
 * so is U = exp(-i H dt).  These calls work on one block.  With c >= n and
 * k = n the block is the paper's own model of Sec. II, Eq. (2): the 2^n atom
 * patterns |l>, each with n - |l| photons, starting from all atoms excited
 * (Sec. IV); the sector's states are ordered by increasing basis index.
 * All are host-only except the builder, and fail with
 * TC_ERR_INVALID_ARGUMENT unless 0 <= k <= n + c. */
/* d_k = sum_m binom(n, k - m) over m = max(0, k - n) .. min(k, c). */
int tc_sector_dim(const tc_model* m, int32_t k, int64_t* d);
/* The basis indices s of sector k, increasing (states: host [d_k]). */
int tc_sector_states(const tc_model* m, int32_t k, int64_t* states);
/* Gershgorin interval of the block (a sector state couples only inside it). */
int tc_sector_spectral_bounds(const tc_model* m, int32_t k, double* lam_lo, double* lam_hi);
/* Writes the block H_k[i][j] = H[s_i][s_j] (device, d_k x d_k, ldh >= d_k,
 * row-major, real symmetric) for the states s_0 < s_1 < ... of sector k. */
int tc_build_sector_hamiltonian(const tc_model* m, int32_t k, double* H, int64_t ldh,
                                void* stream);

/* ----------------------------------------------------- a1: Hamiltonian */

/* Writes the dense real symmetric Eq. (4) into H (device, N x N, row-major,
 * leading dimension ldh >= N; columns N..ldh-1 are not touched):
 *   H[s][s]  = w_c m + sum_i w_a,i l_i
 *   H[t][s]  = H[s][t] = g_i sqrt(m + 1)  for s = (m, l) with l_i = 1, m < c and
 *              t = (m + 1, l with l_i cleared)
 *   every other entry exactly 0. */
int tc_build_hamiltonian(const tc_model* m, double* H, int64_t ldh, void* stream);

/* ------------------------------------------------------------ a2: expm */

int tc_expm_workspace_size(int64_t N, int32_t method, size_t* bytes);

/* U = exp(-i H dt) (Eq. (6) with hbar = 1) for real symmetric H (device, N x N,
 * ldh), written to U (device, tc_c128 N x N, ldu).
 * TC_EXPM_SS_TAYLOR: with mu = (lam_lo + lam_hi)/2 and the smallest s >= 0 such
 * that (lam_hi - lam_lo)/2 |dt| 2^-s <= 1/2, B = (H - mu I) dt 2^-s, cos B and
 * sin B from their Taylor series to degree 18 / 19 (remainder < 1e-17), then
 * U = e^{-i mu dt} (cos B - i sin B)^(2^s), symmetrised.  lam_lo/hi must bound
 * the spectrum (tc_spectral_bounds gives such bounds).
 * TC_EXPM_TAYLOR10: Eq. (10), L = sum_{k=0}^{10} (-i H dt)^k / k!; lam_lo/hi
 * are ignored.  The right factor of Eq. (11) is L^dag, which the stepper forms
 * by conjugation.  ws: device workspace of tc_expm_workspace_size bytes. */
int tc_expm(const double* H, int64_t N, int64_t ldh, double dt,
            double lam_lo, double lam_hi, int32_t method,
            tc_c128* U, int64_t ldu, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------- a3..a8: time stepping */

typedef struct {
  const tc_model* model;    /* host; its n, c define N                              */
  int64_t N;                /* must equal (c + 1) 2^n                               */
  const tc_c128* U;         /* device N x N propagator (tc_expm output), complex symmetric */
  int64_t ldu;
  void* rho;                /* device N x N, type opts.rho_dtype; in: rho(0), out: rho(steps) */
  int64_t ldr;
  double* pop_out;          /* device [steps/record_every + 1] or NULL: sum_i <s_i^+ s_i^-> */
  double* photon_dist_out;  /* device [steps/record_every + 1][c + 1] or NULL: photon-number
                               distribution, sum of rho_ss over the states with m photons */
  void* checkpoints;        /* device [steps/checkpoint_every + 1][N][N] of rho_dtype, or NULL */
  double* photon_state_out; /* device [steps/record_every + 1][min(n, c) + 1] or NULL:
                               P({m>) of Sec. IV, Eq. (13), read on the sector of the
                               all-excited start: the sum of rho_ss over the states with
                               m photons and n - m excited atoms (m = 0 .. min(n, c));
                               equals photon_dist_out[m] only while rho lies in the
                               excitation-n sector                                  */
} tc_instance;

typedef struct {
  int64_t steps;            /* >= 0                                                 */
  double  dt;               /* time step of U (used by the rotating frame)          */
  int32_t gemm_mode;        /* TC_GEMM_*                                            */
  int32_t rho_dtype;        /* TC_C64 or TC_C128                                    */
  int32_t frame;            /* TC_FRAME_*                                           */
  int32_t renorm_every;     /* 0 = never; else Hermitise and divide by Re Tr rho in FP64
                               after every renorm_every-th step                      */
  int32_t record_every;     /* >= 1 when pop_out / photon_dist_out are given        */
  int32_t checkpoint_every; /* 0 = none; else rho after every checkpoint_every-th step */
  int32_t use_graph;        /* 1: the launches of a chunk of steps (a whole number of
                               periods lcm(record_every, renorm_every), about 16
                               steps) are captured once in a hipGraph and replayed,
                               single instances and batches alike; the leftover
                               steps run eagerly.  Ignored with checkpoints or
                               fewer steps than a chunk.  Same results bit for bit */
  int32_t full_product;     /* 0: rho' = X U^dag is Hermitian, so its upper tile
                               triangle is multiplied and mirrored (rho(0) must be
                               Hermitian); 1: every tile of both products        */
  int32_t no_resident;      /* 0: a single instance with N <= 48 (FP64 products) or
                               N <= 64 (complex FP32), stepped densely with no
                               checkpoints and no Lindblad term, runs every step
                               in one launch of one workgroup that keeps U (or D),
                               rho and X in LDS (the per-step launches of such a
                               run would cost more than its arithmetic); same
                               results to rounding.  1: never                      */
  int32_t sectors;          /* 0: dense N x N products.  1: excitation-sector
                               block stepping, in every gemm_mode (count > 1:
                               the blocks of all instances in one grouped
                               launch per product):
                               H of Eq. (4) conserves k = m + |l|, so in the
                               basis sorted by k (stable within a sector) U is
                               block diagonal, U = diag(U_0 .. U_{n+c}), and
                               rho'_{jk} = U_j rho_{jk} U_k^dag for every block
                               pair.  Only the blocks j <= k are formed (rho is
                               Hermitian; rho(0) must be), by two grouped
                               products per step, X_{k,k:} = U_k rho_{k,k:} and
                               rho'_{:k,k} = X_{:k,k} U_k^dag.  Same result as
                               the dense products up to rounding (U's entries
                               between sectors are exact zeros); the work per
                               step is 8 sum_k d_k^2 (N + d_k) flop instead of
                               16 N^3.  U is read at the call's start only;
                               full_product is ignored; with a Lindblad term each
                               step converts to the basis order and back around
                               the damping channels.                            */
} tc_evolve_opts;

int tc_evolve_workspace_size(const tc_instance* inst, int32_t count,
                             const tc_evolve_opts* o, size_t* bytes);

/* Steps each of the count instances o->steps times: rho <- U rho U^dag (Eq. (6);
 * the paper's product order L (rho R) of Eq. (12) is the same product).
 * Record r (r = 0 .. steps/record_every) holds the readout after r*record_every
 * steps; record 0 is rho(0).  On return rho holds rho(steps) in the lab frame.
 * count > 1 steps uneven instances together (all share o).  ws: device
 * workspace of tc_evolve_workspace_size bytes.  Synchronises the stream only
 * when a renormalisation finds a non-finite trace (then TC_ERR_NONFINITE).
 * Results are bitwise reproducible on a given device; a product whose last
 * round of tiles would leave at least half of the compute units idle has
 * those tiles' K sums split into ranges that are added in order, and how it
 * is split depends on the device's compute-unit count. */
int tc_evolve(const tc_instance* inst, int32_t count, const tc_evolve_opts* o,
              void* ws, size_t ws_bytes, void* stream);

/* tc_evolve within excitation sector k: inst->N = d_k, inst->U the d_k x d_k
 * propagator of the block (tc_expm of tc_build_sector_hamiltonian's H_k),
 * inst->rho the d_k x d_k density matrix on the sector's states in the order
 * of tc_sector_states.  Every step is Eq. (6) on the block; records use the
 * basis states of the block (P(m) for m outside the sector is 0);
 * checkpoints are d_k x d_k.  The rotating frame's factor is the scalar
 * e^{i w_c k dt} here, so its operand is D = e^{i w_c k dt} U_k - I and the
 * result needs no phase.  opts.sectors must be 0; a model with a Lindblad term
 * gives TC_ERR_UNSUPPORTED (its damping channels lead out of the sector).
 * One instance per call. */
int tc_evolve_sector_workspace_size(const tc_instance* inst, int32_t k,
                                    const tc_evolve_opts* o, size_t* bytes);
int tc_evolve_sector(const tc_instance* inst, int32_t k, const tc_evolve_opts* o,
                     void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------ a5/a7: observables */

/* Readout of one density matrix (device, N x N, ldr, type rho_dtype): the
 * expectations Tr(O rho) of the diagonal operators of Eq. (4)'s model, the
 * invariants of Eq. (6)'s unitary step (trace, purity, Hermiticity, the
 * excitation-number distribution) and both readings of the {m> probability of
 * Sec. IV, Eq. (13), whose normalisation factors the paper leaves open.
 * scalars (device [8]): Re Tr, Im Tr, purity sum |rho_ij|^2, max |rho - rho^dag|,
 *   sum_i <s_i^+ s_i^->, <a^dag a>, <N_exc>, non-finite flag (1.0 if any entry
 *   is NaN/Inf).  Diagonal readouts use Re rho_ss.
 * atom_pop (device [n]) p_i, photon_dist (device [c + 1]) P(m),
 * exc_dist (device [n + c + 1]) P_k,
 * photon_state (device [min(n, c) + 1]) Eq. (13) on the sector: sum of rho_ss
 *   over the states with m photons and n - m excited atoms,
 * dicke (device [min(n, c) + 1]) Eq. (13) on the symmetric state: <v_m| rho |v_m>
 *   with v_m = binom(n, m)^(-1/2) times the sum of those same basis states, i.e.
 *   the sum of Re rho_st over pairs of them divided by binom(n, m) (equal to
 *   photon_state[m] only when rho has no coherence between them);
 * each output but scalars may be NULL.
 * ws: device workspace of tc_observables_workspace_size bytes (partial sums;
 * the reductions run in a fixed order, so reruns are bitwise identical). */
int tc_observables_workspace_size(int64_t N, size_t* bytes);
int tc_observables(const tc_model* m, const void* rho, int32_t rho_dtype,
                   int64_t N, int64_t ldr, double* scalars, double* atom_pop,
                   double* photon_dist, double* exc_dist, double* photon_state,
                   double* dicke, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * readout and results as tc_observables, bit for bit, with no workspace
 * argument.  The partial sums live in a 16 MiB device array inside the
 * library, one per GPU, held until the process ends; its address is looked up
 * on the first call on each device.  No call allocates or frees device
 * memory.  Every call on one GPU shares that GPU's array (it needs no
 * clearing: each pass writes all of its partials before they are read), so
 * calls that overlap on one GPU, e.g. on two streams, race; calls ordered on
 * one stream do not.  N beyond tc_observables_noalloc_max_dim (37 120) gives
 * TC_ERR_UNSUPPORTED before any device work. */
int tc_observables_noalloc_max_dim(int64_t* N);
int tc_observables_noalloc(const tc_model* m, const void* rho, int32_t rho_dtype,
                           int64_t N, int64_t ldr, double* scalars, double* atom_pop,
                           double* photon_dist, double* exc_dist, double* photon_state,
                           double* dicke, void* stream);

/* ------------------------------------------------- a9: differentiation */

int tc_evolve_backward_workspace_size(const tc_model* m, int64_t N,
                                      const tc_evolve_opts* o, size_t* bytes);

/* With o->sectors = 1 the sweep runs by excitation sectors: O, U and every
 * dH/dtheta conserve the excitation number, so L and its gradient depend on
 * the diagonal blocks of rho only and the adjoint splits into one independent
 * sweep per sector on d_k x d_k blocks (grouped products, G_k = L(A_k, M_k)
 * per block); the checkpoints are the same full matrices.
 * Gradient of L = Tr(O rho(steps)), O = sum_i s_i^+ s_i^- (TC_OBS_EXCITED_TOTAL),
 * with respect to g_i and delta_i (w_a,i = 1 + delta_i), for a run of tc_evolve
 * with the same model, U and opts (frame lab, no renormalisation) whose
 * checkpoints (device [steps/checkpoint_every + 1][N][N], rho_dtype) were
 * recorded.  Adjoint: O_S = O, O_{s-1} = U^dag O_s U, M = sum_s rho_{s-1} U^dag O_s,
 * G = L(A, M) the Frechet derivative of exp at A = -i H dt, and
 * dL/dtheta = 2 Re Tr(dA/dtheta G).  H (device, N x N) is the Hamiltonian that
 * built U.  loss_out (device [1] or NULL), grad_g / grad_delta (device [n]). */
int tc_evolve_backward(const tc_model* m, const double* H, int64_t ldh,
                       const tc_c128* U, int64_t ldu, int64_t N,
                       const tc_evolve_opts* o, const void* checkpoints,
                       int32_t observable, double* loss_out,
                       double* grad_g, double* grad_delta,
                       void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------ kernel-level entry points */

/* C = alpha op(A) op(B) + beta C for complex FP64 N x N matrices (device,
 * tc_c128, row-major, leading dimensions lda/ldb/ldc >= N), op = identity,
 * conjugate (op_* = 1) or transpose (op_* = 2) or conjugate transpose (3).
 * ws: device workspace of tc_gemm_workspace_size bytes.  Runs the same MFMA
 * kernel as the FP64 step. */
int tc_gemm_workspace_size(int64_t M, int64_t N, int64_t K, int32_t mode, size_t* bytes);
int tc_zgemm(int64_t M, int64_t N, int64_t K, tc_c128 alpha,
             const tc_c128* A, int64_t lda, int32_t op_a,
             const tc_c128* B, int64_t ldb, int32_t op_b,
             tc_c128 beta, tc_c128* C, int64_t ldc, int32_t mode,
             void* ws, size_t ws_bytes, void* stream);

/* hi = RNE_bf16(x), lo = RNE_bf16(x - hi) for count binary32 values (device);
 * hi, lo: device uint16 bit patterns.  The rounding used by TC_GEMM_SPLIT_BF16. */
int tc_split_bf16(const float* x, int64_t count, uint16_t* hi, uint16_t* lo, void* stream);

/* ------------------------------------------------- a8: tile autotuner */

/* tc_evolve with count > 1 and FP64 / FP32 products runs each product phase
 * of a step as one persistent launch per tile shape over the tiles of every
 * instance; the shape of each instance comes from a table indexed by its
 * dimension bucket (N <= 256, <= 1024, <= 4096, larger).  tc_autotune times
 * both shapes (1: 128 x 128 tiles, 2: 64 x 64 tiles) on an N x N x N complex
 * product per bucket (N capped at max_N) with hipEvents, stores the faster
 * one in the process-wide table and, if the environment variable
 * TC_AUTOTUNE_CACHE names a file, writes the table there; the table is read
 * from that file on first use.  Synchronises the stream.  ws: device
 * workspace of tc_autotune_workspace_size bytes (three max_N^2 matrices). */
int tc_autotune_workspace_size(int32_t gemm_mode, int64_t max_N, size_t* bytes);
int tc_autotune(int32_t gemm_mode, int64_t max_N, void* ws, size_t ws_bytes, void* stream);
/* Host-only: the tile shape (1 or 2) the table holds for dimension N. */
int tc_autotune_query(int32_t gemm_mode, int64_t N, int32_t* variant);

/* ------------------------------------------------------ kernel timing */

/* Kernel classes of tc_profile_read. */
#define TC_KERNEL_GEMM_F64    0   /* FP64 MFMA products (step, expm)            */
#define TC_KERNEL_GEMM_F32    1   /* FP32 MFMA products                         */
#define TC_KERNEL_SPLIT_BF16  2   /* split-BF16 MFMA products                   */

/* enable != 0: from now on every product-kernel launch is bracketed by two
 * hipEvents recorded on the stream it is launched on (process-wide; previous
 * records are dropped).  enable == 0 stops recording.  Host-only. */
int tc_profile_enable(int32_t enable);
/* Waits for the recorded events of one kernel class and returns the summed
 * kernel time (ms) and the number of launches since tc_profile_enable(1). */
int tc_profile_read(int32_t kernel, double* total_ms, int64_t* launches);

/* ------------------------------------------------------ MFMA rate probe */

/* A diagnostic for reading the product kernels' rooflines (not a step of the
 * method; for callers that measure the hardware).  Every wave of one
 * 512-thread workgroup per compute unit issues `iters` rounds of MFMAs of one
 * kind back to back on operands held in registers, with no memory traffic:
 *   TC_PROBE_BF16_16X16X32  v_mfma_f32_16x16x32_bf16, 16 accumulators (the
 *                           instruction of the split-BF16 products)
 *   TC_PROBE_BF16_32X32X16  v_mfma_f32_32x32x16_bf16, 4 accumulators
 *   TC_PROBE_F64_16X16X4    v_mfma_f64_16x16x4_f64, 8 accumulators (the FP64
 *                           products)
 * random_operands != 0: operand bits from a fixed integer sequence per thread
 * (finite values); 0: zero operands.  out: device buffer of out_count floats,
 * caller-owned, at least 512 x (compute units); it receives each thread's
 * accumulator sum, which keeps the work from being optimised away.  iters in
 * 1 .. 1e7.  Returns the elapsed milliseconds (hipEvents on the stream) and
 * the flops issued (2 per multiply-add); synchronises the stream. */
#define TC_PROBE_BF16_16X16X32 0
#define TC_PROBE_BF16_32X32X16 1
#define TC_PROBE_F64_16X16X4   2
int tc_mfma_probe(int32_t kind, int32_t random_operands, int32_t iters, float* out,
                  int64_t out_count, double* ms, double* flop, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* TCM_H */
