// tc_evolve: the time-stepping loop rho <- U rho U^dag (Eq. (6)) with readouts,
// renormalisation, checkpoints and the frame change; plus tc_observables,
// tc_zgemm and tc_split_bf16.
#include <cmath>
#include <string>
#include <vector>
#include <algorithm>

#include "common.h"
#include "gemm_mfma.h"
#include "gemm_bf16.h"
#include "kernels.h"
#include "profile.h"

namespace tcm {
namespace {

size_t elem_bytes(int dtype) { return dtype == TC_C128 ? 16 : 8; }

// Buffers of one instance, carved from the workspace.
struct InstPlan {
  ModelArgs m;
  int64_t N = 0;
  // product operand (U in the lab frame, D = U~ - I in the rotating frame)
  const void* op = nullptr; int64_t ldop = 0;
  void* op_own = nullptr;       // workspace copy when converted
  // master state (c128 for F64, c64 for F32 / split)
  void* rho = nullptr; int64_t ldr = 0;
  bool rho_converted = false;
  void* X = nullptr; int64_t ldx = 0;
  double* scratch = nullptr;    // [4]: trace, non-finite flag, ...
  // graph-captured single-instance steps read their record index on the device
  ReadoutItem* ritem = nullptr;
  int* counter = nullptr;
  SplitPlanes planes;           // split-BF16 operand planes
  // FP64 / FP32: partial sums of a product's last round split over K
  // (shared by the instances that are stepped one after another)
  void* tail_ws = nullptr; size_t tail_ws_bytes = 0;
  // excitation-sector stepping (opts.sectors): rho and X in the sorted order
  // Each sector's positions are padded to a multiple of the product tile
  // (padding states hold exact zeros), so every block product is whole tiles.
  // stepping within one excitation sector (tc_evolve_sector): rho, U are the
  // d_k x d_k blocks; inv maps every basis state to its position or -1
  int in_sector = -1;
  bool sectors = false;
  int64_t Np = 0;                    // padded dimension of the sorted order
  int svar = 2;                      // tile shape of the grouped block products (1: 128, 2: 64)
  std::vector<int64_t> sdim;         // d_k: states of sector k
  std::vector<int64_t> spo, spd;     // sector k: padded positions [spo[k], spo[k] + spd[k])
  std::vector<size_t> boff;          // element offset of block k (spd[k]^2) in blocks
  int32_t* perm = nullptr;           // device [Np]: basis state at a position, -1 = padding
  int32_t* inv = nullptr;            // device [N]: position of basis state
  int32_t* secpos = nullptr;         // device [Np]: sector of a position
  void* blocks = nullptr;            // U_k (lab) or D_k = e^{i w_c k dt} U_k - I (rotating)
  char* items = nullptr;             // descriptors of the two grouped products
  GroupedProducts g1, g2;
  // split-BF16 by sectors: planes of each block (op and conj(op)^T), of X
  // (rows) and of rho hat^T (rows = columns of rho hat), Np x Np
  std::vector<Planes4> sopA, sopB;
  Planes4 sXp, sRt;
  SplitGrouped sg1, sg2;
  // the block products of one step, largest blocks first (kept so that a
  // batch of instances can launch all of theirs together)
  std::vector<GemmDesc> sd1, sd2;
  std::vector<SplitProduct> ssd1, ssd2;
};

int validate_opts(const tc_evolve_opts* o) {
  TC_CHECK_ARG(o != nullptr, "opts is NULL");
  TC_CHECK_ARG(o->steps >= 0, "steps < 0");
  TC_CHECK_ARG(o->gemm_mode == TC_GEMM_F64 || o->gemm_mode == TC_GEMM_F32 ||
               o->gemm_mode == TC_GEMM_SPLIT_BF16, "unknown gemm_mode");
  TC_CHECK_ARG(o->rho_dtype == TC_C64 || o->rho_dtype == TC_C128, "unknown rho_dtype");
  TC_CHECK_ARG(o->frame == TC_FRAME_LAB || o->frame == TC_FRAME_ROTATING, "unknown frame");
  TC_CHECK_ARG(o->renorm_every >= 0, "renorm_every < 0");
  TC_CHECK_ARG(o->record_every >= 0, "record_every < 0");
  TC_CHECK_ARG(o->checkpoint_every >= 0, "checkpoint_every < 0");
  TC_CHECK_ARG(std::isfinite(o->dt), "dt not finite");
  TC_CHECK_ARG(o->sectors == 0 || o->sectors == 1, "sectors must be 0 or 1");
  return TC_OK;
}

int validate_instance(const tc_instance* in, const tc_evolve_opts* o, ModelArgs* m) {
  TC_CHECK_ARG(in != nullptr, "instance is NULL");
  TC_RETURN_IF(make_model_args(in->model, m));
  TC_CHECK_ARG(in->N == m->N, "instance N != (c+1) 2^n");
  TC_CHECK_ARG(in->U != nullptr && in->rho != nullptr, "U / rho is NULL");
  TC_CHECK_ARG(in->ldu >= in->N && in->ldr >= in->N, "leading dimension < N");
  if (in->pop_out || in->photon_dist_out || in->photon_state_out)
    TC_CHECK_ARG(o->record_every >= 1, "record_every must be >= 1 when records are requested");
  if (in->checkpoints)
    TC_CHECK_ARG(o->checkpoint_every >= 1, "checkpoint_every must be >= 1 with checkpoints");
  return TC_OK;
}

// Sector sizes d_k = sum_m binom(n, k - m) (m = 0..min(k, c)), k = 0..n + c.
void sector_sizes(int n, int c, std::vector<int64_t>& dim, std::vector<int64_t>& off) {
  std::vector<int64_t> binom(n + 1, 0);
  binom[0] = 1;
  for (int i = 1; i <= n; ++i)
    for (int j = i; j >= 1; --j) binom[j] += binom[j - 1];
  dim.assign(n + c + 1, 0);
  off.assign(n + c + 1, 0);
  for (int k = 0; k <= n + c; ++k) {
    for (int mm = 0; mm <= std::min(k, c); ++mm)
      if (k - mm <= n) dim[k] += binom[k - mm];
    if (k > 0) off[k] = off[k - 1] + dim[k - 1];
  }
}

void plan_sectors(const tc_evolve_opts& o, Arena& ar, InstPlan* p) {
  const int64_t N = p->N;
  const bool f64 = o.gemm_mode == TC_GEMM_F64;
  const size_t eb = f64 ? 16 : 8;
  // pad to the edge of the grouped product's tile (128 or 64; the split
  // product's tile is 128)
  const bool split = o.gemm_mode == TC_GEMM_SPLIT_BF16;
  p->sectors = true;
  std::vector<int64_t> off;
  sector_sizes(p->m.n, p->m.c, p->sdim, off);
  // FP64 blocks above 1024 states take 128 x 128 tiles (0.81 of the FP64 peak
  // on the padded work at N = 12288 against 0.75 with 64 x 64, for slightly
  // less time despite the extra padding); otherwise the autotuner's table
  const int64_t maxd = *std::max_element(p->sdim.begin(), p->sdim.end());
  p->svar = (f64 && maxd > 1024) ? 1 : tile_variant_for(N, f64);
  const int64_t q = split ? SPLIT_BM : (p->svar == 1 ? 128 : 64);
  const int ns = int(p->sdim.size());
  p->spo.assign(ns, 0);
  p->spd.assign(ns, 0);
  p->boff.assign(ns, 0);
  int64_t pos = 0;
  size_t tot = 0;
  for (int k = 0; k < ns; ++k) {
    p->spo[k] = pos;
    p->spd[k] = (p->sdim[k] + q - 1) / q * q;
    pos += p->spd[k];
    p->boff[k] = tot;
    tot += size_t(p->spd[k]) * size_t(p->spd[k]);
  }
  p->Np = pos;
  const size_t NN = size_t(pos) * size_t(pos);
  p->rho = ar.take(NN * eb); p->ldr = pos; p->rho_converted = true;
  p->X = ar.take(NN * eb); p->ldx = pos;
  p->blocks = ar.take(tot * eb);
  p->perm = static_cast<int32_t*>(ar.take(size_t(pos) * 4));
  p->inv = static_cast<int32_t*>(ar.take(size_t(N) * 4));
  p->secpos = static_cast<int32_t*>(ar.take(size_t(pos) * 4));
  p->items = static_cast<char*>(ar.take(2 * (split ? split_grouped_bytes(ns) : grouped_bytes(ns))));
  if (split) {
    p->sopA.resize(ns);
    p->sopB.resize(ns);
    for (int k = 0; k < ns; ++k) {
      p->sopA[k] = split_take_planes(ar, p->spd[k], p->spd[k]);
      p->sopB[k] = split_take_planes(ar, p->spd[k], p->spd[k]);
    }
    p->sXp = split_take_planes(ar, pos, pos);
    p->sRt = split_take_planes(ar, pos, pos);
  }
}

// Slots for the partial sums of a dense product's last round split over K:
// one 128 x 128 tile of complex elements per slot (16 B in FP64, 8 B as FP32
// in the FP32 and split-BF16 products), 8 per tile of the N x N product and
// at most 256 (64 MB in FP64); none for a single tile row, whose K is too
// short to split.
size_t tail_bytes(const InstPlan& p, const tc_evolve_opts& o) {
  if (o.sectors) return 0;
  const int64_t t = (p.N + 127) / 128;
  if (t < 2) return 0;
  const size_t eb = o.gemm_mode == TC_GEMM_F64 ? 16 : 8;
  return size_t(std::min<int64_t>(256, 8 * t * t)) * 128 * 128 * eb;
}

// One region of slots for instances stepped one after another on one
// stream (a single instance, or a batch that is not a grouped launch).
void take_tail(Arena& ar, const tc_evolve_opts& o, InstPlan* plans, int count) {
  size_t bytes = 0;
  for (int b = 0; b < count; ++b) bytes = std::max(bytes, tail_bytes(plans[b], o));
  if (bytes == 0) return;
  void* ws = ar.take(bytes);
  for (int b = 0; b < count; ++b) {
    if (tail_bytes(plans[b], o) == 0) continue;
    if (o.gemm_mode == TC_GEMM_SPLIT_BF16) {
      plans[b].planes.tail_acc = static_cast<float*>(ws);
      plans[b].planes.tail_slots = int(bytes / (size_t(128) * 128 * 8));
    } else {
      plans[b].tail_ws = ws;
      plans[b].tail_ws_bytes = bytes;
    }
  }
}

void plan_instance(const tc_instance& in, const tc_evolve_opts& o, const ModelArgs& m, Arena& ar,
                   InstPlan* p) {
  const int64_t N = in.N;
  const size_t NN = size_t(N) * size_t(N);
  p->m = m;
  p->N = N;
  p->scratch = static_cast<double*>(ar.take(4 * sizeof(double)));
  if (o.use_graph) {
    p->ritem = static_cast<ReadoutItem*>(ar.take(sizeof(ReadoutItem)));
    p->counter = static_cast<int*>(ar.take(sizeof(int)));
  }
  if (o.sectors) {
    plan_sectors(o, ar, p);
    return;
  }
  if (p->in_sector >= 0) p->inv = static_cast<int32_t*>(ar.take(size_t(m.N) * 4));
  if (o.gemm_mode == TC_GEMM_F64) {
    if (o.rho_dtype == TC_C128) {
      p->rho = in.rho; p->ldr = in.ldr; p->rho_converted = false;
    } else {
      p->rho = ar.take(NN * 16); p->ldr = N; p->rho_converted = true;
    }
    if (o.frame == TC_FRAME_LAB) {
      p->op = in.U; p->ldop = in.ldu;
    } else {
      p->op_own = ar.take(NN * 16); p->op = p->op_own; p->ldop = N;
    }
    p->X = ar.take(NN * 16); p->ldx = N;
  } else {
    // FP32 and split-BF16 keep an FP32 master
    if (o.rho_dtype == TC_C64) {
      p->rho = in.rho; p->ldr = in.ldr; p->rho_converted = false;
    } else {
      p->rho = ar.take(NN * 8); p->ldr = N; p->rho_converted = true;
    }
    p->op_own = ar.take(NN * 8); p->op = p->op_own; p->ldop = N;
    p->X = ar.take(NN * 8); p->ldx = N;
    if (o.gemm_mode == TC_GEMM_SPLIT_BF16) split_plan(ar, N, &p->planes);
  }
}

int readout(const InstPlan& p, const tc_evolve_opts& o, double* pop, double* pdist,
            double* pstate, hipStream_t s) {
  if (o.gemm_mode == TC_GEMM_F64)
    return launch_readout_c128(p.m, static_cast<const c128*>(p.rho), p.ldr, pop, pdist, s,
                               p.inv, pstate);
  return launch_readout_c64(p.m, static_cast<const c64*>(p.rho), p.ldr, pop, pdist, s, p.inv,
                            pstate);
}

// Sector order: rebuilds the lower block triangle of rho hat from the upper one
// (the stepper forms only blocks j <= k).
int mirror(InstPlan& p, const tc_evolve_opts& o, hipStream_t s) {
  if (o.gemm_mode == TC_GEMM_F64)
    return launch_mirror_lower_c128(static_cast<c128*>(p.rho), p.ldr, p.Np, p.secpos, s);
  return launch_mirror_lower_c64(static_cast<c64*>(p.rho), p.ldr, p.Np, p.secpos, s);
}

// Sector order -> basis order: dst[s][t] = rho hat[inv[s]][inv[t]] (after mirror).
int unpermute_to(InstPlan& p, const tc_evolve_opts& o, void* dst, int64_t ldd, int dst_dtype,
                 hipStream_t s) {
  const int64_t N = p.N;
  if (o.gemm_mode == TC_GEMM_F64) {
    const c128* r = static_cast<const c128*>(p.rho);
    return dst_dtype == TC_C128
        ? launch_gather_c128_c128(r, p.ldr, p.inv, 0, 0, N, N, 1.0, 0.0, false,
                                  static_cast<c128*>(dst), ldd, s)
        : launch_gather_c128_c64(r, p.ldr, p.inv, 0, 0, N, N, 1.0, 0.0, false,
                                 static_cast<c64*>(dst), ldd, s);
  }
  const c64* r = static_cast<const c64*>(p.rho);
  return dst_dtype == TC_C128
      ? launch_gather_c64_c128(r, p.ldr, p.inv, 0, 0, N, N, 1.0, 0.0, false,
                               static_cast<c128*>(dst), ldd, s)
      : launch_gather_c64_c64(r, p.ldr, p.inv, 0, 0, N, N, 1.0, 0.0, false,
                              static_cast<c64*>(dst), ldd, s);
}

// Basis order -> sector order: rho hat[i][j] = src[perm[i]][perm[j]] (0 at padding).
int permute_from(InstPlan& p, const tc_evolve_opts& o, const void* src, int64_t lds, int src_dtype,
                 hipStream_t s) {
  const int64_t Np = p.Np;
  if (o.gemm_mode == TC_GEMM_F64) {
    c128* r = static_cast<c128*>(p.rho);
    return src_dtype == TC_C128
        ? launch_gather_c128_c128(static_cast<const c128*>(src), lds, p.perm, 0, 0, Np, Np, 1.0,
                                  0.0, false, r, p.ldr, s)
        : launch_gather_c64_c128(static_cast<const c64*>(src), lds, p.perm, 0, 0, Np, Np, 1.0,
                                 0.0, false, r, p.ldr, s);
  }
  c64* r = static_cast<c64*>(p.rho);
  return src_dtype == TC_C128
      ? launch_gather_c128_c64(static_cast<const c128*>(src), lds, p.perm, 0, 0, Np, Np, 1.0,
                               0.0, false, r, p.ldr, s)
      : launch_gather_c64_c64(static_cast<const c64*>(src), lds, p.perm, 0, 0, Np, Np, 1.0, 0.0,
                              false, r, p.ldr, s);
}

// exp(dt L) after a unitary step when the model has a Lindblad term; in the
// split form the next step's rho^T planes are re-split from the damped master.
int dissipate(InstPlan& p, const tc_evolve_opts& o, hipStream_t s) {
  if (!(p.m.kappa > 0.0 || p.m.gamma > 0.0)) return TC_OK;
  if (p.sectors) {
    // the damping channels act on the basis order: convert into X (free
    // between steps), damp, convert back
    const int md = o.gemm_mode == TC_GEMM_F64 ? TC_C128 : TC_C64;
    TC_RETURN_IF(mirror(p, o, s));
    TC_RETURN_IF(unpermute_to(p, o, p.X, p.N, md, s));
    if (md == TC_C128)
      TC_RETURN_IF(launch_dissipation_c128(p.m, static_cast<c128*>(p.X), p.N, o.dt, s));
    else
      TC_RETURN_IF(launch_dissipation_c64(p.m, static_cast<c64*>(p.X), p.N, o.dt, s));
    TC_RETURN_IF(permute_from(p, o, p.X, p.N, md, s));
    if (o.gemm_mode == TC_GEMM_SPLIT_BF16)
      TC_RETURN_IF(split_matrix(static_cast<const c64*>(p.rho), p.ldr, p.Np, p.Np, true, false,
                                p.sRt, s));
    return TC_OK;
  }
  if (o.gemm_mode == TC_GEMM_F64)
    return launch_dissipation_c128(p.m, static_cast<c128*>(p.rho), p.ldr, o.dt, s);
  TC_RETURN_IF(launch_dissipation_c64(p.m, static_cast<c64*>(p.rho), p.ldr, o.dt, s));
  if (o.gemm_mode == TC_GEMM_SPLIT_BF16)
    TC_RETURN_IF(split_state(static_cast<const c64*>(p.rho), p.ldr, p.N, p.planes, s));
  return TC_OK;
}

int renorm(InstPlan& p, const tc_evolve_opts& o, hipStream_t s) {
  const int64_t n = p.sectors ? p.Np : p.N;
  if (p.sectors) TC_RETURN_IF(mirror(p, o, s));
  if (o.gemm_mode == TC_GEMM_F64)
    return launch_renorm_c128(static_cast<c128*>(p.rho), p.ldr, n, p.scratch, s);
  TC_RETURN_IF(launch_renorm_c64(static_cast<c64*>(p.rho), p.ldr, n, p.scratch, s));
  if (o.gemm_mode == TC_GEMM_SPLIT_BF16 && p.sectors)
    TC_RETURN_IF(split_matrix(static_cast<const c64*>(p.rho), p.ldr, p.Np, p.Np, true, false,
                              p.sRt, s));
  else if (o.gemm_mode == TC_GEMM_SPLIT_BF16)
    TC_RETURN_IF(split_state(static_cast<const c64*>(p.rho), p.ldr, p.N, p.planes, s));
  return TC_OK;
}

void step_descs(const InstPlan& p, const tc_evolve_opts& o, GemmDesc& g1, GemmDesc& g2);

// One step of Eq. (6) for FP64 / FP32:
//   lab:      X = U rho,          rho' = X U^dag = X conj(U)   (U symmetric)
//   rotating: X = rho + D rho,    rho' = X + X conj(D)         (U~ = I + D symmetric)
// rho' is Hermitian: unless full_product is set, the second product forms only
// its upper tile triangle and mirrors it.
int step_mfma(InstPlan& p, const tc_evolve_opts& o, hipStream_t s) {
  GemmDesc g1, g2;
  step_descs(p, o, g1, g2);
  if (o.gemm_mode == TC_GEMM_F64) {
    TC_RETURN_IF(gemm_f64(g1, s));
    TC_RETURN_IF(gemm_f64(g2, s));
  } else {
    TC_RETURN_IF(gemm_f32(g1, s));
    TC_RETURN_IF(gemm_f32(g2, s));
  }
  return TC_OK;
}

int copy_checkpoint(const InstPlan& p, const tc_instance& in, const tc_evolve_opts& o, int64_t slot,
                    double t, hipStream_t s) {
  const size_t eb = elem_bytes(o.rho_dtype);
  const size_t NN = size_t(p.N) * size_t(p.N);
  char* dst = static_cast<char*>(in.checkpoints) + size_t(slot) * NN * eb;
  const bool master128 = o.gemm_mode == TC_GEMM_F64;
  if (p.sectors) {
    TC_RETURN_IF(mirror(const_cast<InstPlan&>(p), o, s));
    TC_RETURN_IF(unpermute_to(const_cast<InstPlan&>(p), o, dst, p.N, o.rho_dtype, s));
  } else if (master128 && o.rho_dtype == TC_C128) {
    TC_TRY_HIP(hipMemcpy2DAsync(dst, p.N * 16, p.rho, p.ldr * 16, p.N * 16, p.N,
                                hipMemcpyDeviceToDevice, s));
  } else if (!master128 && o.rho_dtype == TC_C64) {
    TC_TRY_HIP(hipMemcpy2DAsync(dst, p.N * 8, p.rho, p.ldr * 8, p.N * 8, p.N,
                                hipMemcpyDeviceToDevice, s));
  } else if (master128) {
    TC_RETURN_IF(launch_copy_c128_to_c64(static_cast<const c128*>(p.rho), p.ldr,
                                         reinterpret_cast<c64*>(dst), p.N, p.N, p.N, s));
  } else {
    TC_RETURN_IF(launch_copy_c64_to_c128(static_cast<const c64*>(p.rho), p.ldr,
                                         reinterpret_cast<c128*>(dst), p.N, p.N, p.N, s));
  }
  if (o.frame == TC_FRAME_ROTATING && t != 0.0 && p.in_sector < 0) {
    if (o.rho_dtype == TC_C128)
      TC_RETURN_IF(launch_frame_phase_c128(p.m, reinterpret_cast<c128*>(dst), p.N, t, s));
    else
      TC_RETURN_IF(launch_frame_phase_c64(p.m, reinterpret_cast<c64*>(dst), p.N, t, s));
  }
  return TC_OK;
}

// Sector stepping: sorted order, blocks of U (or D), and the descriptors of
// the two grouped products of a step (largest sectors first, so the
// persistent launch starts on the longest tiles).
// Split-BF16 by sectors: planes of every block and of rho hat^T, then the two
// grouped split products of a step,
//   X_{k,k:} = U_k rho_{k,k:}   (rotating: + rho_{k,k:}), planes of X written by rows
//   rho'_{:k,k} = X_{:k,k} U_k^dag (rotating: + X_{:k,k}), planes of rho'^T written
// with K offsets at sector starts (multiples of 128).
int prepare_sector_split(InstPlan& p, const tc_evolve_opts& o, const std::vector<int>& order,
                         bool build, hipStream_t s) {
  const int64_t Np = p.Np;
  const bool rot = o.frame == TC_FRAME_ROTATING;
  c64* rho = static_cast<c64*>(p.rho);
  c64* X = static_cast<c64*>(p.X);
  for (size_t k = 0; k < p.spd.size(); ++k) {
    const c64* blk = static_cast<const c64*>(p.blocks) + p.boff[k];
    const int64_t d = p.spd[k];
    TC_RETURN_IF(split_matrix(blk, d, d, d, false, false, p.sopA[k], s));
    TC_RETURN_IF(split_matrix(blk, d, d, d, true, true, p.sopB[k], s));
  }
  TC_TRY_HIP(hipMemsetAsync(p.sXp.base, 0, size_t(4) * p.sXp.rows * p.sXp.ld * 2, s));
  TC_RETURN_IF(split_matrix(rho, p.ldr, Np, Np, true, false, p.sRt, s));
  std::vector<SplitProduct>& d1 = p.ssd1;
  std::vector<SplitProduct>& d2 = p.ssd2;
  d1.clear(); d2.clear();
  for (int k : order) {
    const int64_t off = p.spo[k], d = p.spd[k];
    SplitProduct g1;                    // X_{k, k:} = op_k rho_{k, k:}
    g1.A = p.sopA[k].base; g1.lda = p.sopA[k].ld;
    g1.B = p.sRt.base + plane_offset(p.sRt.ld, off, off, 0); g1.ldb = p.sRt.ld;
    g1.M = d; g1.N = Np - off; g1.Kp = d;
    if (rot) { g1.br = 1.f; g1.Cin = rho + off * p.ldr + off; g1.ldcin = p.ldr; }
    g1.Cf = X + off * p.ldx + off; g1.ldcf = p.ldx;
    g1.P = p.sXp.base + plane_offset(p.sXp.ld, off, off, 0); g1.ldp = p.sXp.ld;
    SplitProduct g2;                    // rho'_{:k, k} = X_{:k, k} op_k^dag
    g2.A = p.sXp.base + plane_offset(p.sXp.ld, 0, off, 0); g2.lda = p.sXp.ld;
    g2.B = p.sopB[k].base; g2.ldb = p.sopB[k].ld;
    g2.M = off + d; g2.N = d; g2.Kp = d;
    if (rot) { g2.br = 1.f; g2.Cin = X + off; g2.ldcin = p.ldx; }
    g2.Cf = rho + off; g2.ldcf = p.ldr;
    g2.P = p.sRt.base + plane_offset(p.sRt.ld, off, 0, 0); g2.ldp = p.sRt.ld; g2.p_trans = true;
    d1.push_back(g1);
    d2.push_back(g2);
  }
  if (!build) return TC_OK;
  const int ns = int(p.spd.size());
  TC_RETURN_IF(split_grouped_build(d1, p.items, &p.sg1, s));
  TC_RETURN_IF(split_grouped_build(d2, p.items + split_grouped_bytes(ns), &p.sg2, s));
  return TC_OK;
}

// build: also upload the grouped products of the instance's own step (false
// when a batch launches the blocks of all its instances together).
int prepare_sectors(InstPlan& p, const tc_instance& in, const tc_evolve_opts& o, hipStream_t s,
                    bool build = true) {
  TC_TRY_HIP(hipMemsetAsync(p.scratch, 0, 4 * sizeof(double), s));
  const int64_t N = p.N, Np = p.Np;
  const int n = p.m.n;
  const int ns = int(p.sdim.size());
  std::vector<int32_t> perm(Np, -1), inv(N), sec(Np);
  std::vector<int64_t> next(p.spo);
  const uint64_t mask = (uint64_t(1) << n) - 1;
  for (int64_t st = 0; st < N; ++st) {
    const int k = int(st >> n) + __builtin_popcountll(uint64_t(st) & mask);
    const int64_t pos = next[k]++;
    perm[pos] = int32_t(st);
    inv[st] = int32_t(pos);
  }
  for (int k = 0; k < ns; ++k)
    for (int64_t i = 0; i < p.spd[k]; ++i) sec[p.spo[k] + i] = k;
  TC_TRY_HIP(hipMemcpyAsync(p.perm, perm.data(), size_t(Np) * 4, hipMemcpyHostToDevice, s));
  TC_TRY_HIP(hipMemcpyAsync(p.inv, inv.data(), size_t(N) * 4, hipMemcpyHostToDevice, s));
  TC_TRY_HIP(hipMemcpyAsync(p.secpos, sec.data(), size_t(Np) * 4, hipMemcpyHostToDevice, s));
  TC_TRY_HIP(hipStreamSynchronize(s));   // the maps are host memory of this call
  TC_RETURN_IF(permute_from(p, o, in.rho, in.ldr, o.rho_dtype, s));
  const bool rot = o.frame == TC_FRAME_ROTATING;
  const bool f64 = o.gemm_mode == TC_GEMM_F64;
  const size_t eb = f64 ? 16 : 8;
  const c128* U = reinterpret_cast<const c128*>(in.U);
  for (int k = 0; k < ns; ++k) {
    // rotating frame: within sector k the frame factor e^{i w_c N dt} is the
    // scalar e^{i w_c k dt}, so D_k = e^{i w_c k dt} U_k - I (0 at padding)
    double ph_re = 1.0, ph_im = 0.0;
    if (rot) {
      ph_re = std::cos(p.m.omega_c * double(k) * o.dt);
      ph_im = std::sin(p.m.omega_c * double(k) * o.dt);
    }
    const int64_t off = p.spo[k], d = p.spd[k];
    char* blk = static_cast<char*>(p.blocks) + p.boff[k] * eb;
    if (f64)
      TC_RETURN_IF(launch_gather_c128_c128(U, in.ldu, p.perm, off, off, d, d, ph_re, ph_im, rot,
                                           reinterpret_cast<c128*>(blk), d, s));
    else
      TC_RETURN_IF(launch_gather_c128_c64(U, in.ldu, p.perm, off, off, d, d, ph_re, ph_im, rot,
                                          reinterpret_cast<c64*>(blk), d, s));
  }
  std::vector<int> order(ns);
  for (int k = 0; k < ns; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return p.spd[a] > p.spd[b]; });
  if (o.gemm_mode == TC_GEMM_SPLIT_BF16) return prepare_sector_split(p, o, order, build, s);
  auto at = [&](void* base, int64_t r, int64_t c, int64_t ld) {
    return static_cast<void*>(static_cast<char*>(base) + (size_t(r) * size_t(ld) + size_t(c)) * eb);
  };
  std::vector<GemmDesc>& d1 = p.sd1;
  std::vector<GemmDesc>& d2 = p.sd2;
  d1.clear(); d2.clear();
  for (int k : order) {
    const int64_t off = p.spo[k], d = p.spd[k];
    const void* blk = static_cast<char*>(p.blocks) + p.boff[k] * eb;
    GemmDesc g1;                        // X_{k, k:} = U_k rho_{k, k:}
    g1.M = d; g1.N = Np - off; g1.K = d;
    g1.A = blk; g1.lda = d; g1.a_kmaj = false;
    g1.B = at(p.rho, off, off, p.ldr); g1.ldb = p.ldr; g1.b_kmaj = true;
    g1.C = at(p.X, off, off, p.ldx); g1.ldc = p.ldx;
    if (rot) { g1.Cin = g1.B; g1.ldcin = p.ldr; g1.beta_re = 1.0; }
    GemmDesc g2;                        // rho'_{:k, k} = X_{:k, k} U_k^dag
    g2.M = off + d; g2.N = d; g2.K = d;
    g2.A = at(p.X, 0, off, p.ldx); g2.lda = p.ldx; g2.a_kmaj = false;
    g2.B = blk; g2.ldb = d; g2.b_kmaj = true; g2.conj_b = true;
    g2.C = at(p.rho, 0, off, p.ldr); g2.ldc = p.ldr;
    if (rot) { g2.Cin = g2.A; g2.ldcin = p.ldx; g2.beta_re = 1.0; }
    d1.push_back(g1);
    d2.push_back(g2);
  }
  if (!build) return TC_OK;
  const int v = p.svar;
  TC_RETURN_IF(grouped_build(d1, f64, v, p.items, &p.g1, s));
  TC_RETURN_IF(grouped_build(d2, f64, v, p.items + grouped_bytes(ns), &p.g2, s));
  p.g1.persistent = p.g2.persistent = false;     // whole tiles: one workgroup each
  return TC_OK;
}

// One-sector run: position of every basis state in the sector's order (-1 outside).
int upload_sector_map(InstPlan& p, hipStream_t s) {
  const int n = p.m.n, k = p.in_sector;
  const uint64_t mask = (uint64_t(1) << n) - 1;
  std::vector<int32_t> map(p.m.N, -1);
  int32_t pos = 0;
  for (int64_t st = 0; st < p.m.N; ++st)
    if (int(st >> n) + __builtin_popcountll(uint64_t(st) & mask) == k) map[st] = pos++;
  TC_TRY_HIP(hipMemcpyAsync(p.inv, map.data(), map.size() * 4, hipMemcpyHostToDevice, s));
  TC_TRY_HIP(hipStreamSynchronize(s));   // map is host memory of this call
  return TC_OK;
}

int prepare(InstPlan& p, const tc_instance& in, const tc_evolve_opts& o, hipStream_t s) {
  if (p.sectors) return prepare_sectors(p, in, o, s);
  if (p.in_sector >= 0) TC_RETURN_IF(upload_sector_map(p, s));
  TC_TRY_HIP(hipMemsetAsync(p.scratch, 0, 4 * sizeof(double), s));
  // master state
  if (p.rho_converted) {
    if (o.gemm_mode == TC_GEMM_F64)
      TC_RETURN_IF(launch_copy_c64_to_c128(static_cast<const c64*>(in.rho), in.ldr,
                                           static_cast<c128*>(p.rho), p.ldr, p.N, p.N, s));
    else
      TC_RETURN_IF(launch_copy_c128_to_c64(static_cast<const c128*>(in.rho), in.ldr,
                                           static_cast<c64*>(p.rho), p.ldr, p.N, p.N, s));
  }
  // product operand
  const c128* U = reinterpret_cast<const c128*>(in.U);
  // within one sector the frame factor e^{i w_c N dt} is the scalar e^{i w_c k dt}
  const double ph = p.m.omega_c * double(p.in_sector) * o.dt;
  if (o.gemm_mode == TC_GEMM_F64) {
    if (o.frame == TC_FRAME_ROTATING && p.in_sector >= 0)
      TC_RETURN_IF(launch_phase_minus_identity_c128(U, in.ldu, std::cos(ph), std::sin(ph),
                                                    static_cast<c128*>(p.op_own), p.ldop, p.N, s));
    else if (o.frame == TC_FRAME_ROTATING)
      TC_RETURN_IF(launch_rotating_d(p.m, U, in.ldu, o.dt, static_cast<c128*>(p.op_own), p.ldop, s));
  } else {
    if (o.frame == TC_FRAME_ROTATING && p.in_sector >= 0)
      TC_RETURN_IF(launch_phase_minus_identity_c64(U, in.ldu, std::cos(ph), std::sin(ph),
                                                   static_cast<c64*>(p.op_own), p.ldop, p.N, s));
    else if (o.frame == TC_FRAME_ROTATING)
      TC_RETURN_IF(launch_rotating_d_c64(p.m, U, in.ldu, o.dt, static_cast<c64*>(p.op_own), p.ldop, s));
    else
      TC_RETURN_IF(launch_copy_c128_to_c64(U, in.ldu, static_cast<c64*>(p.op_own), p.ldop, p.N, p.N, s));
  }
  if (o.gemm_mode == TC_GEMM_SPLIT_BF16) {
    TC_RETURN_IF(split_operand(static_cast<const c64*>(p.op), p.ldop, p.N, p.planes, s));
    TC_RETURN_IF(split_state(static_cast<const c64*>(p.rho), p.ldr, p.N, p.planes, s));
  }
  return TC_OK;
}

int finish(InstPlan& p, const tc_instance& in, const tc_evolve_opts& o, hipStream_t s) {
  const double T = double(o.steps) * o.dt;
  if (p.sectors) {
    TC_RETURN_IF(mirror(p, o, s));
    TC_RETURN_IF(unpermute_to(p, o, in.rho, in.ldr, o.rho_dtype, s));
    if (o.frame == TC_FRAME_ROTATING && T != 0.0) {
      if (o.rho_dtype == TC_C128)
        TC_RETURN_IF(launch_frame_phase_c128(p.m, static_cast<c128*>(in.rho), in.ldr, T, s));
      else
        TC_RETURN_IF(launch_frame_phase_c64(p.m, static_cast<c64*>(in.rho), in.ldr, T, s));
    }
    return TC_OK;
  }
  // (one sector: the frame's phase is global, e^{i w_c k t} rho e^{-i w_c k t} = rho)
  if (o.frame == TC_FRAME_ROTATING && T != 0.0 && p.in_sector < 0) {
    if (o.gemm_mode == TC_GEMM_F64)
      TC_RETURN_IF(launch_frame_phase_c128(p.m, static_cast<c128*>(p.rho), p.ldr, T, s));
    else
      TC_RETURN_IF(launch_frame_phase_c64(p.m, static_cast<c64*>(p.rho), p.ldr, T, s));
  }
  if (p.rho_converted) {
    if (o.gemm_mode == TC_GEMM_F64)
      TC_RETURN_IF(launch_copy_c128_to_c64(static_cast<const c128*>(p.rho), p.ldr,
                                           static_cast<c64*>(in.rho), in.ldr, p.N, p.N, s));
    else
      TC_RETURN_IF(launch_copy_c64_to_c128(static_cast<const c64*>(p.rho), p.ldr,
                                           static_cast<c128*>(in.rho), in.ldr, p.N, p.N, s));
  }
  return TC_OK;
}

int step(InstPlan& p, const tc_evolve_opts& o, hipStream_t s) {
  if (p.sectors && o.gemm_mode == TC_GEMM_SPLIT_BF16) {
    TC_RETURN_IF(split_grouped_run(p.sg1, s));
    return split_grouped_run(p.sg2, s);
  }
  if (p.sectors) {
    TC_RETURN_IF(grouped_run(p.g1, s));
    return grouped_run(p.g2, s);
  }
  if (o.gemm_mode == TC_GEMM_SPLIT_BF16)
    return step_split(static_cast<c64*>(p.rho), p.ldr, static_cast<c64*>(p.X), p.ldx, p.N,
                      o.frame == TC_FRAME_ROTATING, o.full_product == 0, p.planes, s);
  return step_mfma(p, o, s);
}

// The step pattern repeats with period lcm(record_every, renorm_every); a
// captured chunk is a whole number of periods of about 16 steps.
int64_t gcd64(int64_t a, int64_t b) { while (b) { const int64_t t = a % b; a = b; b = t; } return a; }

int64_t graph_chunk(const tc_evolve_opts& o, bool rec) {
  int64_t L = 1;
  if (rec && o.record_every > 0) L = o.record_every;
  if (o.renorm_every > 0) L = L / gcd64(L, o.renorm_every) * o.renorm_every;
  return L * std::max<int64_t>(1, 16 / L);
}

// Steps 1..steps through one_step(st, stream).  With graph, the launches of
// steps 1..chunk are captured once into a hipGraph on a stream of its own
// (ordered after and before s by events) and replayed steps / chunk times;
// the remaining steps run eagerly on that stream.  Every launch of a captured
// step must address the same memory in every period (record indices come from
// a device counter), and nothing in it may be a memset node.
template <class StepFn>
int run_steps(StepFn&& one_step, int64_t steps, int64_t chunk, bool graph, hipStream_t s) {
  if (!graph) {
    for (int64_t st = 1; st <= steps; ++st) TC_RETURN_IF(one_step(st, s));
    return TC_OK;
  }
  hipStream_t cs = nullptr;
  hipEvent_t ev = nullptr;
  hipGraph_t gr = nullptr;
  hipGraphExec_t ex = nullptr;
  TC_TRY_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  int rc = TC_OK;
  auto hip_ok = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && rc == TC_OK) {
      set_error(std::string("hipGraph step chunk: ") + what + ": " + hipGetErrorString(e));
      rc = TC_ERR_HIP;
    }
    return e == hipSuccess;
  };
  if (hip_ok(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event") &&
      hip_ok(hipEventRecord(ev, s), "record") && hip_ok(hipStreamWaitEvent(cs, ev, 0), "wait") &&
      hip_ok(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture")) {
    profile_suspend(true);
    for (int64_t st = 1; st <= chunk && rc == TC_OK; ++st) rc = one_step(st, cs);
    profile_suspend(false);
    const bool ended = hip_ok(hipStreamEndCapture(cs, &gr), "end capture");
    if (rc == TC_OK && ended && hip_ok(hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0), "instantiate")) {
      const int64_t reps = steps / chunk;
      for (int64_t r = 0; r < reps && rc == TC_OK; ++r) hip_ok(hipGraphLaunch(ex, cs), "launch");
      for (int64_t st = reps * chunk + 1; st <= steps && rc == TC_OK; ++st) rc = one_step(st, cs);
    }
    hip_ok(hipEventRecord(ev, cs), "record");
    hip_ok(hipStreamWaitEvent(s, ev, 0), "wait");
    hip_ok(hipStreamSynchronize(cs), "sync");
  }
  if (ex) (void)hipGraphExecDestroy(ex);
  if (gr) (void)hipGraphDestroy(gr);
  if (ev) (void)hipEventDestroy(ev);
  (void)hipStreamDestroy(cs);
  return rc;
}

// One small instance stepped densely, without checkpoints or damping, runs
// in the LDS-resident kernel (one launch for all steps).
bool use_resident(const InstPlan& p, const tc_instance& in, const tc_evolve_opts& o) {
  if (o.no_resident || p.sectors || p.in_sector >= 0 || in.checkpoints) return false;
  if (p.m.kappa > 0.0 || p.m.gamma > 0.0) return false;
  if (o.gemm_mode == TC_GEMM_F64) return p.N <= RESIDENT_MAX_N_C128;
  if (o.gemm_mode == TC_GEMM_F32) return p.N <= RESIDENT_MAX_N_C64;
  return false;
}

int evolve_resident(InstPlan& p, const tc_instance& in, const tc_evolve_opts& o, hipStream_t s) {
  TC_RETURN_IF(prepare(p, in, o, s));
  ResidentArgs a;
  a.op = p.op; a.ldop = p.ldop;
  a.rho = p.rho; a.ldr = p.ldr;
  a.rot = o.frame == TC_FRAME_ROTATING;
  a.steps = o.steps;
  a.renorm_every = o.renorm_every;
  a.record_every = o.record_every;
  a.pop = in.pop_out; a.pdist = in.photon_dist_out; a.pstate = in.photon_state_out;
  a.scratch = p.scratch;
  TC_RETURN_IF(o.gemm_mode == TC_GEMM_F64 ? launch_resident_c128(p.m, a, s)
                                          : launch_resident_c64(p.m, a, s));
  return finish(p, in, o, s);
}

int evolve_one(InstPlan& p, const tc_instance& in, const tc_evolve_opts& o, hipStream_t s) {
  if (use_resident(p, in, o)) return evolve_resident(p, in, o, s);
  TC_RETURN_IF(prepare(p, in, o, s));
  const int c1 = p.m.c + 1, ns = std::min(p.m.n, p.m.c) + 1;
  const bool rec = (in.pop_out || in.photon_dist_out || in.photon_state_out);
  const int64_t chunk = graph_chunk(o, rec);
  const bool graph = o.use_graph && !in.checkpoints && chunk <= 256 && o.steps >= chunk;
  const bool c128s = o.gemm_mode == TC_GEMM_F64;
  if (graph && rec) {
    // the record index lives on the device, so that a captured chunk replays
    ReadoutItem ri;
    ri.rho = p.rho; ri.ld = p.ldr; ri.n = p.m.n; ri.c = p.m.c;
    ri.pop = in.pop_out; ri.pdist = in.photon_dist_out; ri.pstate = in.photon_state_out;
    ri.map = p.inv;
    TC_TRY_HIP(hipMemcpyAsync(p.ritem, &ri, sizeof(ri), hipMemcpyHostToDevice, s));
    TC_TRY_HIP(hipMemsetAsync(p.counter, 0, sizeof(int), s));
    TC_TRY_HIP(hipStreamSynchronize(s));   // ri is host memory of this call
    TC_RETURN_IF(launch_grouped_readout(p.ritem, 1, c128s, p.counter, s, true));
  } else if (rec) {
    TC_RETURN_IF(readout(p, o, in.pop_out, in.photon_dist_out, in.photon_state_out, s));
  }
  if (in.checkpoints) TC_RETURN_IF(copy_checkpoint(p, in, o, 0, 0.0, s));
  auto one_step = [&](int64_t st, hipStream_t q) -> int {
    TC_RETURN_IF(step(p, o, q));
    TC_RETURN_IF(dissipate(p, o, q));
    if (o.renorm_every > 0 && st % o.renorm_every == 0) TC_RETURN_IF(renorm(p, o, q));
    if (rec && st % o.record_every == 0) {
      if (graph) {
        TC_RETURN_IF(launch_grouped_readout(p.ritem, 1, c128s, p.counter, q, true));
      } else {
        const int64_t r = st / o.record_every;
        TC_RETURN_IF(readout(p, o, in.pop_out ? in.pop_out + r : nullptr,
                             in.photon_dist_out ? in.photon_dist_out + r * c1 : nullptr,
                             in.photon_state_out ? in.photon_state_out + r * ns : nullptr, q));
      }
    }
    if (in.checkpoints && st % o.checkpoint_every == 0)
      TC_RETURN_IF(copy_checkpoint(p, in, o, st / o.checkpoint_every, double(st) * o.dt, q));
    return TC_OK;
  };
  TC_RETURN_IF(run_steps(one_step, o.steps, chunk, graph, s));
  return finish(p, in, o, s);
}

// ------------------------------------------------------------------ batching
// count > 1 instances with FP64 / FP32 products: each product phase of a step
// is one persistent grouped launch per tile shape over every instance's
// tiles, the readout is one launch for all instances (record index kept in a
// device counter), and with use_graph the launches of a chunk of steps are
// captured once in a hipGraph and replayed.
struct BatchBufs {
  char* items = nullptr;          // 8 groups of count GroupItem descriptors
  ReadoutItem* ritems = nullptr;  // count readout descriptors
  int* counter = nullptr;         // record index
};

bool use_batched(int count, const tc_evolve_opts& o) {
  return count > 1 && (o.gemm_mode != TC_GEMM_SPLIT_BF16 || o.sectors);
}

// sector_items: total sector blocks of the batch (0 without sectors); the
// block products of all instances share two groups per tile shape
void plan_batch(Arena& ar, int count, int64_t sector_items, BatchBufs* b) {
  const size_t blocks = std::max(grouped_bytes(int(sector_items)),
                                 split_grouped_bytes(int(sector_items)));
  b->items = static_cast<char*>(ar.take(std::max(8 * grouped_bytes(count), 4 * blocks)));
  b->ritems = static_cast<ReadoutItem*>(ar.take(size_t(count) * sizeof(ReadoutItem)));
  b->counter = static_cast<int*>(ar.take(sizeof(int)));
}

void step_descs(const InstPlan& p, const tc_evolve_opts& o, GemmDesc& g1, GemmDesc& g2) {
  const bool rot = o.frame == TC_FRAME_ROTATING;
  g1 = GemmDesc();
  g1.M = g1.N = g1.K = p.N;
  g1.A = p.op; g1.lda = p.ldop; g1.a_kmaj = false;
  g1.B = p.rho; g1.ldb = p.ldr; g1.b_kmaj = true;
  g1.C = p.X; g1.ldc = p.ldx;
  if (rot) { g1.Cin = p.rho; g1.ldcin = p.ldr; g1.beta_re = 1.0; }
  g1.tail_ws = p.tail_ws; g1.tail_ws_bytes = p.tail_ws_bytes;
  g2 = GemmDesc();
  g2.M = g2.N = g2.K = p.N;
  g2.A = p.X; g2.lda = p.ldx; g2.a_kmaj = false;
  g2.B = p.op; g2.ldb = p.ldop; g2.b_kmaj = true; g2.conj_b = true;
  g2.C = p.rho; g2.ldc = p.ldr;
  if (rot) { g2.Cin = p.X; g2.ldcin = p.ldx; g2.beta_re = 1.0; }
  g2.herm = o.full_product == 0;
  g2.tail_ws = p.tail_ws; g2.tail_ws_bytes = p.tail_ws_bytes;
}

// Sector blocks of all instances of a batch (0 without sectors).
int64_t sector_items(const tc_instance* inst, int count, const tc_evolve_opts& o) {
  if (!o.sectors) return 0;
  int64_t t = 0;
  for (int b = 0; b < count; ++b)
    t += inst[b].model->n_atoms + inst[b].model->photon_cutoff + 1;
  return t;
}

int evolve_batched(std::vector<InstPlan>& plans, const tc_instance* inst, int count,
                   const tc_evolve_opts& o, const BatchBufs& bb, hipStream_t s) {
  const bool f64 = o.gemm_mode == TC_GEMM_F64;
  const bool sec = o.sectors != 0, split = o.gemm_mode == TC_GEMM_SPLIT_BF16;
  for (int b = 0; b < count; ++b)
    TC_RETURN_IF(sec ? prepare_sectors(plans[b], inst[b], o, s, false)
                     : prepare(plans[b], inst[b], o, s));
  // group the products by tile shape (autotuner table per dimension bucket)
  // and by whether N is a multiple of the tile: those run one workgroup per
  // tile with the unchecked tile (fewer registers), the rest persistently.
  // By sectors, the block products of every instance (whole tiles of the
  // instance's padding) go into one group per tile shape, largest K first.
  std::vector<GemmDesc> d1[3][2], d2[3][2];
  std::vector<SplitProduct> sp1, sp2;
  for (int b = 0; b < count; ++b) {
    const int v = sec ? plans[b].svar : tile_variant_for(plans[b].N, f64);
    if (sec && split) {
      sp1.insert(sp1.end(), plans[b].ssd1.begin(), plans[b].ssd1.end());
      sp2.insert(sp2.end(), plans[b].ssd2.begin(), plans[b].ssd2.end());
    } else if (sec) {
      d1[v][0].insert(d1[v][0].end(), plans[b].sd1.begin(), plans[b].sd1.end());
      d2[v][0].insert(d2[v][0].end(), plans[b].sd2.begin(), plans[b].sd2.end());
    } else {
      GemmDesc g1, g2;
      step_descs(plans[b], o, g1, g2);
      const int edge = v == 1 ? 128 : 64;
      const int e = plans[b].N % edge == 0 ? 0 : 1;
      d1[v][e].push_back(g1);
      d2[v][e].push_back(g2);
    }
  }
  auto by_k = [](const auto& x, const auto& y) { return x.K > y.K; };
  auto by_kp = [](const SplitProduct& x, const SplitProduct& y) { return x.Kp > y.Kp; };
  std::stable_sort(sp1.begin(), sp1.end(), by_kp);
  std::stable_sort(sp2.begin(), sp2.end(), by_kp);
  GroupedProducts G1[3][2], G2[3][2];
  SplitGrouped S1, S2;
  char* it = bb.items;
  const size_t gstep = sec ? std::max(grouped_bytes(int(d1[1][0].size() + d1[2][0].size())),
                                      split_grouped_bytes(int(sp1.size())))
                           : grouped_bytes(count);
  if (sec && split) {
    TC_RETURN_IF(split_grouped_build(sp1, it, &S1, s));
    it += gstep;
    TC_RETURN_IF(split_grouped_build(sp2, it, &S2, s));
    it += gstep;
  }
  for (int v = 1; v <= 2; ++v)
    for (int e = 0; e < 2; ++e) {
      if (d1[v][e].empty()) continue;
      if (sec) {
        std::stable_sort(d1[v][e].begin(), d1[v][e].end(), by_k);
        std::stable_sort(d2[v][e].begin(), d2[v][e].end(), by_k);
      }
      TC_RETURN_IF(grouped_build(d1[v][e], f64, v, it, &G1[v][e], s));
      it += gstep;
      TC_RETURN_IF(grouped_build(d2[v][e], f64, v, it, &G2[v][e], s));
      it += gstep;
      G1[v][e].persistent = G2[v][e].persistent = e == 1;
    }
  bool rec = false, ckpt = false;
  std::vector<ReadoutItem> ri(count);
  for (int b = 0; b < count; ++b) {
    ri[b].rho = plans[b].rho;
    ri[b].ld = plans[b].ldr;
    ri[b].n = plans[b].m.n;
    ri[b].c = plans[b].m.c;
    ri[b].pop = inst[b].pop_out;
    ri[b].pdist = inst[b].photon_dist_out;
    ri[b].map = sec ? plans[b].inv : nullptr;
    ri[b].pstate = inst[b].photon_state_out;
    rec = rec || inst[b].pop_out || inst[b].photon_dist_out || inst[b].photon_state_out;
    ckpt = ckpt || inst[b].checkpoints;
  }
  TC_TRY_HIP(hipMemcpyAsync(bb.ritems, ri.data(), ri.size() * sizeof(ReadoutItem),
                            hipMemcpyHostToDevice, s));
  TC_TRY_HIP(hipMemsetAsync(bb.counter, 0, sizeof(int), s));
  TC_TRY_HIP(hipStreamSynchronize(s));   // ri is host memory of this call
  const bool c128s = f64;
  if (rec) {
    TC_RETURN_IF(launch_grouped_readout(bb.ritems, count, c128s, bb.counter, s));
    TC_RETURN_IF(launch_advance_counter(bb.counter, s));
  }
  for (int b = 0; b < count; ++b)
    if (inst[b].checkpoints) TC_RETURN_IF(copy_checkpoint(plans[b], inst[b], o, 0, 0.0, s));

  auto one_step = [&](int64_t st, hipStream_t q) -> int {
    TC_RETURN_IF(split_grouped_run(S1, q));
    for (int v = 1; v <= 2; ++v)
      for (int e = 0; e < 2; ++e) TC_RETURN_IF(grouped_run(G1[v][e], q));
    TC_RETURN_IF(split_grouped_run(S2, q));
    for (int v = 1; v <= 2; ++v)
      for (int e = 0; e < 2; ++e) TC_RETURN_IF(grouped_run(G2[v][e], q));
    for (int b = 0; b < count; ++b) TC_RETURN_IF(dissipate(plans[b], o, q));
    if (o.renorm_every > 0 && st % o.renorm_every == 0)
      for (int b = 0; b < count; ++b) TC_RETURN_IF(renorm(plans[b], o, q));
    if (rec && st % o.record_every == 0) {
      TC_RETURN_IF(launch_grouped_readout(bb.ritems, count, c128s, bb.counter, q));
      TC_RETURN_IF(launch_advance_counter(bb.counter, q));
    }
    if (ckpt && o.checkpoint_every > 0 && st % o.checkpoint_every == 0)
      for (int b = 0; b < count; ++b)
        if (inst[b].checkpoints)
          TC_RETURN_IF(copy_checkpoint(plans[b], inst[b], o, st / o.checkpoint_every,
                                       double(st) * o.dt, q));
    return TC_OK;
  };

  const int64_t chunk = graph_chunk(o, rec);
  const bool graph = o.use_graph && !ckpt && chunk <= 256 && o.steps >= chunk;
  TC_RETURN_IF(run_steps(one_step, o.steps, chunk, graph, s));
  for (int b = 0; b < count; ++b) TC_RETURN_IF(finish(plans[b], inst[b], o, s));
  return TC_OK;
}

}  // namespace
}  // namespace tcm

using namespace tcm;

extern "C" {

int tc_evolve_workspace_size(const tc_instance* inst, int32_t count, const tc_evolve_opts* o,
                             size_t* bytes) {
  clear_error();
  TC_CHECK_ARG(bytes != nullptr, "bytes is NULL");
  TC_CHECK_ARG(count >= 1, "count < 1");
  TC_CHECK_ARG(inst != nullptr, "instances is NULL");
  TC_RETURN_IF(validate_opts(o));
  Arena ar(nullptr, 0);
  std::vector<InstPlan> plans(count);
  for (int b = 0; b < count; ++b) {
    ModelArgs m;
    TC_RETURN_IF(validate_instance(&inst[b], o, &m));
    plan_instance(inst[b], *o, m, ar, &plans[b]);
  }
  if (use_batched(count, *o)) {
    BatchBufs bb;
    plan_batch(ar, count, sector_items(inst, count, *o), &bb);
  } else {
    take_tail(ar, *o, plans.data(), count);
  }
  *bytes = ar.used;
  return TC_OK;
}

int tc_evolve(const tc_instance* inst, int32_t count, const tc_evolve_opts* o, void* ws,
              size_t ws_bytes, void* stream) {
  clear_error();
  size_t need = 0;
  TC_RETURN_IF(tc_evolve_workspace_size(inst, count, o, &need));
  TC_CHECK_ARG(ws != nullptr || need == 0, "workspace is NULL");
  if (ws_bytes < need) {
    set_error("workspace too small for tc_evolve: need " + std::to_string(need) + " bytes");
    return TC_ERR_WORKSPACE;
  }
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);
  std::vector<InstPlan> plans(count);
  for (int b = 0; b < count; ++b) {
    ModelArgs m;
    TC_RETURN_IF(validate_instance(&inst[b], o, &m));
    plan_instance(inst[b], *o, m, ar, &plans[b]);
  }
  if (use_batched(count, *o)) {
    BatchBufs bb;
    plan_batch(ar, count, sector_items(inst, count, *o), &bb);
    TC_RETURN_IF(evolve_batched(plans, inst, count, *o, bb, s));
  } else {
    take_tail(ar, *o, plans.data(), count);
    for (int b = 0; b < count; ++b) TC_RETURN_IF(evolve_one(plans[b], inst[b], *o, s));
  }
  if (o->renorm_every > 0 && o->steps >= o->renorm_every) {
    // one flag read per call: a renormalisation met a non-finite or non-positive trace
    for (int b = 0; b < count; ++b) {
      double flag = 0.0;
      TC_TRY_HIP(hipMemcpyAsync(&flag, plans[b].scratch + 1, sizeof(double),
                                hipMemcpyDeviceToHost, s));
      TC_TRY_HIP(hipStreamSynchronize(s));
      if (flag != 0.0) {
        set_error("renormalisation found a non-finite or non-positive trace (instance " +
                  std::to_string(b) + ")");
        return TC_ERR_NONFINITE;
      }
    }
  }
  return TC_OK;
}

int tc_evolve_sector_workspace_size(const tc_instance* inst, int32_t k, const tc_evolve_opts* o,
                                    size_t* bytes) {
  clear_error();
  TC_CHECK_ARG(bytes != nullptr, "bytes is NULL");
  TC_CHECK_ARG(inst != nullptr, "instance is NULL");
  TC_RETURN_IF(validate_opts(o));
  TC_CHECK_ARG(o->sectors == 0, "sectors must be 0 for a one-sector run");
  int64_t d = 0;
  TC_RETURN_IF(tc_sector_dim(inst->model, k, &d));
  ModelArgs m;
  TC_RETURN_IF(make_model_args(inst->model, &m));
  if (m.kappa > 0.0 || m.gamma > 0.0) {
    set_error("the damping channels lead out of an excitation sector");
    return TC_ERR_UNSUPPORTED;
  }
  TC_CHECK_ARG(inst->N == d, "instance N != d_k of the sector");
  TC_CHECK_ARG(inst->U != nullptr && inst->rho != nullptr, "U / rho is NULL");
  TC_CHECK_ARG(inst->ldu >= d && inst->ldr >= d, "leading dimension < d_k");
  if (inst->pop_out || inst->photon_dist_out || inst->photon_state_out)
    TC_CHECK_ARG(o->record_every >= 1, "record_every must be >= 1 when records are requested");
  if (inst->checkpoints)
    TC_CHECK_ARG(o->checkpoint_every >= 1, "checkpoint_every must be >= 1 with checkpoints");
  Arena ar(nullptr, 0);
  InstPlan p;
  p.in_sector = k;
  plan_instance(*inst, *o, m, ar, &p);
  take_tail(ar, *o, &p, 1);
  *bytes = ar.used;
  return TC_OK;
}

int tc_evolve_sector(const tc_instance* inst, int32_t k, const tc_evolve_opts* o, void* ws,
                     size_t ws_bytes, void* stream) {
  clear_error();
  size_t need = 0;
  TC_RETURN_IF(tc_evolve_sector_workspace_size(inst, k, o, &need));
  TC_CHECK_ARG(ws != nullptr || need == 0, "workspace is NULL");
  if (ws_bytes < need) {
    set_error("workspace too small for tc_evolve_sector: need " + std::to_string(need) + " bytes");
    return TC_ERR_WORKSPACE;
  }
  hipStream_t s = as_stream(stream);
  ModelArgs m;
  TC_RETURN_IF(make_model_args(inst->model, &m));
  Arena ar(ws, ws_bytes);
  InstPlan p;
  p.in_sector = k;
  plan_instance(*inst, *o, m, ar, &p);
  take_tail(ar, *o, &p, 1);
  TC_RETURN_IF(evolve_one(p, *inst, *o, s));
  if (o->renorm_every > 0 && o->steps >= o->renorm_every) {
    double flag = 0.0;
    TC_TRY_HIP(hipMemcpyAsync(&flag, p.scratch + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    TC_TRY_HIP(hipStreamSynchronize(s));
    if (flag != 0.0) {
      set_error("renormalisation found a non-finite or non-positive trace");
      return TC_ERR_NONFINITE;
    }
  }
  return TC_OK;
}

int tc_observables_workspace_size(int64_t N, size_t* bytes) {
  clear_error();
  TC_CHECK_ARG(bytes != nullptr, "bytes is NULL");
  TC_CHECK_ARG(N >= 0, "N < 0");
  *bytes = observables_partials_count(N) * sizeof(double);
  return TC_OK;
}

int tc_observables(const tc_model* m, const void* rho, int32_t rho_dtype, int64_t N, int64_t ldr,
                   double* scalars, double* atom_pop, double* photon_dist, double* exc_dist,
                   double* photon_state, double* dicke, void* ws, size_t ws_bytes,
                   void* stream) {
  clear_error();
  ModelArgs a;
  TC_RETURN_IF(make_model_args(m, &a));
  TC_CHECK_ARG(N == a.N, "N != (c+1) 2^n");
  TC_CHECK_ARG(rho != nullptr && scalars != nullptr, "rho / scalars is NULL");
  TC_CHECK_ARG(rho_dtype == TC_C64 || rho_dtype == TC_C128, "unknown rho_dtype");
  TC_CHECK_ARG(ldr >= N, "ldr < N");
  size_t need = 0;
  TC_RETURN_IF(tc_observables_workspace_size(N, &need));
  TC_CHECK_ARG(ws != nullptr, "workspace is NULL");
  if (ws_bytes < need) {
    set_error("workspace too small for tc_observables");
    return TC_ERR_WORKSPACE;
  }
  return launch_observables(a, rho, rho_dtype, ldr, static_cast<double*>(ws), scalars, atom_pop,
                            photon_dist, exc_dist, photon_state, dicke, as_stream(stream));
}

int tc_gemm_workspace_size(int64_t M, int64_t N, int64_t K, int32_t mode, size_t* bytes) {
  clear_error();
  TC_CHECK_ARG(bytes != nullptr, "bytes is NULL");
  TC_CHECK_ARG(M >= 0 && N >= 0 && K >= 0, "negative size");
  TC_CHECK_ARG(mode == TC_GEMM_F64 || mode == TC_GEMM_F32 || mode == TC_GEMM_SPLIT_BF16,
               "unknown mode");
  if (mode == TC_GEMM_F64) { *bytes = 0; return TC_OK; }
  // c64 copies of A (M x K), B (K x N) and C (M x N), plus split planes
  Arena ar(nullptr, 0);
  ar.take(size_t(M) * size_t(K) * 8);
  ar.take(size_t(K) * size_t(N) * 8);
  ar.take(size_t(M) * size_t(N) * 8);
  if (mode == TC_GEMM_SPLIT_BF16) split_gemm_plan(ar, M, N, K, nullptr);
  *bytes = ar.used;
  return TC_OK;
}

int tc_zgemm(int64_t M, int64_t N, int64_t K, tc_c128 alpha, const tc_c128* A, int64_t lda,
             int32_t op_a, const tc_c128* B, int64_t ldb, int32_t op_b, tc_c128 beta, tc_c128* C,
             int64_t ldc, int32_t mode, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  TC_CHECK_ARG(M >= 0 && N >= 0 && K >= 0, "negative size");
  TC_CHECK_ARG(op_a >= 0 && op_a <= 3 && op_b >= 0 && op_b <= 3, "op must be 0..3");
  TC_CHECK_ARG(C != nullptr, "C is NULL");
  TC_CHECK_ARG(K == 0 || (A != nullptr && B != nullptr), "A / B is NULL");
  const bool ta = op_a >= 2, tb = op_b >= 2;
  TC_CHECK_ARG(lda >= std::max<int64_t>(1, ta ? M : K), "lda too small");
  TC_CHECK_ARG(ldb >= std::max<int64_t>(1, tb ? K : N), "ldb too small");
  TC_CHECK_ARG(ldc >= std::max<int64_t>(1, N), "ldc too small");
  size_t need = 0;
  TC_RETURN_IF(tc_gemm_workspace_size(M, N, K, mode, &need));
  if (need) {
    TC_CHECK_ARG(ws != nullptr, "workspace is NULL");
    if (ws_bytes < need) { set_error("workspace too small for tc_zgemm"); return TC_ERR_WORKSPACE; }
  }
  hipStream_t s = as_stream(stream);
  GemmDesc d;
  d.M = M; d.N = N; d.K = K;
  d.a_kmaj = ta; d.conj_a = (op_a & 1) != 0;
  d.b_kmaj = !tb; d.conj_b = (op_b & 1) != 0;
  d.alpha_re = alpha.re; d.alpha_im = alpha.im;
  d.beta_re = beta.re; d.beta_im = beta.im;
  if (mode == TC_GEMM_F64) {
    d.A = A; d.lda = lda; d.B = B; d.ldb = ldb;
    d.C = C; d.ldc = ldc; d.Cin = C; d.ldcin = ldc;
    return gemm_f64(d, s);
  }
  // reduced precision: operate on c64 copies
  Arena ar(ws, ws_bytes);
  const int64_t ar_rows = ta ? K : M, ar_cols = ta ? M : K;
  const int64_t br_rows = tb ? N : K, br_cols = tb ? K : N;
  c64* A32 = static_cast<c64*>(ar.take(size_t(M) * size_t(K) * 8));
  c64* B32 = static_cast<c64*>(ar.take(size_t(K) * size_t(N) * 8));
  c64* C32 = static_cast<c64*>(ar.take(size_t(M) * size_t(N) * 8));
  if (K > 0) {
    TC_RETURN_IF(launch_copy_c128_to_c64(reinterpret_cast<const c128*>(A), lda, A32, ar_cols,
                                         ar_rows, ar_cols, s));
    TC_RETURN_IF(launch_copy_c128_to_c64(reinterpret_cast<const c128*>(B), ldb, B32, br_cols,
                                         br_rows, br_cols, s));
  }
  TC_RETURN_IF(launch_copy_c128_to_c64(reinterpret_cast<const c128*>(C), ldc, C32, N, M, N, s));
  d.A = A32; d.lda = ar_cols; d.B = B32; d.ldb = br_cols;
  d.C = C32; d.ldc = N; d.Cin = C32; d.ldcin = N;
  if (mode == TC_GEMM_F32) {
    TC_RETURN_IF(gemm_f32(d, s));
  } else {
    SplitGemmPlan sp;
    split_gemm_plan(ar, M, N, K, &sp);
    TC_RETURN_IF(split_gemm(d, sp, s));
  }
  return launch_copy_c64_to_c128(C32, N, reinterpret_cast<c128*>(C), ldc, M, N, s);
}

int tc_split_bf16(const float* x, int64_t count, uint16_t* hi, uint16_t* lo, void* stream) {
  clear_error();
  TC_CHECK_ARG(count >= 0, "count < 0");
  TC_CHECK_ARG(count == 0 || (x && hi && lo), "NULL pointer");
  return launch_split_bf16(x, count, hi, lo, as_stream(stream));
}

}  // extern "C"
