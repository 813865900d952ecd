// LDS-resident stepping of one small instance: every step of Eq. (6) in a
// single launch of one workgroup, with the product operand, rho and the
// intermediate X held in LDS for the whole run.
//
// At N = 32 a step is two 32 x 32 x 32 complex products (0.5 Mflop), far too
// little to fill even one CU; launched as separate kernels per step the run
// is bound by launch latency.  Here the launch is paid once per run and each
// step costs the products' arithmetic and two workgroup barriers.
//
// Per step, for every output (i, j):
//   X[i][j]  = sum_k op[i][k] R[k][j]        (+ R[i][j] in the rotating frame)
//   R'[i][j] = sum_k X[i][k] conj(op[j][k])  (+ X[i][j] in the rotating frame)
// i.e. X = op R, R' = X op^dag: op = U in the lab frame, D = U~ - I in the
// rotating frame (U~ = I + D).  The matrices sit in LDS padded with zeros to
// a multiple of 16, and each wave forms 16 x 16 output blocks with the
// 16 x 16 x 4 MFMA of the storage precision (four real products per complex
// block, FP64 or FP32 accumulation), so a K step reads one complex element
// per lane and operand from LDS.  (A form with 2 x 2 outputs per thread and
// vector FMAs read four elements per 16 multiply-adds and was bound by LDS
// bandwidth.)  Renormalisation (every renorm_every steps) is Hermitisation
// and division by Re Tr R in FP64, and the records (excited-atom population,
// photon-number distribution, P({m>) of Eq. (13)) are read from the diagonal
// in FP64 by one wavefront.
#include "kernels.h"

namespace tcm {
namespace {

constexpr int PWAVES = 4;                  // waves that form the product blocks
constexpr int RTPB = 64 * (PWAVES + 1);    // plus one wave for the records

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// 16 x 16 x 4 MFMA in the storage precision: lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; output r of lane l is row l/16 + 4r (FP64) or
// 4(l/16) + r (FP32) of column l%16.
__device__ __forceinline__ d4 mma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> struct Acc;
template <> struct Acc<double> {
  typedef d4 type;
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Acc<float> {
  typedef f4 type;
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename T, int MAXN>
__global__ void __launch_bounds__(RTPB) resident_kernel(ModelArgs m, ResidentArgs a) {
  typedef cplx<T> E;
  typedef typename Acc<T>::type V;
  constexpr int MAXP = (MAXN + 15) / 16 * 16;
  // one element of padding per row: the 16 rows of a fragment read fall on
  // distinct banks
  constexpr int LD = MAXP + 1;
  __shared__ E sU[MAXP * LD];
  __shared__ E sA[MAXP * LD];
  __shared__ E sB[MAXP * LD];
  __shared__ int bad;
  __shared__ double trace;
  const int N = int(m.N);
  const int NP = (N + 15) & ~15;
  const int NN = N * N;
  const E* __restrict__ op = static_cast<const E*>(a.op);
  E* __restrict__ rho = static_cast<E*>(a.rho);
  for (int idx = threadIdx.x; idx < NP * NP; idx += RTPB) {
    const int i = idx / NP, j = idx - (idx / NP) * NP;
    E u{T(0), T(0)}, r{T(0), T(0)};
    if (i < N && j < N) {
      u = op[int64_t(i) * a.ldop + j];
      r = rho[int64_t(i) * a.ldr + j];
    }
    sU[i * LD + j] = u;
    sA[i * LD + j] = r;
  }
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  E* R = sA;
  E* X = sB;
  const int n = m.n, c = m.c;
  const int per = 1 << n;
  const int ns = (n < c ? n : c) + 1;
  const bool rec = a.pop || a.pdist || a.pstate;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int nb = NP / 16, nblk = nb * nb;

  // records of R's diagonal, by the last wave while the others start the next
  // step's first product (which only reads R): lane l takes the states
  // s = l, l + 64, ... of each photon block, then each readout is a butterfly
  // sum over the wave (every lane ends with the same bits, lane 0 writes)
  auto record = [&](int64_t r) {
    if (wave != PWAVES) return;
    double pop = 0.0;
    for (int mm = 0; mm <= c; ++mm) {
      double part = 0.0, st = 0.0;
      for (int l = lane; l < per; l += 64) {
        const int s = mm * per + l;
        const double d = double(R[s * LD + s].re);
        const int pc = __popc(unsigned(l));
        part += d;
        pop += double(pc) * d;
        if (pc == n - mm) st += d;
      }
      if (a.pdist) {
        part = wave_sum(part);
        if (lane == 0) a.pdist[r * (c + 1) + mm] = part;
      }
      if (a.pstate && mm < ns) {
        st = wave_sum(st);
        if (lane == 0) a.pstate[r * ns + mm] = st;
      }
    }
    pop = wave_sum(pop);
    if (a.pop && lane == 0) a.pop[r] = pop;
  };

  if (rec) record(0);
  // step counts at which the next renormalisation and record fall
  int64_t next_renorm = a.renorm_every > 0 ? a.renorm_every : -1;
  int64_t next_record = a.record_every, rindex = 0;
  for (int64_t step = 1; step <= a.steps; ++step) {
    // X = op R (+ R): A[i][k] = op[i][k], B[k][j] = R[k][j].  The padding of
    // op and R is zero, so X's padding is too.
    for (int b = wave; wave < PWAVES && b < nblk; b += PWAVES) {
      const int i0 = (b / nb) * 16, j0 = (b - (b / nb) * nb) * 16;
      V re = V{0, 0, 0, 0}, im = V{0, 0, 0, 0};
      for (int k16 = 0; k16 < NP; k16 += 16) {   // NP is a multiple of 16
        E x[4], y[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int k = k16 + 4 * q + lk;
          x[q] = sU[(i0 + lr) * LD + k];
          y[q] = R[k * LD + j0 + lr];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          re = mma(x[q].re, y[q].re, re);
          re = mma(-x[q].im, y[q].im, re);
          im = mma(x[q].re, y[q].im, im);
          im = mma(x[q].im, y[q].re, im);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = (i0 + Acc<T>::row(lane, r)) * LD + j0 + lr;
        T xr = re[r], xi = im[r];
        if (a.rot) {
          xr += R[o].re;
          xi += R[o].im;
        }
        X[o] = E{xr, xi};
      }
    }
    __syncthreads();
    // R = X op^dag (+ X): A[i][k] = X[i][k], B[k][j] = conj(op[j][k])
    for (int b = wave; wave < PWAVES && b < nblk; b += PWAVES) {
      const int i0 = (b / nb) * 16, j0 = (b - (b / nb) * nb) * 16;
      V re = V{0, 0, 0, 0}, im = V{0, 0, 0, 0};
      for (int k16 = 0; k16 < NP; k16 += 16) {
        E x[4], y[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int k = k16 + 4 * q + lk;
          x[q] = X[(i0 + lr) * LD + k];
          y[q] = sU[(j0 + lr) * LD + k];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          re = mma(x[q].re, y[q].re, re);
          re = mma(x[q].im, y[q].im, re);
          im = mma(x[q].im, y[q].re, im);
          im = mma(-x[q].re, y[q].im, im);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = (i0 + Acc<T>::row(lane, r)) * LD + j0 + lr;
        T yr = re[r], yi = im[r];
        if (a.rot) {
          yr += X[o].re;
          yi += X[o].im;
        }
        R[o] = E{yr, yi};
      }
    }
    __syncthreads();
    if (step == next_renorm) {
      next_renorm += a.renorm_every;
      if (threadIdx.x == 0) {
        double tr = 0.0;
        for (int s = 0; s < N; ++s) tr += double(R[s * LD + s].re);
        trace = tr;
        a.scratch[0] = tr;
        if (!(tr > 0.0) || !isfinite(tr)) {
          bad = 1;
          a.scratch[1] = 1.0;
        }
      }
      __syncthreads();
      if (!bad) {                       // once a trace was bad, rho is left as it is
        const double inv = 1.0 / trace;
        for (int idx = threadIdx.x; idx < NN; idx += RTPB) {
          const int i = idx / N, j = idx - (idx / N) * N;
          const E p = R[i * LD + j], q = R[j * LD + i];
          const double re = 0.5 * (double(p.re) + double(q.re)) * inv;
          const double im = i == j ? 0.0 : 0.5 * (double(p.im) - double(q.im)) * inv;
          X[i * LD + j] = E{T(re), T(im)};
        }
        __syncthreads();
        E* t = R;
        R = X;
        X = t;
      }
    }
    // the record wave reads R's diagonal while the product waves start the
    // next step's first product, which only reads R; R is next written after
    // the barrier that follows it
    if (rec && step == next_record) {
      next_record += a.record_every;
      record(++rindex);
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < NN; idx += RTPB) {
    const int i = idx / N, j = idx - (idx / N) * N;
    rho[int64_t(i) * a.ldr + j] = R[i * LD + j];
  }
}

}  // namespace

int launch_resident_c128(const ModelArgs& m, const ResidentArgs& a, hipStream_t s) {
  if (m.N > RESIDENT_MAX_N_C128) {
    set_error("LDS-resident stepping: N too large for complex FP64");
    return TC_ERR_UNSUPPORTED;
  }
  hipLaunchKernelGGL((resident_kernel<double, RESIDENT_MAX_N_C128>), dim3(1), dim3(RTPB), 0, s,
                     m, a);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_resident_c64(const ModelArgs& m, const ResidentArgs& a, hipStream_t s) {
  if (m.N > RESIDENT_MAX_N_C64) {
    set_error("LDS-resident stepping: N too large for complex FP32");
    return TC_ERR_UNSUPPORTED;
  }
  hipLaunchKernelGGL((resident_kernel<float, RESIDENT_MAX_N_C64>), dim3(1), dim3(RTPB), 0, s, m,
                     a);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

}  // namespace tcm
