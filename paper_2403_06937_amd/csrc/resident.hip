// LDS-resident stepping of one small instance: every step of Eq. (6) in a
// single launch of one workgroup, with the product operand, rho and the
// intermediate X held in LDS for the whole run.
//
// At N = 32 a step is two 32 x 32 x 32 complex products (0.5 Mflop), far too
// little to fill even one CU; launched as separate kernels per step the run
// is bound by launch latency.  Here the launch is paid once per run and each
// step costs the products' arithmetic and two workgroup barriers.
//
// Per step, for every output (i, j) (2 x 2 blocks of outputs per thread):
//   X[i][j]  = sum_k op[i][k] R[k][j]        (+ R[i][j] in the rotating frame)
//   R'[i][j] = sum_k X[i][k] conj(op[j][k])  (+ X[i][j] in the rotating frame)
// i.e. X = op R, R' = X op^dag: op = U in the lab frame, D = U~ - I in the
// rotating frame (U~ = I + D).  The sums run over k in increasing order with
// fused multiply-adds in the storage precision.  Renormalisation (every
// renorm_every steps) is Hermitisation and division by Re Tr R in FP64, and
// the records (excited-atom population, photon-number distribution, P({m>)
// of Eq. (13)) are read from the diagonal in FP64 by one wavefront.
#include "kernels.h"

namespace tcm {
namespace {

constexpr int RTPB = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T, int MAXN>
__global__ void __launch_bounds__(RTPB) resident_kernel(ModelArgs m, ResidentArgs a) {
  typedef cplx<T> E;
  constexpr int LD = MAXN + 1;
  __shared__ E sU[MAXN * LD];
  __shared__ E sA[MAXN * LD];
  __shared__ E sB[MAXN * LD];
  __shared__ int bad;
  __shared__ double trace;
  const int N = int(m.N);
  const int NN = N * N;
  const E* __restrict__ op = static_cast<const E*>(a.op);
  E* __restrict__ rho = static_cast<E*>(a.rho);
  for (int idx = threadIdx.x; idx < NN; idx += RTPB) {
    const int i = idx / N, j = idx - (idx / N) * N;
    sU[i * LD + j] = op[int64_t(i) * a.ldop + j];
    sA[i * LD + j] = rho[int64_t(i) * a.ldr + j];
  }
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  E* R = sA;
  E* X = sB;
  const int n = m.n, c = m.c;
  const int per = 1 << n;
  const int ns = (n < c ? n : c) + 1;
  const bool rec = a.pop || a.pdist || a.pstate;

  // records of R's diagonal, by wave 0: lane l takes the states s = l, l + 64,
  // ... of each photon block, then each readout is a butterfly sum over the
  // wave (every lane ends with the same bits, lane 0 writes)
  auto record = [&](int64_t r) {
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
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

  // outputs in 2 x 2 blocks (N is even: N = (c + 1) 2^n with n >= 1), so each
  // k step loads two elements of each operand for four products
  const int NB = N >> 1, NBB = NB * NB;
  if (rec) record(0);
  for (int64_t step = 1; step <= a.steps; ++step) {
    // X = op R (+ R)
    for (int idx = threadIdx.x; idx < NBB; idx += RTPB) {
      const int i = 2 * (idx / NB), j = 2 * (idx - (idx / NB) * NB);
      T xr[2][2] = {{0, 0}, {0, 0}}, xi[2][2] = {{0, 0}, {0, 0}};
      for (int k = 0; k < N; ++k) {
        const E u[2] = {sU[i * LD + k], sU[(i + 1) * LD + k]};
        const E r[2] = {R[k * LD + j], R[k * LD + j + 1]};
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            xr[p][q] = fma(u[p].re, r[q].re, xr[p][q]);
            xr[p][q] = fma(-u[p].im, r[q].im, xr[p][q]);
            xi[p][q] = fma(u[p].re, r[q].im, xi[p][q]);
            xi[p][q] = fma(u[p].im, r[q].re, xi[p][q]);
          }
      }
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int o = (i + p) * LD + j + q;
          if (a.rot) {
            xr[p][q] += R[o].re;
            xi[p][q] += R[o].im;
          }
          X[o] = E{xr[p][q], xi[p][q]};
        }
    }
    __syncthreads();
    // R = X op^dag (+ X)
    for (int idx = threadIdx.x; idx < NBB; idx += RTPB) {
      const int i = 2 * (idx / NB), j = 2 * (idx - (idx / NB) * NB);
      T yr[2][2] = {{0, 0}, {0, 0}}, yi[2][2] = {{0, 0}, {0, 0}};
      for (int k = 0; k < N; ++k) {
        const E x[2] = {X[i * LD + k], X[(i + 1) * LD + k]};
        const E u[2] = {sU[j * LD + k], sU[(j + 1) * LD + k]};
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            yr[p][q] = fma(x[p].re, u[q].re, yr[p][q]);
            yr[p][q] = fma(x[p].im, u[q].im, yr[p][q]);
            yi[p][q] = fma(x[p].im, u[q].re, yi[p][q]);
            yi[p][q] = fma(-x[p].re, u[q].im, yi[p][q]);
          }
      }
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int o = (i + p) * LD + j + q;
          if (a.rot) {
            yr[p][q] += X[o].re;
            yi[p][q] += X[o].im;
          }
          R[o] = E{yr[p][q], yi[p][q]};
        }
    }
    __syncthreads();
    if (a.renorm_every > 0 && step % a.renorm_every == 0) {
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
    // wave 0 reads R's diagonal while the others start the next product,
    // which only reads R; R is next written after the barrier that follows
    if (rec && step % a.record_every == 0) record(step / a.record_every);
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
