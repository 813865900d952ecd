// HBM-bound and latency-bound kernels of libtcm: the Hamiltonian of Eq. (4),
// helpers of the matrix exponential, frame changes, per-step diagonal readout,
// FP64 renormalisation, full observables and the bfloat16 split.
//
// Reductions are deterministic: fixed per-thread strides, a butterfly of
// cross-lane exchanges inside each wavefront, then the wave results added in
// a fixed order (no atomics), so reruns are bitwise identical.
#include "kernels.h"

#include <algorithm>
#include <cstdint>
#include <type_traits>
#include "ham_entry.h"

namespace tcm {
namespace {

constexpr int TPB = 256;

__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }

// Wavefront sum by a butterfly of cross-lane exchanges: every lane ends with
// the same bits (each exchange adds the same two values, and IEEE addition
// commutes).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide sum (all threads get the result): a wavefront sum per wave, then
// the TPB / 64 wave results added in wave order.
__device__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int w = 1; w < TPB / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
}
__device__ double block_max(double v, double* sh) {
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int w = 1; w < TPB / 64; ++w) r = fmax(r, sh[w]);
  __syncthreads();
  return r;
}

// ------------------------------------------------------------ Eq. (4)
__global__ void ham_fill_kernel(ModelArgs m, double* __restrict__ H, int64_t ldh) {
  const int64_t col = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (col >= m.N) return;
  for (int64_t row = blockIdx.y; row < m.N; row += gridDim.y)
    H[row * ldh + col] = ham_entry(m, row, col);
}

// ----------------------------------------------------- expm helpers
__global__ void axpb_identity_kernel(const double* __restrict__ X, int64_t ldx, double a, double b,
                                     double* __restrict__ out, int64_t ldo, int64_t N) {
  const int64_t col = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (col >= N) return;
  for (int64_t row = blockIdx.y; row < N; row += gridDim.y)
    out[row * ldo + col] = a * X[row * ldx + col] + (row == col ? b : 0.0);
}

__global__ void assemble_cs_kernel(const double* __restrict__ Cm, const double* __restrict__ Sm,
                                   int64_t ld, double pr, double pi, c128* __restrict__ U,
                                   int64_t ldu, int64_t N) {
  const int64_t col = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (col >= N) return;
  for (int64_t row = blockIdx.y; row < N; row += gridDim.y) {
    const double c = Cm[row * ld + col], sv = Sm[row * ld + col];
    // (pr + i pi) (c - i s)
    U[row * ldu + col] = c128{pr * c + pi * sv, pi * c - pr * sv};
  }
}

__global__ void symmetrize_kernel(c128* __restrict__ U, int64_t ldu, int64_t N) {
  const int64_t col = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (col >= N) return;
  for (int64_t row = blockIdx.y; row < col; row += gridDim.y) {
    const c128 a = U[row * ldu + col], b = U[col * ldu + row];
    const c128 v{0.5 * (a.re + b.re), 0.5 * (a.im + b.im)};
    U[row * ldu + col] = v;
    U[col * ldu + row] = v;
  }
}

// ----------------------------------------------------------- copies
__global__ void c128_to_c64_kernel(const c128* __restrict__ s, int64_t lds, c64* __restrict__ d,
                                   int64_t ldd, int64_t rows, int64_t cols) {
  const int64_t col = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (col >= cols) return;
  for (int64_t row = blockIdx.y; row < rows; row += gridDim.y) {
    const c128 v = s[row * lds + col];
    d[row * ldd + col] = c64{float(v.re), float(v.im)};
  }
}
__global__ void c64_to_c128_kernel(const c64* __restrict__ s, int64_t lds, c128* __restrict__ d,
                                   int64_t ldd, int64_t rows, int64_t cols) {
  const int64_t col = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (col >= cols) return;
  for (int64_t row = blockIdx.y; row < rows; row += gridDim.y) {
    const c64 v = s[row * lds + col];
    d[row * ldd + col] = c128{double(v.re), double(v.im)};
  }
}

// ------------------------------------------------------ rotating frame
__device__ __forceinline__ int exc_number(int64_t s, int n) {
  const uint64_t mask = (uint64_t(1) << n) - 1;
  return int(s >> n) + popc64(uint64_t(s) & mask);
}

template <typename E>
__global__ void rotating_d_kernel(ModelArgs m, const c128* __restrict__ U, int64_t ldu, double dt,
                                  E* __restrict__ D, int64_t ldd) {
  const int64_t col = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (col >= m.N) return;
  for (int64_t row = blockIdx.y; row < m.N; row += gridDim.y) {
    double sn, cs;
    sincos(m.omega_c * double(exc_number(row, m.n)) * dt, &sn, &cs);
    const c128 u = U[row * ldu + col];
    c128 v{cs * u.re - sn * u.im, cs * u.im + sn * u.re};
    if (row == col) v.re -= 1.0;
    typedef decltype(E().re) T;
    D[row * ldd + col] = E{T(v.re), T(v.im)};
  }
}

template <typename E>
__global__ void frame_phase_kernel(ModelArgs m, E* __restrict__ rho, int64_t ld, double t) {
  const int64_t col = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (col >= m.N) return;
  const int kc = exc_number(col, m.n);
  for (int64_t row = blockIdx.y; row < m.N; row += gridDim.y) {
    const int kr = exc_number(row, m.n);
    if (kr == kc) continue;
    double sn, cs;
    sincos(-m.omega_c * double(kr - kc) * t, &sn, &cs);
    const E v = rho[row * ld + col];
    const double re = double(v.re), im = double(v.im);
    rho[row * ld + col] = E{decltype(v.re)(cs * re - sn * im), decltype(v.re)(cs * im + sn * re)};
  }
}

// ------------------------------------------------------- dissipation
// Amplitude damping of the atoms on index bits b0 and b1 (b1 < 0: b0 only;
// atom i is bit n - 1 - i), probability p = 1 - e^{-gamma dt}, f = sqrt(1 - p).
// For one atom and the 2 x 2 block of rows {r, r + e} and columns {s, s + e}
// (both with the atom's bit clear) the channel K0 . K0^dag + K1 . K1^dag is
//   x00 <- x00 + p x11,  x01 <- f x01,  x10 <- f x10,  x11 <- (1 - p) x11.
// A thread owns the (2^k x 2^k) block over the k bits of the pass, so the
// update is in place with no other thread touching its elements.
__device__ __forceinline__ int64_t insert_zero_bit(int64_t q, int b) {
  return ((q >> b) << (b + 1)) | (q & ((int64_t(1) << b) - 1));
}

template <typename E, int K>
__global__ void damp_atoms_kernel(E* __restrict__ rho, int64_t ld, int64_t N, int b0, int b1,
                                  double p, double f) {
  constexpr int B = 1 << K;
  const int64_t R = N >> K;                  // reduced row / column count
  const int64_t qs = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (qs >= R) return;
  int64_t s0 = insert_zero_bit(qs, b0);
  if (K == 2) s0 = insert_zero_bit(s0, b1);
  const int64_t e[2] = {int64_t(1) << b0, K == 2 ? int64_t(1) << b1 : 0};
  for (int64_t qr = blockIdx.y; qr < R; qr += gridDim.y) {
    int64_t r0 = insert_zero_bit(qr, b0);
    if (K == 2) r0 = insert_zero_bit(r0, b1);
    double xr[B][B], xi[B][B];
#pragma unroll
    for (int u = 0; u < B; ++u)
#pragma unroll
      for (int v = 0; v < B; ++v) {
        const int64_t r = r0 + ((u & 1) ? e[0] : 0) + ((u & 2) ? e[1] : 0);
        const int64_t c = s0 + ((v & 1) ? e[0] : 0) + ((v & 2) ? e[1] : 0);
        const E x = rho[r * ld + c];
        xr[u][v] = double(x.re);
        xi[u][v] = double(x.im);
      }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int bit = 1 << k;
#pragma unroll
      for (int u = 0; u < B; ++u)
#pragma unroll
        for (int v = 0; v < B; ++v) {
          if ((u & bit) || (v & bit)) continue;
          const int u1 = u | bit, v1 = v | bit;
          xr[u][v] += p * xr[u1][v1];
          xi[u][v] += p * xi[u1][v1];
          xr[u][v1] *= f; xi[u][v1] *= f;
          xr[u1][v] *= f; xi[u1][v] *= f;
          xr[u1][v1] *= 1.0 - p; xi[u1][v1] *= 1.0 - p;
        }
    }
#pragma unroll
    for (int u = 0; u < B; ++u)
#pragma unroll
      for (int v = 0; v < B; ++v) {
        const int64_t r = r0 + ((u & 1) ? e[0] : 0) + ((u & 2) ? e[1] : 0);
        const int64_t c = s0 + ((v & 1) ? e[0] : 0) + ((v & 2) ? e[1] : 0);
        rho[r * ld + c] = E{decltype(E::re)(xr[u][v]), decltype(E::re)(xi[u][v])};
      }
  }
}

// The three channels on one 8 x 8 block held by two neighbouring lanes: lane
// h has rows u = 4 h + uu (uu = 0..3) and all 8 columns; bit k of a row or
// column index is the state of atom k of the three.
__device__ __forceinline__ void damp3_block(float (&xr)[4][8], float (&xi)[4][8], int h, float p,
                                            float f) {
  const float q1 = 1.f - p;
  // atom b2: lane 0 gains p x[u|4][v|4] (the partner's columns 4..7), then
  // scales its columns 4..7 by f; lane 1 scales columns 0..3 by f and 4..7
  // by 1 - p
#pragma unroll
  for (int uu = 0; uu < 4; ++uu)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float pr = __shfl_xor(xr[uu][v + 4], 1, 64);
      const float pi = __shfl_xor(xi[uu][v + 4], 1, 64);
      if (h == 0) {
        xr[uu][v] += p * pr;
        xi[uu][v] += p * pi;
        xr[uu][v + 4] *= f;
        xi[uu][v + 4] *= f;
      } else {
        xr[uu][v] *= f;
        xi[uu][v] *= f;
        xr[uu][v + 4] *= q1;
        xi[uu][v + 4] *= q1;
      }
    }
  // atoms b0, b1 inside the half (row bits 0, 1 of uu; column bits 0, 1 of v)
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int bit = 1 << k;
#pragma unroll
    for (int uu = 0; uu < 4; ++uu)
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        if ((uu & bit) || (v & bit)) continue;
        const int u1 = uu | bit, v1 = v | bit;
        xr[uu][v] += p * xr[u1][v1];
        xi[uu][v] += p * xi[u1][v1];
        xr[uu][v1] *= f; xi[uu][v1] *= f;
        xr[u1][v] *= f; xi[u1][v] *= f;
        xr[u1][v1] *= q1; xi[u1][v1] *= q1;
      }
  }
}

// Three atoms per pass (bits b0 < b1 < b2) for the complex FP32 state, in
// FP32 arithmetic: the same channel as above for each of the three bits, so a
// state of n atoms takes ceil(n / 3) passes over the matrix instead of
// ceil(n / 2).  The 8 x 8 block of one row and column triple is shared by two
// neighbouring lanes: lane h of the pair holds its rows u with u's bit 2
// (atom b2) equal to h, 32 complex values, so the kernel fits three waves per
// SIMD (one lane holding all 64 values needed more than 256 registers and ran
// one wave per SIMD at half of HBM bandwidth).  The channels of different
// atoms commute, so the b2 channel goes first: its only coupling between the
// halves, x[u][v] += p x[u|4][v|4] for u, v with bit 2 clear, takes the
// partner's 16 values x[u|4][v|4] by a cross-lane exchange before either lane
// changes them; the b0 and b1 channels then act inside each half.
__global__ void __launch_bounds__(TPB)
damp_atoms3_c64_kernel(c64* __restrict__ rho, int64_t ld, int64_t N, int b0, int b1, int b2,
                       float p, float f) {
  const int64_t R = N >> 3;
  const int64_t tid = int64_t(blockIdx.x) * TPB + threadIdx.x;
  const int64_t qs = tid >> 1;
  const int h = int(tid & 1);
  if (qs >= R) return;                       // both lanes of a pair leave together
  const int64_t s0 = insert_zero_bit(insert_zero_bit(insert_zero_bit(qs, b0), b1), b2);
  const int64_t e0 = int64_t(1) << b0, e1 = int64_t(1) << b1, e2 = int64_t(1) << b2;
  for (int64_t qr = blockIdx.y; qr < R; qr += gridDim.y) {
    const int64_t r0 = insert_zero_bit(insert_zero_bit(insert_zero_bit(qr, b0), b1), b2) +
                       (h ? e2 : 0);
    float xr[4][8], xi[4][8];                // rows u = 4 h + uu, all 8 columns
#pragma unroll
    for (int uu = 0; uu < 4; ++uu)
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int64_t r = r0 + ((uu & 1) ? e0 : 0) + ((uu & 2) ? e1 : 0);
        const int64_t c = s0 + ((v & 1) ? e0 : 0) + ((v & 2) ? e1 : 0) + ((v & 4) ? e2 : 0);
        const c64 x = rho[r * ld + c];
        xr[uu][v] = x.re;
        xi[uu][v] = x.im;
      }
    damp3_block(xr, xi, h, p, f);
#pragma unroll
    for (int uu = 0; uu < 4; ++uu)
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int64_t r = r0 + ((uu & 1) ? e0 : 0) + ((uu & 2) ? e1 : 0);
        const int64_t c = s0 + ((v & 1) ? e0 : 0) + ((v & 2) ? e1 : 0) + ((v & 4) ? e2 : 0);
        rho[r * ld + c] = c64{xr[uu][v], xi[uu][v]};
      }
  }
}

// The same three-atom pass for atoms b, b + 1, b + 2 with coalesced memory
// access.  Each 8 x 8 block's columns lie 2^b apart, so a lane pair reading its
// own block touches a different cache line with almost every load.  Here a
// workgroup takes one row triple group (the 8 rows r0 + u 2^b) and a window of
// W consecutive columns (W a multiple of 8 2^b, so the window holds W / 8 whole
// column groups): it reads the 8 x W values with 16-byte loads that cover
// contiguous rows, stages them in LDS, applies damp3_block to each block with
// two lanes per block as above, and writes the window back the same way.  LDS
// holds column w of a row at w + w / 8 (rows W + W / 8 + 2 long), which keeps
// the block reads of a wave on distinct banks for every b.
__device__ __forceinline__ int damp3_pos(int w) { return w + (w >> 3); }

__global__ void __launch_bounds__(512)
damp_atoms3_lds_c64_kernel(c64* __restrict__ rho, int64_t ld, int64_t N, int b, int W, float p,
                           float f) {
  extern __shared__ float2 sx[];
  const int pitch = W + (W >> 3) + 2;
  const int nt = W >> 2;                      // two lanes per block, W / 8 blocks
  const int t = threadIdx.x;
  const int64_t e = int64_t(1) << b;
  const int64_t c0 = int64_t(blockIdx.x) * W;
  // this lane's block and half
  const int blk = t >> 1, h = t & 1;
  const int j = blk & int(e - 1), gi = blk >> b;
  for (int64_t rg = blockIdx.y; rg < (N >> 3); rg += gridDim.y) {
    const int64_t r0 = insert_zero_bit(insert_zero_bit(insert_zero_bit(rg, b), b + 1), b + 2);
    // 8 rows x W columns: piece k * nt + t (two complex values) of every row
    float4 v[8][2];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int64_t col = c0 + 2 * (k * nt + t);
        v[u][k] = *reinterpret_cast<const float4*>(rho + (r0 + u * e) * ld + col);
      }
    __syncthreads();                          // the previous group's window is written out
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int w = 2 * (k * nt + t);       // even: w and w + 1 share a group of 8
        sx[u * pitch + damp3_pos(w)] = make_float2(v[u][k].x, v[u][k].y);
        sx[u * pitch + damp3_pos(w) + 1] = make_float2(v[u][k].z, v[u][k].w);
      }
    __syncthreads();
    {
      float xr[4][8], xi[4][8];
#pragma unroll
      for (int uu = 0; uu < 4; ++uu)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int w = (gi << (b + 3)) | (c << b) | j;
          const float2 x = sx[(4 * h + uu) * pitch + damp3_pos(w)];
          xr[uu][c] = x.x;
          xi[uu][c] = x.y;
        }
      damp3_block(xr, xi, h, p, f);
#pragma unroll
      for (int uu = 0; uu < 4; ++uu)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int w = (gi << (b + 3)) | (c << b) | j;
          sx[(4 * h + uu) * pitch + damp3_pos(w)] = make_float2(xr[uu][c], xi[uu][c]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int w = 2 * (k * nt + t);
        const float2 a = sx[u * pitch + damp3_pos(w)], c = sx[u * pitch + damp3_pos(w) + 1];
        *reinterpret_cast<float4*>(rho + (r0 + u * e) * ld + c0 + w) = make_float4(a.x, a.y, c.x, c.y);
      }
  }
}

// Cavity damping with eta = e^{-kappa dt}: Kraus operators
// E_l = sum_m sqrt(binom(m, l)) eta^{(m-l)/2} (1 - eta)^{l/2} |m - l><m|, so
//   rho'[(m,a),(m',a')] = sum_{l >= 0} sqrt(binom(m+l, l) binom(m'+l, l))
//                         eta^{(m+m')/2} (1 - eta)^l rho[(m+l,a),(m'+l,a')].
// A thread owns one chain (a, a', m' - m = d) and walks it from the lowest
// photon numbers up, so each new value reads only entries not yet rewritten.
template <typename E>
__global__ void damp_cavity_kernel(E* __restrict__ rho, int64_t ld, int n, int c, double eta) {
  const int64_t per = int64_t(1) << n;
  const int64_t ac = int64_t(blockIdx.x) * TPB + threadIdx.x;   // column atom index a'
  if (ac >= per) return;
  const int d = int(blockIdx.z) - c;                             // m' - m
  const int mlo = d < 0 ? -d : 0;
  const int len = c + 1 - (d < 0 ? -d : d);
  const double q = 1.0 - eta;
  for (int64_t ar = blockIdx.y; ar < per; ar += gridDim.y) {
    for (int j = 0; j < len; ++j) {
      const int m = mlo + j, mp = m + d;
      double coef = pow(eta, 0.5 * double(m + mp));
      double yr = 0.0, yi = 0.0;
      for (int l = 0; j + l < len; ++l) {
        if (l > 0) coef *= sqrt(double(m + l) * double(mp + l)) / double(l) * q;
        const E x = rho[(int64_t(m + l) * per + ar) * ld + int64_t(mp + l) * per + ac];
        yr += coef * double(x.re);
        yi += coef * double(x.im);
      }
      rho[(int64_t(m) * per + ar) * ld + int64_t(mp) * per + ac] =
          E{decltype(E::re)(yr), decltype(E::re)(yi)};
    }
  }
}

// The same channel with each chain held in registers (c + 1 <= L): a thread
// owns the (c + 1)^2 elements of one (a, a') pair and walks its 2c + 1
// chains, so every element is read once and written once and a workgroup
// touches only the c + 1 rows of one a.
template <typename E, int L>
__global__ void damp_cavity_reg_kernel(E* __restrict__ rho, int64_t ld, int n, int c,
                                       double eta) {
  const int64_t per = int64_t(1) << n;
  const int64_t ac = int64_t(blockIdx.x) * TPB + threadIdx.x;   // column atom index a'
  if (ac >= per) return;
  const double q = 1.0 - eta, se = sqrt(eta);
  for (int64_t ar = blockIdx.y; ar < per; ar += gridDim.y) {
    for (int d = -c; d <= c; ++d) {                              // m' - m
      const int mlo = d < 0 ? -d : 0;
      const int len = c + 1 - (d < 0 ? -d : d);
      double xr[L], xi[L];
#pragma unroll
      for (int j = 0; j < L; ++j) {
        if (j < len) {
          const E x = rho[(int64_t(mlo + j) * per + ar) * ld + int64_t(mlo + j + d) * per + ac];
          xr[j] = double(x.re);
          xi[j] = double(x.im);
        }
      }
#pragma unroll
      for (int j = 0; j < L; ++j) {
        if (j >= len) continue;
        const int m = mlo + j, mp = m + d;
        double coef = 1.0;                     // eta^{(m + m')/2}
        for (int e = 0; e < m + mp; ++e) coef *= se;
        double yr = 0.0, yi = 0.0;
#pragma unroll
        for (int l = 0; l < L; ++l) {
          if (j + l >= len) break;
          if (l > 0) coef *= sqrt(double(m + l) * double(mp + l)) / double(l) * q;
          yr += coef * xr[j + l];
          yi += coef * xi[j + l];
        }
        rho[(int64_t(m) * per + ar) * ld + int64_t(mp) * per + ac] =
            E{decltype(E::re)(yr), decltype(E::re)(yi)};
      }
    }
  }
}

// ------------------------------------------------------- per-step readout
// map == NULL: rho is in the basis order; else basis state s sits at row and
// column map[s] of rho (the excitation-sorted order of the sector stepper, or
// the order of one sector, where states outside it have map[s] = -1).
// Writes pop = sum_s |l(s)| Re rho_ss, pdist[m] = sum_{photon(s) = m} Re rho_ss
// and pstate[m] = P({m>) of Eq. (13) (m photons and n - m excited atoms),
// m = 0 .. min(n, c); each output may be NULL.
template <typename E>
__device__ __forceinline__ void readout_body(int n, int c, const E* __restrict__ rho, int64_t ld,
                                             const int32_t* __restrict__ map,
                                             double* __restrict__ pop, double* __restrict__ pdist,
                                             double* __restrict__ pstate, double* sh) {
  const int64_t per = int64_t(1) << n;
  const uint64_t mask = uint64_t(per - 1);
  double tot = 0.0;
  for (int mm = 0; mm <= c; ++mm) {
    double part = 0.0, ex = 0.0, st = 0.0;
    for (int64_t s = mm * per + threadIdx.x; s < (mm + 1) * per; s += TPB) {
      const int64_t q = map ? int64_t(map[s]) : s;
      if (q < 0) continue;                     // state outside a one-sector rho
      const double d = double(rho[q * ld + q].re);
      const int pc = popc64(uint64_t(s) & mask);
      part += d;
      ex += double(pc) * d;
      if (pc == n - mm) st += d;
    }
    if (pdist) {
      const double pm = block_sum(part, sh);
      if (threadIdx.x == 0) pdist[mm] = pm;
    }
    if (pstate && mm <= n) {
      const double pm = block_sum(st, sh);
      if (threadIdx.x == 0) pstate[mm] = pm;
    }
    tot += ex;
  }
  const double t = block_sum(tot, sh);
  if (threadIdx.x == 0 && pop) *pop = t;
}

template <typename E>
__global__ void readout_kernel(ModelArgs m, const E* __restrict__ rho, int64_t ld,
                               const int32_t* __restrict__ map, double* __restrict__ pop,
                               double* __restrict__ pdist, double* __restrict__ pstate) {
  __shared__ double sh[TPB / 64];
  readout_body(m.n, m.c, rho, ld, map, pop, pdist, pstate, sh);
}

// advance (a launch of one item only): the kernel also moves the record
// index on, after the block's last barrier, by which point every thread has
// read it; a captured step then needs no separate counter launch.
template <typename E>
__global__ void grouped_readout_kernel(const ReadoutItem* __restrict__ items,
                                       int* __restrict__ counter, int advance) {
  __shared__ double sh[TPB / 64];
  const ReadoutItem it = items[blockIdx.x];
  const int64_t r = *counter;
  const int ns = (it.n < it.c ? it.n : it.c) + 1;
  readout_body(it.n, it.c, static_cast<const E*>(it.rho), it.ld, it.map,
               it.pop ? it.pop + r : nullptr, it.pdist ? it.pdist + r * (it.c + 1) : nullptr,
               it.pstate ? it.pstate + r * ns : nullptr, sh);
  if (advance && threadIdx.x == 0) *counter = int(r) + 1;
}

__global__ void advance_counter_kernel(int* counter) {
  if (threadIdx.x == 0) *counter += 1;
}

// ---------------------------------------------------- FP64 renormalisation
template <typename E>
__global__ void trace_kernel(const E* __restrict__ rho, int64_t ld, int64_t N, double* scratch) {
  __shared__ double sh[TPB / 64];
  double part = 0.0;
  for (int64_t s = threadIdx.x; s < N; s += TPB) part += double(rho[s * ld + s].re);
  const double tr = block_sum(part, sh);
  if (threadIdx.x == 0) {
    scratch[0] = tr;
    if (!(tr > 0.0) || !isfinite(tr)) scratch[1] = 1.0;
  }
}

constexpr int RT = 32;  // tile edge of the pair kernels

__device__ __forceinline__ void pair_index(int64_t b, int64_t& bi, int64_t& bj) {
  // b -> (bi <= bj) over the upper triangle of tile pairs, row by row of bj:
  // bj = floor((sqrt(8b+1)-1)/2), bi = b - bj(bj+1)/2
  int64_t j = int64_t((sqrt(8.0 * double(b) + 1.0) - 1.0) * 0.5);
  while (j * (j + 1) / 2 > b) --j;
  while ((j + 1) * (j + 2) / 2 <= b) ++j;
  bj = j;
  bi = b - j * (j + 1) / 2;
}

template <typename E>
__global__ void renorm_kernel(E* __restrict__ rho, int64_t ld, int64_t N, const double* scratch) {
  __shared__ double2 tA[RT][RT + 1];
  __shared__ double2 tB[RT][RT + 1];
  if (scratch[1] != 0.0) return;   // non-finite / non-positive trace: leave rho as is
  const double inv = 1.0 / scratch[0];
  int64_t bi, bj;
  pair_index(blockIdx.x, bi, bj);
  const int tx = threadIdx.x % RT, ty = threadIdx.x / RT;   // 32 x 8
  // load tile (bi, bj) and (bj, bi)
  for (int r = ty; r < RT; r += TPB / RT) {
    const int64_t i = bi * RT + r, j = bj * RT + tx;
    if (i < N && j < N) { const E v = rho[i * ld + j]; tA[r][tx] = make_double2(v.re, v.im); }
    const int64_t i2 = bj * RT + r, j2 = bi * RT + tx;
    if (i2 < N && j2 < N) { const E v = rho[i2 * ld + j2]; tB[r][tx] = make_double2(v.re, v.im); }
  }
  __syncthreads();
  // element (i, j) in tile A pairs with (j, i) = tB[tx][r]
  for (int r = ty; r < RT; r += TPB / RT) {
    const int64_t i = bi * RT + r, j = bj * RT + tx;
    if (i < N && j < N) {
      const double2 a = tA[r][tx], b = tB[tx][r];
      double re = 0.5 * (a.x + b.x) * inv, im = 0.5 * (a.y - b.y) * inv;
      if (i == j) im = 0.0;
      typedef decltype(E().re) T;
      rho[i * ld + j] = E{T(re), T(im)};
      if (bi != bj) rho[j * ld + i] = E{T(re), T(-im)};
    }
  }
}

// ------------------------------------------------------------ observables
// Pass 1: per tile pair (bi <= bj): purity partial, Hermiticity max,
// non-finite count; diagonal tiles also copy their diagonal to diag[].
template <typename E>
__global__ void obs_pass1(const E* __restrict__ rho, int64_t ld, int64_t N,
                          double* __restrict__ partials, double* __restrict__ diag) {
  __shared__ double2 tA[RT][RT + 1];
  __shared__ double2 tB[RT][RT + 1];
  __shared__ double sh[TPB / 64];
  int64_t bi, bj;
  pair_index(blockIdx.x, bi, bj);
  const int tx = threadIdx.x % RT, ty = threadIdx.x / RT;
  for (int r = ty; r < RT; r += TPB / RT) {
    const int64_t i = bi * RT + r, j = bj * RT + tx;
    tA[r][tx] = (i < N && j < N) ? make_double2(rho[i * ld + j].re, rho[i * ld + j].im) : make_double2(0, 0);
    const int64_t i2 = bj * RT + r, j2 = bi * RT + tx;
    tB[r][tx] = (i2 < N && j2 < N) ? make_double2(rho[i2 * ld + j2].re, rho[i2 * ld + j2].im) : make_double2(0, 0);
  }
  __syncthreads();
  double pur = 0.0, herm = 0.0, bad = 0.0;
  for (int r = ty; r < RT; r += TPB / RT) {
    const double2 a = tA[r][tx], b = tB[tx][r];
    const double2 b2 = tB[r][tx];
    if (!isfinite(a.x) || !isfinite(a.y)) bad += 1.0;
    pur += a.x * a.x + a.y * a.y;
    if (bi != bj) {
      if (!isfinite(b2.x) || !isfinite(b2.y)) bad += 1.0;
      pur += b2.x * b2.x + b2.y * b2.y;
    }
    herm = fmax(herm, hypot(a.x - b.x, a.y + b.y));
    if (bi == bj && r == tx) {
      const int64_t i = bi * RT + r;
      if (i < N) diag[i] = a.x;
    }
  }
  const double P = block_sum(pur, sh);
  const double Hm = block_max(herm, sh);
  const double B = block_sum(bad, sh);
  if (threadIdx.x == 0) {
    partials[3 * blockIdx.x + 0] = P;
    partials[3 * blockIdx.x + 1] = Hm;
    partials[3 * blockIdx.x + 2] = B;
  }
}

__global__ void obs_pass2(ModelArgs m, const double* __restrict__ partials, int64_t npairs,
                          const double* __restrict__ diag, const double* __restrict__ trace_im_src,
                          double* __restrict__ scalars, double* __restrict__ atom_pop,
                          double* __restrict__ photon_dist, double* __restrict__ exc_dist,
                          double* __restrict__ photon_state) {
  __shared__ double sh[TPB / 64];
  const int n = m.n;
  const int64_t N = m.N;
  const uint64_t mask = (uint64_t(1) << n) - 1;
  double pur = 0.0, herm = 0.0, bad = 0.0;
  for (int64_t b = threadIdx.x; b < npairs; b += TPB) {
    pur += partials[3 * b];
    herm = fmax(herm, partials[3 * b + 1]);
    bad += partials[3 * b + 2];
  }
  pur = block_sum(pur, sh);
  herm = block_max(herm, sh);
  bad = block_sum(bad, sh);
  double tr = 0.0, ex = 0.0, ph = 0.0, nx = 0.0;
  for (int64_t s = threadIdx.x; s < N; s += TPB) {
    const double d = diag[s];
    const int pc = popc64(uint64_t(s) & mask);
    const int64_t mm = s >> n;
    tr += d;
    ex += double(pc) * d;
    ph += double(mm) * d;
    nx += double(mm + pc) * d;
  }
  tr = block_sum(tr, sh);
  ex = block_sum(ex, sh);
  ph = block_sum(ph, sh);
  nx = block_sum(nx, sh);
  if (threadIdx.x == 0) {
    scalars[0] = tr;
    scalars[1] = trace_im_src ? *trace_im_src : 0.0;
    scalars[2] = pur;
    scalars[3] = herm;
    scalars[4] = ex;
    scalars[5] = ph;
    scalars[6] = nx;
    scalars[7] = bad > 0.0 ? 1.0 : 0.0;
  }
  if (atom_pop) {
    for (int i = 0; i < n; ++i) {
      double p = 0.0;
      for (int64_t s = threadIdx.x; s < N; s += TPB)
        if ((uint64_t(s) >> (n - 1 - i)) & 1) p += diag[s];
      p = block_sum(p, sh);
      if (threadIdx.x == 0) atom_pop[i] = p;
    }
  }
  if (photon_dist) {
    const int64_t per = int64_t(1) << n;
    for (int mm = 0; mm <= m.c; ++mm) {
      double p = 0.0;
      for (int64_t s = mm * per + threadIdx.x; s < (mm + 1) * per; s += TPB) p += diag[s];
      p = block_sum(p, sh);
      if (threadIdx.x == 0) photon_dist[mm] = p;
    }
  }
  if (photon_state) {
    // Eq. (13), sector reading: m photons and n - m excited atoms
    const int64_t per = int64_t(1) << n;
    for (int mm = 0; mm <= m.c && mm <= n; ++mm) {
      double p = 0.0;
      for (int64_t s = mm * per + threadIdx.x; s < (mm + 1) * per; s += TPB)
        if (popc64(uint64_t(s) & mask) == n - mm) p += diag[s];
      p = block_sum(p, sh);
      if (threadIdx.x == 0) photon_state[mm] = p;
    }
  }
  if (exc_dist) {
    for (int k = 0; k <= n + m.c; ++k) {
      double p = 0.0;
      for (int64_t s = threadIdx.x; s < N; s += TPB)
        if (int(s >> n) + popc64(uint64_t(s) & mask) == k) p += diag[s];
      p = block_sum(p, sh);
      if (threadIdx.x == 0) exc_dist[k] = p;
    }
  }
}

// Eq. (13), symmetric reading: <v_m| rho |v_m> with v_m the normalised equal
// sum of the binom(n, m) basis states with m photons and n - m excited atoms,
// i.e. the sum of Re rho_st over those pairs divided by binom(n, m).
// Pass 1: grid (ceil(2^n / 4), min(n, c) + 1); wave w of block b takes atom
// pattern l = 4 b + w as its row and sums its row of the photon block m over
// the columns with the same excitation count; partials[m * gridDim.x + b].
template <typename E>
__global__ void dicke_pass1(int n, const E* __restrict__ rho, int64_t ld,
                            double* __restrict__ partials) {
  __shared__ double sh[TPB / 64];
  const int mm = blockIdx.y;
  const int64_t per = int64_t(1) << n;
  const int64_t l = int64_t(blockIdx.x) * (TPB / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  double acc = 0.0;
  if (l < per && popc64(uint64_t(l)) == n - mm) {
    const E* row = rho + (mm * per + l) * ld + mm * per;
    for (int64_t t = lane; t < per; t += 64)
      if (popc64(uint64_t(t)) == n - mm) acc += double(row[t].re);
  }
  acc = wave_sum(acc);
  if (lane == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int w = 1; w < TPB / 64; ++w) r += sh[w];
    partials[int64_t(mm) * gridDim.x + blockIdx.x] = r;
  }
}

// Pass 2: one block per m: dicke[m] = (sum of its partials) / binom(n, m).
__global__ void dicke_pass2(int n, const double* __restrict__ partials, int64_t nblk,
                            double* __restrict__ dicke) {
  __shared__ double sh[TPB / 64];
  const int mm = blockIdx.x;
  double p = 0.0;
  for (int64_t b = threadIdx.x; b < nblk; b += TPB) p += partials[int64_t(mm) * nblk + b];
  p = block_sum(p, sh);
  if (threadIdx.x == 0) {
    double binom = 1.0;
    for (int j = 1; j <= mm; ++j) binom = binom * double(n - mm + j) / double(j);
    dicke[mm] = p / binom;
  }
}

// Im Tr rho (separate, one block).
template <typename E>
__global__ void trace_im_kernel(const E* __restrict__ rho, int64_t ld, int64_t N, double* out) {
  __shared__ double sh[TPB / 64];
  double part = 0.0;
  for (int64_t s = threadIdx.x; s < N; s += TPB) part += double(rho[s * ld + s].im);
  const double t = block_sum(part, sh);
  if (threadIdx.x == 0) *out = t;
}

// ------------------------------------------------------------ adjoint helpers
template <typename E>
__global__ void excitation_op_kernel(ModelArgs m, E* __restrict__ O, int64_t ld) {
  const int64_t col = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (col >= m.N) return;
  const uint64_t mask = (uint64_t(1) << m.n) - 1;
  typedef decltype(E().re) T;
  for (int64_t row = blockIdx.y; row < m.N; row += gridDim.y) {
    const T v = row == col ? T(popc64(uint64_t(row) & mask)) : T(0);
    O[row * ld + col] = E{v, T(0)};
  }
}

__global__ void accumulate_c64_kernel(const c64* __restrict__ T, int64_t ldt, c128* __restrict__ M,
                                      int64_t ldm, int64_t N) {
  const int64_t col = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (col >= N) return;
  for (int64_t row = blockIdx.y; row < N; row += gridDim.y) {
    const c64 t = T[row * ldt + col];
    c128 v = M[row * ldm + col];
    v.re += double(t.re);
    v.im += double(t.im);
    M[row * ldm + col] = v;
  }
}

__global__ void minus_i_shifted_kernel(ModelArgs m, const double* __restrict__ H, int64_t ldh,
                                       double mu, double scale, c128* __restrict__ out,
                                       int64_t ldo) {
  const int64_t col = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (col >= m.N) return;
  for (int64_t row = blockIdx.y; row < m.N; row += gridDim.y) {
    double h = H[row * ldh + col];
    if (row == col) h -= m.omega_c * double(exc_number(row, m.n)) + mu;
    out[row * ldo + col] = c128{0.0, -h * scale};
  }
}

__global__ void scale_c128_kernel(c128* __restrict__ X, int64_t ld, double a, int64_t N) {
  const int64_t col = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (col >= N) return;
  for (int64_t row = blockIdx.y; row < N; row += gridDim.y) {
    c128 v = X[row * ld + col];
    X[row * ld + col] = c128{a * v.re, a * v.im};
  }
}

__global__ void identity_c128_kernel(c128* __restrict__ X, int64_t ld, int64_t N) {
  const int64_t col = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (col >= N) return;
  for (int64_t row = blockIdx.y; row < N; row += gridDim.y)
    X[row * ld + col] = c128{row == col ? 1.0 : 0.0, 0.0};
}

// One workgroup per parameter: blocks 0..n-1 give dL/dg_i, n..2n-1 dL/ddelta_i.
__global__ void grad_trace_kernel(ModelArgs m, const c128* __restrict__ G, int64_t ld, double pr,
                                  double pi, double dt, double* __restrict__ grad_g,
                                  double* __restrict__ grad_delta) {
  __shared__ double sh[TPB / 64];
  const int n = m.n;
  const int p = blockIdx.x;
  const int i = p % n;
  const int64_t per = int64_t(1) << n;
  const uint64_t bit = uint64_t(1) << (n - 1 - i);
  double acc = 0.0;   // Im(ph * sum)
  if (p < n) {
    // pairs s = (mm, l) with bit set, mm < c; t = s + 2^n - bit
    for (int64_t s = threadIdx.x; s < int64_t(m.c) * per; s += TPB) {
      if (!(uint64_t(s) & bit)) continue;
      const int64_t t = s + per - int64_t(bit);
      const double w = sqrt(double((s >> n) + 1));
      const c128 a = G[s * ld + t], b = G[t * ld + s];
      const double zr = w * (a.re + b.re), zi = w * (a.im + b.im);
      acc += pr * zi + pi * zr;
    }
  } else {
    for (int64_t s = threadIdx.x; s < m.N; s += TPB) {
      if (!(uint64_t(s) & bit)) continue;
      const c128 a = G[s * ld + s];
      acc += pr * a.im + pi * a.re;
    }
  }
  const double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    if (p < n) grad_g[i] = 2.0 * dt * tot;
    else grad_delta[i] = 2.0 * dt * tot;
  }
}

// --------------------------------------------------------- bfloat16 split
__device__ __forceinline__ uint16_t rne_bf16(float x) {
  const uint32_t b = __float_as_uint(x);
  if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu) != 0)
    return uint16_t((b >> 16) | 0x40u);                       // NaN stays (quiet) NaN
  const uint32_t upper = b >> 16, rem = b & 0xFFFFu;
  const uint32_t up = (rem > 0x8000u) || (rem == 0x8000u && (upper & 1u));
  return uint16_t(upper + up);
}

__global__ void split_bf16_kernel(const float* __restrict__ x, int64_t count,
                                  uint16_t* __restrict__ hi, uint16_t* __restrict__ lo) {
  for (int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * TPB) {
    const float v = x[i];
    const uint16_t h = rne_bf16(v);
    const float r = v - __uint_as_float(uint32_t(h) << 16);
    hi[i] = h;
    lo[i] = rne_bf16(r);
  }
}

dim3 grid2(int64_t cols, int64_t rows) {
  const int64_t gx = (cols + TPB - 1) / TPB;
  const int64_t gy = rows < 4096 ? rows : 4096;
  return dim3(unsigned(gx > 0 ? gx : 1), unsigned(gy > 0 ? gy : 1));
}

int64_t npairs_of(int64_t N) {
  const int64_t T = (N + RT - 1) / RT;
  return T * (T + 1) / 2;
}

}  // namespace

int launch_ham_fill(const ModelArgs& m, double* H, int64_t ldh, hipStream_t s) {
  if (m.N == 0) return TC_OK;
  hipLaunchKernelGGL(ham_fill_kernel, grid2(m.N, m.N), dim3(TPB), 0, s, m, H, ldh);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_axpb_identity(const double* X, int64_t ldx, double a, double b, double* out,
                         int64_t ldo, int64_t N, hipStream_t s) {
  if (N == 0) return TC_OK;
  hipLaunchKernelGGL(axpb_identity_kernel, grid2(N, N), dim3(TPB), 0, s, X, ldx, a, b, out, ldo, N);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_assemble_cs(const double* Cm, const double* Sm, int64_t ld, double pr, double pi,
                       c128* U, int64_t ldu, int64_t N, hipStream_t s) {
  if (N == 0) return TC_OK;
  hipLaunchKernelGGL(assemble_cs_kernel, grid2(N, N), dim3(TPB), 0, s, Cm, Sm, ld, pr, pi, U, ldu, N);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_symmetrize(c128* U, int64_t ldu, int64_t N, hipStream_t s) {
  if (N == 0) return TC_OK;
  hipLaunchKernelGGL(symmetrize_kernel, grid2(N, N), dim3(TPB), 0, s, U, ldu, N);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_copy_c128_to_c64(const c128* src, int64_t lds, c64* dst, int64_t ldd, int64_t rows,
                            int64_t cols, hipStream_t s) {
  if (rows == 0 || cols == 0) return TC_OK;
  hipLaunchKernelGGL(c128_to_c64_kernel, grid2(cols, rows), dim3(TPB), 0, s, src, lds, dst, ldd, rows, cols);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_copy_c64_to_c128(const c64* src, int64_t lds, c128* dst, int64_t ldd, int64_t rows,
                            int64_t cols, hipStream_t s) {
  if (rows == 0 || cols == 0) return TC_OK;
  hipLaunchKernelGGL(c64_to_c128_kernel, grid2(cols, rows), dim3(TPB), 0, s, src, lds, dst, ldd, rows, cols);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_rotating_d(const ModelArgs& m, const c128* U, int64_t ldu, double dt, c128* D,
                      int64_t ldd, hipStream_t s) {
  if (m.N == 0) return TC_OK;
  hipLaunchKernelGGL(rotating_d_kernel<c128>, grid2(m.N, m.N), dim3(TPB), 0, s, m, U, ldu, dt, D, ldd);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_rotating_d_c64(const ModelArgs& m, const c128* U, int64_t ldu, double dt, c64* D,
                          int64_t ldd, hipStream_t s) {
  if (m.N == 0) return TC_OK;
  hipLaunchKernelGGL(rotating_d_kernel<c64>, grid2(m.N, m.N), dim3(TPB), 0, s, m, U, ldu, dt, D, ldd);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_frame_phase_c128(const ModelArgs& m, c128* rho, int64_t ld, double t, hipStream_t s) {
  if (m.N == 0) return TC_OK;
  hipLaunchKernelGGL(frame_phase_kernel<c128>, grid2(m.N, m.N), dim3(TPB), 0, s, m, rho, ld, t);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_frame_phase_c64(const ModelArgs& m, c64* rho, int64_t ld, double t, hipStream_t s) {
  if (m.N == 0) return TC_OK;
  hipLaunchKernelGGL(frame_phase_kernel<c64>, grid2(m.N, m.N), dim3(TPB), 0, s, m, rho, ld, t);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

template <typename E>
int launch_dissipation_t(const ModelArgs& m, E* rho, int64_t ld, double dt, hipStream_t s) {
  if (m.N == 0) return TC_OK;
  if (m.gamma > 0.0) {
    const double p = -expm1(-m.gamma * dt);        // 1 - e^{-gamma dt}
    const double f = sqrt(1.0 - p);
    int b = 0;
    if constexpr (std::is_same<E, c64>::value) {
      for (; b + 3 <= m.n; b += 3) {
        // column window of the coalesced pass: 512 columns, or the 2^n of a
        // photon block if fewer (so it divides N); it must hold whole column
        // groups of 8 2^b.  Wider groups (b >= 7, whose window would need more
        // than the default 64 KB of dynamic LDS) and row strides that break
        // 16-byte alignment take the per-block kernel.
        const int64_t per = int64_t(1) << m.n;
        const int64_t W = std::min<int64_t>(512, per);
        if ((int64_t(8) << b) <= W && ld % 2 == 0 &&
            (reinterpret_cast<uintptr_t>(rho) & 15) == 0) {
          const size_t lds = size_t(8) * size_t(W + W / 8 + 2) * sizeof(float2);
          const int64_t groups = m.N >> 3;
          hipLaunchKernelGGL(damp_atoms3_lds_c64_kernel,
                             dim3(unsigned(m.N / W), unsigned(groups < 4096 ? groups : 4096)),
                             dim3(unsigned(W / 4)), lds, s, rho, ld, m.N, b, int(W), float(p),
                             float(f));
        } else {
          const int64_t R = m.N >> 3;            // two lanes per 8 x 8 block
          hipLaunchKernelGGL(damp_atoms3_c64_kernel, grid2(2 * R, R), dim3(TPB), 0, s, rho, ld,
                             m.N, b, b + 1, b + 2, float(p), float(f));
        }
        TC_TRY_HIP(hipGetLastError());
      }
    }
    for (; b < m.n; b += 2) {
      if (b + 1 < m.n) {
        const int64_t R = m.N >> 2;
        hipLaunchKernelGGL((damp_atoms_kernel<E, 2>), grid2(R, R), dim3(TPB), 0, s, rho, ld, m.N,
                           b, b + 1, p, f);
      } else {
        const int64_t R = m.N >> 1;
        hipLaunchKernelGGL((damp_atoms_kernel<E, 1>), grid2(R, R), dim3(TPB), 0, s, rho, ld, m.N,
                           b, -1, p, f);
      }
      TC_TRY_HIP(hipGetLastError());
    }
  }
  if (m.kappa > 0.0 && m.c > 0) {
    const int64_t per = int64_t(1) << m.n;
    const dim3 grid(unsigned((per + TPB - 1) / TPB), unsigned(per < 4096 ? per : 4096),
                    unsigned(2 * m.c + 1));
    if (m.c + 1 <= 8)
      hipLaunchKernelGGL((damp_cavity_reg_kernel<E, 8>), dim3(grid.x, grid.y), dim3(TPB), 0, s,
                         rho, ld, m.n, m.c, exp(-m.kappa * dt));
    else
      hipLaunchKernelGGL(damp_cavity_kernel<E>, grid, dim3(TPB), 0, s, rho, ld, m.n, m.c,
                         exp(-m.kappa * dt));
    TC_TRY_HIP(hipGetLastError());
  }
  return TC_OK;
}

int launch_dissipation_c128(const ModelArgs& m, c128* rho, int64_t ld, double dt, hipStream_t s) {
  return launch_dissipation_t(m, rho, ld, dt, s);
}

int launch_dissipation_c64(const ModelArgs& m, c64* rho, int64_t ld, double dt, hipStream_t s) {
  return launch_dissipation_t(m, rho, ld, dt, s);
}

int launch_readout_c128(const ModelArgs& m, const c128* rho, int64_t ld, double* pop,
                        double* pdist, hipStream_t s, const int32_t* map, double* pstate) {
  hipLaunchKernelGGL(readout_kernel<c128>, dim3(1), dim3(TPB), 0, s, m, rho, ld, map, pop, pdist,
                     pstate);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_readout_c64(const ModelArgs& m, const c64* rho, int64_t ld, double* pop,
                       double* pdist, hipStream_t s, const int32_t* map, double* pstate) {
  hipLaunchKernelGGL(readout_kernel<c64>, dim3(1), dim3(TPB), 0, s, m, rho, ld, map, pop, pdist,
                     pstate);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

template <typename E>
static int renorm_impl(E* rho, int64_t ld, int64_t N, double* scratch, hipStream_t s) {
  if (N == 0) return TC_OK;
  hipLaunchKernelGGL(trace_kernel<E>, dim3(1), dim3(TPB), 0, s, rho, ld, N, scratch);
  TC_TRY_HIP(hipGetLastError());
  const int64_t np = npairs_of(N);
  hipLaunchKernelGGL(renorm_kernel<E>, dim3(unsigned(np)), dim3(TPB), 0, s, rho, ld, N, scratch);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_renorm_c128(c128* rho, int64_t ld, int64_t N, double* scratch, hipStream_t s) {
  return renorm_impl(rho, ld, N, scratch, s);
}
int launch_renorm_c64(c64* rho, int64_t ld, int64_t N, double* scratch, hipStream_t s) {
  return renorm_impl(rho, ld, N, scratch, s);
}

// Layout of the partials buffer: 3 per tile pair, the diagonal (N), Im Tr
// (8 slots), then the Dicke partials (min(n, c) + 1) ceil(2^n / 4) <= N.
size_t observables_partials_count(int64_t N) {
  return size_t(3 * npairs_of(N) + N + 8 + N);
}

int launch_observables(const ModelArgs& m, const void* rho, int dtype, int64_t ld,
                       double* partials, double* scalars, double* atom_pop,
                       double* photon_dist, double* exc_dist, double* photon_state,
                       double* dicke, hipStream_t s) {
  const int64_t N = m.N;
  const int64_t np = npairs_of(N);
  double* diag = partials + 3 * np;
  double* tim = diag + N;
  double* dpart = tim + 8;
  const int64_t per = int64_t(1) << m.n;
  const int64_t nblk = (per + TPB / 64 - 1) / (TPB / 64);
  const int ns = (m.n < m.c ? m.n : m.c) + 1;
  if (dtype == TC_C128) {
    const c128* r = static_cast<const c128*>(rho);
    hipLaunchKernelGGL(obs_pass1<c128>, dim3(unsigned(np)), dim3(TPB), 0, s, r, ld, N, partials, diag);
    hipLaunchKernelGGL(trace_im_kernel<c128>, dim3(1), dim3(TPB), 0, s, r, ld, N, tim);
    if (dicke)
      hipLaunchKernelGGL(dicke_pass1<c128>, dim3(unsigned(nblk), unsigned(ns)), dim3(TPB), 0, s,
                         m.n, r, ld, dpart);
  } else {
    const c64* r = static_cast<const c64*>(rho);
    hipLaunchKernelGGL(obs_pass1<c64>, dim3(unsigned(np)), dim3(TPB), 0, s, r, ld, N, partials, diag);
    hipLaunchKernelGGL(trace_im_kernel<c64>, dim3(1), dim3(TPB), 0, s, r, ld, N, tim);
    if (dicke)
      hipLaunchKernelGGL(dicke_pass1<c64>, dim3(unsigned(nblk), unsigned(ns)), dim3(TPB), 0, s,
                         m.n, r, ld, dpart);
  }
  TC_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(obs_pass2, dim3(1), dim3(TPB), 0, s, m, partials, np, diag, tim, scalars,
                     atom_pop, photon_dist, exc_dist, photon_state);
  TC_TRY_HIP(hipGetLastError());
  if (dicke) {
    hipLaunchKernelGGL(dicke_pass2, dim3(unsigned(ns)), dim3(TPB), 0, s, m.n, dpart, nblk, dicke);
    TC_TRY_HIP(hipGetLastError());
  }
  return TC_OK;
}

int launch_split_bf16(const float* x, int64_t count, uint16_t* hi, uint16_t* lo, hipStream_t s) {
  if (count == 0) return TC_OK;
  int64_t blocks = (count + TPB - 1) / TPB;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(split_bf16_kernel, dim3(unsigned(blocks)), dim3(TPB), 0, s, x, count, hi, lo);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_grouped_readout(const ReadoutItem* items_dev, int count, bool c128_storage,
                           int* counter, hipStream_t s, bool advance) {
  if (count == 0) return TC_OK;
  if (advance && count != 1) {
    set_error("readout: only a single-item launch can advance the record index");
    return TC_ERR_INVALID_ARGUMENT;
  }
  if (c128_storage)
    hipLaunchKernelGGL(grouped_readout_kernel<c128>, dim3(unsigned(count)), dim3(TPB), 0, s,
                       items_dev, counter, advance ? 1 : 0);
  else
    hipLaunchKernelGGL(grouped_readout_kernel<c64>, dim3(unsigned(count)), dim3(TPB), 0, s,
                       items_dev, counter, advance ? 1 : 0);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_advance_counter(int* counter, hipStream_t s) {
  hipLaunchKernelGGL(advance_counter_kernel, dim3(1), dim3(64), 0, s, counter);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_excitation_op_c128(const ModelArgs& m, c128* O, int64_t ld, hipStream_t s) {
  if (m.N == 0) return TC_OK;
  hipLaunchKernelGGL(excitation_op_kernel<c128>, grid2(m.N, m.N), dim3(TPB), 0, s, m, O, ld);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_excitation_op_c64(const ModelArgs& m, c64* O, int64_t ld, hipStream_t s) {
  if (m.N == 0) return TC_OK;
  hipLaunchKernelGGL(excitation_op_kernel<c64>, grid2(m.N, m.N), dim3(TPB), 0, s, m, O, ld);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_accumulate_c64(const c64* T, int64_t ldt, c128* M, int64_t ldm, int64_t N,
                          hipStream_t s) {
  if (N == 0) return TC_OK;
  hipLaunchKernelGGL(accumulate_c64_kernel, grid2(N, N), dim3(TPB), 0, s, T, ldt, M, ldm, N);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_minus_i_shifted(const ModelArgs& m, const double* H, int64_t ldh, double mu,
                           double scale, c128* out, int64_t ldo, hipStream_t s) {
  if (m.N == 0) return TC_OK;
  hipLaunchKernelGGL(minus_i_shifted_kernel, grid2(m.N, m.N), dim3(TPB), 0, s, m, H, ldh, mu,
                     scale, out, ldo);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_scale_c128(c128* X, int64_t ld, double a, int64_t N, hipStream_t s) {
  if (N == 0) return TC_OK;
  hipLaunchKernelGGL(scale_c128_kernel, grid2(N, N), dim3(TPB), 0, s, X, ld, a, N);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_identity_c128(c128* X, int64_t ld, int64_t N, hipStream_t s) {
  if (N == 0) return TC_OK;
  hipLaunchKernelGGL(identity_c128_kernel, grid2(N, N), dim3(TPB), 0, s, X, ld, N);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_grad_trace(const ModelArgs& m, const c128* G, int64_t ld, double ph_re, double ph_im,
                      double dt, double* grad_g, double* grad_delta, hipStream_t s) {
  hipLaunchKernelGGL(grad_trace_kernel, dim3(unsigned(2 * m.n)), dim3(TPB), 0, s, m, G, ld, ph_re,
                     ph_im, dt, grad_g, grad_delta);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

}  // namespace tcm
