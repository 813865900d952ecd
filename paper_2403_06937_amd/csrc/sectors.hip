// Kernels of the excitation-sector stepper.
//
// H of Eq. (4) only couples |m, l> to |m +- 1, l -+ e_i>, so the excitation
// number k = m + |l| is conserved and, in the basis sorted by k (stable within
// a sector), H and U = exp(-i H dt) are block diagonal.  The stepper keeps rho
// in that sorted order ("rho hat"), multiplies the blocks, and converts at the
// boundary with the gathers below.  Each sector's positions are padded to a
// multiple of the product tile with padding states that stay exactly zero.
// Position i holds basis state perm[i] (-1 for padding) of sector sec[i];
// basis state s sits at position inv[s].
#include "kernels.h"
#include "ham_entry.h"

namespace tcm {
namespace {

constexpr int TPB = 256;
constexpr int RT = 32;   // tile edge of the mirror kernel

template <typename E> struct real_of;
template <> struct real_of<c128> { typedef double type; };
template <> struct real_of<c64> { typedef float type; };

// dst[i][j] = ph * src[map[ro + i]][map[co + j]] - sub * [ro + i == co + j];
// a negative map entry (a padding position) gives exactly 0.
template <typename Ein, typename Eout>
__global__ void gather_kernel(const Ein* __restrict__ src, int64_t lds,
                              const int32_t* __restrict__ map, int64_t ro, int64_t co,
                              int64_t rows, int64_t cols, double ph_re, double ph_im, int sub,
                              Eout* __restrict__ dst, int64_t ldd) {
  typedef typename real_of<Eout>::type T;
  const int64_t j = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (j >= cols) return;
  const int64_t sc = map[co + j];
  for (int64_t i = blockIdx.y; i < rows; i += gridDim.y) {
    const int64_t sr = map[ro + i];
    double re = 0.0, im = 0.0;
    if (sr >= 0 && sc >= 0) {
      const Ein v = src[sr * lds + sc];
      re = ph_re * double(v.re) - ph_im * double(v.im);
      im = ph_re * double(v.im) + ph_im * double(v.re);
      if (sub && ro + i == co + j) re -= 1.0;
    }
    dst[i * ldd + j] = Eout{T(re), T(im)};
  }
}

// Tile pair (bi <= bj) of the upper tile triangle, row by row of bj.
__device__ __forceinline__ void pair_of(int64_t b, int64_t& bi, int64_t& bj) {
  int64_t j = int64_t((sqrt(8.0 * double(b) + 1.0) - 1.0) * 0.5);
  while (j * (j + 1) / 2 > b) --j;
  while ((j + 1) * (j + 2) / 2 <= b) ++j;
  bj = j;
  bi = b - j * (j + 1) / 2;
}

// Workgroup b rebuilds the lower tile (bj, bi) from the upper tile (bi, bj):
// element (i, j) of the lower tile with sector(i) > sector(j) becomes
// conj(rho[j][i]).  Every element read that way lies in the upper block
// triangle, which no workgroup writes, and the source tile is read into LDS
// before any write, so the pass is race-free in place.
template <typename E>
__global__ void mirror_lower_kernel(E* __restrict__ rho, int64_t ld, int64_t N,
                                    const int32_t* __restrict__ sec) {
  typedef typename real_of<E>::type T;
  __shared__ E tS[RT][RT + 1];
  int64_t bi, bj;
  pair_of(blockIdx.x, bi, bj);
  const int64_t r0 = bj * RT, c0 = bi * RT;            // destination tile origin
  const int64_t rlast = min(r0 + RT, N) - 1;
  // nothing to write when the last row's sector does not exceed the first column's
  if (sec[rlast] <= sec[c0]) return;
  const int tx = threadIdx.x % RT, ty = threadIdx.x / RT;
  for (int r = ty; r < RT; r += TPB / RT) {
    const int64_t i = bi * RT + r, j = bj * RT + tx;
    if (i < N && j < N) tS[r][tx] = rho[i * ld + j];
  }
  __syncthreads();
  for (int r = ty; r < RT; r += TPB / RT) {
    const int64_t i = r0 + r, j = c0 + tx;
    if (i < N && j < N && sec[i] > sec[j]) {
      const E v = tS[tx][r];
      rho[i * ld + j] = E{v.re, T(-v.im)};
    }
  }
}

// The i-th basis state (increasing index) of excitation sector k: photon
// numbers m from max(0, k - n) upward, and within one m the n-bit atom
// patterns with k - m ones in increasing order (combinatorial unranking,
// binom[a * (n + 1) + b] = C(a, b)).  -1 if i >= d_k.
__device__ int64_t sector_state(int64_t i, int k, int n, int c, const int64_t* binom) {
  const int mlo = k - n > 0 ? k - n : 0, mhi = k < c ? k : c;
  for (int m = mlo; m <= mhi; ++m) {
    int p = k - m;
    const int64_t cnt = binom[n * (n + 1) + p];
    if (i < cnt) {
      uint64_t l = 0;
      for (int b = n - 1; b >= 0; --b) {
        // patterns whose bit b is 0 place all p ones among the b lower bits
        const int64_t c0 = p <= b ? binom[b * (n + 1) + p] : 0;
        if (i >= c0) { l |= uint64_t(1) << b; i -= c0; --p; }
      }
      return (int64_t(m) << n) | int64_t(l);
    }
    i -= cnt;
  }
  return -1;
}

// H_k[i][j] = H[state_i][state_j] over the d_k states of sector k.
__global__ void ham_sector_kernel(ModelArgs m, int k, int64_t d, double* __restrict__ H,
                                  int64_t ldh) {
  __shared__ int64_t binom[(TC_MAX_ATOMS + 1) * (TC_MAX_ATOMS + 1)];
  const int n = m.n;
  for (int e = threadIdx.x; e < (n + 1) * (n + 1); e += TPB) {
    const int a = e / (n + 1), b = e % (n + 1);
    int64_t v = 0;
    if (b <= a) {
      v = 1;
      for (int q = 1; q <= b; ++q) v = v * (a - b + q) / q;
    }
    binom[e] = v;
  }
  __syncthreads();
  const int64_t j = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (j >= d) return;
  const int64_t sj = sector_state(j, k, n, m.c, binom);
  for (int64_t i = blockIdx.y; i < d; i += gridDim.y)
    H[i * ldh + j] = ham_entry(m, sector_state(i, k, n, m.c, binom), sj);
}

// out = ph * U - I (the rotating-frame operand of one sector, where the frame
// factor e^{i w_c N dt} is the scalar e^{i w_c k dt}).
template <typename Eout>
__global__ void phase_minus_identity_kernel(const c128* __restrict__ U, int64_t ldu, double ph_re,
                                            double ph_im, Eout* __restrict__ out, int64_t ldo,
                                            int64_t N) {
  typedef typename real_of<Eout>::type T;
  const int64_t j = int64_t(blockIdx.x) * TPB + threadIdx.x;
  if (j >= N) return;
  for (int64_t i = blockIdx.y; i < N; i += gridDim.y) {
    const c128 v = U[i * ldu + j];
    double re = ph_re * v.re - ph_im * v.im;
    const double im = ph_re * v.im + ph_im * v.re;
    if (i == j) re -= 1.0;
    out[i * ldo + j] = Eout{T(re), T(im)};
  }
}

template <typename Ein, typename Eout>
int gather_impl(const Ein* src, int64_t lds, const int32_t* map, int64_t ro, int64_t co,
                int64_t rows, int64_t cols, double ph_re, double ph_im, bool sub, Eout* dst,
                int64_t ldd, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return TC_OK;
  const dim3 grid(unsigned((cols + TPB - 1) / TPB), unsigned(rows < 4096 ? rows : 4096));
  hipLaunchKernelGGL((gather_kernel<Ein, Eout>), grid, dim3(TPB), 0, s, src, lds, map, ro, co,
                     rows, cols, ph_re, ph_im, sub ? 1 : 0, dst, ldd);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

template <typename E>
int mirror_impl(E* rho, int64_t ld, int64_t N, const int32_t* sec, hipStream_t s) {
  if (N <= 1) return TC_OK;
  const int64_t T = (N + RT - 1) / RT;
  const int64_t np = T * (T + 1) / 2;
  hipLaunchKernelGGL(mirror_lower_kernel<E>, dim3(unsigned(np)), dim3(TPB), 0, s, rho, ld, N,
                     sec);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

template <typename Eout>
int phase_minus_identity_impl(const c128* U, int64_t ldu, double ph_re, double ph_im, Eout* out,
                              int64_t ldo, int64_t N, hipStream_t s) {
  if (N <= 0) return TC_OK;
  const dim3 grid(unsigned((N + TPB - 1) / TPB), unsigned(N < 4096 ? N : 4096));
  hipLaunchKernelGGL(phase_minus_identity_kernel<Eout>, grid, dim3(TPB), 0, s, U, ldu, ph_re,
                     ph_im, out, ldo, N);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

// ---- block-diagonal storage of padded sectors (the sector adjoint)
// Block k is D_k x D_k (row-major, ld D_k) at element offset boff[k];
// boff[nb] is the total.  Position p of the padded sorted order lies in the
// block whose spo[k] <= p < spo[k] + D_k; perm[p] is its basis state or -1.
__device__ __forceinline__ int block_of(const int64_t* __restrict__ off, int nb, int64_t e) {
  int lo = 0, hi = nb - 1;               // last k with off[k] <= e
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// what = 0: identity blocks; 1: diag(sum_i s_i^+ s_i^-) of the block's states
template <typename E>
__global__ void block_fill_kernel(BlockTable t, int what, int n, E* __restrict__ out) {
  typedef typename real_of<E>::type T;
  const int64_t total = t.boff[t.nb];
  const uint64_t mask = (uint64_t(1) << n) - 1;
  for (int64_t e = int64_t(blockIdx.x) * TPB + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * TPB) {
    const int k = block_of(t.boff, t.nb, e);
    const int64_t D = t.dim[k], r = e - t.boff[k], i = r / D, j = r % D;
    double v = 0.0;
    if (i == j) {
      if (what == 0) {
        v = 1.0;
      } else {
        const int32_t st = t.perm[t.spo[k] + i];
        v = st >= 0 ? double(__popcll(uint64_t(st) & mask)) : 0.0;
      }
    }
    out[e] = E{T(v), T(0)};
  }
}

// out = -i scale (H_k - (w_c k + mu) I) on every block (0 at padding)
__global__ void block_minus_i_shift_kernel(BlockTable t, const double* __restrict__ H, int64_t ldh,
                                           double omega_c, double mu, double scale,
                                           c128* __restrict__ out) {
  const int64_t total = t.boff[t.nb];
  for (int64_t e = int64_t(blockIdx.x) * TPB + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * TPB) {
    const int k = block_of(t.boff, t.nb, e);
    const int64_t D = t.dim[k], r = e - t.boff[k], i = r / D, j = r % D;
    const int32_t si = t.perm[t.spo[k] + i], sj = t.perm[t.spo[k] + j];
    double h = 0.0;
    if (si >= 0 && sj >= 0) {
      h = H[int64_t(si) * ldh + sj];
      if (i == j) h -= omega_c * double(k) + mu;
    }
    out[e] = c128{0.0, -scale * h};
  }
}

// full[s_i][s_j] = blocks (entries outside the blocks are left alone)
__global__ void block_scatter_kernel(BlockTable t, const c128* __restrict__ G,
                                     c128* __restrict__ full, int64_t ld) {
  const int64_t total = t.boff[t.nb];
  for (int64_t e = int64_t(blockIdx.x) * TPB + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * TPB) {
    const int k = block_of(t.boff, t.nb, e);
    const int64_t D = t.dim[k], r = e - t.boff[k], i = r / D, j = r % D;
    const int32_t si = t.perm[t.spo[k] + i], sj = t.perm[t.spo[k] + j];
    if (si >= 0 && sj >= 0) full[int64_t(si) * ld + sj] = G[e];
  }
}

// diag[p] = the diagonal element of position p
template <typename E>
__global__ void block_diag_kernel(BlockTable t, const E* __restrict__ blocks, int64_t Np,
                                  E* __restrict__ diag) {
  for (int64_t p = int64_t(blockIdx.x) * TPB + threadIdx.x; p < Np;
       p += int64_t(gridDim.x) * TPB) {
    const int k = block_of(t.spo, t.nb, p);
    const int64_t i = p - t.spo[k];
    diag[p] = blocks[t.boff[k] + i * (t.dim[k] + 1)];
  }
}

__global__ void scale_vec_kernel(c128* __restrict__ x, int64_t count, double a) {
  for (int64_t e = int64_t(blockIdx.x) * TPB + threadIdx.x; e < count;
       e += int64_t(gridDim.x) * TPB) {
    x[e].re *= a;
    x[e].im *= a;
  }
}

__global__ void accumulate_vec_kernel(const c64* __restrict__ t, c128* __restrict__ m,
                                      int64_t count) {
  for (int64_t e = int64_t(blockIdx.x) * TPB + threadIdx.x; e < count;
       e += int64_t(gridDim.x) * TPB) {
    m[e].re += double(t[e].re);
    m[e].im += double(t[e].im);
  }
}

unsigned grid1(int64_t count) {
  int64_t g = (count + TPB - 1) / TPB;
  return unsigned(g < 65536 ? (g > 0 ? g : 1) : 65536);
}

}  // namespace

int launch_block_fill_c128(const BlockTable& t, int64_t total, int what, int n, c128* out,
                           hipStream_t s) {
  if (total <= 0) return TC_OK;
  hipLaunchKernelGGL(block_fill_kernel<c128>, dim3(grid1(total)), dim3(TPB), 0, s, t, what, n, out);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}
int launch_block_fill_c64(const BlockTable& t, int64_t total, int what, int n, c64* out,
                          hipStream_t s) {
  if (total <= 0) return TC_OK;
  hipLaunchKernelGGL(block_fill_kernel<c64>, dim3(grid1(total)), dim3(TPB), 0, s, t, what, n, out);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}
int launch_block_minus_i_shift(const BlockTable& t, int64_t total, const double* H, int64_t ldh,
                               double omega_c, double mu, double scale, c128* out, hipStream_t s) {
  if (total <= 0) return TC_OK;
  hipLaunchKernelGGL(block_minus_i_shift_kernel, dim3(grid1(total)), dim3(TPB), 0, s, t, H, ldh,
                     omega_c, mu, scale, out);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}
int launch_block_scatter(const BlockTable& t, int64_t total, const c128* G, c128* full, int64_t ld,
                         hipStream_t s) {
  if (total <= 0) return TC_OK;
  hipLaunchKernelGGL(block_scatter_kernel, dim3(grid1(total)), dim3(TPB), 0, s, t, G, full, ld);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}
int launch_block_diag_c128(const BlockTable& t, const c128* blocks, int64_t Np, c128* diag,
                           hipStream_t s) {
  if (Np <= 0) return TC_OK;
  hipLaunchKernelGGL(block_diag_kernel<c128>, dim3(grid1(Np)), dim3(TPB), 0, s, t, blocks, Np, diag);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}
int launch_block_diag_c64(const BlockTable& t, const c64* blocks, int64_t Np, c64* diag,
                          hipStream_t s) {
  if (Np <= 0) return TC_OK;
  hipLaunchKernelGGL(block_diag_kernel<c64>, dim3(grid1(Np)), dim3(TPB), 0, s, t, blocks, Np, diag);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}
int launch_scale_vec_c128(c128* x, int64_t count, double a, hipStream_t s) {
  if (count <= 0) return TC_OK;
  hipLaunchKernelGGL(scale_vec_kernel, dim3(grid1(count)), dim3(TPB), 0, s, x, count, a);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}
int launch_accumulate_vec_c64(const c64* t, c128* m, int64_t count, hipStream_t s) {
  if (count <= 0) return TC_OK;
  hipLaunchKernelGGL(accumulate_vec_kernel, dim3(grid1(count)), dim3(TPB), 0, s, t, m, count);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_ham_sector(const ModelArgs& m, int k, int64_t d, double* H, int64_t ldh,
                      hipStream_t s) {
  if (d <= 0) return TC_OK;
  const dim3 grid(unsigned((d + TPB - 1) / TPB), unsigned(d < 4096 ? d : 4096));
  hipLaunchKernelGGL(ham_sector_kernel, grid, dim3(TPB), 0, s, m, k, d, H, ldh);
  TC_TRY_HIP(hipGetLastError());
  return TC_OK;
}

int launch_phase_minus_identity_c128(const c128* U, int64_t ldu, double ph_re, double ph_im,
                                     c128* out, int64_t ldo, int64_t N, hipStream_t s) {
  return phase_minus_identity_impl(U, ldu, ph_re, ph_im, out, ldo, N, s);
}
int launch_phase_minus_identity_c64(const c128* U, int64_t ldu, double ph_re, double ph_im,
                                    c64* out, int64_t ldo, int64_t N, hipStream_t s) {
  return phase_minus_identity_impl(U, ldu, ph_re, ph_im, out, ldo, N, s);
}

int launch_gather_c128_c128(const c128* src, int64_t lds, const int32_t* map, int64_t ro,
                            int64_t co, int64_t rows, int64_t cols, double ph_re, double ph_im,
                            bool sub_identity, c128* dst, int64_t ldd, hipStream_t s) {
  return gather_impl(src, lds, map, ro, co, rows, cols, ph_re, ph_im, sub_identity, dst, ldd, s);
}
int launch_gather_c128_c64(const c128* src, int64_t lds, const int32_t* map, int64_t ro,
                           int64_t co, int64_t rows, int64_t cols, double ph_re, double ph_im,
                           bool sub_identity, c64* dst, int64_t ldd, hipStream_t s) {
  return gather_impl(src, lds, map, ro, co, rows, cols, ph_re, ph_im, sub_identity, dst, ldd, s);
}
int launch_gather_c64_c64(const c64* src, int64_t lds, const int32_t* map, int64_t ro,
                          int64_t co, int64_t rows, int64_t cols, double ph_re, double ph_im,
                          bool sub_identity, c64* dst, int64_t ldd, hipStream_t s) {
  return gather_impl(src, lds, map, ro, co, rows, cols, ph_re, ph_im, sub_identity, dst, ldd, s);
}
int launch_gather_c64_c128(const c64* src, int64_t lds, const int32_t* map, int64_t ro,
                           int64_t co, int64_t rows, int64_t cols, double ph_re, double ph_im,
                           bool sub_identity, c128* dst, int64_t ldd, hipStream_t s) {
  return gather_impl(src, lds, map, ro, co, rows, cols, ph_re, ph_im, sub_identity, dst, ldd, s);
}

int launch_mirror_lower_c128(c128* rho, int64_t ld, int64_t N, const int32_t* sec,
                             hipStream_t s) {
  return mirror_impl(rho, ld, N, sec, s);
}
int launch_mirror_lower_c64(c64* rho, int64_t ld, int64_t N, const int32_t* sec, hipStream_t s) {
  return mirror_impl(rho, ld, N, sec, s);
}

}  // namespace tcm
