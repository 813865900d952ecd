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

}  // namespace

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
