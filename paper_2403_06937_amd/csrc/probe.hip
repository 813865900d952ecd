// MFMA issue-rate probe: a diagnostic for reading the product kernels'
// rooflines, not a step of the method.  Every wave of one 512-thread
// workgroup per compute unit issues MFMAs of one kind back to back on
// operands held in registers (no memory traffic inside the loop), so the
// elapsed time is the rate at which the chip sustains that instruction on
// those operand bits.  The datasheet peaks assume the full clock; with
// random operands the BF16 MFMA draws enough power that the chip holds a
// lower clock, which bounds every BF16 product kernel from above.
#include "kernels.h"

namespace tcm {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

constexpr int PTPB = 512;

// Operand bits from a linear congruential sequence seeded by the thread
// index; the mask keeps every bf16 exponent below the top of the range, so
// the values are finite.  random == 0 gives zero operands.
__device__ void operand_bits(u4 (&a)[4], u4 (&b)[4], uint32_t t, int random) {
  uint32_t x = 0x9E3779B9u ^ (t * 2654435761u);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x = x * 1664525u + 1013904223u;
      a[i][k] = random ? (x & 0x3FFF3FFFu) : 0u;
      x = x * 1664525u + 1013904223u;
      b[i][k] = random ? (x & 0x3FFF3FFFu) : 0u;
    }
  }
}

__global__ void __launch_bounds__(PTPB) probe_bf16_16(float* out, int iters, int random) {
  const uint32_t t = threadIdx.x + blockIdx.x * PTPB;
  u4 a[4], b[4];
  operand_bits(a, b, t, random);
  f4 acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = f4{0, 0, 0, 0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 16; ++i)
      acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a[i & 3]),
                                                       __builtin_bit_cast(bf8, b[i >> 2]), acc[i],
                                                       0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[t] = s;
}

__global__ void __launch_bounds__(PTPB) probe_bf16_32(float* out, int iters, int random) {
  const uint32_t t = threadIdx.x + blockIdx.x * PTPB;
  u4 a[4], b[4];
  operand_bits(a, b, t, random);
  f16v acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            __builtin_bit_cast(bf8, a[(i + q) & 3]), __builtin_bit_cast(bf8, b[(i >> 1) + 2 * q]),
            acc[i], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += acc[i][r];
  out[t] = s;
}

__global__ void __launch_bounds__(PTPB) probe_f64(float* out, int iters, int random) {
  const uint32_t t = threadIdx.x + blockIdx.x * PTPB;
  double a[4], b[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    a[i] = random ? 1.0 + 1e-3 * double((t + i) % 97) : 0.0;
    b[i] = random ? 0.5 - 1e-3 * double((t * 3 + i) % 89) : 0.0;
  }
  d4 acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = d4{0, 0, 0, 0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
      acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i & 3], b[(i >> 1) & 3], acc[i], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[t] = float(s);
}

}  // namespace
}  // namespace tcm

using namespace tcm;

extern "C" int tc_mfma_probe(int32_t kind, int32_t random_operands, int32_t iters, float* out,
                             int64_t out_count, double* ms, double* flop, void* stream) {
  clear_error();
  TC_CHECK_ARG(kind == TC_PROBE_BF16_16X16X32 || kind == TC_PROBE_BF16_32X32X16 ||
                   kind == TC_PROBE_F64_16X16X4,
               "unknown probe kind");
  TC_CHECK_ARG(iters >= 1 && iters <= 10000000, "iters outside 1 .. 1e7");
  TC_CHECK_ARG(out != nullptr && ms != nullptr && flop != nullptr, "NULL argument");
  int dev = 0, cus = 0;
  TC_TRY_HIP(hipGetDevice(&dev));
  TC_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  TC_CHECK_ARG(cus > 0, "the device reports no compute units");
  TC_CHECK_ARG(out_count >= int64_t(cus) * PTPB, "out holds fewer than 512 x CUs floats");
  hipStream_t s = as_stream(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TC_TRY_HIP(hipEventCreate(&e0));
  hipError_t err = hipEventCreate(&e1);
  if (err != hipSuccess) {
    (void)hipEventDestroy(e0);
    TC_TRY_HIP(err);
  }
  double per_wave_iter = 0.0;   // flops per wave and loop iteration
  err = hipEventRecord(e0, s);
  if (err == hipSuccess) {
    if (kind == TC_PROBE_BF16_16X16X32) {
      hipLaunchKernelGGL(probe_bf16_16, dim3(cus), dim3(PTPB), 0, s, out, iters, random_operands);
      per_wave_iter = 16.0 * 16 * 16 * 32 * 2;
    } else if (kind == TC_PROBE_BF16_32X32X16) {
      hipLaunchKernelGGL(probe_bf16_32, dim3(cus), dim3(PTPB), 0, s, out, iters, random_operands);
      per_wave_iter = 8.0 * 32 * 32 * 16 * 2;
    } else {
      hipLaunchKernelGGL(probe_f64, dim3(cus), dim3(PTPB), 0, s, out, iters, random_operands);
      per_wave_iter = 8.0 * 16 * 16 * 4 * 2;
    }
    err = hipGetLastError();
  }
  if (err == hipSuccess) err = hipEventRecord(e1, s);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float t = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  TC_TRY_HIP(err);
  *ms = double(t);
  *flop = per_wave_iter * double(iters) * double(cus) * (PTPB / 64);
  return TC_OK;
}
