// tc_observables_noalloc: tc_observables for callers that cannot allocate
// device memory (code under graph capture, tight serving loops).  Its kernels
// take their partial sums from one file-scope device array instead of a
// caller workspace; each GPU the library runs on holds its own copy of the
// array until the process ends.
#include <mutex>
#include <string>

#include "kernels.h"

namespace tcm {
namespace {

// Partial sums of the observables' reductions: 16 MiB, enough for every N up
// to 37 120 (3 per 32 x 32 tile pair, the diagonal, Im Tr and the Dicke pass).
constexpr size_t SCRATCH_BYTES = size_t(16) << 20;
static __device__ __align__(256) double scratch[SCRATCH_BYTES / sizeof(double)];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};   // device address of scratch, per device (nullptr: not yet)

// The address of this device's copy of scratch, looked up once per device
// with that device current.  The array's host-side name is not a device
// address; only this pointer may be passed to kernels.
int scratch_address(void** out) {
  int dev = 0;
  TC_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) {
    set_error("tc_observables_noalloc: device id beyond the library's table");
    return TC_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    TC_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("hipGetSymbolAddress returned a null address for the scratch array");
      return TC_ERR_HIP;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return TC_OK;
}

}  // namespace
}  // namespace tcm

using namespace tcm;

extern "C" {

int tc_observables_noalloc_max_dim(int64_t* N) {
  clear_error();
  TC_CHECK_ARG(N != nullptr, "N is NULL");
  int64_t lo = 0, hi = int64_t(1) << 20;
  while (lo < hi) {                          // largest N whose partials fit
    const int64_t mid = (lo + hi + 1) / 2;
    if (observables_partials_count(mid) * sizeof(double) <= SCRATCH_BYTES) lo = mid;
    else hi = mid - 1;
  }
  *N = lo;
  return TC_OK;
}

int tc_observables_noalloc(const tc_model* m, const void* rho, int32_t rho_dtype, int64_t N,
                           int64_t ldr, double* scalars, double* atom_pop, double* photon_dist,
                           double* exc_dist, double* photon_state, double* dicke,
                           void* stream) {
  clear_error();
  ModelArgs a;
  TC_RETURN_IF(make_model_args(m, &a));
  TC_CHECK_ARG(N == a.N, "N != (c+1) 2^n");
  TC_CHECK_ARG(rho != nullptr && scalars != nullptr, "rho / scalars is NULL");
  TC_CHECK_ARG(rho_dtype == TC_C64 || rho_dtype == TC_C128, "unknown rho_dtype");
  TC_CHECK_ARG(ldr >= N, "ldr < N");
  const size_t need = observables_partials_count(N) * sizeof(double);
  if (need > SCRATCH_BYTES) {
    set_error("tc_observables_noalloc: N = " + std::to_string(N) + " needs " +
              std::to_string(need) + " bytes of partial sums, more than its " +
              std::to_string(SCRATCH_BYTES) + "-byte device array; use tc_observables");
    return TC_ERR_UNSUPPORTED;
  }
  void* ws = nullptr;
  TC_RETURN_IF(scratch_address(&ws));
  return launch_observables(a, rho, rho_dtype, ldr, static_cast<double*>(ws), scalars, atom_pop,
                            photon_dist, exc_dist, photon_state, dicke, as_stream(stream));
}

}  // extern "C"
