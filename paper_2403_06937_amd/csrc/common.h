// Internal definitions shared by the HIP sources of libtcm (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <string>

#include "../../include/tcm.h"

namespace tcm {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
void clear_error();

struct Status {
  int code = TC_OK;
  static Status ok() { return Status(); }
};

#define TC_TRY_HIP(expr)                                                       \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ::tcm::set_error(std::string("HIP error in ") + #expr + ": " +           \
                       hipGetErrorString(e_));                                 \
      return TC_ERR_HIP;                                                       \
    }                                                                          \
  } while (0)

#define TC_CHECK_ARG(cond, msg)                                                \
  do {                                                                         \
    if (!(cond)) {                                                             \
      ::tcm::set_error(std::string("invalid argument: ") + (msg));             \
      return TC_ERR_INVALID_ARGUMENT;                                          \
    }                                                                          \
  } while (0)

#define TC_RETURN_IF(err)                                                      \
  do {                                                                         \
    int r_ = (err);                                                            \
    if (r_ != TC_OK) return r_;                                                \
  } while (0)

// ------------------------------------------------------------ value types
template <typename T> struct cplx { T re, im; };
typedef cplx<double> c128;
typedef cplx<float> c64;

static_assert(sizeof(c128) == 16, "c128 layout");
static_assert(sizeof(c64) == 8, "c64 layout");

// Model parameters passed to kernels by value (n <= TC_MAX_ATOMS).
constexpr int TC_MAX_ATOMS = 24;
struct ModelArgs {
  int n;           // atoms
  int c;           // photon cutoff
  int64_t N;       // (c+1) 2^n
  double omega_c;
  double omega_a[TC_MAX_ATOMS];
  double g[TC_MAX_ATOMS];
  double kappa, gamma;   // dissipation rates of the Lindblad term (0: unitary)
};

int make_model_args(const tc_model* m, ModelArgs* out);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Simple bump allocator over a caller workspace.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  Arena(void* p, size_t n) : base(static_cast<char*>(p)), cap(n) {}
  // Sizing mode (base == nullptr): only accumulates.
  void* take(size_t bytes) {
    size_t off = align_up(used, 256);
    used = off + align_up(bytes, 256);
    return base ? base + off : nullptr;
  }
  bool fits() const { return used <= cap; }
};

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace tcm
