// Entry (row, col) of the Tavis-Cummings Hamiltonian of Eq. (4) in the
// photon-major basis |m>|l_1 .. l_n> (index m 2^n + l, atom i on bit n - 1 - i,
// photon cutoff c): the diagonal w_c m + sum_i w_a,i l_i, the coupling
// g_i sqrt(m + 1) between (m, l) with l_i = 1 and (m + 1, l - e_i), else 0.
#pragma once
#include "common.h"

namespace tcm {

__device__ __forceinline__ double ham_entry(const ModelArgs& m, int64_t row, int64_t col) {
  const int n = m.n;
  const uint64_t mask = (uint64_t(1) << n) - 1;
  const int64_t mr = row >> n, mc = col >> n;
  const uint64_t lr = uint64_t(row) & mask, lc = uint64_t(col) & mask;
  double v = 0.0;
  if (row == col) {
    v = m.omega_c * double(mr);
    for (int i = 0; i < n; ++i)
      if ((lr >> (n - 1 - i)) & 1) v += m.omega_a[i];
  } else if (mr - mc == 1 || mc - mr == 1) {
    // the state with fewer photons carries the one extra excited atom
    const uint64_t llo = mr < mc ? lr : lc, lhi = mr < mc ? lc : lr;
    const int64_t mhi = mr < mc ? mc : mr;
    const uint64_t x = llo ^ lhi;
    if (x != 0 && (x & (x - 1)) == 0 && (llo & x) != 0) {
      const int bit = __ffsll((unsigned long long)x) - 1;
      v = m.g[n - 1 - bit] * sqrt(double(mhi));
    }
  }
  return v;
}

}  // namespace tcm
