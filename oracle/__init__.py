"""CPU oracle for the Tavis-Cummings density-matrix stepper (test infrastructure).

This package is a plain, slow, FP64 reference of what the GPU library
computes, written from the paper (Miao & Ozhigov, "Distributed computing
quantum unitary evolution", arXiv 2403.06937).  It exists only to check the
GPU path: only the test suite, the smoke check and the benchmark's CPU
baseline may import it.  It shares no code with the GPU library and never
imports it; both read their inputs from the separate ``tcm_inputs`` module.

Modules
  model        Hamiltonian of Eq. (4) from Kronecker products of the operators
  evolve       exact propagator (Hermitian eigendecomposition), dense stepping
               of Eq. (6), the excitation-sector route, brute-force state vector,
               and the truncated Taylor factors of Eq. (10)-(11)
  observables  populations and the photon-number readout of Eq. (13),
               trace / purity / Hermiticity invariants
  renorm       Hermitisation and trace renormalisation of rho
  bf16         round-to-nearest-even bfloat16 and the hi/lo split
  gradient     d(final excitation)/d(g_i, delta_i) by the Daleckii-Krein
               formula and by central finite differences
  linalg       plain matrix-product definitions used for kernel-level checks
  open_system  the Lindblad term of Eq. (5) restored: Liouvillian, exact
               damping channels, and the split step rho <- exp(dt L)(U rho U^dag)
"""
