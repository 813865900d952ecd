"""The usual call sequence of the C ABI on torch device tensors.

  build H (tc_build_hamiltonian) -> bounds (tc_spectral_bounds) -> U (tc_expm)
  -> time steps (tc_evolve) -> readout (tc_observables)

Each function only allocates device tensors and calls the library; no
arithmetic of the method happens here.
"""
from __future__ import annotations

import torch

from . import (Model, TC_C128, TC_C64, TC_EXPM_SS_TAYLOR, TC_FRAME_LAB, TC_GEMM_F64,
               make_instance, make_opts, tc_build_hamiltonian, tc_build_sector_hamiltonian,
               tc_evolve, tc_evolve_sector, tc_expm, tc_observables, tc_sector_dim,
               tc_sector_spectral_bounds, tc_spectral_bounds)


def model_of(inst) -> Model:
    """Model from an object with n, c, g, omega_a (and optionally omega_c, kappa,
    gamma) attributes."""
    return Model(int(inst.n), int(inst.c), list(map(float, inst.g)),
                 list(map(float, inst.omega_a)), float(getattr(inst, "omega_c", 1.0)),
                 float(getattr(inst, "kappa", 0.0)), float(getattr(inst, "gamma", 0.0)))


def hamiltonian(model: Model, device="cuda") -> torch.Tensor:
    N = model.N
    H = torch.empty((N, N), dtype=torch.float64, device=device)
    tc_build_hamiltonian(model, H)
    return H


def propagator(model: Model, dt: float, method: int = TC_EXPM_SS_TAYLOR, device="cuda",
               H: torch.Tensor = None):
    """(H, U) with U = exp(-i H dt) formed on the device."""
    if H is None:
        H = hamiltonian(model, device)
    lo, hi = tc_spectral_bounds(model)
    U = torch.empty((model.N, model.N), dtype=torch.complex128, device=device)
    tc_expm(H, dt, lo, hi, U, method)
    return H, U


def evolve(model: Model, U: torch.Tensor, rho: torch.Tensor, steps: int, dt: float,
           gemm_mode: int = TC_GEMM_F64, frame: int = TC_FRAME_LAB, renorm_every: int = 0,
           record_every: int = 1, checkpoint_every: int = 0, record_photons: bool = False,
           ws=None, full_product: bool = False, sectors: bool = False,
           record_states: bool = False, use_graph: bool = False, no_resident: bool = False):
    """Steps rho (device, complex128 or complex64) in place; returns the records
    (pop [R], photon distribution [R, c+1] or None, checkpoints or None), and
    with record_states also the Eq. (13) records [R, min(n, c)+1] as a fourth."""
    rho_dtype = TC_C128 if rho.dtype == torch.complex128 else TC_C64
    R = steps // record_every + 1 if record_every else 0
    pop = torch.zeros(R, dtype=torch.float64, device=rho.device) if R else None
    pd = (torch.zeros((R, model.c + 1), dtype=torch.float64, device=rho.device)
          if (R and record_photons) else None)
    ps = (torch.zeros((R, min(model.n, model.c) + 1), dtype=torch.float64, device=rho.device)
          if (R and record_states) else None)
    ck = None
    if checkpoint_every:
        ck = torch.empty((steps // checkpoint_every + 1, model.N, model.N), dtype=rho.dtype,
                         device=rho.device)
    opts = make_opts(steps, dt, gemm_mode, rho_dtype, frame, renorm_every,
                     record_every if record_every else 0, checkpoint_every,
                     use_graph=int(use_graph), full_product=int(full_product),
                     sectors=int(sectors), no_resident=int(no_resident))
    inst = make_instance(model, U, rho, pop, pd, ck, ps)
    tc_evolve([inst], opts, ws=ws, device=rho.device)
    if record_states:
        return pop, pd, ck, ps
    return pop, pd, ck


def sector_hamiltonian(model: Model, k: int, device="cuda") -> torch.Tensor:
    """The d_k x d_k block of Eq. (4) on excitation sector k (the paper's 2^n
    model for c >= n, k = n)."""
    d = tc_sector_dim(model, k)
    H = torch.empty((d, d), dtype=torch.float64, device=device)
    tc_build_sector_hamiltonian(model, k, H)
    return H


def sector_propagator(model: Model, k: int, dt: float, method: int = TC_EXPM_SS_TAYLOR,
                      device="cuda", H: torch.Tensor = None):
    """(H_k, U_k) with U_k = exp(-i H_k dt) (or Eq. (10)'s series) on the device."""
    if H is None:
        H = sector_hamiltonian(model, k, device)
    lo, hi = tc_sector_spectral_bounds(model, k)
    U = torch.empty(H.shape, dtype=torch.complex128, device=device)
    tc_expm(H, dt, lo, hi, U, method)
    return H, U


def evolve_sector(model: Model, k: int, U: torch.Tensor, rho: torch.Tensor, steps: int,
                  dt: float, gemm_mode: int = TC_GEMM_F64, frame: int = TC_FRAME_LAB,
                  renorm_every: int = 0, record_every: int = 1, checkpoint_every: int = 0,
                  record_photons: bool = False, ws=None, full_product: bool = False):
    """Steps the d_k x d_k block rho of sector k in place; returns the records
    as evolve() does."""
    rho_dtype = TC_C128 if rho.dtype == torch.complex128 else TC_C64
    R = steps // record_every + 1 if record_every else 0
    pop = torch.zeros(R, dtype=torch.float64, device=rho.device) if R else None
    pd = (torch.zeros((R, model.c + 1), dtype=torch.float64, device=rho.device)
          if (R and record_photons) else None)
    ck = None
    if checkpoint_every:
        ck = torch.empty((steps // checkpoint_every + 1,) + tuple(rho.shape), dtype=rho.dtype,
                         device=rho.device)
    opts = make_opts(steps, dt, gemm_mode, rho_dtype, frame, renorm_every,
                     record_every if record_every else 0, checkpoint_every,
                     full_product=int(full_product))
    inst = make_instance(model, U, rho, pop, pd, ck)
    inst.N = rho.shape[0]
    tc_evolve_sector(inst, k, opts, ws=ws, device=rho.device)
    return pop, pd, ck


def observables(model: Model, rho: torch.Tensor) -> dict:
    s = torch.zeros(8, dtype=torch.float64, device=rho.device)
    ap = torch.zeros(model.n, dtype=torch.float64, device=rho.device)
    pd = torch.zeros(model.c + 1, dtype=torch.float64, device=rho.device)
    ed = torch.zeros(model.n + model.c + 1, dtype=torch.float64, device=rho.device)
    ns = min(model.n, model.c) + 1
    ps = torch.zeros(ns, dtype=torch.float64, device=rho.device)
    dk = torch.zeros(ns, dtype=torch.float64, device=rho.device)
    tc_observables(model, rho, s, ap, pd, ed, ps, dk)
    v = s.cpu().numpy()
    return {"trace_re": v[0], "trace_im": v[1], "purity": v[2], "herm_err": v[3],
            "excitation_total": v[4], "photon_mean": v[5], "excitation_mean": v[6],
            "nonfinite": v[7], "atom_pop": ap.cpu().numpy(), "photon_dist": pd.cpu().numpy(),
            "exc_dist": ed.cpu().numpy(), "photon_state": ps.cpu().numpy(),
            "dicke": dk.cpu().numpy()}
