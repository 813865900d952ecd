"""Pins of the oracle's bfloat16 rounding / hi-lo split and its gradient routes."""
import math

import numpy as np
import pytest
import torch

import tcm_inputs as ti
from oracle import bf16, gradient, model


def _torch_rne_bits(x):
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16)


def test_rne_matches_library_conversion():
    """Round-to-nearest-even to bfloat16 equals torch's float32->bfloat16 cast
    on random values and on exact ties / carries / extremes."""
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(200000) * np.exp(rng.uniform(-60, 60, 200000))).astype(np.float32)
    ties = np.array([0x3F808000, 0x3F818000, 0x3F80FFFF, 0x3F7FFFFF, 0x7F7FFFFF,
                     0x00008000, 0x00018000, 0x80008000, 0x3F800001, 0x7F7F8000],
                    dtype=np.uint32).view(np.float32)
    x = np.concatenate([x, ties, np.array([0.0, -0.0, 1.0, -3.5, 1e-40, np.inf, -np.inf], np.float32)])
    assert np.array_equal(bf16.rne_bits(x), _torch_rne_bits(x))


def test_split_reconstruction_bound():
    """hi + lo reproduces x to within 2^-16 |x| (hi keeps 8 significant bits,
    lo the next 8, with one rounding each)."""
    rng = np.random.default_rng(2)
    x = (rng.standard_normal(100000) * np.exp(rng.uniform(-20, 20, 100000))).astype(np.float32)
    v = bf16.split_value(x)
    assert np.all(np.abs(v - x.astype(np.float64)) <= 2.0 ** -16 * np.abs(x.astype(np.float64)))
    hi, lo = bf16.split(x)
    # hi alone is only 8-bit accurate
    assert np.max(np.abs(bf16.bits_to_float(hi) - x) / np.abs(x)) > 2.0 ** -10


def test_grad_jc_closed_form():
    """n=1, resonant, psi0 = |0>|e>: L(T) = cos^2(g T) so dL/dg = -T sin(2 g T);
    dL/ddelta = 0 at delta = 0 (L is even in delta)."""
    g, T, c = 0.017, 37.0, 2
    psi0 = ti.basis_state(1, c, 0, [1])
    rho0 = np.outer(psi0, psi0)
    L, gg, gd = gradient.grad_daleckii_krein(1, c, [g], [0.0], rho0, T)
    assert abs(L - math.cos(g * T) ** 2) < 1e-13
    assert abs(gg[0] - (-T * math.sin(2 * g * T))) < 1e-11
    assert abs(gd[0]) < 1e-12


def test_grad_jc_detuned_closed_form():
    """n=1 detuned: L = 1 - (4 g^2 / W^2) sin^2(W T / 2), W^2 = D^2 + 4 g^2.
    The closed form is differentiated by central differences of the formula
    itself (no Hamiltonian involved)."""
    g, D, T, c = 0.013, 0.021, 25.0, 1
    psi0 = ti.basis_state(1, c, 0, [1])

    def closed(g, D):
        W = math.sqrt(D * D + 4 * g * g)
        return 1 - (4 * g * g / (W * W)) * math.sin(W * T / 2) ** 2

    L, gg, gd = gradient.grad_daleckii_krein(1, c, [g], [D], np.outer(psi0, psi0), T)
    h = 1e-6
    assert abs(L - closed(g, D)) < 1e-13
    assert abs(gg[0] - (closed(g + h, D) - closed(g - h, D)) / (2 * h)) < 1e-7
    assert abs(gd[0] - (closed(g, D + h) - closed(g, D - h)) / (2 * h)) < 1e-7


@pytest.mark.parametrize("state", ["excited", "gaussian"])
def test_grad_dk_matches_fd(state):
    n, c = 3, 3
    inst = ti.random_model(n, c, 41, delta_sigma=0.01, state=state)
    delta = inst.omega_a - 1
    rho0 = inst.rho0()
    T = 40 * 0.5
    L, gg, gd = gradient.grad_daleckii_krein(n, c, inst.g, delta, rho0, T)
    fg, fd = gradient.grad_fd(n, c, inst.g, delta, rho0, T)
    scale = max(np.max(np.abs(gg)), np.max(np.abs(gd)))
    assert np.max(np.abs(gg - fg)) < 1e-6 * scale
    assert np.max(np.abs(gd - fd)) < 1e-6 * scale
    # the sector restriction is exact
    L2, gg2, gd2 = gradient.grad_daleckii_krein(n, c, inst.g, delta, rho0, T, restrict=False)
    assert abs(L - L2) < 1e-13
    assert np.max(np.abs(gg - gg2)) < 1e-11 and np.max(np.abs(gd - gd2)) < 1e-11


def test_grad_symmetries():
    """delta = 0 and a basis-state start: populations are even in delta, so every
    dL/ddelta_i vanishes; equal g: all dL/dg_i are equal (atoms interchangeable)."""
    n, c = 3, 3
    psi0 = ti.basis_state(n, c, 0, [1] * n)
    rho0 = np.outer(psi0, psi0)
    _, gg, gd = gradient.grad_daleckii_krein(n, c, [0.01] * n, [0.0] * n, rho0, 60.0)
    assert np.max(np.abs(gd)) < 1e-12
    assert np.max(gg) - np.min(gg) < 1e-11
    assert np.max(np.abs(gg)) > 1.0
