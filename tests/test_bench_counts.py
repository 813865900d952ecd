"""The work counts behind the reported TFLOP/s (bench.py) against brute-force
enumeration on small models: sector sizes from the oracle's excitation
labels, the sector-block products' multiply-adds counted element by element,
the padded sector work, and the dense step's tiles (the second product on
the upper tile triangle of its Hermitian result)."""
import itertools

import numpy as np
import pytest

import bench
from oracle import model as omodel


def _sector_labels(n, c):
    secs = omodel.sectors(n, c)
    lab = np.empty(sum(v.size for v in secs.values()), dtype=int)
    for k, idx in secs.items():
        lab[idx] = k
    return lab


@pytest.mark.parametrize("n,c", [(1, 1), (2, 3), (3, 2), (4, 1), (3, 0), (2, 5)])
def test_sector_flops_by_enumeration(n, c):
    """X_{k,k:} = U_k rho_{k,k:} and rho'_{:k,k} = X_{:k,k} U_k^dag: one complex
    multiply-add (8 flop) per (i, l, j) with i, l in sector k and j in a sector
    >= k (first product), or j in sector k, l in sector k and i in a sector
    <= k (second)."""
    lab = _sector_labels(n, c)
    N = lab.size
    macs = 0
    for i, l, j in itertools.product(range(N), repeat=3):
        if lab[i] == lab[l] and lab[j] >= lab[i]:
            macs += 1                                   # first product, row i
        if lab[j] == lab[l] and lab[i] <= lab[j]:
            macs += 1                                   # second product, column j
    assert bench.sector_flop_per_step(n, c) == 8.0 * macs


@pytest.mark.parametrize("n,c,q", [(3, 2, 4), (4, 1, 8), (2, 3, 3)])
def test_sector_executed_flops_padding(n, c, q):
    """Executed work: the same enumeration over sectors padded to multiples of q."""
    secs = omodel.sectors(n, c)
    D = [-(-secs[k].size // q) * q for k in sorted(secs)]
    lab = np.repeat(np.arange(len(D)), D)               # padded sorted order
    Np = lab.size
    macs = 0
    for k, Dk in enumerate(D):
        rows = np.sum(lab == k)
        # first product: Dk x Dk x (columns of sectors >= k); second: (rows of
        # sectors <= k) x Dk x Dk
        macs += rows * Dk * np.sum(lab >= k) + np.sum(lab <= k) * Dk * Dk
    assert np.sum(D) == Np
    assert bench.sector_executed_flop_per_step(n, c, q) == 8.0 * macs


@pytest.mark.parametrize("T", [1, 2, 5, 96])
def test_dense_executed_flops_triangle(T):
    """Second product on the tiles (tm, tn) with tm <= tn of a T x T grid."""
    N = T * bench.TILE
    tiles = sum(1 for tm in range(T) for tn in range(T) if tm <= tn)
    full = 8.0 * N ** 3
    assert bench.executed_flop_per_step(N) == pytest.approx(full * (1 + tiles / T ** 2), rel=1e-15)
    assert bench.executed_flop_per_step(N, full=True) == 2 * full
