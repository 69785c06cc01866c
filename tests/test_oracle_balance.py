"""Pins for the oracle's workload rebalancing (Sec. 6), independent of its code:

* a uniform histogram over M = k P blocks splits into P equal ranges;
* each processor's workload is below total / P + max W (the CDF map puts at
  most one block across each slice boundary), and on tiny inputs the largest
  workload is within max W of the best contiguous split found by brute force;
* the paper's picture: with a coverage gradient the busy cells are spread
  over more processors (fewer cells each) than the idle ones;
* with a capacity, ranges never exceed it, still tile the blocks, equal the
  unconstrained map whenever that already respects the capacity, and pack an
  idle stretch at full capacity;
* a histogram without mass splits as a uniform one.
"""
import itertools

import numpy as np
import pytest

from oracle import balance


def _check_tiling(b, M, P):
    assert b[0] == 0 and b[-1] == M and len(b) == P + 1
    assert all(x <= y for x, y in zip(b, b[1:]))


@pytest.mark.parametrize("M,P", [(64, 8), (4096, 2048), (12, 3), (5, 5)])
def test_uniform_histogram_equal_ranges(M, P):
    b = balance.cdf_partition([7] * M, P)
    assert b == [l * M // P for l in range(P + 1)]


def test_mass_bound_and_brute_force():
    rng = np.random.default_rng(3)
    for _ in range(300):
        M = int(rng.integers(1, 9))
        P = int(rng.integers(1, 5))
        W = [int(x) for x in rng.integers(0, 20, size=M)]
        if rng.random() < 0.2:
            W[int(rng.integers(0, M))] += 100  # a spike
        b = balance.cdf_partition(W, P)
        _check_tiling(b, M, P)
        masses = balance.part_masses(W, b)
        total, wmax = sum(W), max(W)
        if total > 0:
            assert max(masses) * P < total + P * wmax or max(masses) * P == total
        best = None
        for cuts in itertools.combinations_with_replacement(range(M + 1), P - 1):
            bb = [0, *cuts, M]
            m = max(balance.part_masses(W, bb))
            best = m if best is None else min(best, m)
        assert best <= max(masses) <= best + wmax


def test_gradient_spreads_busy_cells():
    """1D adsorption strip with coverage growing along it: jumps are frequent
    where coverage is low, so the low-coverage end gets small ranges."""
    M, P = 256, 16
    W = [int(1000 * (1.0 - m / M)) + 1 for m in range(M)]
    b = balance.cdf_partition(W, P)
    sizes = [y - x for x, y in zip(b, b[1:])]
    assert sizes[0] < sizes[-1]
    assert all(s1 <= s2 + 1 for s1, s2 in zip(sizes, sizes[1:]))
    masses = balance.part_masses(W, b)
    assert max(masses) - min(masses) <= 2 * max(W)


def test_capacity_respected_and_neutral_when_slack():
    rng = np.random.default_rng(5)
    for _ in range(300):
        P = int(rng.integers(1, 40))
        cap = int(rng.integers(1, 9))
        M = int(rng.integers(1, P * cap + 1))
        W = [int(x) for x in rng.integers(0, 50, size=M)]
        if rng.random() < 0.5:  # an idle half, as in a half-filled lattice
            W = [0] * (M // 2) + W[M // 2:]
        b = balance.cdf_partition(W, P, cap)
        _check_tiling(b, M, P)
        assert all(0 <= y - x <= cap for x, y in zip(b, b[1:]))
        free = balance.cdf_partition(W, P)
        if all(y - x <= cap for x, y in zip(free, free[1:])):
            assert b == free


def test_capacity_packs_idle_stretch():
    """Half the blocks idle (cost 1), half busy (cost 100), 4 processors per
    8 blocks of capacity 4: the idle half is packed 4 per processor and the
    busy half gets the remaining processors."""
    W = [1] * 64 + [100] * 64
    b = balance.cdf_partition(W, 32, 8)
    sizes = [y - x for x, y in zip(b, b[1:])]
    idle = [s for s, x in zip(sizes, b) if x < 64]
    assert max(sizes) <= 8 and all(s == 8 for s in idle[:-1])
    assert len(idle) <= 9


def test_no_mass_is_uniform_and_errors():
    assert balance.cdf_partition([0] * 12, 4) == [0, 3, 6, 9, 12]
    with pytest.raises(ValueError):
        balance.cdf_partition([1] * 10, 2, cap=4)  # 10 blocks do not fit 2 x 4
    with pytest.raises(ValueError):
        balance.cdf_partition([1, -1], 1)


def test_block_costs():
    assert balance.block_costs([5, 0, 2], [0, 1, 0], [13, 12], 3) == [44, 36, 41]
