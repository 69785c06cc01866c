"""Workload histogram and mass-transport rebalancing (Sec. 6) -- TEST
INFRASTRUCTURE ONLY: the oracle of the library's workload partition.

The workload W(m) of block m over a period is the number of jumps the block
made in it (Sec. 6, eq. wload); normalised it is a histogram over the blocks.
Rebalancing maps the mass of the cumulative distribution of W onto equal
masses of the uniform distribution over P processors (Sec. 6): processor l
(l = 1..P) receives the blocks, taken in their given order, whose cumulative
workload lies in the l-th of P equal slices of the total.  Written out on
integers: with C(k) = W(0) + ... + W(k-1), boundary l is the smallest k with
P * C(k) >= l * total, and processor l owns blocks [boundary l-1, boundary l).
A histogram with no mass is treated as uniform.

A processor of the GPU library (a resident wave) holds at most `cap` blocks,
and a boundary must leave the remaining processors able to cover the rest:
when `cap` is given, boundary l is clamped into
[max(b_{l-1}, M - (P-l) cap), min(b_{l-1} + cap, M)], taken in order.  The
capacity clamp, and the block cost the library feeds in (jumps plus a fixed
cost per block and window, `block_costs`), are the library's additions to
the paper's map.
"""
import os

# test hook: a planted mistake for tests/test_oracle_plants.py
_PLANT = int(os.environ.get("FSKMC_ORACLE_PLANT", "0"))


def cdf_partition(W, P, cap=None):
    """Boundaries b_0 = 0 <= b_1 <= ... <= b_P = M of the CDF map of W onto
    P processors; processor l owns blocks [b_{l-1}, b_l)."""
    W = [int(w) for w in W]
    M = len(W)
    if P < 1 or any(w < 0 for w in W):
        raise ValueError("need P >= 1 and non-negative workloads")
    if cap is not None and (cap < 1 or M > P * cap):
        raise ValueError("the blocks do not fit P processors of capacity cap")
    weights = W if sum(W) > 0 else [1] * M
    total = sum(weights)
    bounds = [0]
    cum, k = 0, 0
    for l in range(1, P):
        # quantile: smallest k with P * C(k) >= l * total
        while k < M and (cum * P <= l * total if _PLANT == 11 else cum * P < l * total):
            cum += weights[k]
            k += 1
        b = k
        if cap is not None:
            prev = bounds[-1]
            lo = max(prev, M - (P - l) * cap)
            hi = min(prev + cap, M)
            b = min(max(b, lo), hi)
        bounds.append(b)
    bounds.append(M)
    return bounds


def block_costs(W, colours, active, base):
    """The library's block cost for rebalancing: jumps of block m plus `base`
    for every window its colour took part in (active[c] windows of colour c)."""
    return [int(w) + base * int(active[int(c)]) for w, c in zip(W, colours)]


def part_masses(W, bounds):
    """Workload of each processor's range."""
    return [sum(int(w) for w in W[bounds[l]:bounds[l + 1]]) for l in range(len(bounds) - 1)]
