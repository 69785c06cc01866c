"""Nested (hierarchical) fractional-step decomposition (Sec. 5, eqs. sublatt2
and opdecomp2) -- TEST INFRASTRUCTURE ONLY: the oracle of the library's
nested schedule and colour map.

Two levels of sub-lattices.  Coarse cells C_m, each made of cx x cy fine
blocks, carry the outer colouring of the lattice (eq. sublatt), which splits
the generator into one operator per outer colour (eq. opdecomp).  Inside every
coarse cell the fine blocks D_ml carry an inner colouring (eq. sublatt2), and
each coarse-cell operator splits again over the inner colours (eq. opdecomp2).
A splitting scheme (Lie or Strang) applied at both levels replaces every outer
factor exp(d L^c) by the inner scheme of step dtau over the inner colours of
the coarse cells of colour c.

The coarse cells of one outer colour are independent, so the nested scheme is
the flat fractional-step scheme on the product colour c_outer * k_inner +
c_inner, with the window list below; the blockwise oracle `fs_run` runs it
unchanged.  Both the outer list and every inner list come from the oracle's
own flat `schedule`.  The random schedule is not nested here.
"""
import os

import numpy as np

# test hook: a planted mistake for tests/test_oracle_plants.py
_PLANT = int(os.environ.get("FSKMC_ORACLE_PLANT", "0"))


def _builtin(k, i, j):
    """The built-in colourings of a grid: 1 colour; 2 colours (i+j)%2; 4 colours (i%2)+2(j%2)."""
    if k == 1:
        return 0
    if k == 2:
        return (i + j) % 2
    if k == 4:
        return (i % 2) + 2 * (j % 2)
    raise ValueError(f"no built-in colouring with {k} colours")


def nested_colour_map(Lx, Ly, bx, by, cx, cy, k_outer, k_inner):
    """Flat colour of every fine block (row-major block index bj*NBX + bi):
    outer colour of its coarse cell (bi//cx, bj//cy) times k_inner plus the
    inner colour of its position (bi%cx, bj%cy) inside the cell."""
    if Lx % bx or Ly % by:
        raise ValueError("fine blocks do not tile the lattice")
    NBX, NBY = Lx // bx, Ly // by
    if NBX % cx or NBY % cy:
        raise ValueError("coarse cells do not tile the block grid")
    out = np.zeros(NBX * NBY, np.int32)
    for bj in range(NBY):
        for bi in range(NBX):
            co = _builtin(k_outer, bi // cx, bj // cy)
            ci = _builtin(k_inner, bi % cx, bj % cy)
            out[bj * NBX + bi] = co * k_inner + ci
    return out


def nested_schedule(outer_split, k_outer, inner_split, k_inner, dt, dtau, T):
    """(colours, durations, step_end) of the nested scheme: the outer scheme
    of step dt over the outer colours, each outer window (c, d) expanded into
    the inner scheme of step dtau over the inner colours for time d (d must
    be a whole number of inner steps); step_end marks the last inner window
    of every outer step."""
    from . import LIE, STRANG, schedule
    if outer_split not in (LIE, STRANG) or inner_split not in (LIE, STRANG):
        raise ValueError("the nested schedule takes Lie or Strang at both levels")
    oc, od, oe = schedule(outer_split, k_outer, dt, T)
    cols, durs, ends = [], [], []
    for c, d, e in zip(oc, od, oe):
        span = dt if _PLANT == 13 else d
        ic, idur, _ = schedule(inner_split, k_inner, dtau, span)
        cols.extend(int(c) * k_inner + int(x) for x in ic)
        durs.extend(float(x) for x in idur)
        ends.extend([0] * (len(ic) - 1) + [int(e)])
    return (np.array(cols, np.int32), np.array(durs, np.float64), np.array(ends, np.uint8))
