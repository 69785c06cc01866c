"""Pins for the oracle's rates (test infrastructure).

* Spin-flip Arrhenius rates (Sec. 4.1 eq. adsdesrate, Sec. 7 eq. Arrhenius)
  against a 50-digit mpmath evaluation of k_d exp(-beta (J n + h)).
* Reaction-model rates (Sec. 7.1, Table COrates): for all 3^5 neighbourhood
  patterns, the oracle's 13 channels and site total against the independent
  event enumeration of oracle/exact.py on a 3x3 lattice (brute force).
"""
import math

import mpmath
import numpy as np

from oracle import exact


def test_flip_table_vs_mpmath(orc):
    mpmath.mp.dps = 50
    for (ka, kd, J, h, beta, dim) in [(1.0, 1.0, 1.0, 0.0, 1.0, 2), (0.3, 2.5, 2.0, -1.0, 1.7, 2),
                                      (1.0, 1.0, 0.5, 0.25, 4.0, 1)]:
        m = orc.Model("flip", 8, 8 if dim == 2 else 1, k_a=ka, k_d=kd, J=J, h=h, beta=beta)
        tab = orc.rate_table(m)
        z = m.z
        for n in range(z + 1):
            assert tab[n] == ka
            # the contract evaluates the argument in IEEE doubles; exp of it
            # must be accurate, and the argument itself within a few ulp
            arg = -(beta * (J * float(n) + h))
            exact_arg = -mpmath.mpf(beta) * (mpmath.mpf(J) * n + mpmath.mpf(h))
            assert abs(mpmath.mpf(arg) - exact_arg) <= 4 * abs(exact_arg) * mpmath.mpf(2) ** -53
            ref = mpmath.mpf(kd) * mpmath.exp(mpmath.mpf(arg))
            got = tab[(z + 1) + n]
            assert abs(mpmath.mpf(got) - ref) <= 2 * math.ulp(float(ref))


def test_flip_site_rate_counts_neighbours(orc):
    m = orc.Model("flip", 5, 4, k_a=0.7, k_d=1.3, J=1.1, h=0.2, beta=0.9)
    rng = np.random.default_rng(0)
    lat = rng.integers(0, 2, 20).astype(np.uint8)
    tab = orc.rate_table(m)
    g = lat.reshape(4, 5)
    for s in range(20):
        x, y = s % 5, s // 5
        n = g[y, (x + 1) % 5] + g[y, (x - 1) % 5] + g[(y + 1) % 4, x] + g[(y - 1) % 4, x]
        assert orc.site_rate(m, lat, s) == tab[lat[s] * 5 + n]


def test_zgb_table_vs_event_enumeration(orc):
    y, kr, D = 0.37, 11.0, 3.0
    m = orc.Model("zgb", 3, 3, y=y, k_r=kr, D=D)
    tab = orc.rate_table(m).reshape(243, 14)
    centre = 4
    nbr = {0: 5, 1: 3, 2: 7, 3: 1}  # E, W, N, S of (1,1) on a 3x3 torus
    for pat in range(243):
        r = pat
        conf = [0] * 9
        conf[centre] = r % 3
        r //= 3
        for d in range(4):
            conf[nbr[d]] = r % 3
            r //= 3
        evs = [e for e in exact.events("zgb", (y, kr, D), 3, 3, tuple(conf)) if e[0] == centre]
        total = math.fsum(e[1] for e in evs)
        assert abs(tab[pat, 13] - total) <= 8 * math.ulp(max(total, 1e-300)), pat
        assert abs(math.fsum(tab[pat, :13]) - total) <= 8 * math.ulp(max(total, 1e-300))
        # each channel's update: compare the multiset of (rate, new configuration)
        got = []
        for c in range(13):
            if tab[pat, c] == 0:
                continue
            new = list(conf)
            if c == 0:
                new[centre] = 1
            else:
                q = nbr[(c - 1) % 4]
                if c <= 4:
                    new[centre], new[q] = 2, 2
                elif c <= 8:
                    new[centre], new[q] = 0, 0
                else:
                    new[centre], new[q] = 0, 1
            got.append((tab[pat, c], tuple(new)))
        want = sorted((e[1], e[2]) for e in evs)
        assert sorted(got) == want, pat
