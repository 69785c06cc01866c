"""Exact references for the oracle -- TEST INFRASTRUCTURE ONLY.

Everything here is written from the mathematics of the paper, independently of
the C oracle:

* ``single_site_coverage``: the two-state chain of one site with
  adsorption k_a and desorption k_d (eq. adsdesrate with J = 0) solved in closed
  form.
* ``exact_equilibrium_small`` / ``transfer_matrix_1d``: the equilibrium measure of the
  Arrhenius spin-flip dynamics (Sec. 7, eq. Arrhenius).  Detailed balance of
  those rates fixes pi(sigma) ~ exp(beta*J*B(sigma) + (beta*h + ln(k_a/k_d))*S(sigma))
  with B the number of occupied nearest-neighbour bonds and S the number of
  occupied sites; it is evaluated by brute force on tiny lattices and with the
  finite transfer matrix on rings.
* ``generator``: the master-equation generator Q of eq. generator over all
  configurations of a tiny lattice, built from the same event list as the model
  definition (per site, per update omega: rate and new configuration), with
  an ``owner`` mask restricting it to the events owned by one colour (the
  operators L^E, L^O of eq. opdecomp).
* ``propagate`` / ``split_propagate``: p0 exp(tQ) and the fractional-step
  product p0 prod_w exp(d_w Q_{c_w}) (eqs. lie, strang).
"""
import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg


# ----------------------------------------------------------------------------
# closed forms
def single_site_coverage(k_a, k_d, s0, t):
    """P(sigma_t = 1) for one site flipping 0->1 at k_a and 1->0 at k_d."""
    th = k_a / (k_a + k_d)
    return th + (s0 - th) * np.exp(-(k_a + k_d) * np.asarray(t, dtype=np.float64))


def effective_field(k_a, k_d, h, beta):
    """The chemical potential mu with pi ~ exp(beta J B + beta mu S)."""
    return h + np.log(k_a / k_d) / beta


def transfer_matrix_1d(N, J, h, beta, k_a=1.0, k_d=1.0):
    """Finite periodic ring of N sites: (coverage, occupied-bond density).

    Bond density = E[#bonds with both ends occupied] / N (N bonds on a ring)."""
    mu = effective_field(k_a, k_d, h, beta)
    s = np.array([0.0, 1.0])
    # symmetric transfer matrix T(s,s') = exp(beta J s s' + beta mu (s+s')/2)
    T = np.exp(beta * J * np.outer(s, s) + 0.5 * beta * mu * (s[:, None] + s[None, :]))
    w, Uv = np.linalg.eigh(T)
    D = np.diag(s)

    def tr_pow(k):
        return (Uv * w ** k) @ Uv.T

    TN = tr_pow(N)
    Z = np.trace(TN)
    cov = np.trace(D @ TN) / Z
    bond = np.trace(D @ T @ D @ tr_pow(N - 1)) / Z
    return cov, bond


def exact_equilibrium_small(Lx, Ly, J, h, beta, k_a=1.0, k_d=1.0):
    """Brute-force Gibbs averages on a tiny periodic lattice (N <= 20 sites):
    (coverage, occupied-bond density per site), bonds along +x and (2D) +y."""
    N = Lx * Ly
    mu = effective_field(k_a, k_d, h, beta)
    dim = 1 if Ly == 1 else 2
    idx = np.arange(2 ** N, dtype=np.int64)
    conf = ((idx[:, None] >> np.arange(N)[None, :]) & 1).astype(np.float64)  # site i = bit i
    g = conf.reshape(-1, Ly, Lx)
    B = (g * np.roll(g, -1, axis=2)).sum(axis=(1, 2))
    if dim == 2:
        B = B + (g * np.roll(g, -1, axis=1)).sum(axis=(1, 2))
    S = conf.sum(axis=1)
    logw = beta * J * B + beta * mu * S
    w = np.exp(logw - logw.max())
    Z = w.sum()
    return float((w * S).sum() / Z / N), float((w * B).sum() / Z / N)


# ----------------------------------------------------------------------------
# master equation on tiny lattices
def _neighbours(Lx, Ly, dim, site):
    x, y = site % Lx, site // Lx
    out = [y * Lx + (x + 1) % Lx, y * Lx + (x - 1) % Lx]
    if dim == 2:
        out += [((y + 1) % Ly) * Lx + x, ((y - 1) % Ly) * Lx + x]
    return out


def events(kind, params, Lx, Ly, conf):
    """All events (x, rate, new configuration) of eq. generator for one
    configuration (a tuple of states).  kind 'flip': params (k_a,k_d,J,h,beta);
    kind 'zgb': params (y,k_r,D); kind 'kawasaki': params (D,J,beta), a
    particle at x moves to an empty neighbour q (spin exchange) at rate
    D/4 exp(-beta J n), n = occupied neighbours of x."""
    dim = 1 if Ly == 1 else 2
    N = Lx * Ly
    ev = []
    for x in range(N):
        nb = _neighbours(Lx, Ly, dim, x)
        s = conf[x]
        if kind == "flip":
            k_a, k_d, J, h, beta = params
            if s == 0:
                r = k_a
            else:
                n = sum(conf[q] for q in nb)
                r = k_d * np.exp(-beta * (J * n + h))
            new = list(conf)
            new[x] = 1 - s
            ev.append((x, r, tuple(new)))
        elif kind == "kawasaki":
            D, J, beta = params
            if s != 1:
                continue
            n = sum(1 for q in nb if conf[q] == 1)
            for q in nb:
                if conf[q] == 0:
                    new = list(conf)
                    new[x], new[q] = 0, 1
                    ev.append((x, D / 4.0 * np.exp(-beta * J * n), tuple(new)))
        else:
            y_, kr, D = params
            if s == 0:
                new = list(conf)
                new[x] = 1
                ev.append((x, y_, tuple(new)))
            for q in nb:
                sq = conf[q]
                if s == 0 and sq == 0:
                    new = list(conf)
                    new[x] = 2
                    new[q] = 2
                    ev.append((x, (1.0 - y_) / 4.0, tuple(new)))
                if (s == 1 and sq == 2) or (s == 2 and sq == 1):
                    new = list(conf)
                    new[x] = 0
                    new[q] = 0
                    ev.append((x, kr / 4.0, tuple(new)))
                if s == 1 and sq == 0 and D > 0:
                    new = list(conf)
                    new[x] = 0
                    new[q] = 1
                    ev.append((x, D / 4.0, tuple(new)))
    return [e for e in ev if e[1] > 0.0]


def state_index(conf, K):
    idx = 0
    for s in reversed(conf):
        idx = idx * K + s
    return idx


def all_states(N, K):
    """Configurations in index order: index = sum_i conf[i] * K**i."""
    for idx in range(K ** N):
        conf = []
        r = idx
        for _ in range(N):
            conf.append(r % K)
            r //= K
        yield tuple(conf)


def generator(kind, params, Lx, Ly, owner=None, sparse=False):
    """Generator matrix Q[i,j] = rate(i -> j), Q[i,i] = -sum.  ``owner`` is an
    optional boolean array over sites: only events whose site x is owned count
    (the restriction of L to one colour, eq. opdecomp)."""
    K = 3 if kind == "zgb" else 2
    N = Lx * Ly
    S = K ** N
    rows, cols, vals = [], [], []
    for i, conf in enumerate(all_states(N, K)):
        out = 0.0
        for (x, r, new) in events(kind, params, Lx, Ly, conf):
            if owner is not None and not owner[x]:
                continue
            j = state_index(new, K)
            rows.append(i)
            cols.append(j)
            vals.append(r)
            out += r
        rows.append(i)
        cols.append(i)
        vals.append(-out)
    Q = scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(S, S))
    return Q if sparse else Q.toarray()


def propagate(p0, Q, t):
    """Row vector p0 exp(tQ)."""
    if scipy.sparse.issparse(Q):
        return scipy.sparse.linalg.expm_multiply((Q.T * t).tocsr(), p0)
    return p0 @ scipy.linalg.expm(Q * t)


def split_propagate(p0, Qc, colours, durs):
    """Fractional-step propagator p0 * prod_w exp(d_w Q_{c_w}) in window order."""
    p = np.asarray(p0, dtype=np.float64)
    cache = {}
    for c, d in zip(colours, durs):
        c = int(c)
        d = float(d)
        if scipy.sparse.issparse(Qc[c]):
            p = scipy.sparse.linalg.expm_multiply((Qc[c].T * d).tocsr(), p)
        else:
            key = (c, d)
            if key not in cache:
                cache[key] = scipy.linalg.expm(Qc[c] * d)
            p = p @ cache[key]
    return p


def site_owner_by_colour(Lx, Ly, bx, by, cmap, colour):
    """Boolean array over sites: the site's block has the given colour."""
    NBX = Lx // bx
    own = np.zeros(Lx * Ly, bool)
    for s in range(Lx * Ly):
        x, y = s % Lx, s // Lx
        m = (y // by) * NBX + (x // bx)
        own[s] = cmap[m] == colour
    return own


def observable_vectors(kind, Lx, Ly):
    """Per-configuration observables matching the oracle's count layout:
    [#0, #1, #2, #bonds 0-0, #bonds 1-1, #bonds 2-2, #bonds A-B]."""
    K = 3 if kind == "zgb" else 2
    N = Lx * Ly
    dim = 1 if Ly == 1 else 2
    out = []
    for conf in all_states(N, K):
        v = [0] * 7
        for x in range(N):
            s = conf[x]
            v[s] += 1
            nbs = _neighbours(Lx, Ly, dim, x)
            pos = [nbs[0]] + ([nbs[2]] if dim == 2 else [])
            for q in pos:
                if conf[q] == s:
                    v[3 + s] += 1
                if {s, conf[q]} == {1, 2}:
                    v[6] += 1
        out.append(v)
    return np.array(out, dtype=np.float64)
