"""Independent brute-force re-derivations used to pin the oracle on tiny inputs.

Nothing here is shared with the oracle or with the GPU library: each routine is
a literal, whole-array (numpy) or exhaustive-search restatement of a definition
from the paper, written separately so that a mistake in one place shows up as a
disagreement.
"""
from collections import deque

import numpy as np

# D2Q9 (paper Sec. 2.1.1) and D3Q19 (textbook) written out as sets, in an order
# different from the oracle's so that index slips cannot cancel.
D2Q9 = [((0, 0, 0), 4 / 9)] + [((a, b, 0), 1 / 9) for a, b in ((0, 1), (1, 0), (0, -1), (-1, 0))] + \
       [((a, b, 0), 1 / 36) for a in (1, -1) for b in (1, -1)]
D3Q19 = [((0, 0, 0), 1 / 3)]
for k in range(3):
    for s in (1, -1):
        v = [0, 0, 0]
        v[k] = s
        D3Q19.append((tuple(v), 1 / 18))
for k1 in range(3):
    for k2 in range(k1 + 1, 3):
        for s1 in (1, -1):
            for s2 in (1, -1):
                v = [0, 0, 0]
                v[k1] = s1
                v[k2] = s2
                D3Q19.append((tuple(v), 1 / 36))


def velset(lattice):
    return D2Q9 if lattice == 0 else D3Q19


def shift(a, e):
    """a(x - e) as a whole-array periodic roll (arrays indexed [z, y, x])."""
    return np.roll(a, shift=(e[2], e[1], e[0]), axis=(0, 1, 2))


def literal_step(f, lattice, G, tau, rho0=1.0):
    """One plain Shan-Chen BGK step on populations f[q, z, y, x] (film off).

    Moments (Eq. vel_dens), psi (Eq. pseudopotential), neighbour-sum force
    (Eq. shanchen3) summed over every direction, u_eq = u + tau F / rho,
    BGK towards f^eq, then streaming f_i(x + e_i) = f*_i(x).
    """
    vs = velset(lattice)
    rho = f.sum(axis=0)
    j = np.zeros((3,) + rho.shape)
    for q, (e, _) in enumerate(vs):
        for k in range(3):
            j[k] += e[k] * f[q]
    psi = rho0 * (1 - np.exp(-rho / rho0))
    F = np.zeros_like(j)
    for e, w in vs:
        nb = shift(psi, tuple(-c for c in e))  # psi(x + e)
        for k in range(3):
            F[k] += w * e[k] * nb
    F *= -G * psi
    u = (j + tau * F) / rho
    uu = (u * u).sum(axis=0)
    out = np.empty_like(f)
    for q, (e, w) in enumerate(vs):
        eu = e[0] * u[0] + e[1] * u[1] + e[2] * u[2]
        feq = w * rho * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * uu)
        post = f[q] - (f[q] - feq) / tau
        out[q] = shift(post, e)
    return out


def to_velset_order(f_oracle, e_oracle, lattice):
    """Reorder populations given in the oracle's direction order into velset order."""
    vs = velset(lattice)
    idx = [next(i for i in range(len(e_oracle)) if tuple(e_oracle[i]) == e) for e, _ in vs]
    return f_oracle[idx]


def neighbours(shape, lattice):
    nz, ny, nx = shape
    vs = velset(lattice)
    return [e for e, _ in vs if e != (0, 0, 0)]


def bfs_labels(gas, lattice):
    """Canonical periodic component labels by flood fill from each unlabelled gas cell
    visited in increasing linear index (x fastest); 1-based, 0 = not gas."""
    nz, ny, nx = gas.shape
    lab = np.zeros(gas.shape, np.int32)
    links = neighbours(gas.shape, lattice)
    nb = 0
    for idx in range(gas.size):
        z, y, x = idx // (nx * ny), (idx // nx) % ny, idx % nx
        if not gas[z, y, x] or lab[z, y, x]:
            continue
        nb += 1
        lab[z, y, x] = nb
        dq = deque([(z, y, x)])
        while dq:
            cz, cy, cx = dq.popleft()
            for e in links:
                tz, ty, tx = (cz + e[2]) % nz, (cy + e[1]) % ny, (cx + e[0]) % nx
                if gas[tz, ty, tx] and not lab[tz, ty, tx]:
                    lab[tz, ty, tx] = nb
                    dq.append((tz, ty, tx))
    return lab, nb


def hop_distances_from(src, shape, lattice):
    """Exact lattice-link hop distance from one cell to every cell (periodic BFS)."""
    nz, ny, nx = shape
    d = -np.ones(shape, np.int64)
    d[src] = 0
    dq = deque([src])
    links = neighbours(shape, lattice)
    while dq:
        c = dq.popleft()
        for e in links:
            t = ((c[0] + e[2]) % nz, (c[1] + e[1]) % ny, (c[2] + e[0]) % nx)
            if d[t] < 0:
                d[t] = d[c] + 1
                dq.append(t)
    return d


def exhaustive_owner(labels, lattice, zone_width):
    """For every cell: min hop distance to any gas cell, and the min / max label
    among gas cells at that distance; truncated at zone_width - 1 hops."""
    shape = labels.shape
    best = np.full(shape, 1 << 30, np.int64)
    lo = np.zeros(shape, np.int64)
    hi = np.zeros(shape, np.int64)
    for src in zip(*np.nonzero(labels)):
        d = hop_distances_from(src, shape, lattice)
        L = labels[src]
        closer = d < best
        tie = d == best
        best = np.where(closer, d, best)
        lo = np.where(closer, L, np.where(tie, np.minimum(lo, L), lo))
        hi = np.where(closer, L, np.where(tie, np.maximum(hi, L), hi))
    far = best > zone_width - 1
    dist = np.where(far, -1, best)
    lo = np.where(far, 0, lo)
    hi = np.where(far, 0, hi)
    return lo.astype(np.int32), hi.astype(np.int32), dist.astype(np.int32)
