"""Pins of the oracle's film model: labels, owner/dist maps, barrier links,
rupture criterion and the film behaviour the paper describes (Sec. 2.1.5, Sec. 4).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage

from oracle import OracleSim, lattice, p0

from . import bruteforce as bf


def _sim_with_density(kind, rho3, **kw):
    """Oracle sim whose state has exactly the density rho3[z, y, x] (rest populations)."""
    nz, ny, nx = rho3.shape
    s = OracleSim(lattice=kind, nx=nx, ny=ny, nz=nz, **kw)
    e, w = lattice(kind)
    f = w[:, None, None, None] * rho3[None]
    s.set_populations(f if kind == 1 else f[:, 0])
    return s


# --------------------------------------------------------------------------
# connected-component labels (T9)
# --------------------------------------------------------------------------
def _labels_of(kind, gas):
    rho = np.where(gas, 0.1, 2.0).astype(np.float64)
    s = _sim_with_density(kind, rho)
    lab, nb = s.label_field(rho if kind == 1 else rho[0])
    return lab.reshape(gas.shape), nb


def test_labels_hand_patterns_2d():
    g = np.zeros((1, 6, 8), bool)
    g[0, 2, 0] = g[0, 2, 7] = True          # joined across the x wrap
    g[0, 0, 3] = g[0, 5, 3] = True          # joined across the y wrap
    g[0, 3, 5] = g[0, 4, 6] = True          # diagonal-only neighbours
    lab, nb = _labels_of(0, g)
    assert nb == 3
    assert lab[0, 0, 3] == lab[0, 5, 3] == 1  # min index 3 comes first
    assert lab[0, 2, 0] == lab[0, 2, 7] == 2
    assert lab[0, 3, 5] == lab[0, 4, 6] == 3


def test_labels_hand_patterns_3d():
    g = np.zeros((8, 8, 8), bool)            # indexed [z, y, x]
    g[1, 1, 1] = g[2, 2, 2] = True          # body diagonal: not a D3Q19 link
    g[4, 0, 0] = g[4, 1, 1] = True          # face diagonal: a link
    g[6, 5, 0] = g[6, 5, 7] = True          # x wrap
    lab, nb = _labels_of(1, g)
    assert nb == 4
    assert lab[4, 0, 0] == lab[4, 1, 1]
    assert lab[1, 1, 1] != lab[2, 2, 2]
    assert lab[6, 5, 0] == lab[6, 5, 7]


def test_labels_spiral_one_component():
    n = 15
    g = np.zeros((1, n, n), bool)
    x = y = n // 2
    dx, dy, steps = 1, 0, 1
    g[0, y, x] = True
    while 0 < x < n - 1 and 0 < y < n - 1:
        for _ in range(2):
            for _ in range(steps):
                x, y = x + dx, y + dy
                if 0 <= x < n and 0 <= y < n:
                    g[0, y, x] = True
            dx, dy = -dy, dx
        steps += 2
    lab, nb = _labels_of(0, g)
    assert nb == 1 and np.all((lab > 0) == g)


def _periodic_equiv_scipy(gas, kind):
    """Periodic components from scipy.ndimage.label on a 3x3(x3) tiling."""
    D = 2 if kind == 0 else 3
    a = gas[0] if kind == 0 else gas
    tiled = np.tile(a, (3,) * D)
    struct = ndimage.generate_binary_structure(D, 2 if kind == 1 else 2)
    tl, _ = ndimage.label(tiled, structure=struct)
    shape = a.shape
    idx = list(zip(*np.nonzero(a)))
    parent = {c: c for c in idx}

    def find(c):
        while parent[c] != c:
            c = parent[c]
        return c

    centre = tuple(s for s in shape)
    by_label = {}
    for c in idx:
        L = tl[tuple(ci + si for ci, si in zip(c, centre))]
        by_label.setdefault(L, []).append(c)
    for copies in np.ndindex(*(3,) * D):
        for c in idx:
            L = tl[tuple(ci + k * si for ci, k, si in zip(c, copies, shape))]
            if L in by_label:
                a0, b0 = find(c), find(by_label[L][0])
                if a0 != b0:
                    parent[a0] = b0
    return {c: find(c) for c in idx}


@pytest.mark.parametrize("kind,shape,p", [(0, (1, 20, 24), 0.35), (0, (1, 17, 13), 0.5),
                                          (1, (6, 7, 8), 0.25), (1, (5, 5, 5), 0.4)])
def test_labels_random_vs_bruteforce_and_scipy(kind, shape, p):
    rng = np.random.default_rng(int(p * 100) + kind)
    gas = rng.random(shape) < p
    lab, nb = _labels_of(kind, gas)
    ref, nbr = bf.bfs_labels(gas, kind)
    assert nb == nbr and np.array_equal(lab, ref)
    eq = _periodic_equiv_scipy(gas, kind)
    idx = list(eq)
    for a in idx[:200]:
        for b in idx[:200]:
            same = lab[a if kind == 1 else (0,) + a] == lab[b if kind == 1 else (0,) + b]
            if eq[a] == eq[b]:
                assert same
    # canonical order: component k has the k-th smallest minimum linear index
    flat = lab.reshape(-1)
    mins = [np.flatnonzero(flat == k).min() for k in range(1, nb + 1)]
    assert mins == sorted(mins)


# --------------------------------------------------------------------------
# owner / dist maps (T10)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind,shape,p,zw", [(0, (1, 16, 12), 0.06, 6), (0, (1, 11, 13), 0.1, 4),
                                             (1, (6, 5, 7), 0.05, 5), (1, (4, 6, 5), 0.08, 6)])
def test_owner_dist_vs_exhaustive(kind, shape, p, zw):
    rng = np.random.default_rng(31 + kind)
    gas = rng.random(shape) < p
    lab, nb = bf.bfs_labels(gas, kind)
    rho = np.where(gas, 0.1, 2.0)
    s = _sim_with_density(kind, rho, zone_width=zw)
    o1, o2, d = s.owner_dist(lab if kind == 1 else lab[0])
    lo, hi, dist = bf.exhaustive_owner(lab, kind, zw)
    if kind == 0:
        lo, hi, dist = lo[0], hi[0], dist[0]
    assert np.array_equal(d, dist)
    assert np.array_equal(o1, lo)
    assert np.array_equal(o2, hi)
    assert np.any(o1 != o2)  # the fields above do contain ties


def test_barrier_masks_match_definition():
    kind, zw = 0, 6
    ny, nx = 24, 40
    y, x = np.mgrid[0:ny, 0:nx]
    gas = ((x - 10) ** 2 + (y - 12) ** 2 <= 36) | ((x - 24) ** 2 + (y - 12) ** 2 <= 36) | \
          ((x - 36) ** 2 + (y - 3) ** 2 <= 4)
    rho = np.where(gas, 0.1, 2.0)[None]
    s = _sim_with_density(kind, rho, film_on=1, k_own=1, zone_width=zw, rupture_warmup=10 ** 9)
    s.step(1)
    m = s.maps()
    lab, nb = bf.bfs_labels(gas[None], kind)
    lo, hi, dist = bf.exhaustive_owner(lab, kind, zw)
    lo, hi, dist = lo[0], hi[0], dist[0]
    assert np.array_equal(m["label"], lab[0]) and m["n_bubbles"] == nb == 3
    e, _ = lattice(kind)
    expect = np.zeros((ny, nx), np.uint32)
    for i in range(1, len(e)):
        ylo, yhi = np.roll(lo, (-e[i][1], -e[i][0]), (0, 1)), np.roll(hi, (-e[i][1], -e[i][0]), (0, 1))
        yd = np.roll(dist, (-e[i][1], -e[i][0]), (0, 1))
        bar = (lo > 0) & (ylo > 0) & ((lo != ylo) | (hi != yhi)) & (dist + yd + 1 <= zw)
        expect |= np.where(bar, np.uint32(1 << i), np.uint32(0))
    assert np.array_equal(m["mask"], expect)
    assert np.count_nonzero(expect) > 0


# --------------------------------------------------------------------------
# rupture criterion on synthetic symmetric films (T12)
# --------------------------------------------------------------------------
def _liquid_spinodal(G):
    q = (1 - math.sqrt(1 + 4 / G)) / 2
    return -math.log(q)


@pytest.mark.parametrize("G", [-4.5, -5.0, -5.5, -6.0])
def test_rupture_indicator_flips_at_liquid_spinodal(G):
    rs = _liquid_spinodal(G)
    # the spinodal is where dp0/drho changes sign (Eq. Pequ with psi = 1 - e^-rho)
    h = 1e-6
    assert (p0(rs + h, G) - p0(rs - h, G)) / (2 * h) == pytest.approx(0, abs=1e-7)
    # gas | smooth symmetric film centred on x0 | gas | thick liquid slab (so the two
    # gas regions are distinct bubbles on the periodic line)
    nx, x0, width = 200, 64, 12.0
    x = np.arange(nx)
    fired = {}
    for dc in (+0.04, -0.04):
        rc, rg = rs + dc, 0.12
        rho = rg + (rc - rg) * np.exp(-(((x - x0) / width) ** 2))
        rho = np.where((x >= 140) & (x < 190), 2.2, rho)
        s = _sim_with_density(0, rho[None, None], G=G, film_on=1, k_own=1, zone_width=40,
                              rupture_warmup=0)
        s.step(1)
        fired[dc] = len(s.events()) > 0
        assert s.maps()["n_bubbles"] == 2
    assert fired == {+0.04: False, -0.04: True}


# --------------------------------------------------------------------------
# film behaviour (T11)
# --------------------------------------------------------------------------
def test_one_bubble_film_is_exact_noop():
    runs = []
    for film in (0, 1):
        s = OracleSim(lattice=0, nx=128, ny=128, G=-5.0, film_on=film, seed=1)
        s.set_nuclei([[64, 64, 0, 20]])
        s.step(2000)
        runs.append(s.populations())
    assert np.array_equal(runs[0], runs[1])


def _two_bubbles(film, warmup, on_rupture=0, steps=1500, every=100):
    R, gap = 14.0, 2.0
    s = OracleSim(lattice=0, nx=96, ny=64, G=-5.5, rho_liquid=2.3, rho_gas=0.11, film_on=film,
                  rupture_warmup=warmup, zone_width=6, k_own=1, seed=3, on_rupture=on_rupture)
    s.set_nuclei([[48 - R - gap / 2 - 0.5, 32, 0, R], [48 + R + gap / 2 + 0.5, 32, 0, R]])
    nbs = []
    for _ in range(steps // every):
        if s.step(every):
            break
        nbs.append(s.labels()[1])
    return s, nbs


@pytest.mark.slow
def test_two_bubbles_merge_without_film():
    s, nbs = _two_bubbles(0, 0)
    assert nbs[0] == 2 and nbs[-1] == 1


@pytest.mark.slow
def test_barrier_keeps_film_without_rupture():
    s, nbs = _two_bubbles(1, 10 ** 9)
    assert all(n == 2 for n in nbs)
    assert s.n_ruptures == 0


@pytest.mark.slow
def test_rupture_then_merge():
    s, nbs = _two_bubbles(1, 50)
    ev = s.events()
    assert len(ev) > 0 and ev[0][0] == 50 and tuple(ev[0][1:]) == (1, 2)
    assert s.n_ruptures == 1
    assert nbs[0] == 2 and nbs[-1] == 1
    # the two bubbles stay aliased across relabelling until they join
    s2, _ = _two_bubbles(1, 50, steps=200)
    m = s2.maps()
    assert m["n_bubbles"] == 2 and m["alias_root"][1] == m["alias_root"][2]


def _disc(gas, cx, cy, r):
    y, x = np.mgrid[0:gas.shape[0], 0:gas.shape[1]]
    gas[(x - cx) ** 2 + (y - cy) ** 2 <= r * r] = True


def test_alias_carry_hand_built_relabel():
    # R21 (Sec. 2.1.5, the film between a pair is removed once they are one
    # bubble): at a refresh, new bubbles whose gas overlaps old bubbles of one
    # alias class become aliases of each other.  Hand-built: old A ~ B by a
    # rupture; new P overlaps A and Q overlaps B (carried: P ~ Q); old C splits
    # into C1, C2 (split: C1 ~ C2); old F and H merge into M (merge: one
    # label, in a class of its own); E' overlaps only E, N overlaps nothing
    # (non-aliased neighbours).  The films P|Q and C1|C2 then carry no barrier
    # links, the film M|N does.
    ny, nx = 40, 72
    old = np.zeros((ny, nx), bool)
    for cx, cy, r in ((7, 8, 2), (15, 8, 2), (32, 8, 4), (60, 8, 3), (10, 28, 3), (20, 28, 3)):
        _disc(old, cx, cy, r)
    new = np.zeros((ny, nx), bool)
    for cx, cy, r in ((8, 8, 2), (14, 8, 2), (30, 8, 2), (36, 8, 2), (60, 8, 2), (26, 28, 2)):
        _disc(new, cx, cy, r)
    new[26:31, 8:23] = True  # M covers F and H
    kw = dict(G=-5.5, film_on=1, k_own=1, zone_width=6, rupture_warmup=10 ** 9)
    s = _sim_with_density(0, np.where(old, 0.1, 2.0)[None], **kw)
    s.step(1)  # refresh at step 0 labels the old field
    m1 = s.maps()
    lab1 = m1["label"]
    assert m1["n_bubbles"] == 6
    A, B = lab1[8, 7], lab1[8, 15]
    assert s.alias_unite(A, B) == 1  # as a rupture of the A|B film would
    e, w = lattice(0)
    s.set_populations(w[:, None, None] * np.where(new, 0.1, 2.0)[None])
    s.step(1)  # refresh at step 1 labels the new field and carries the aliases
    m2 = s.maps()
    lab, root = m2["label"], m2["alias_root"]
    ref, nb = bf.bfs_labels(new[None], 0)
    assert np.array_equal(lab.reshape(ref.shape), ref) and nb == 7
    P, Q, C1, C2, E2, M, N = (lab[8, 8], lab[8, 14], lab[8, 30], lab[8, 36], lab[8, 60], lab[28, 15], lab[28, 26])
    assert len({P, Q, C1, C2, E2, M, N}) == 7 and 0 not in (P, Q, C1, C2, E2, M, N)
    assert root[P] == root[Q]                      # carried through the rupture of A|B
    assert root[C1] == root[C2]                    # split of one old bubble
    classes = {root[P], root[C1], root[M], root[E2], root[N]}
    assert len(classes) == 5                       # merge, E', N each in a class of their own
    assert root[M] == M and root[E2] == E2 and root[N] == N
    mask = m2["mask"]
    assert mask[8, 11] == 0 and mask[8, 10] == 0 and mask[8, 12] == 0   # P|Q film: no barrier
    assert mask[8, 33] == 0 and mask[8, 32] == 0 and mask[8, 34] == 0   # C1|C2 film: no barrier
    assert mask[28, 23] != 0                                          # M|N film: barrier


def test_stop_on_first_rupture():
    s, _ = _two_bubbles(1, 50, on_rupture=1, steps=300, every=300)
    assert s.stopped and s.steps_done == 51
    f = s.populations().copy()
    assert s.step(10) == 1 and s.steps_done == 51
    assert np.array_equal(s.populations(), f)


def test_histogram_equivalent_diameters():
    rho = np.full((1, 40, 50), 2.0)
    y, x = np.mgrid[0:40, 0:50]
    rho[0][(x - 10) ** 2 + (y - 10) ** 2 <= 25] = 0.1     # 81 cells
    rho[0][(x - 35) ** 2 + (y - 25) ** 2 <= 64] = 0.1     # 197 cells
    s = _sim_with_density(0, rho)
    lab, nb = s.label_field(rho[0])
    counts, sizes = s.histogram(lab, nb, 20, 1.0)
    assert nb == 2 and list(sizes[1:]) == [81, 197]
    d = [2 * math.sqrt(81 / math.pi), 2 * math.sqrt(197 / math.pi)]
    expect = np.zeros(20, np.int64)
    for v in d:
        expect[int(v)] += 1
    assert np.array_equal(counts, expect)


@pytest.mark.parametrize("mode", [0, 1])
def test_barrier_force_substitution(mode):
    # F(x) = -G psi(x) sum_i w_i psi~(x+e_i) e_i with psi~ = psi_bar on barrier links
    # (psi(rho_liquid) in mode 0, psi(x) in mode 1), recomputed here from the masks
    kind, zw, G = 0, 6, -5.5
    ny, nx = 20, 36
    y, x = np.mgrid[0:ny, 0:nx]
    gas = ((x - 9) ** 2 + (y - 10) ** 2 <= 30) | ((x - 22) ** 2 + (y - 10) ** 2 <= 30)
    rng = np.random.default_rng(5)
    rho = np.where(gas, 0.1, 2.0) + 0.05 * rng.random((ny, nx))
    s = _sim_with_density(kind, rho[None], G=G, film_on=1, k_own=1, zone_width=zw,
                          rupture_warmup=10 ** 9, psi_bar_mode=mode, rho_liquid=2.3)
    f0 = s.populations().copy()
    s.step(1)                       # refreshes the maps from this density
    s.set_populations(f0)           # back to the same state, maps kept
    m = s.maps()
    assert np.count_nonzero(m["mask"]) > 0
    F = s.force(with_film=1)
    e, w = lattice(kind)
    psi = 1 - np.exp(-rho)
    bar = np.full_like(psi, 1 - math.exp(-2.3)) if mode == 0 else psi
    acc = np.zeros((2, ny, nx))
    for i in range(1, len(e)):
        nb = np.roll(psi, (-e[i][1], -e[i][0]), (0, 1))
        on = (m["mask"] >> i) & 1
        val = np.where(on == 1, bar, nb)
        acc[0] += w[i] * e[i][0] * val
        acc[1] += w[i] * e[i][1] * val
    ref = -G * psi * acc
    assert np.abs(F - ref).max() < 1e-13
    Fplain = s.force(with_film=0)
    assert np.abs(F - Fplain).max() > 1e-3


@pytest.mark.parametrize("src", [0, 1])
@pytest.mark.parametrize("kind,dims", [(0, (1, 40, 48)), (1, (14, 15, 16))])
def test_refresh_labels_density_reading(kind, dims, src):
    # R12: the maps refreshed at step n (n = 0 mod k_own) label the gas of the
    # density that enters step n (refresh_src 0, the default), or of the one
    # that entered step n - 1 (refresh_src 1); at n = 0, and after the state
    # was replaced, both label the density of the current state.  Each is
    # checked against a brute-force flood fill of that density < ln 2.
    nz, ny, nx = dims
    rng = np.random.default_rng(3 + kind)
    nuc = [[rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz) if kind else 0.0, rng.uniform(2.5, 4.5)]
           for _ in range(6)]
    k = 3
    kw = dict(lattice=kind, nx=nx, ny=ny, nz=nz, G=-5.5, rho_liquid=2.3, rho_gas=0.11, film_on=1, k_own=k,
              zone_width=6, rupture_warmup=10 ** 6, seed=2, refresh_src=src)
    s = OracleSim(**kw)
    s.set_nuclei(nuc)
    s.step(1)
    gas0 = (s.maps()["label"] > 0).reshape(dims)
    s.set_nuclei(nuc)
    assert np.array_equal(gas0, s.density().reshape(dims) < math.log(2.0))  # step 0: current state
    s.step(k - 1)
    prev = s.density().reshape(dims)  # enters step k - 1
    s.step(1)
    cur = s.density().reshape(dims)  # enters step k, at which the maps are refreshed
    s.step(1)
    lab = s.maps()["label"].reshape(dims)
    ref, nb = bf.bfs_labels((cur if src == 0 else prev) < math.log(2.0), kind)
    assert np.array_equal(lab, ref) and nb > 1
    assert not np.array_equal(prev < math.log(2.0), cur < math.log(2.0))  # the two readings differ here
    # after the state is replaced the next refresh labels the new state
    s2 = OracleSim(**kw)
    s2.set_nuclei(nuc)
    s2.step(k)
    s2.set_populations(s2.populations())
    s2.step(1)
    ref2, _ = bf.bfs_labels(cur < math.log(2.0), kind)
    assert np.array_equal(s2.maps()["label"].reshape(dims), ref2)


def test_foam_statistics_hand_built():
    # Table 5 of Sec. 5: bubble percentage, foam density (the melt density
    # times one minus that fraction: 2.7 (1 - 0.443) = 1.50 g/cm^3 as printed)
    # and the mean bubble size, here from labels of two hand-drawn discs and,
    # in 3-D, two boxes of known volume
    rho = np.full((1, 40, 50), 2.0)
    y, x = np.mgrid[0:40, 0:50]
    rho[0][(x - 10) ** 2 + (y - 10) ** 2 <= 25] = 0.1     # 81 cells
    rho[0][(x - 35) ** 2 + (y - 25) ** 2 <= 64] = 0.1     # 197 cells
    s = _sim_with_density(0, rho)
    lab, nb = s.label_field(rho[0])
    st = s.foam_stats(lab, nb)
    d = [2 * math.sqrt(81 / math.pi), 2 * math.sqrt(197 / math.pi)]
    assert st["gas_fraction"] == 278 / 2000 and st["relative_density"] == 1 - 278 / 2000
    assert abs(st["mean_diameter"] - sum(d) / 2) < 1e-14 and st["max_diameter"] == max(d)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    t5 = gold["table5_simulation"]
    assert abs(t5["melt_density_g_cm3"] * (1 - t5["bubble_fraction"]) - t5["foam_density_g_cm3"]) < 0.005
    rho3 = np.full((10, 12, 14), 2.0)
    rho3[1:4, 2:5, 3:8] = 0.1    # 3 x 3 x 5 = 45 cells
    rho3[6:9, 7:11, 9:11] = 0.1  # 3 x 4 x 2 = 24 cells
    s3 = _sim_with_density(1, rho3)
    lab3, nb3 = s3.label_field(rho3)
    st3 = s3.foam_stats(lab3, nb3)
    d3 = [(6 * 45 / math.pi) ** (1 / 3), (6 * 24 / math.pi) ** (1 / 3)]
    assert nb3 == 2 and st3["gas_fraction"] == 69 / rho3.size
    assert abs(st3["mean_diameter"] - sum(d3) / 2) < 1e-14
    empty = s.foam_stats(np.zeros((40, 50), np.int32), 0)
    assert empty["gas_fraction"] == 0 and empty["mean_diameter"] == 0
