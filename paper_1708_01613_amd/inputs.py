"""Seeded synthetic workloads: nuclei lists, batch draws and arrival traces.

This module generates inputs only; it holds none of the method's arithmetic
and is shared by the GPU tests, the benchmark and the CPU-oracle checks.
All draws use numpy's PCG64 with explicit seeds.  Sizes follow the foam
workloads: a 128^2 single-bubble case, a 1024^2 D2Q9 foam with 200
Poisson-disk nuclei, a 256^3 D3Q19 foam with 2000 nuclei, a 64-lattice
uneven D2Q9 ensemble and a Poisson arrival stream of mixed jobs.
"""
import math

import numpy as np


def single_bubble(n=128, radius=20.0):
    """One centred bubble (cell centres at integer coordinates)."""
    return np.array([[n / 2, n / 2, 0.0, radius]])


def poisson_disk_2d(nx, ny, count, min_sep, rmin, rmax, seed, max_tries=200000):
    """Dart throwing: centres uniform in the periodic box, rejected if closer than
    min_sep (minimum image) to an accepted centre; radii uniform in [rmin, rmax]."""
    rng = np.random.default_rng(seed)
    pts = []
    tries = 0
    while len(pts) < count and tries < max_tries:
        tries += 1
        c = rng.random(2) * (nx, ny)
        ok = True
        for q in pts:
            dx = abs(c[0] - q[0])
            dy = abs(c[1] - q[1])
            dx = min(dx, nx - dx)
            dy = min(dy, ny - dy)
            if dx * dx + dy * dy < min_sep * min_sep:
                ok = False
                break
        if ok:
            pts.append(c)
    pts = np.array(pts)
    r = rng.uniform(rmin, rmax, len(pts))
    return np.column_stack([pts[:, 0], pts[:, 1], np.zeros(len(pts)), r])


def uniform_nuclei(dims, count, rmin, rmax, seed):
    """Centres uniform in the periodic box (overlaps allowed: union of disks/balls)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    c = rng.random((count, 3)) * (nx, ny, nz)
    if nz == 1:
        c[:, 2] = 0.0
    r = rng.uniform(rmin, rmax, count)
    return np.column_stack([c, r])


def nonoverlapping_2d(n, count, rmin, rmax, rng, attempts=10000):
    """Disks placed one by one, rejected when closer than r1 + r2 + 2 (minimum
    image) to an accepted disk; stops after `attempts` draws."""
    out = []
    for _ in range(attempts):
        if len(out) >= count:
            break
        c = rng.random(2) * n
        r = rng.uniform(rmin, rmax)
        ok = True
        for q in out:
            dx = abs(c[0] - q[0])
            dy = abs(c[1] - q[1])
            dx = min(dx, n - dx)
            dy = min(dy, n - dy)
            if dx * dx + dy * dy < (r + q[3] + 2) ** 2:
                ok = False
                break
        if ok:
            out.append((c[0], c[1], 0.0, r))
    return np.array(out).reshape(-1, 4)


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------
def config_single_bubble():
    """D2Q9 128^2 FP64, tau 1, G -5, one centred bubble R 20 (rho 0.15 in 2.0),
    noise 0.01 (seed 1), film on, 2000 steps."""
    params = dict(lattice=0, storage="f64", nx=128, ny=128, nz=1, tau=1.0, G=-5.0, rho0=1.0,
                  rho_liquid=2.0, rho_gas=0.15, noise_amp=0.01, seed=1, film_on=1)
    return params, single_bubble(128, 20.0), 2000


def config_foam2d():
    """D2Q9 1024^2 FP32, G -5.5, 200 Poisson-disk nuclei (min separation 30,
    radii U[4, 12], seed 2), film on, 20000 steps, labels every 500 steps."""
    params = dict(lattice=0, storage="f32", nx=1024, ny=1024, nz=1, tau=1.0, G=-5.5, rho0=1.0,
                  rho_liquid=2.0, rho_gas=0.15, noise_amp=0.01, seed=2, film_on=1)
    return params, poisson_disk_2d(1024, 1024, 200, 30.0, 4.0, 12.0, seed=2), 20000


def config_foam3d(storage="f32", n=256):
    """D3Q19 256^3, G -5.5, 2000 uniform nuclei with radii U[3, 8] (seed 3),
    film on, 5000 steps."""
    params = dict(lattice=1, storage=storage, nx=n, ny=n, nz=n, tau=1.0, G=-5.5, rho0=1.0,
                  rho_liquid=2.0, rho_gas=0.15, noise_amp=0.01, seed=3, film_on=1)
    count = max(1, int(round(2000 * (n / 256) ** 3)))
    return params, uniform_nuclei((n, n, n), count, 3.0, 8.0, seed=3), 5000


def config_ensemble(count=64, seed=4):
    """Uneven D2Q9 ensemble: side round(exp U[ln 64, ln 512]), G U[-6, -4.5],
    10..150 non-overlapping nuclei with radii U[3, 10], FP32, 10000 steps."""
    rng = np.random.default_rng(seed)
    members = []
    for k in range(count):
        n = int(round(math.exp(rng.uniform(math.log(64), math.log(512)))))
        G = float(rng.uniform(-6.0, -4.5))
        want = int(rng.integers(10, 151))
        nuc = nonoverlapping_2d(n, want, 3.0, 10.0, rng)
        params = dict(lattice=0, storage="f32", nx=n, ny=n, nz=1, tau=1.0, G=G, rho0=1.0,
                      rho_liquid=2.0, rho_gas=0.15, noise_amp=0.01, seed=1000 + k, film_on=1)
        members.append((params, nuc))
    return members, 10000


def arrival_trace(n_requests=256, rate=20.0, d3_fraction=0.5, seed=5):
    """Poisson arrivals (rate per second) of mixed jobs: D2Q9 side logU[128, 1024]
    or D3Q19 side logU[64, 192]; G, nuclei and radii as in the ensemble; 5000 steps."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    jobs = []
    for k in range(n_requests):
        G = float(rng.uniform(-6.0, -4.5))
        if rng.random() < d3_fraction:
            n = int(round(math.exp(rng.uniform(math.log(64), math.log(192)))))
            cnt = int(rng.integers(10, 151))
            nuc = uniform_nuclei((n, n, n), cnt, 3.0, 10.0, seed=int(rng.integers(1 << 31)))
            params = dict(lattice=1, storage="f32", nx=n, ny=n, nz=n, G=G, film_on=1, seed=2000 + k)
        else:
            n = int(round(math.exp(rng.uniform(math.log(128), math.log(1024)))))
            nuc = nonoverlapping_2d(n, int(rng.integers(10, 151)), 3.0, 10.0, rng)
            params = dict(lattice=0, storage="f32", nx=n, ny=n, nz=1, G=G, film_on=1, seed=2000 + k)
        jobs.append(dict(arrival=float(t[k]), params=params, nuclei=nuc, steps=5000))
    return jobs
