"""Pins of the oracle's container boundary (Sec. 5: the two-bubble case is
run in a container closed for the gas and open for the liquid, so that the
liquid the growing bubbles displace leaves it) and of the gas release into
the gas lattice of the two-lattice model (Sec. 2.1.3 with Sec. 2.1.5).

The container is read as two open planes across the last axis (z on D3Q19,
y on D2Q9) facing a liquid reservoir at rest at density rho_res: a
population that streams in across such a plane comes from the reservoir,
w_i rho_res, one that streams out leaves; neighbours beyond the planes are
the reservoir's.  The other axes stay periodic.
"""
import numpy as np
import pytest

from oracle.oracle import OracleSim, lattice

TL = dict(model=1, G=-5.0, G_mg=0.3, rho_g_bubble=0.4, rho_g_liquid=0.05)


@pytest.mark.parametrize("kind,shape", [(0, (9, 11, 1)), (1, (5, 6, 7))])
@pytest.mark.parametrize("model", [0, 1])
def test_reservoir_state_is_steady(kind, shape, model):
    # a container filled with the reservoir's own state stays exactly so
    nx, ny, nz = shape
    kw = dict(TL) if model else dict(G=-5.0)
    s = OracleSim(lattice=kind, nx=nx, ny=ny, nz=nz, open_z=1, rho_res=1.7, tau=0.8, **kw)
    e, w = lattice(kind)
    sh = s.shape
    f = w.reshape((-1,) + (1,) * len(sh)) * np.full(sh, 1.7)[None]
    if model:
        g = w.reshape((-1,) + (1,) * len(sh)) * np.full(sh, TL["rho_g_liquid"])[None]
        f = np.concatenate([f, g])
    s.set_populations(f)
    s.step(15)
    assert np.allclose(s.populations(), f, rtol=0, atol=1e-15)


@pytest.mark.parametrize("kind,shape", [(0, (10, 12, 1)), (1, (6, 5, 8))])
def test_mass_flux_through_open_planes(kind, shape):
    # without forces, at rest, with tau = 1 a cell's post-collision
    # populations are w_i rho, so one step changes the mass by what streams
    # in from the reservoir minus what streams out, plane by plane:
    #   sum_{first, last planes} (rho_res - rho_c) * (sum of w_i over e_i crossing the plane inwards)
    nx, ny, nz = shape
    s = OracleSim(lattice=kind, nx=nx, ny=ny, nz=nz, open_z=1, rho_res=1.3, G=0.0, tau=1.0)
    e, w = lattice(kind)
    ax = 1 if kind == 0 else 2
    rng = np.random.default_rng(9)
    rho = 1.0 + rng.random(s.shape)
    s.set_populations(w.reshape((-1,) + (1,) * rho.ndim) * rho[None])
    m0 = s.stats()[0]
    s.step(1)
    w_in = sum(w[i] for i in range(len(w)) if e[i][ax] > 0)  # crossing one plane inwards
    first = rho[0] if kind == 1 else rho[0, :]   # the plane at the start of the last axis
    last = rho[-1] if kind == 1 else rho[-1, :]
    expect = w_in * ((1.3 - first).sum() + (1.3 - last).sum())
    assert abs(s.stats()[0] - m0 - expect) < 1e-12 * m0
    # a periodic lattice keeps its mass
    p = OracleSim(lattice=kind, nx=nx, ny=ny, nz=nz, G=0.0, tau=1.0)
    p.set_populations(w.reshape((-1,) + (1,) * rho.ndim) * rho[None])
    p.step(1)
    assert abs(p.stats()[0] - m0) < 1e-12 * m0


@pytest.mark.parametrize("kind", [0, 1])
def test_gas_release_goes_to_the_gas_lattice(kind):
    # Sec. 2.1.3 in the two-lattice model: every step the gas lattice gains
    # exactly 3 A (dn/dt), the melt lattice nothing
    dims = dict(nx=24, ny=20, nz=1) if kind == 0 else dict(nx=12, ny=10, nz=9)
    s = OracleSim(lattice=kind, **dims, growth_on=1, gas_A=2.0, gas_dndt=0.05, **TL)
    c = [12.0, 10.0, 0.0, 4.0] if kind == 0 else [6.0, 5.0, 4.0, 3.0]
    s.set_nuclei([c])
    mm, mg = s.density().sum(), s.density_gas().sum()
    s.step(12)
    assert abs(s.density().sum() - mm) < 1e-12 * mm
    assert abs(s.density_gas().sum() - (mg + 12 * 3.0 * 2.0 * 0.05)) < 1e-12 * mg


@pytest.mark.slow
def test_growth_in_the_container_ruptures_the_film_sooner():
    # two bubbles 16 cells apart in a container open for the liquid: their
    # growth thins the film between them to the rupture criterion, earlier
    # than with the dissolved gas alone, and the displaced liquid leaves
    def first_event(dndt):
        nx, ny, R, gap = 128, 96, 10.0, 16.0
        c = (nx - 1) / 2
        s = OracleSim(lattice=0, nx=nx, ny=ny, noise_amp=0.0, growth_on=int(dndt > 0), gas_A=1.0, gas_dndt=dndt,
                      open_z=1, rho_res=2.0, rho_liquid=2.0, rho_gas=0.15, film_on=1, rupture_warmup=20, k_own=5,
                      zone_width=6, **TL)
        s.set_nuclei([[c - R - gap / 2 - 0.5, ny / 2, 0, R], [c + R + gap / 2 + 0.5, ny / 2, 0, R]])
        m0 = s.density().sum()
        for _ in range(12):
            s.step(100)
            if len(s.events()):
                break
        ev = s.events()
        return (int(ev[0][0]) if len(ev) else None), s.density().sum() - m0, s.labels()[1]
    grown, dm, nb = first_event(0.1)
    still, _, _ = first_event(0.0)
    assert grown is not None and still is not None and 20 < grown < still
    assert dm < 0  # melt left the container


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("model", [0, 1])
def test_force_sees_the_reservoir_beyond_the_planes(kind, model):
    # the force of a state in the container equals, on its cells, the force
    # of the same state on a periodic lattice with one plane of the
    # reservoir's state added at each end of the last axis
    dims = dict(nx=7, ny=6, nz=1) if kind == 0 else dict(nx=5, ny=4, nz=6)
    kw = dict(TL) if model else dict(G=-5.0)
    e, w = lattice(kind)
    ax = 1 if kind == 0 else 2
    s = OracleSim(lattice=kind, **dims, open_z=1, rho_res=1.8, **kw)
    rng = np.random.default_rng(3)
    shape = s.shape
    sets = [0.2 + 2.0 * rng.random(shape)]
    if model:
        sets.append(0.05 + 0.5 * rng.random(shape))

    def pops(fields):
        return np.concatenate([w.reshape((-1,) + (1,) * len(shape)) * r[None] for r in fields])

    s.set_populations(pops(sets))
    ext_dims = dict(dims)
    key = "ny" if ax == 1 else "nz"
    ext_dims[key] += 2
    x = OracleSim(lattice=kind, **ext_dims, **kw)
    lead = 0  # the last axis is the first array axis
    pads = [1.8, TL["rho_g_liquid"]]
    ext = [np.concatenate([np.full((1,) + shape[1:], pads[k]), sets[k], np.full((1,) + shape[1:], pads[k])], axis=lead)
           for k in range(len(sets))]
    x.set_populations(pops(ext))
    assert np.allclose(s.force(0), x.force(0)[(slice(None), slice(1, -1))], rtol=0, atol=1e-14)
