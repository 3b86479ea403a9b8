"""Pins of the oracle's two-lattice model (melt and gas lattices coupled
every step, Sec. 2.1.5 and Fig. Mainflowchart "Domain coupling").

Each test checks the oracle against something other than itself: the
single-lattice oracle on a case the two-lattice model must reduce to, the
conservation laws of the coupling, the mechanical equilibrium of a flat
interface (which fixes the relative weights of the force terms and of the
equation of state), mirror symmetry of a film between two bubbles, and the
behaviour the film model exists for.
"""
import numpy as np
import pytest

from oracle.oracle import OracleSim, lattice

TL = dict(model=1, G=-5.0, G_mg=0.5, G_gg=0.0, rho_g_bubble=0.5, rho_g_liquid=0.05)


def _random_state(kind, shape, seed, scale=0.02):
    """Positive populations near rest equilibria of random densities, with
    random momenta: a state far from any steady state."""
    e, w = lattice(kind)
    rng = np.random.default_rng(seed)
    out = []
    for rho0 in (1.5, 0.3):
        rho = rho0 * (1.0 + 0.2 * rng.random(shape))
        f = w.reshape((-1,) + (1,) * len(shape)) * rho[None]
        out.append(f * (1.0 + scale * rng.standard_normal(f.shape)))
    return np.concatenate(out)


@pytest.mark.parametrize("kind,nx,ny,nz", [(0, 9, 7, 1), (1, 5, 4, 3)])
def test_without_forces_the_sum_is_one_lattice(kind, nx, ny, nz):
    # G = G_mg = G_gg = 0 and one relaxation time: each lattice relaxes to the
    # equilibrium of its own density at the common velocity, and equilibria
    # are linear in the density, so f_m + f_g steps exactly like one lattice
    # of the summed density (Sec. 2.1.1 collision and streaming)
    kw = dict(lattice=kind, nx=nx, ny=ny, nz=nz, tau=0.8, G=0.0)
    s2 = OracleSim(**kw, model=1, G_mg=0.0, G_gg=0.0, tau_g=0.8)
    shape = s2.shape
    f = _random_state(kind, shape, 4)
    s2.set_populations(f)
    s1 = OracleSim(**kw)
    s1.set_populations(f[: s1.Q] + f[s1.Q:])
    s1.step(25)
    s2.step(25)
    g = s2.populations()
    assert np.allclose(g[: s1.Q] + g[s1.Q:], s1.populations(), rtol=0, atol=1e-13)


@pytest.mark.parametrize("taus", [(1.0, 1.0), (0.7, 1.3)])
def test_momentum_and_component_masses_conserved(taus):
    # the Shan-Chen pair forces cancel over the lattice (the cross terms act
    # on both lattices with the same coupling), and the common velocity
    # weights each lattice's momentum by 1 / tau, so the collisions of the
    # two lattices together change no momentum even with unequal relaxation
    # times; streaming moves populations only
    tau, tau_g = taus
    s = OracleSim(lattice=0, nx=11, ny=9, tau=tau, tau_g=tau_g, **TL)
    s.set_populations(_random_state(0, s.shape, 7))
    m0 = (s.density().sum(), s.density_gas().sum())
    _, p0 = s.stats()
    s.step(40)
    _, p1 = s.stats()
    assert abs(s.density().sum() - m0[0]) < 1e-12 * m0[0]
    assert abs(s.density_gas().sum() - m0[1]) < 1e-12 * m0[1]
    assert np.all(np.abs(p1 - p0) < 1e-12 * (m0[0] + m0[1]))
    # and the momentum does change per lattice: the coupling exchanges it
    assert np.abs(s.velocity()).max() > 1e-4


def test_flat_interface_bulk_pressures_balance():
    # a gas slab in melt on an odd periodic lattice (odd, so no staggered
    # mode): at rest, the momentum balance across each interface leaves the
    # bulk pressures of melt and slab equal.  The two-component equation of
    # state (rho_m + rho_g)/3 + (G psi_m^2 + 2 G_mg psi_m psi_g + G_gg
    # psi_g^2)/6 is the one the pair forces integrate to, so any other weight
    # of a term (the cross term once instead of twice, say) leaves a gap
    e, w = lattice(0)
    nx, ny = 65, 3
    s = OracleSim(lattice=0, nx=nx, ny=ny, tau_g=0.8, noise_amp=0.0, **TL)
    rm = np.full((ny, nx), 2.0)
    rg = np.full((ny, nx), 0.05)
    rm[:, 16:49] = 0.1
    rg[:, 16:49] = 0.5
    s.set_populations(np.concatenate([w[:, None, None] * rm[None], w[:, None, None] * rg[None]]))
    s.step(8000)
    p = s.pressure()
    assert abs(p[1, 32] - p[1, 0]) < 1e-6 * p[1, 0]
    # the slab is a genuine second phase of the gas lattice
    assert s.density_gas()[1, 32] > 5 * s.density_gas()[1, 0]


def test_one_bubble_film_is_exact_noop():
    runs = []
    for film in (0, 1):
        s = OracleSim(lattice=0, nx=48, ny=48, film_on=film, k_own=1, seed=2, **TL)
        s.set_nuclei([[24, 24, 0, 8]])
        s.step(120)
        runs.append(s.populations())
    assert np.array_equal(runs[0], runs[1])


def _two_bubbles(film, warmup, steps, every=100, nx=95, **kw):
    R, gap = 14.0, 2.0
    c = (nx - 1) / 2.0
    s = OracleSim(lattice=0, nx=nx, ny=64, film_on=film, rupture_warmup=warmup, zone_width=6, k_own=1,
                  noise_amp=0.0, **TL, **kw)
    s.set_nuclei([[c - R - gap / 2 - 0.5, 32, 0, R], [c + R + gap / 2 + 0.5, 32, 0, R]])
    nbs = []
    for _ in range(steps // every):
        if s.step(every):
            break
        nbs.append(s.labels()[1])
    return s, nbs


def test_film_between_mirror_bubbles_is_mirror_symmetric():
    # two equal bubbles placed symmetrically about x = (nx - 1) / 2: with the
    # barrier active, the substitution on the links x -> x + e_i and on their
    # opposites must keep the melt and gas fields mirror images
    s, nbs = _two_bubbles(1, 10 ** 9, 200)
    assert nbs[-1] == 2 and s.maps()["mask"].any()
    for f in (s.density(), s.density_gas()):
        assert np.allclose(f, f[:, ::-1], rtol=0, atol=1e-11)
    u = s.velocity()
    assert np.allclose(u[0], -u[0][:, ::-1], rtol=0, atol=1e-11)


@pytest.mark.slow
def test_two_bubble_film_behaves_as_the_single_lattice_reading():
    # the behaviour the film model exists for, as in the single-lattice
    # reading: without the barrier the bubbles merge, with it they stay apart,
    # and once the test runs the first crossing unites them and they merge
    _, nbs = _two_bubbles(0, 0, 800)
    assert nbs[-1] == 1
    s, nbs = _two_bubbles(1, 10 ** 9, 1200)
    assert all(n == 2 for n in nbs) and s.n_ruptures == 0
    s, nbs = _two_bubbles(1, 50, 800)
    ev = s.events()
    assert len(ev) > 0 and ev[0][0] == 50 and tuple(ev[0][1:]) == (1, 2)
    assert s.n_ruptures == 1 and nbs[-1] == 1


def test_rejects_bad_two_lattice_parameters():
    # (the gas release goes to the gas lattice; a body force is not part of the model)
    for bad in (dict(gx=1e-5), dict(tau_g=0.5), dict(rho_g_liquid=0.0), dict(rho_g_bubble=-1.0)):
        with pytest.raises(ValueError):
            OracleSim(lattice=0, nx=8, ny=8, **dict(TL, **bad))
