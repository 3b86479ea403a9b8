"""Pins of the oracle's bubble-growth source: the gas-release law of
Sec. 2.1.3 (dp/dt = A (dn/dt) / N at each of the N domain gas points; the
"Bubble growth" box of Fig. Mainflowchart).  Reading R25: the domain gas
points are the cells of the nuclei, fixed at nucleation; the pressure
increment of a step is taken as the ideal-gas density increment
drho = dp / c_s^2 = 3 A (dn/dt) / N, added isotropically (w_i drho to
population i) after the collision.
"""
import numpy as np
import pytest

from oracle import OracleSim, lattice

NUC2 = [[10.5, 12.0, 0, 5.0], [30.0, 22.0, 0, 6.5], [47.0, 3.0, 0, 4.0]]
NUC3 = [[4.0, 5.0, 6.0, 3.0], [12.5, 3.0, 1.0, 2.5]]


def _sim(kind, growth, A=1.5, dndt=0.02, **kw):
    dims = dict(nx=48, ny=32) if kind == 0 else dict(nx=16, ny=14, nz=12)
    s = OracleSim(lattice=kind, G=-5.5, rho_liquid=2.3, rho_gas=0.11, growth_on=growth, gas_A=A, gas_dndt=dndt,
                  seed=4, **dims, **kw)
    s.set_nuclei(NUC2 if kind == 0 else NUC3)
    return s


@pytest.mark.parametrize("kind", [0, 1])
def test_gas_points_are_the_nucleus_cells(kind):
    s = _sim(kind, 1, noise_amp=0.0)
    pts, n = s.gas_points()
    assert n == int(pts.sum()) > 0
    assert np.array_equal(pts, s.density() < 1.0)  # the initial gas cells, noise off


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("film", [0, 1])
def test_mass_grows_by_the_released_amount(kind, film):
    # every step adds A (dn/dt) / N of pressure at N points: 3 A (dn/dt) of mass
    A, dndt, steps = 1.5, 0.02, 60
    s = _sim(kind, 1, A, dndt, film_on=film, k_own=5, rupture_warmup=20)
    m0, _ = s.stats()
    s.step(steps)
    m1, _ = s.stats()
    assert abs((m1 - m0) - steps * 3 * A * dndt) <= 1e-13 * m0
    # and without the source the mass is conserved
    s0 = _sim(kind, 0, A, dndt, film_on=film, k_own=5, rupture_warmup=20)
    s0.step(steps)
    assert abs(s0.stats()[0] - m0) <= steps * 2.0 ** -52 * m0


@pytest.mark.parametrize("kind", [0, 1])
def test_one_step_increment_closed_form(kind):
    # From one state, one step with and one without the source: the source
    # cell c adds w_i drho to f_i, which streams to c + e_i, so the density
    # difference is drho * sum_i w_i [c + e_i is reached from a gas point],
    # and the momentum difference is drho * sum_i w_i e_i = 0.
    A, dndt = 2.0, 0.01
    on, off = _sim(kind, 1, A, dndt), _sim(kind, 0, A, dndt)
    pts, n = on.gas_points()
    drho = 3 * A * dndt / n
    on.step(1)
    off.step(1)
    e, w = lattice(kind)
    D = 2 if kind == 0 else 3
    inc = np.zeros(pts.shape)
    for i in range(len(w)):
        shift = tuple(int(e[i][k]) for k in reversed(range(D)))
        inc += w[i] * np.roll(pts.astype(float), shift, tuple(range(D)))
    assert np.abs((on.density() - off.density()) - drho * inc).max() <= 1e-15
    _, p_on = on.stats()
    _, p_off = off.stats()
    assert np.abs(p_on - p_off).max() <= 1e-13


def test_source_off_when_no_gas_points():
    s = OracleSim(lattice=0, nx=20, ny=20, growth_on=1, gas_A=1.0, gas_dndt=0.1)
    s.set_nuclei([])
    m0, _ = s.stats()
    s.step(10)
    assert s.gas_points()[1] == 0 and abs(s.stats()[0] - m0) <= 1e-12 * m0
