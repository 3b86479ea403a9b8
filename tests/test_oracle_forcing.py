"""Pins of the oracle's body force: the forcing term of Sec. 2.1.1 for gravity,
read as He's term F_i = w_i rho' [(e_i - u).g / c_s^2 + (e_i.u)(e_i.g) / c_s^4]
with rho' = rho - g_rho_ref and u the velocity of the equilibrium (R29; the
printed term lacks the e_i of its second part and one power of c_s^2).
It adds rho' g of momentum and no mass per cell and step.
"""
import numpy as np
import pytest

from oracle import OracleSim, lattice

G3 = (2e-4, -3e-4, 1.5e-4)


def _uniform(kind, rho, g, rho_ref):
    dims = dict(nx=6, ny=5, nz=1) if kind == 0 else dict(nx=4, ny=5, nz=3)
    s = OracleSim(lattice=kind, G=-5.0, noise_amp=0.0, rho_liquid=rho, gx=g[0], gy=g[1],
                  gz=g[2] if kind == 1 else 0.0, g_rho_ref=rho_ref, **dims)
    s.set_nuclei([])
    return s


@pytest.mark.parametrize("rho_ref", [0.0, 0.7])
@pytest.mark.parametrize("kind", [0, 1])
def test_uniform_fluid_two_steps_closed_form(kind, rho_ref):
    # a uniform fluid feels no interaction force; with tau = 1 the state after
    # one step is w_i rho (1 + 3 e_i.a), a = (rho'/rho) g, and after two it is
    # the equilibrium at velocity a plus F_i evaluated at u = a
    rho = 1.3
    g = np.array(G3 if kind == 1 else (G3[0], G3[1], 0.0))
    s = _uniform(kind, rho, g, rho_ref)
    e, w = lattice(kind)
    rb = rho - rho_ref
    a = rb / rho * g
    s.step(1)
    f1 = s.populations().reshape(len(w), -1)
    ref1 = w * rho * (1 + 3 * (e @ a))
    assert np.abs(f1 - ref1[:, None]).max() < 1e-15
    s.step(1)
    f2 = s.populations().reshape(len(w), -1)
    ea, eg = e @ a, e @ g
    feq = w * rho * (1 + 3 * ea + 4.5 * ea ** 2 - 1.5 * (a @ a))
    F = w * rb * (3 * (eg - a @ g) + 9 * ea * eg)
    assert np.abs(f2 - (feq + F)[:, None]).max() < 1e-15


@pytest.mark.parametrize("kind", [0, 1])
def test_momentum_grows_by_the_body_force(kind):
    # film off, several bubbles: the interaction forces cancel pairwise, so
    # the total momentum gains (M - N rho_ref) g per step; with rho_ref the
    # mean density it is conserved (the buoyancy form for periodic boxes)
    dims = dict(nx=48, ny=40, nz=1) if kind == 0 else dict(nx=18, ny=16, nz=14)
    nuc = [[10, 12, 0, 6], [30, 25, 0, 8]] if kind == 0 else [[5, 5, 5, 4], [12, 10, 8, 3.5]]
    g = np.array(G3 if kind == 1 else (G3[0], G3[1], 0.0))
    N = dims["nx"] * dims["ny"] * dims["nz"]
    for mode in ("plain", "buoyancy"):
        s0 = OracleSim(lattice=kind, G=-5.5, rho_liquid=2.3, rho_gas=0.11, seed=5, **dims)
        s0.set_nuclei(nuc)
        M, P0 = s0.stats()
        ref = 0.0 if mode == "plain" else M / N
        s = OracleSim(lattice=kind, G=-5.5, rho_liquid=2.3, rho_gas=0.11, seed=5, gx=g[0], gy=g[1],
                      gz=g[2] if kind == 1 else 0.0, g_rho_ref=ref, **dims)
        s.set_nuclei(nuc)
        n = 60
        s.step(n)
        m, P = s.stats()
        # no mass added: a mass term of the force would move it by ~1e-6 M per
        # step here; what remains is the rounding of the moving equilibrium
        assert abs(m - M) <= 1e-13 * n * M
        expect = P0 + n * (M - N * ref) * g
        assert np.abs(P - expect).max() <= 1e-12 * M, (mode, P, expect)
