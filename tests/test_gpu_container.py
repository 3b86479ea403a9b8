"""GPU against the FP64 oracle on the container open for the liquid (Sec. 5:
open planes across the last axis facing a liquid reservoir) and on the gas
release into the gas lattice of the two-lattice model (Sec. 2.1.3 with Sec.
2.1.5): densities, velocity, totals (no longer conserved), pressure, film
maps and rupture events, D2Q9 and D3Q19, FP64 and FP32 storage.
"""
import math
import sys

import numpy as np
import pytest

from .gpu_helpers import active_links, max_rel, oracle_for, oracle_order, vel_err

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def flb():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1708_01613_amd import foamlbm

    return foamlbm


def _case(kind, storage, model, **kw):
    p = dict(lattice=kind, storage=storage, tau=1.0, rho_th=math.log(2.0), noise_amp=0.01, film_on=1, k_own=3,
             zone_width=6, rupture_warmup=30, velocity_mode=1, seed=5, open_z=1)
    if model == 0:
        p.update(G=-5.5, rho_liquid=2.3 if kind == 0 else 2.0, rho_gas=0.11)
        p.update(rho_res=p["rho_liquid"])
    else:
        p.update(model=1, G=-5.0, rho_liquid=2.0, rho_gas=0.15, G_mg=0.3, tau_g=0.9, rho_g_bubble=0.4,
                 rho_g_liquid=0.05, rho_res=2.0, growth_on=1, gas_A=1.0, gas_dndt=0.05)
    if kind == 0:
        p.update(nx=72, ny=44, nz=1)
        nuc = [[20.0, 22.0, 0, 9.0], [40.5, 22.0, 0, 9.0], [60.0, 8.0, 0, 5.0]]
        steps = 90
    else:
        p.update(nx=32, ny=24, nz=22)
        nuc = [[7.5, 12.0, 11.0, 6.0], [24.5, 12.0, 11.0, 6.0], [28.0, 4.0, 4.0, 3.5]]
        steps = 50
    p.update(kw)
    print(f"\n[case] {p}", flush=True)
    sys.stdout.flush()
    return p, nuc, steps


@pytest.mark.parametrize("model", [0, 1])
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("kind", [0, 1])
def test_open_container_parity(flb, kind, storage, model):
    p, nuc, steps = _case(kind, storage, model)
    g = flb.Sim(**p)
    g.set_nuclei(nuc)
    o = oracle_for(p, nuc)
    m_start = o.stats()[0]
    g.step(steps)
    o.step(steps)
    tol = TOL[storage]
    assert max_rel(g.density(), o.density()) <= tol
    if model == 1:
        assert max_rel(g.gas_density(), o.density_gas()) <= tol
    assert vel_err(g.velocity(), o.velocity()) <= tol
    st = g.stats()
    m, mom = o.stats()
    assert abs(m - m_start) > 1e3 * tol * m  # mass did cross the open planes
    assert abs(st["mass"] - m) <= tol * m
    assert np.abs(st["mom"] - mom).max() <= tol * m
    # the pressure is a difference of terms of the size of the density
    assert np.abs(g.pressure() - o.pressure()).max() <= tol * o.density().max()
    gm, om = g.maps(), o.maps()
    for key in ("label", "owner", "owner2", "dist"):
        assert np.array_equal(gm[key], om[key]), key
    order = oracle_order(kind, flb.DIRECTIONS[kind])
    oa = active_links(kind, om)
    omask = np.zeros_like(gm["mask"])
    for i, j in enumerate(order):
        omask |= ((oa >> np.uint32(j)) & np.uint32(1)) << np.uint32(i)
    assert np.array_equal(gm["mask"], omask)
    ge = {tuple(r) for r in g.rupture_events().tolist()}
    oe = {tuple(r) for r in o.events().tolist()}
    assert ge == oe
    assert st["n_ruptures"] == o.n_ruptures


def test_open_container_state_round_trip(flb):
    # populations written back into an open container come back unchanged
    # (the reservoir enters only when a step streams)
    p, nuc, _ = _case(0, "f64", 0)
    g = flb.Sim(**p)
    g.set_nuclei(nuc)
    g.step(5)
    f = g.populations()
    g.set_populations(f)
    assert np.array_equal(g.populations(), f)


def test_open_container_rejected_in_batches(flb):
    p, _, _ = _case(0, "f32", 0)
    with pytest.raises(RuntimeError):
        flb.Batch([p, p])


def test_growth_in_container_ruptures_at_the_oracles_step(flb):
    # the validation case of Sec. 5 in lattice units: two bubbles growing in
    # a container open for the liquid reach the rupture criterion; FP64 on
    # the GPU takes the first event at the oracle's step, with the same pair
    nx, ny, R, gap = 128, 96, 10.0, 16.0
    c = (nx - 1) / 2
    p = dict(lattice=0, storage="f64", nx=nx, ny=ny, nz=1, tau=1.0, G=-5.0, rho_liquid=2.0, rho_gas=0.15,
             noise_amp=0.0, model=1, G_mg=0.3, tau_g=1.0, rho_g_bubble=0.4, rho_g_liquid=0.05, growth_on=1,
             gas_A=1.0, gas_dndt=0.1, open_z=1, rho_res=2.0, film_on=1, rupture_warmup=20, k_own=5, zone_width=6)
    nuc = [[c - R - gap / 2 - 0.5, ny / 2, 0, R], [c + R + gap / 2 + 0.5, ny / 2, 0, R]]
    print(f"\n[case] {p}", flush=True)
    g = flb.Sim(**p)
    g.set_nuclei(nuc)
    o = oracle_for(p, nuc)
    first = None
    for _ in range(12):
        g.step(50)
        o.step(50)
        oe = o.events()
        if len(oe):
            first = oe
            break
    assert first is not None and first[0][0] > 20
    ge = g.rupture_events()
    assert {tuple(r) for r in ge.tolist()} == {tuple(r) for r in first.tolist()}
    assert max_rel(g.gas_density(), o.density_gas()) <= 1e-11
