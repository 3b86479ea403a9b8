"""Persistent batch runs (D2Q9): one cooperative launch per stretch of steps
between film-map refreshes, with grid-wide barriers between the step tiles,
the rupture test, the mask pruning and the finishers of each step (marked
gpu).  Every member must equal its solo run bit for bit in populations, maps,
events and step counts, as it does under per-step launches; the FP64 totals
are summed in another order and agree to rounding."""
import sys

import numpy as np
import pytest

from .test_gpu_batch import _members_2d, _solo

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def flb():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1708_01613_amd import foamlbm

    return foamlbm


def _say(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


def _members(storage, stop):
    members = _members_2d(storage)
    for k, (p, _) in enumerate(members):
        if k % 3 == 0:
            p.update(growth_on=1, gas_A=1.0 + k, gas_dndt=0.01)
        if k == 3:
            p.update(gx=1e-5, gy=-2e-5, g_rho_ref=1.5)
    if stop:
        # film members stop after their first rupture
        for p, _ in members:
            if p["film_on"]:
                p.update(on_rupture=1)
    return members


def _check_member(m, s, p):
    assert np.array_equal(m.populations(), s.populations())
    sm, ss = m.stats(), s.stats()
    assert sm["step"] == ss["step"]
    assert sm["stopped"] == ss["stopped"]
    assert sm["n_ruptures"] == ss["n_ruptures"]
    assert abs(sm["mass"] - ss["mass"]) <= 1e-12 * abs(ss["mass"])
    assert np.abs(sm["mom"] - ss["mom"]).max() <= 1e-12 * abs(ss["mass"])
    if p["film_on"]:
        gm, sm_ = m.maps(), s.maps()
        for key in ("label", "owner", "dist", "mask"):
            assert np.array_equal(gm[key], sm_[key]), key
        assert {tuple(r) for r in m.rupture_events().tolist()} == {tuple(r) for r in s.rupture_events().tolist()}
    return ss


@pytest.mark.parametrize("max_steps", [0, 7])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
def test_persistent_members_match_solo_runs(flb, storage, max_steps):
    members = _members(storage, stop=max_steps == 7)
    _say(f"persistent batch of {len(members)} D2Q9 {storage}, max_steps {max_steps}")
    b = flb.Batch([p for p, _ in members])
    b.set_persistent(True, max_steps)
    assert b.tuning()["tile"] == 2
    for k, (_, nuc) in enumerate(members):
        b.members[k].set_nuclei(nuc)
    steps = 83
    b.step(steps)
    b.synchronize()
    any_rupture = stopped = False
    for k, (p, nuc) in enumerate(members):
        _say(f"member {k}")
        ss = _check_member(b.members[k], _solo(flb, p, nuc, steps), p)
        any_rupture |= p["film_on"] and ss["n_ruptures"] > 0
        stopped |= ss["stopped"]
    assert any_rupture and stopped == (max_steps == 7)


def test_persistent_and_graph_runs_interleave(flb):
    # switching between persistent runs and graph replay mid-run, with an
    # autotune in between, keeps every member on its solo trajectory
    members = _members("f32", stop=False)
    _say("persistent / graph interleave, D2Q9 f32")
    b = flb.Batch([p for p, _ in members])
    for k, (_, nuc) in enumerate(members):
        b.members[k].set_nuclei(nuc)
    b.set_persistent(True, 5)
    b.step(21)
    b.set_persistent(False)
    b.step(19)
    b.set_persistent(True)
    assert b.autotune(reps=2) > 0
    assert b.tuning()["tile"] == 2
    b.step(23)
    b.synchronize()
    for k, (p, nuc) in enumerate(members):
        _check_member(b.members[k], _solo(flb, p, nuc, 63), p)


def test_persistent_rejections(flb):
    _say("persistent rejections")
    p2 = dict(lattice=0, storage="f32", nx=32, ny=32)
    b = flb.Batch([p2, p2])
    b.set_persistent(True)
    with pytest.raises(flb.FlbError):
        b.set_tuning(tile=0)
    b.set_persistent(False)
    b.set_tuning(tile=0)
    b.close()
    p3 = dict(lattice=1, storage="f32", nx=16, ny=16, nz=16)
    b3 = flb.Batch([p3])
    with pytest.raises(flb.FlbError):
        b3.set_persistent(True)
    b3.close()
