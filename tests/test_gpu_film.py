"""The two-bubble film workload (Sec. 4: Table 2, Fig. 7, Fig. plot) and the
foam statistics of Sec. 5 (Table 5) on the GPU against the FP64 oracle
(marked gpu).  The workload module samples the library's queries; the oracle
is given the same query names by a small view, so both runs are sampled by
the same code."""
import sys

import numpy as np
import pytest

from .gpu_helpers import oracle_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def flb():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1708_01613_amd import foamlbm

    return foamlbm


class OracleView:
    """The oracle under the query names of the binding's Sim."""

    def __init__(self, o):
        self.o = o

    def step(self, n):
        self.o.step(n)

    def density(self):
        return self.o.density()

    def pressure(self):
        return self.o.pressure()

    def velocity(self):
        return self.o.velocity()

    def labels(self):
        return self.o.labels()

    def rupture_events(self):
        return self.o.events()

    def foam_stats(self):
        lab, nb = self.o.labels()
        st = self.o.foam_stats(lab, nb)
        return dict(st, n_bubbles=nb, gas_cells=int((lab > 0).sum()))


def _say(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


def _film_params(n):
    return dict(lattice=0, storage="f64", nx=n, ny=n, G=-5.5, rho_liquid=2.0, rho_gas=0.15, film_on=1, k_own=2,
                zone_width=6, rupture_warmup=60, seed=7)


def test_two_bubble_film_workload_matches_oracle(flb):
    from paper_1708_01613_amd import film

    n, nuc = film.table2_geometry(gap=2.0, cells_per_mm=2)
    p = _film_params(n)
    _say(f"two-bubble film {n}^2, R {nuc[0][3]}")
    g = flb.Sim(**p)
    g.set_nuclei(nuc)
    o = OracleView(oracle_for(p, nuc))
    rg, sg = film.run(g, nuc, 400, 25)
    ro, so = film.run(o, nuc, 400, 25)
    assert len(rg) == len(ro)
    for a, b in zip(rg, ro):
        assert a["step"] == b["step"] and a["n_bubbles"] == b["n_bubbles"] and a["events"] == b["events"]
        assert a["first_event_step"] == b["first_event_step"]
        for key in ("line_pressure", "centres_density"):
            assert np.abs(a[key] - b[key]).max() <= 1e-11 * np.abs(b[key]).max(), (a["step"], key)
        umax = max(np.abs(b["line_velocity"]).max(), 1e-300)
        assert np.abs(a["line_velocity"] - b["line_velocity"]).max() <= 1e-10 * umax, a["step"]
        assert a["foam"]["gas_cells"] == b["foam"]["gas_cells"] and a["foam"]["n_bubbles"] == b["foam"]["n_bubbles"]
        assert abs(a["foam"]["mean_diameter"] - b["foam"]["mean_diameter"]) <= 1e-12 * b["foam"]["mean_diameter"]
    assert sg["rupture_step"] == so["rupture_step"] is not None
    assert sg["merged_by_step"] == so["merged_by_step"]
    assert sg["probe_sign_changes_before_rupture"] == so["probe_sign_changes_before_rupture"]
    assert sg["profile_before"] is not None and sg["profile_after"] is not None


@pytest.mark.parametrize("kind", [0, 1])
def test_foam_stats_match_oracle(flb, kind):
    rng = np.random.default_rng(21 + kind)
    if kind == 0:
        p = dict(lattice=0, storage="f64", nx=150, ny=110, G=-5.5, rho_liquid=2.0, rho_gas=0.15, seed=3)
        nuc = [[float(rng.uniform(0, 150)), float(rng.uniform(0, 110)), 0.0, float(rng.uniform(4, 9))]
               for _ in range(14)]
    else:
        p = dict(lattice=1, storage="f64", nx=40, ny=34, nz=30, G=-5.5, rho_liquid=2.0, rho_gas=0.15, seed=3)
        nuc = [[float(rng.uniform(0, 40)), float(rng.uniform(0, 34)), float(rng.uniform(0, 30)),
                float(rng.uniform(3, 6))] for _ in range(8)]
    _say(f"foam stats lattice {kind}")
    g = flb.Sim(**p)
    g.set_nuclei(nuc)
    o = oracle_for(p, nuc)
    g.step(40)
    o.step(40)
    gs = g.foam_stats()
    lab, nb = o.labels()
    os_ = o.foam_stats(lab, nb)
    assert gs["n_bubbles"] == nb >= 2 and gs["gas_cells"] == int((lab > 0).sum())
    assert gs["gas_fraction"] == os_["gas_fraction"] and gs["relative_density"] == os_["relative_density"]
    assert abs(gs["mean_diameter"] - os_["mean_diameter"]) <= 1e-13 * os_["mean_diameter"]
    assert abs(gs["max_diameter"] - os_["max_diameter"]) <= 1e-14 * os_["max_diameter"]
