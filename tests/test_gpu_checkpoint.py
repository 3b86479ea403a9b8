"""Checkpoint / resume and imported film maps (runs on an MI355X; marked gpu)."""
import numpy as np
import pytest

from .gpu_helpers import oracle_for, oracle_order

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def flb():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1708_01613_amd import foamlbm

    return foamlbm


def _two_bubbles(storage, **kw):
    R, gap = 14.0, 2.0
    p = dict(lattice=0, storage=storage, nx=96, ny=64, G=-5.5, rho_liquid=2.3, rho_gas=0.11, film_on=1,
             rupture_warmup=20, zone_width=6, k_own=4, seed=3)
    p.update(kw)
    print(f"\n[case] {p}", flush=True)
    return p, [[48 - R - gap / 2 - 0.5, 32, 0, R], [48 + R + gap / 2 + 0.5, 32, 0, R]]


def _snapshot(s):
    st = s.stats()
    return (s.populations(), sorted(map(tuple, s.rupture_events().tolist())), st["step"], st["n_ruptures"],
            st["n_bubbles"], s.maps())


def _assert_same(a, b):
    assert np.array_equal(a[0], b[0])
    assert a[1:5] == b[1:5]
    for k in a[5]:
        assert np.array_equal(a[5][k], b[5][k]), k


@pytest.mark.parametrize("storage,save_at", [("f32", 37), ("f16s", 42), ("f64", 13)])
def test_resume_is_exact(flb, tmp_path, storage, save_at):
    # saved mid refresh cycle and, for odd steps, from the second buffer;
    # the resumed run must reproduce the uninterrupted one bit for bit,
    # ruptures (warmup at step 20, unions after it) included
    p, nuc = _two_bubbles(storage)
    a = flb.Sim(**p)
    a.set_nuclei(nuc)
    a.step(save_at)
    path = tmp_path / "a.ckpt"
    a.save(path)
    a.step(150)
    ref = _snapshot(a)
    assert ref[3] > 0, "the case must rupture"
    b = flb.Sim(**p)
    b.set_nuclei([[10.0, 10.0, 0, 5.0]])  # a different state, overwritten by the load
    b.step(3)
    b.load(path)
    assert b.stats()["step"] == save_at
    b.step(150)
    _assert_same(_snapshot(b), ref)
    # rewinding a context to its own earlier state
    a.load(path)
    a.step(150)
    _assert_same(_snapshot(a), ref)


def test_resume_without_film(flb, tmp_path):
    p, nuc = _two_bubbles("f32", film_on=0)
    a = flb.Sim(**p)
    a.set_nuclei(nuc)
    a.step(9)
    a.save(tmp_path / "n.ckpt")
    a.step(20)
    b = flb.Sim(**p)
    b.load(tmp_path / "n.ckpt")
    b.step(20)
    assert np.array_equal(a.populations(), b.populations())


def test_load_rejects_other_parameters(flb, tmp_path):
    p, nuc = _two_bubbles("f32")
    a = flb.Sim(**p)
    a.set_nuclei(nuc)
    a.step(2)
    a.save(tmp_path / "c.ckpt")
    for change in ({"G": -5.0}, {"storage": "f64"}, {"nx": 97}):
        b = flb.Sim(**dict(p, **change))
        with pytest.raises(flb.FlbError):
            b.load(tmp_path / "c.ckpt")
    with pytest.raises(flb.FlbError):
        a.load(tmp_path / "missing.ckpt")
    (tmp_path / "junk.ckpt").write_bytes(b"not a checkpoint at all" * 10)
    with pytest.raises(flb.FlbError):
        a.load(tmp_path / "junk.ckpt")
    # a failed load leaves the context usable
    a.step(1)
    assert a.stats()["step"] == 3


def test_imported_oracle_maps_give_oracle_masks(flb):
    # film maps computed by the oracle, imported: the library's barrier masks
    # built from them equal the oracle's, cell by cell and link by link
    p, nuc = _two_bubbles("f64", k_own=4, rupture_warmup=10 ** 6)
    o = oracle_for(p, nuc)
    o.step(41)
    om = o.maps()
    g = flb.Sim(**p)
    g.set_nuclei(nuc)
    nb = int(om["label"].max())
    g.import_maps(om["label"], om["owner"], om["owner2"], om["dist"], nb)
    gm = g.maps()
    for key in ("label", "owner", "owner2", "dist"):
        assert np.array_equal(gm[key], om[key]), key
    order = oracle_order(0, flb.DIRECTIONS[0])
    omask = np.zeros_like(gm["mask"])
    for i, j in enumerate(order):
        omask |= ((om["mask"] >> np.uint32(j)) & np.uint32(1)) << np.uint32(i)
    assert np.count_nonzero(omask) > 0
    assert np.array_equal(gm["mask"], omask)
    assert g.stats()["n_bubbles"] == nb


def test_imported_aliases_remove_links(flb):
    # with both bubbles' labels aliased to one root no link is a barrier
    p, nuc = _two_bubbles("f64", k_own=4, rupture_warmup=10 ** 6)
    g = flb.Sim(**p)
    g.set_nuclei(nuc)
    g.step(5)
    m = g.maps()
    nb = int(m["label"].max())
    assert nb == 2 and np.count_nonzero(m["mask"]) > 0
    g.import_maps(m["label"], m["owner"], m["owner2"], m["dist"], nb)
    assert np.array_equal(g.maps()["mask"], m["mask"])
    g.import_maps(m["label"], m["owner"], m["owner2"], m["dist"], nb, alias_root=[0, 1, 1])
    assert np.count_nonzero(g.maps()["mask"]) == 0


def test_import_rejects_inconsistent_maps(flb):
    p, nuc = _two_bubbles("f32")
    g = flb.Sim(**p)
    g.set_nuclei(nuc)
    g.step(1)
    m = g.maps()
    nb = int(m["label"].max())
    bad_dist = m["dist"].copy()
    bad_dist[m["dist"] >= 0] = p["zone_width"]
    bad_owner = m["owner"].copy()
    bad_owner[0, 0] = nb + 5
    for args in ((m["label"], m["owner"], m["owner2"], bad_dist, nb),
                 (m["label"], bad_owner, m["owner2"], m["dist"], nb),
                 (m["label"], m["owner"], m["owner2"], m["dist"], -1)):
        with pytest.raises(flb.FlbError):
            g.import_maps(*args)
    with pytest.raises(flb.FlbError):
        g.import_maps(m["label"], m["owner"], m["owner2"], m["dist"], nb, alias_root=[0, 2, 1])
