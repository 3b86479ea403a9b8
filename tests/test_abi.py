"""The C ABI library loads, exports every function include/foamlbm.h declares,
and rejects invalid arguments before touching a device (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "foamlbm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(flb_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("flb_create", "flb_set_nuclei", "flb_step", "flb_get_density", "flb_get_velocity",
                 "flb_get_labels", "flb_destroy", "flb_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1708_01613_amd import foamlbm

    out = subprocess.run(["nm", "-D", "--defined-only", foamlbm.LIBPATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (flb_[a-z_0-9]+)$", out, flags=re.M))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    # the binding wraps every exported function under the same name
    assert set(_declared()) <= set(foamlbm.EXPORTED)


def test_params_default_and_validation_without_device():
    from paper_1708_01613_amd import foamlbm as F

    p = F.default_params()
    assert (p.lattice, p.storage, p.nx, p.ny, p.nz) == (0, 1, 64, 64, 1)
    assert abs(p.rho_th - 0.6931471805599453) < 1e-16 and p.k_own == 10 and p.zone_width == 6
    assert p.rupture_filter == 1
    h = C.c_void_p()
    bad = [dict(tau=0.5), dict(lattice=2), dict(nx=0), dict(zone_width=16), dict(k_own=0),
           dict(storage=3), dict(rho0=0.0), dict(psi_bar_mode=2), dict(rupture_filter=2)]
    for kw in bad:
        q = F.default_params(**kw)
        rc = F.flb_create(C.byref(q), None, None, C.byref(h))
        assert rc == F.FLB_EINVAL, kw
        assert F.flb_last_error()
        assert not h.value
    q = F.default_params(lattice=0)
    q.nz = 2
    assert F.flb_create(C.byref(q), None, None, C.byref(h)) == F.FLB_EINVAL
    assert F.flb_create(None, None, None, C.byref(h)) == F.FLB_EINVAL
    F.flb_destroy(None)


def test_null_context_is_rejected():
    from paper_1708_01613_amd import foamlbm as F

    assert F.flb_step(None, 1) == F.FLB_EINVAL
    assert F.flb_set_nuclei(None, None, 0) == F.FLB_EINVAL
    assert F.flb_set_tuning(None, 0, 0, 0) == F.FLB_EINVAL
