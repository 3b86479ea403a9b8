"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import numpy as np

from oracle import OracleSim, lattice


def oracle_order(kind, gpu_dirs):
    """Index array mapping the oracle's direction order onto the library's."""
    e, _ = lattice(kind)
    D = 2 if kind == 0 else 3
    return np.array([next(i for i in range(len(e)) if tuple(e[i][:D]) == tuple(v)) for v in gpu_dirs])


def oracle_for(params, nuclei):
    """An oracle run with the same problem definition as a GPU run."""
    keys = ("lattice", "nx", "ny", "nz", "tau", "G", "rho0", "rho_liquid", "rho_gas", "noise_amp", "seed",
            "film_on", "k_own", "zone_width", "rho_th", "psi_bar_mode", "rupture_warmup", "on_rupture",
            "velocity_mode", "refresh_src", "growth_on", "gas_A", "gas_dndt", "gx", "gy", "gz", "g_rho_ref",
            "model", "G_mg", "G_gg", "tau_g", "rho_g_bubble", "rho_g_liquid", "open_z", "rho_res")
    kw = {k: params[k] for k in keys if k in params}
    s = OracleSim(**kw)
    s.set_nuclei(nuclei)
    return s


def max_rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def vel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def active_links(kind, om):
    """The oracle's barrier mask (its direction order) without the links whose
    two ends now have equal alias-root pairs: the links a rupture has removed
    since the refresh, which the library clears from its mask."""
    e, _ = lattice(kind)
    ar = om["alias_root"]
    a, b = ar[om["owner"]], ar[om["owner2"]]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    mask = om["mask"]
    out = np.zeros_like(mask)
    axes = (0, 1, 2) if kind == 1 else (0, 1)
    for j in range(1, len(e)):
        bit = ((mask >> np.uint32(j)) & np.uint32(1)).astype(bool)
        if not bit.any():
            continue
        sh = (-int(e[j][2]), -int(e[j][1]), -int(e[j][0])) if kind == 1 else (-int(e[j][1]), -int(e[j][0]))
        keep = bit & ((np.roll(lo, sh, axes) != lo) | (np.roll(hi, sh, axes) != hi))
        out |= keep.astype(np.uint32) << np.uint32(j)
    return out
