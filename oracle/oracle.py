"""ctypes binding of the FP64 CPU oracle (oracle/foam_oracle.c).

TEST INFRASTRUCTURE: this is the slow reference the GPU library is checked
against; the product path never imports it.
"""
import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FOAM_ORACLE_LIB lets a mutation check load a deliberately broken build of the oracle
_LIBPATH = os.environ.get("FOAM_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None


class _Params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("tau", C.c_double), ("G", C.c_double), ("rho0", C.c_double),
        ("rho_liquid", C.c_double), ("rho_gas", C.c_double), ("noise_amp", C.c_double),
        ("seed", C.c_uint64),
        ("film_on", C.c_int32), ("k_own", C.c_int32), ("zone_width", C.c_int32),
        ("rho_th", C.c_double),
        ("psi_bar_mode", C.c_int32), ("rupture_warmup", C.c_int32),
        ("on_rupture", C.c_int32), ("velocity_mode", C.c_int32),
        ("refresh_src", C.c_int32), ("growth_on", C.c_int32),
        ("gas_A", C.c_double), ("gas_dndt", C.c_double),
        ("gx", C.c_double), ("gy", C.c_double), ("gz", C.c_double), ("g_rho_ref", C.c_double),
        ("model", C.c_int32), ("G_mg", C.c_double), ("G_gg", C.c_double), ("tau_g", C.c_double),
        ("rho_g_bubble", C.c_double), ("rho_g_liquid", C.c_double),
        ("open_z", C.c_int32), ("rho_res", C.c_double),
    ]


DEFAULTS = dict(lattice=0, nx=16, ny=16, nz=1, tau=1.0, G=-5.0, rho0=1.0,
                rho_liquid=2.0, rho_gas=0.15, noise_amp=0.01, seed=1,
                film_on=0, k_own=10, zone_width=6, rho_th=math.log(2.0),
                psi_bar_mode=0, rupture_warmup=200, on_rupture=0, velocity_mode=0,
                refresh_src=0, growth_on=0, gas_A=0.0, gas_dndt=0.0,
                gx=0.0, gy=0.0, gz=0.0, g_rho_ref=0.0,
                model=0, G_mg=0.0, G_gg=0.0, tau_g=1.0, rho_g_bubble=1.0, rho_g_liquid=0.05,
                open_z=0, rho_res=2.0)

_P = C.c_void_p
_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_U = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_L = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from .build_oracle import build
        build()
    lib = C.CDLL(_LIBPATH)
    sig = {
        "or_create": (_P, [C.POINTER(_Params)]),
        "or_destroy": (None, [_P]),
        "or_Q": (C.c_int, [_P]),
        "or_N": (C.c_long, [_P]),
        "or_step_count": (C.c_int64, [_P]),
        "or_stopped": (C.c_int32, [_P]),
        "or_lattice": (None, [C.c_int, _I, _D]),
        "or_set_nuclei": (C.c_int, [_P, _D, C.c_int32]),
        "or_set_populations": (None, [_P, _D]),
        "or_get_populations": (None, [_P, _D]),
        "or_step": (C.c_int, [_P, C.c_int64]),
        "or_density": (None, [_P, _D]),
        "or_velocity": (None, [_P, _D]),
        "or_force": (None, [_P, C.c_int, _D]),
        "or_labels": (C.c_int32, [_P, _I]),
        "or_label_field": (C.c_int32, [_P, _D, _I]),
        "or_owner_dist": (None, [_P, _I, _I, _I, _I]),
        "or_maps": (C.c_int32, [_P, _I, _I, _I, _I, _U, _I]),
        "or_stats": (None, [_P, C.POINTER(C.c_double), _D]),
        "or_n_ruptures": (C.c_int64, [_P]),
        "or_events": (C.c_long, [_P, _L, C.c_long]),
        "or_histogram": (None, [_P, _I, C.c_int32, C.c_int32, C.c_double, _L, _L]),
        "or_p0": (C.c_double, [C.c_double, C.c_double, C.c_double]),
        "or_p_tl": (C.c_double, [C.c_double] * 6),
        "or_density_gas": (None, [_P, _D]),
        "or_gas_points": (C.c_long, [_P, C.c_void_p]),
        "or_pressure": (None, [_P, _D]),
        "or_alias_unite": (C.c_int, [_P, C.c_int32, C.c_int32]),
        "or_foam_stats": (None, [_P, _I, C.c_int32, _D]),
        "or_threads": (C.c_int, []),
        "or_set_threads": (None, [C.c_int]),
        "or_splitmix64": (C.c_uint64, [C.c_uint64]),
        "or_uniform": (C.c_double, [C.c_uint64, C.c_uint64]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def p0(rho, G, rho0=1.0):
    return _load().or_p0(float(rho), float(G), float(rho0))


def p_tl(rho_m, rho_g, G, G_mg, G_gg, rho0=1.0):
    """Two-component bulk pressure of the two-lattice model."""
    return _load().or_p_tl(float(rho_m), float(rho_g), float(G), float(G_mg), float(G_gg), float(rho0))


def splitmix64(x):
    return _load().or_splitmix64(int(x) & 0xFFFFFFFFFFFFFFFF)


def uniform(seed, idx):
    return _load().or_uniform(int(seed), int(idx))


def match_labels(old, new):
    """Overlap of two bubble labellings of one lattice (coalescence tracking
    for the bubble statistics of Sec. 5): for every pair (old bubble a, new
    bubble b) that share at least one cell, (a, b, number of shared cells),
    sorted by (a, b).  Label 0 is liquid.  The definition written out: count
    the cells that are gas in both labellings by their label pair."""
    old = np.asarray(old, np.int64).reshape(-1)
    new = np.asarray(new, np.int64).reshape(-1)
    assert old.shape == new.shape
    both = (old > 0) & (new > 0)
    pairs, counts = np.unique(np.stack([old[both], new[both]], axis=1), axis=0, return_counts=True)
    if pairs.size == 0:
        return np.zeros((0, 3), np.int64)
    return np.concatenate([pairs, counts[:, None]], axis=1).astype(np.int64)


def lattice(kind):
    q = 9 if kind == 0 else 19
    e = np.zeros(3 * q, np.int32)
    w = np.zeros(q, np.float64)
    _load().or_lattice(kind, e, w)
    return e.reshape(q, 3), w


class OracleSim:
    """One lattice advanced by the FP64 oracle.  Arrays are x-fastest."""

    def __init__(self, **params):
        p = dict(DEFAULTS)
        unknown = set(params) - set(p)
        if unknown:
            raise KeyError(f"unknown oracle parameters {sorted(unknown)}")
        p.update(params)
        if p["lattice"] == 0:
            p["nz"] = 1
        self.params = p
        self._lib = _load()
        self._cp = _Params(**{k: p[k] for k, _ in _Params._fields_})
        self._h = self._lib.or_create(C.byref(self._cp))
        if not self._h:
            raise ValueError(f"oracle rejected parameters {p}")
        self.Q = self._lib.or_Q(self._h)
        self.N = self._lib.or_N(self._h)
        self.ncomp = 2 if p["model"] == 1 else 1  # population sets (melt, then gas)
        self.D = 2 if p["lattice"] == 0 else 3
        self.shape = (p["nz"], p["ny"], p["nx"]) if self.D == 3 else (p["ny"], p["nx"])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.or_destroy(h)
            self._h = None

    # -- state --------------------------------------------------------------
    def set_nuclei(self, nuclei):
        arr = np.ascontiguousarray(np.asarray(nuclei, np.float64).reshape(-1, 4))
        if arr.size == 0:
            arr = np.zeros((1, 4), np.float64)
            n = 0
        else:
            n = arr.shape[0]
        if self._lib.or_set_nuclei(self._h, arr.reshape(-1), n) != 0:
            raise MemoryError("oracle: out of host memory")
        return self

    def set_populations(self, f):
        f = np.ascontiguousarray(np.asarray(f, np.float64).reshape(-1))
        assert f.size == self.ncomp * self.Q * self.N
        self._lib.or_set_populations(self._h, f)

    def populations(self):
        """(Q, *shape); with the two-lattice model (2 Q, *shape), the melt's
        populations first."""
        out = np.zeros(self.ncomp * self.Q * self.N, np.float64)
        self._lib.or_get_populations(self._h, out)
        return out.reshape((self.ncomp * self.Q,) + self.shape)

    def step(self, n=1):
        return self._lib.or_step(self._h, int(n))

    @property
    def steps_done(self):
        return self._lib.or_step_count(self._h)

    @property
    def stopped(self):
        return bool(self._lib.or_stopped(self._h))

    # -- queries ------------------------------------------------------------
    def density(self):
        out = np.zeros(self.N, np.float64)
        self._lib.or_density(self._h, out)
        return out.reshape(self.shape)

    def density_gas(self):
        """Two-lattice model: density of the gas lattice."""
        assert self.ncomp == 2
        out = np.zeros(self.N, np.float64)
        self._lib.or_density_gas(self._h, out)
        return out.reshape(self.shape)

    def velocity(self):
        out = np.zeros(self.D * self.N, np.float64)
        self._lib.or_velocity(self._h, out)
        return out.reshape((self.D,) + self.shape)

    def force(self, with_film=None):
        if with_film is None:
            with_film = self.params["film_on"]
        out = np.zeros(3 * self.N, np.float64)
        self._lib.or_force(self._h, int(with_film), out)
        return out.reshape((3,) + self.shape)[: self.D]

    def labels(self):
        out = np.zeros(self.N, np.int32)
        nb = self._lib.or_labels(self._h, out)
        return out.reshape(self.shape), nb

    def label_field(self, rho):
        rho = np.ascontiguousarray(np.asarray(rho, np.float64).reshape(-1))
        out = np.zeros(self.N, np.int32)
        nb = self._lib.or_label_field(self._h, rho, out)
        return out.reshape(self.shape), nb

    def owner_dist(self, labels):
        lab = np.ascontiguousarray(np.asarray(labels, np.int32).reshape(-1))
        owner = np.zeros(self.N, np.int32)
        owner2 = np.zeros(self.N, np.int32)
        dist = np.zeros(self.N, np.int32)
        self._lib.or_owner_dist(self._h, lab, owner, owner2, dist)
        s = self.shape
        return owner.reshape(s), owner2.reshape(s), dist.reshape(s)

    def maps(self):
        label = np.zeros(self.N, np.int32)
        owner = np.zeros(self.N, np.int32)
        owner2 = np.zeros(self.N, np.int32)
        dist = np.zeros(self.N, np.int32)
        mask = np.zeros(self.N, np.uint32)
        alias = np.zeros(self.N + 2, np.int32)
        nb = self._lib.or_maps(self._h, label, owner, owner2, dist, mask, alias)
        s = self.shape
        return dict(label=label.reshape(s), owner=owner.reshape(s), owner2=owner2.reshape(s),
                    dist=dist.reshape(s),
                    mask=mask.reshape(s), alias_root=alias[: nb + 1].copy(), n_bubbles=nb)

    def foam_stats(self, labels, nb):
        """Virtual-metallography statistics of a label field (Sec. 5, Table 5):
        gas fraction, relative foam density, mean and largest equivalent diameter."""
        lab = np.ascontiguousarray(np.asarray(labels, np.int32).reshape(-1))
        out = np.zeros(4, np.float64)
        self._lib.or_foam_stats(self._h, lab, int(nb), out)
        return dict(gas_fraction=out[0], relative_density=out[1], mean_diameter=out[2], max_diameter=out[3])

    def pressure(self):
        """Bulk pressure p0(rho) of the current state (Eq. Pequ)."""
        out = np.zeros(self.N, np.float64)
        self._lib.or_pressure(self._h, out)
        return out.reshape(self.shape)

    def gas_points(self):
        """The domain gas points of the gas-release law (the nucleus cells) and their number N."""
        out = np.zeros(self.N, np.uint8)
        n = self._lib.or_gas_points(self._h, out.ctypes.data_as(C.c_void_p))
        return out.reshape(self.shape).astype(bool), n

    def alias_unite(self, a, b):
        """Test hook: unite the alias classes of labels a and b of the maps in
        force, as a rupture between them would (1 if they were apart)."""
        r = self._lib.or_alias_unite(self._h, int(a), int(b))
        if r < 0:
            raise ValueError("no maps in force, or a label out of range")
        return r

    def stats(self):
        m = C.c_double(0.0)
        mom = np.zeros(3, np.float64)
        self._lib.or_stats(self._h, C.byref(m), mom)
        return m.value, mom

    @property
    def n_ruptures(self):
        return self._lib.or_n_ruptures(self._h)

    def threads(self):
        """OpenMP threads the oracle runs on."""
        return self._lib.or_threads()

    def set_threads(self, n):
        """OpenMP threads for the oracle's later loops (process-wide)."""
        self._lib.or_set_threads(int(n))

    def events(self):
        n = self._lib.or_events(self._h, np.zeros(3, np.int64), 0)
        out = np.zeros(3 * max(n, 1), np.int64)
        self._lib.or_events(self._h, out, n)
        return out[: 3 * n].reshape(n, 3)

    def histogram(self, labels, nb, nbins, bin_width):
        lab = np.ascontiguousarray(np.asarray(labels, np.int32).reshape(-1))
        counts = np.zeros(nbins, np.int64)
        sizes = np.zeros(nb + 1, np.int64)
        self._lib.or_histogram(self._h, lab, int(nb), int(nbins), float(bin_width), counts, sizes)
        return counts, sizes
