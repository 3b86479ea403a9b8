"""Thin ctypes binding of libfoamlbm.so (include/foamlbm.h).

The flb_* functions here have the names and argument order of the C ABI and
only marshal arguments; every step of the method runs in the HIP library.
`Sim` is a convenience wrapper that takes device memory and the stream from
PyTorch.  Importing this module fails loudly when the library is not built.
"""
import ctypes as C
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FOAMLBM_LIB selects another build of the library (e.g. built with other
# compile-time options); the default is the in-tree build
LIBPATH = os.environ.get("FOAMLBM_LIB") or os.path.join(_HERE, "libfoamlbm.so")

FLB_OK, FLB_EINVAL, FLB_ENOMEM, FLB_ENUMERIC, FLB_EBUSY, FLB_EHIP, FLB_STOPPED = 0, -1, -2, -3, -4, -5, 1
FLB_D2Q9, FLB_D3Q19 = 0, 1
FLB_F64, FLB_F32, FLB_F16S = 0, 1, 2
STORAGE = {"f64": FLB_F64, "f32": FLB_F32, "f16s": FLB_F16S}

# direction vectors in the library's population order (lattice coordinates)
DIRECTIONS = {
    FLB_D2Q9: np.array([(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1)]),
    FLB_D3Q19: np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
                         (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1),
                         (1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]),
}


class flb_params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("storage", C.c_int32),
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("tau", C.c_double), ("G", C.c_double), ("rho0", C.c_double),
        ("rho_liquid", C.c_double), ("rho_gas", C.c_double), ("noise_amp", C.c_double),
        ("seed", C.c_uint64),
        ("film_on", C.c_int32), ("k_own", C.c_int32), ("zone_width", C.c_int32),
        ("rho_th", C.c_double),
        ("psi_bar_mode", C.c_int32), ("rupture_warmup", C.c_int32),
        ("on_rupture", C.c_int32), ("velocity_mode", C.c_int32),
        ("rupture_filter", C.c_int32),
        ("refresh_src", C.c_int32), ("growth_on", C.c_int32),
        ("gas_A", C.c_double), ("gas_dndt", C.c_double),
        ("f16_rho_ref", C.c_double),
        ("gx", C.c_double), ("gy", C.c_double), ("gz", C.c_double), ("g_rho_ref", C.c_double),
        ("model", C.c_int32), ("G_mg", C.c_double), ("G_gg", C.c_double), ("tau_g", C.c_double),
        ("rho_g_bubble", C.c_double), ("rho_g_liquid", C.c_double),
        ("open_z", C.c_int32), ("rho_res", C.c_double),
    ]


class flb_nucleus(C.Structure):
    _fields_ = [("x", C.c_double), ("y", C.c_double), ("z", C.c_double), ("r", C.c_double)]


class flb_stats(C.Structure):
    _fields_ = [("mass", C.c_double), ("mom", C.c_double * 3), ("step", C.c_int64),
                ("n_bubbles", C.c_int32), ("n_ruptures", C.c_int32), ("stopped", C.c_int32),
                ("events_lost", C.c_int32)]


class flb_foam_stats(C.Structure):
    _fields_ = [("n_bubbles", C.c_int32), ("gas_cells", C.c_int64), ("gas_fraction", C.c_double),
                ("relative_density", C.c_double), ("mean_diameter", C.c_double), ("max_diameter", C.c_double)]


class flb_server_config(C.Structure):
    _fields_ = [("pool_bytes", C.c_int64), ("max_jobs", C.c_int32), ("chunk_steps", C.c_int32),
                ("graph_steps", C.c_int32), ("max_cells", C.c_int64), ("policy", C.c_int32)]


FLB_JOB_QUEUED, FLB_JOB_RUNNING, FLB_JOB_DONE, FLB_JOB_FAILED, FLB_JOB_CANCELLED = 0, 1, 2, 3, 4
FLB_SERVE_FIFO, FLB_SERVE_SHORTEST = 0, 1

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class flb_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


if not os.path.exists(LIBPATH):
    raise ImportError(f"libfoamlbm.so is not built at {LIBPATH}; run __graft_entry__.build() "
                      "(or python paper_1708_01613_amd/build.py)")
if not os.environ.get("FOAMLBM_LIB"):
    # the in-tree library must have been built from the sources beside it
    from .build import source_hash, stamp_of  # noqa: E402

    _stamp = stamp_of(LIBPATH)
    if _stamp != source_hash():
        raise ImportError(f"{LIBPATH} was built from other sources (stamp {_stamp!r}, sources "
                          f"{source_hash()!r}); rebuild it with __graft_entry__.build()")
# PyTorch ships its own HIP runtime under the same soname: loading torch
# first makes the library bind to that one instance, so device memory and
# streams from torch are valid in the library's calls
import torch  # noqa: E402,F401

_lib = C.CDLL(LIBPATH)

_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_U = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_L = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_CTX = C.c_void_p

_SIGS = {
    "flb_default_params": (None, [C.POINTER(flb_params)]),
    "flb_create": (C.c_int, [C.POINTER(flb_params), C.POINTER(flb_allocator), C.c_void_p, C.POINTER(_CTX)]),
    "flb_set_nuclei": (C.c_int, [_CTX, C.POINTER(flb_nucleus), C.c_int32]),
    "flb_step": (C.c_int, [_CTX, C.c_int64]),
    "flb_get_density": (C.c_int, [_CTX, _D, C.c_size_t]),
    "flb_get_gas_density": (C.c_int, [_CTX, _D, C.c_size_t]),
    "flb_get_velocity": (C.c_int, [_CTX, _D, C.c_size_t]),
    "flb_get_populations": (C.c_int, [_CTX, _D, C.c_size_t]),
    "flb_set_populations": (C.c_int, [_CTX, _D, C.c_size_t]),
    "flb_get_stats": (C.c_int, [_CTX, C.POINTER(flb_stats)]),
    "flb_get_labels": (C.c_int, [_CTX, _I, C.c_size_t, C.POINTER(C.c_int32)]),
    "flb_label_field": (C.c_int, [_CTX, _D, C.c_size_t, _I, C.POINTER(C.c_int32)]),
    "flb_get_maps": (C.c_int, [_CTX, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t]),
    "flb_get_histogram": (C.c_int, [_CTX, C.c_int32, C.c_double, _L, C.POINTER(C.c_int32)]),
    "flb_get_histogram_noalloc": (C.c_int, [_CTX, C.c_int32, C.c_double, _L, C.POINTER(C.c_int32)]),
    "flb_get_foam_stats": (C.c_int, [_CTX, C.POINTER(flb_foam_stats)]),
    "flb_match_labels": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_int64, C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int32)]),
    "flb_get_rupture_events": (C.c_int, [_CTX, C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]),
    "flb_set_tuning": (C.c_int, [_CTX, C.c_int32, C.c_int32, C.c_int32]),
    "flb_get_tuning": (C.c_int, [_CTX] + [C.POINTER(C.c_int32)] * 6),
    "flb_autotune": (C.c_int, [_CTX, C.c_int32, C.POINTER(C.c_double)]),
    "flb_save": (C.c_int, [_CTX, C.c_char_p]),
    "flb_load": (C.c_int, [_CTX, C.c_char_p]),
    "flb_import_maps": (C.c_int, [_CTX, _I, _I, _I, _I, C.c_size_t, C.c_void_p, C.c_int32]),
    "flb_time_steps": (C.c_int, [_CTX, C.c_int64, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "flb_time_phases": (C.c_int, [_CTX, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "flb_copy_bandwidth": (C.c_int, [C.POINTER(flb_allocator), C.c_void_p, C.c_int64, C.c_int32,
                                     C.POINTER(C.c_double)]),
    "flb_get_pressure": (C.c_int, [_CTX, _D, C.c_size_t]),
    "flb_get_gas_points": (C.c_int, [_CTX, C.c_void_p, C.c_size_t, C.POINTER(C.c_int64)]),
    "flb_destroy": (None, [_CTX]),
    "flb_last_error": (C.c_char_p, []),
    "flb_batch_create": (C.c_int, [C.POINTER(flb_params), C.c_int32, C.POINTER(flb_allocator), C.c_void_p,
                                   C.POINTER(C.c_void_p)]),
    "flb_batch_size": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "flb_batch_member": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(_CTX)]),
    "flb_batch_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "flb_batch_set_tuning": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int32, C.c_int32]),
    "flb_batch_get_tuning": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "flb_batch_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    "flb_batch_set_persistent": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "flb_batch_time_steps": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_double)]),
    "flb_batch_destroy": (None, [C.c_void_p]),
    "flb_server_default_config": (None, [C.POINTER(flb_server_config)]),
    "flb_server_create": (C.c_int, [C.POINTER(flb_server_config), C.POINTER(flb_allocator), C.c_void_p,
                                    C.POINTER(C.c_void_p)]),
    "flb_server_submit": (C.c_int, [C.c_void_p, C.POINTER(flb_params), C.POINTER(flb_nucleus), C.c_int32,
                                    C.c_int64, C.POINTER(C.c_int64)]),
    "flb_server_pump": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "flb_server_job": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "flb_server_result": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_size_t, C.POINTER(flb_stats)]),
    "flb_server_release": (C.c_int, [C.c_void_p, C.c_int64]),
    "flb_server_cancel": (C.c_int, [C.c_void_p, C.c_int64]),
    "flb_server_usage": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "flb_server_destroy": (None, [C.c_void_p]),
}
EXPORTED = tuple(_SIGS)
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
    globals()[_name] = _fn


class FlbError(RuntimeError):
    def __init__(self, code, what):
        msg = flb_last_error().decode(errors="replace")
        super().__init__(f"{what} failed with {code}: {msg}")
        self.code = code


def check(code, what):
    if code < 0:
        raise FlbError(code, what)
    return code


def default_params(**kw):
    p = flb_params()
    flb_default_params(C.byref(p))
    for k, v in kw.items():
        if k == "storage" and isinstance(v, str):
            v = STORAGE[v]
        if not hasattr(p, k):
            raise KeyError(f"unknown parameter {k}")
        setattr(p, k, v)
    if p.lattice == FLB_D2Q9:
        p.nz = 1
    return p


def _torch_allocator(device_index, stream):
    """Device memory from PyTorch's caching allocator, tagged with the stream
    the library enqueues its work on (so a block is reused only in that
    stream's order)."""

    def _alloc(nbytes, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device_index, stream)
        except Exception as exc:  # the library reports FLB_ENOMEM; say why
            print(f"foamlbm: device allocation of {int(nbytes)} bytes failed: {exc}", file=sys.stderr, flush=True)
            return None

    def _free(ptr, user):
        torch.cuda.caching_allocator_delete(ptr)

    fa, ff = ALLOC_FN(_alloc), FREE_FN(_free)
    return flb_allocator(fa, ff, None), (fa, ff)


class Sim:
    """One lattice on the GPU.  Arrays are x-fastest: (ny, nx) or (nz, ny, nx)."""

    def __init__(self, stream=None, use_torch_memory=True, **params):
        import torch

        self.params = default_params(**params)
        p = self.params
        self.D = 2 if p.lattice == FLB_D2Q9 else 3
        self.Q = 9 if self.D == 2 else 19
        self.N = p.nx * p.ny * p.nz
        self.shape = (p.ny, p.nx) if self.D == 2 else (p.nz, p.ny, p.nx)
        self.ncomp = 2 if p.model == 1 else 1  # population sets: the melt's, then the gas's
        dev = torch.cuda.current_device()
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._keep = None
        alloc = None
        if use_torch_memory:
            al, self._keep = _torch_allocator(dev, self.stream)
            alloc = C.byref(al)
            self._al = al
        h = _CTX()
        check(flb_create(C.byref(p), alloc, C.c_void_p(self.stream.cuda_stream), C.byref(h)), "flb_create")
        self.h = h

    @classmethod
    def _member(cls, handle, params, owner):
        """A borrowed view of a batch member (the batch owns the context)."""
        self = cls.__new__(cls)
        self.params = params
        p = params
        self.D = 2 if p.lattice == FLB_D2Q9 else 3
        self.Q = 9 if self.D == 2 else 19
        self.N = p.nx * p.ny * p.nz
        self.shape = (p.ny, p.nx) if self.D == 2 else (p.nz, p.ny, p.nx)
        self.ncomp = 1
        self.stream = owner.stream
        self._owner = owner
        self.h = handle
        return self

    def close(self):
        if getattr(self, "_owner", None) is not None:
            self.h = None  # owned by its batch
            return
        if getattr(self, "h", None) is not None and self.h.value:
            flb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_nuclei(self, nuclei):
        arr = np.asarray(nuclei, np.float64).reshape(-1, 4)
        n = arr.shape[0]
        buf = (flb_nucleus * max(n, 1))()
        for k in range(n):
            buf[k] = flb_nucleus(*arr[k])
        check(flb_set_nuclei(self.h, buf, n), "flb_set_nuclei")
        return self

    def step(self, n=1):
        return check(flb_step(self.h, int(n)), "flb_step")

    def density(self):
        out = np.empty(self.N, np.float64)
        check(flb_get_density(self.h, out, out.size), "flb_get_density")
        return out.reshape(self.shape)

    def velocity(self):
        out = np.empty(self.D * self.N, np.float64)
        check(flb_get_velocity(self.h, out, out.size), "flb_get_velocity")
        return out.reshape((self.D,) + self.shape)

    def gas_density(self):
        """Two-lattice model: density of the gas lattice."""
        out = np.empty(self.N, np.float64)
        check(flb_get_gas_density(self.h, out, out.size), "flb_get_gas_density")
        return out.reshape(self.shape)

    def populations(self):
        out = np.empty(self.ncomp * self.Q * self.N, np.float64)
        check(flb_get_populations(self.h, out, out.size), "flb_get_populations")
        return out.reshape((self.ncomp * self.Q,) + self.shape)

    def set_populations(self, f):
        f = np.ascontiguousarray(np.asarray(f, np.float64).reshape(-1))
        check(flb_set_populations(self.h, f, f.size), "flb_set_populations")

    def labels(self):
        out = np.empty(self.N, np.int32)
        nb = C.c_int32(0)
        check(flb_get_labels(self.h, out, out.size, C.byref(nb)), "flb_get_labels")
        return out.reshape(self.shape), nb.value

    def label_field(self, rho):
        rho = np.ascontiguousarray(np.asarray(rho, np.float64).reshape(-1))
        out = np.empty(self.N, np.int32)
        nb = C.c_int32(0)
        check(flb_label_field(self.h, rho, rho.size, out, C.byref(nb)), "flb_label_field")
        return out.reshape(self.shape), nb.value

    def maps(self):
        arrs = {k: np.empty(self.N, np.int32) for k in ("label", "owner", "owner2", "dist")}
        mask = np.empty(self.N, np.uint32)
        ptr = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
        check(flb_get_maps(self.h, ptr(arrs["label"]), ptr(arrs["owner"]), ptr(arrs["owner2"]),
                           ptr(arrs["dist"]), ptr(mask), self.N), "flb_get_maps")
        out = {k: v.reshape(self.shape) for k, v in arrs.items()}
        out["mask"] = mask.reshape(self.shape)
        return out

    def histogram(self, nbins, bin_width):
        counts = np.empty(nbins, np.int64)
        nb = C.c_int32(0)
        check(flb_get_histogram(self.h, nbins, float(bin_width), counts, C.byref(nb)), "flb_get_histogram")
        return counts, nb.value

    def foam_stats(self):
        """Virtual-metallography statistics of the current labels (Sec. 5, Table 5)."""
        s = flb_foam_stats()
        check(flb_get_foam_stats(self.h, C.byref(s)), "flb_get_foam_stats")
        return dict(n_bubbles=s.n_bubbles, gas_cells=s.gas_cells, gas_fraction=s.gas_fraction,
                    relative_density=s.relative_density, mean_diameter=s.mean_diameter,
                    max_diameter=s.max_diameter)

    def match_labels(self, old_labels):
        """(old label, current label, shared cells) for every pair of bubbles of an
        earlier labelling and the current one that overlap, sorted; and the
        current bubble count."""
        old = np.ascontiguousarray(np.asarray(old_labels, np.int32).reshape(-1))
        n, nb = C.c_int64(0), C.c_int32(0)
        check(flb_match_labels(self.h, old.ctypes.data_as(C.c_void_p), old.size, None, 0, C.byref(n), C.byref(nb)),
              "flb_match_labels")
        out = np.zeros(3 * max(n.value, 1), np.int64)
        check(flb_match_labels(self.h, old.ctypes.data_as(C.c_void_p), old.size, out.ctypes.data_as(C.c_void_p),
                               n.value, C.byref(n), C.byref(nb)), "flb_match_labels")
        return out[: 3 * n.value].reshape(-1, 3), nb.value

    def rupture_events(self):
        n = C.c_int64(0)
        check(flb_get_rupture_events(self.h, None, 0, C.byref(n)), "flb_get_rupture_events")
        out = np.zeros(3 * max(n.value, 1), np.int64)
        check(flb_get_rupture_events(self.h, out.ctypes.data_as(C.c_void_p), n.value, C.byref(n)),
              "flb_get_rupture_events")
        return out[: 3 * min(n.value, out.size // 3)].reshape(-1, 3)

    def set_tuning(self, tile=-1, lz=0, xcd=-1):
        check(flb_set_tuning(self.h, tile, lz, xcd), "flb_set_tuning")

    def tuning(self):
        v = [C.c_int32(0) for _ in range(6)]
        check(flb_get_tuning(self.h, *[C.byref(x) for x in v]), "flb_get_tuning")
        return dict(zip(("tile", "lz", "xcd", "n_tiles", "tile_x", "tile_m"), (x.value for x in v)))

    def save(self, path):
        check(flb_save(self.h, os.fsencode(path)), "flb_save")

    def load(self, path):
        check(flb_load(self.h, os.fsencode(path)), "flb_load")

    def import_maps(self, label, owner, owner2, dist, n_bubbles, alias_root=None):
        arrs = [np.ascontiguousarray(np.asarray(a, np.int32).reshape(-1)) for a in (label, owner, owner2, dist)]
        ar = None if alias_root is None else np.ascontiguousarray(np.asarray(alias_root, np.int32).reshape(-1))
        check(flb_import_maps(self.h, *arrs, arrs[0].size, None if ar is None else ar.ctypes.data_as(C.c_void_p),
                              int(n_bubbles)), "flb_import_maps")

    def autotune(self, reps=5):
        """Pick the fastest step-kernel variant for this lattice (state unchanged)."""
        ms = C.c_double(0.0)
        check(flb_autotune(self.h, int(reps), C.byref(ms)), "flb_autotune")
        return ms.value

    def pressure(self):
        """Bulk pressure p0(rho) of the current state (Eq. Pequ), FP64."""
        out = np.empty(self.N, np.float64)
        check(flb_get_pressure(self.h, out, out.size), "flb_get_pressure")
        return out.reshape(self.shape)

    def gas_points(self):
        """Domain gas points of the gas-release source (bool array) and their number."""
        out = np.empty(self.N, np.uint8)
        n = C.c_int64(0)
        check(flb_get_gas_points(self.h, out.ctypes.data_as(C.c_void_p), out.size, C.byref(n)),
              "flb_get_gas_points")
        return out.reshape(self.shape).astype(bool), n.value

    def time_phases(self, n):
        """n steps timed per phase: (total ms, {refresh, step, rupture, finish} ms sums)."""
        ms = C.c_double(0.0)
        ph = (C.c_double * 4)()
        check(flb_time_phases(self.h, int(n), C.byref(ms), ph), "flb_time_phases")
        return ms.value, dict(zip(("refresh", "step", "rupture", "finish"), list(ph)))

    def time_steps(self, n, refresh=True, kernel=False):
        """Milliseconds for n steps; with kernel=True, (total, step-kernel sum)."""
        ms = C.c_double(0.0)
        kms = C.c_double(0.0)
        check(flb_time_steps(self.h, int(n), int(bool(refresh)), C.byref(ms), C.byref(kms) if kernel else None),
              "flb_time_steps")
        return (ms.value, kms.value) if kernel else ms.value

    def stats(self):
        s = flb_stats()
        check(flb_get_stats(self.h, C.byref(s)), "flb_get_stats")
        return dict(mass=s.mass, mom=np.array(list(s.mom)), step=s.step, n_bubbles=s.n_bubbles,
                    n_ruptures=s.n_ruptures, stopped=bool(s.stopped), events_lost=s.events_lost)


def copy_bandwidth(nbytes=1 << 30, reps=10, stream=None):
    """Read + write GB/s of the library's 16-byte-per-lane device copy of
    nbytes (the practical HBM ceiling of the step kernel)."""
    dev = torch.cuda.current_device()
    stream = stream if stream is not None else torch.cuda.current_stream(dev)
    al, keep = _torch_allocator(dev, stream)
    gbs = C.c_double(0.0)
    check(flb_copy_bandwidth(C.byref(al), C.c_void_p(stream.cuda_stream), int(nbytes), int(reps), C.byref(gbs)),
          "flb_copy_bandwidth")
    del keep
    return gbs.value


class Batch:
    """Many lattices of one lattice type and storage advanced together
    (batched launches, replayed from captured HIP graphs).  `members` is a
    list of parameter dicts; `batch.members[k]` is a Sim view of member k."""

    def __init__(self, members, stream=None, use_torch_memory=True):
        import torch

        plist = [default_params(**m) for m in members]
        n = len(plist)
        arr = (flb_params * n)(*plist)
        dev = torch.cuda.current_device()
        # a stream of its own (default priority): graphs cannot be captured on
        # the null stream
        self.stream = stream if stream is not None else torch.cuda.Stream(dev)
        self._keep = None
        alloc = None
        if use_torch_memory:
            al, self._keep = _torch_allocator(dev, self.stream)
            alloc = C.byref(al)
            self._al = al
        h = C.c_void_p()
        check(flb_batch_create(arr, n, alloc, C.c_void_p(self.stream.cuda_stream), C.byref(h)), "flb_batch_create")
        self.h = h
        self.members = []
        for k in range(n):
            mh = _CTX()
            check(flb_batch_member(self.h, k, C.byref(mh)), "flb_batch_member")
            self.members.append(Sim._member(mh, plist[k], self))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            for m in self.members:
                m.h = None
            flb_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return len(self.members)

    def step(self, n=1):
        return check(flb_batch_step(self.h, int(n)), "flb_batch_step")

    def set_tuning(self, tile=-1, target=0, xcd=-1, graph_steps=-1):
        check(flb_batch_set_tuning(self.h, tile, target, xcd, graph_steps), "flb_batch_set_tuning")

    def set_persistent(self, on=True, max_steps=0):
        check(flb_batch_set_persistent(self.h, 1 if on else 0, int(max_steps)), "flb_batch_set_persistent")

    def tuning(self):
        t, x, g, nt = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        tg = C.c_int64()
        check(flb_batch_get_tuning(self.h, C.byref(t), C.byref(tg), C.byref(x), C.byref(g), C.byref(nt)),
              "flb_batch_get_tuning")
        return dict(tile=t.value, target=tg.value, xcd=x.value, graph_steps=g.value, n_tiles=nt.value)

    def autotune(self, reps=5):
        ms = C.c_double(0.0)
        check(flb_batch_autotune(self.h, int(reps), C.byref(ms)), "flb_batch_autotune")
        return ms.value

    def time_steps(self, n):
        ms = C.c_double(0.0)
        check(flb_batch_time_steps(self.h, int(n), C.byref(ms)), "flb_batch_time_steps")
        return ms.value

    def synchronize(self):
        self.stream.synchronize()


def _nuclei_array(nuclei):
    arr = np.asarray(nuclei, np.float64).reshape(-1, 4)
    buf = (flb_nucleus * max(arr.shape[0], 1))()
    for k in range(arr.shape[0]):
        buf[k] = flb_nucleus(*arr[k])
    return buf, arr.shape[0]


class Server:
    """Resident foam jobs advanced together (continuous batching): submit()
    queues a job, pump() runs one scheduling round, result() returns the final
    density and statistics of a finished job."""

    def __init__(self, pool_bytes=None, max_jobs=None, chunk_steps=None, graph_steps=None, max_cells=None,
                 policy=None, stream=None, use_torch_memory=True):
        import torch

        cfg = flb_server_config()
        flb_server_default_config(C.byref(cfg))
        for k, v in (("pool_bytes", pool_bytes), ("max_jobs", max_jobs), ("chunk_steps", chunk_steps),
                     ("graph_steps", graph_steps), ("max_cells", max_cells), ("policy", policy)):
            if v is not None:
                setattr(cfg, k, int(v))
        self.cfg = cfg
        dev = torch.cuda.current_device()
        self.stream = stream if stream is not None else torch.cuda.Stream(dev)
        self._keep = None
        alloc = None
        if use_torch_memory:
            al, self._keep = _torch_allocator(dev, self.stream)
            alloc = C.byref(al)
            self._al = al
        h = C.c_void_p()
        check(flb_server_create(C.byref(cfg), alloc, C.c_void_p(self.stream.cuda_stream), C.byref(h)),
              "flb_server_create")
        self.h = h
        self._shape = {}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            flb_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, steps, nuclei, **params):
        p = default_params(**params)
        buf, n = _nuclei_array(nuclei)
        jid = C.c_int64()
        check(flb_server_submit(self.h, C.byref(p), buf, n, int(steps), C.byref(jid)), "flb_server_submit")
        self._shape[jid.value] = (p.ny, p.nx) if p.lattice == FLB_D2Q9 else (p.nz, p.ny, p.nx)
        return jid.value

    def pump(self):
        r, q, d = C.c_int32(), C.c_int32(), C.c_int64()
        check(flb_server_pump(self.h, C.byref(r), C.byref(q), C.byref(d)), "flb_server_pump")
        return r.value, q.value, d.value

    def state(self, jid):
        st, done = C.c_int32(), C.c_int64()
        check(flb_server_job(self.h, int(jid), C.byref(st), C.byref(done)), "flb_server_job")
        return st.value, done.value

    def result(self, jid):
        shape = self._shape[jid]
        out = np.empty(int(np.prod(shape)), np.float64)
        s = flb_stats()
        check(flb_server_result(self.h, int(jid), out.ctypes.data_as(C.c_void_p), out.size, C.byref(s)),
              "flb_server_result")
        return out.reshape(shape), dict(mass=s.mass, step=s.step, n_bubbles=s.n_bubbles, n_ruptures=s.n_ruptures)

    def release(self, jid):
        check(flb_server_release(self.h, int(jid)), "flb_server_release")
        self._shape.pop(jid, None)

    def cancel(self, jid):
        check(flb_server_cancel(self.h, int(jid)), "flb_server_cancel")

    def usage(self):
        u, p = C.c_int64(), C.c_int64()
        check(flb_server_usage(self.h, C.byref(u), C.byref(p)), "flb_server_usage")
        return u.value, p.value
