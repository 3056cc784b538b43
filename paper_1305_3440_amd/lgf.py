"""ctypes binding of the C ABI in include/lgf.h (argument marshalling only).

Every function keeps its C name and arguments; numpy arrays stand for host
pointers, and a torch tensor may be passed as a borrowed device buffer and a
torch stream as the handle's stream.  All arithmetic happens in the gfx950
library ``liblgf.so``; importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblgf.so")

LGF_OK, LGF_EINVAL, LGF_ENOMEM, LGF_EHIP, LGF_ENOTCONV, LGF_ENUMERIC, LGF_ESTATE = range(7)
STATUS_NAMES = {0: "LGF_OK", 1: "LGF_EINVAL", 2: "LGF_ENOMEM", 3: "LGF_EHIP", 4: "LGF_ENOTCONV",
                5: "LGF_ENUMERIC", 6: "LGF_ESTATE"}
LGF_FP64_18, LGF_FP32_18, LGF_FP32_12, LGF_FP64_12, LGF_FP64_12S = range(5)
FORMAT_NAMES = {0: "fp64-18", 1: "fp32-18", 2: "fp32-12", 3: "fp64-12", 4: "fp64-12s"}
LINK_BYTES = {0: 144, 1: 72, 2: 48, 3: 96}


class lgf_fix_params(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("p_sr", ctypes.c_double),
                ("theta_target", ctypes.c_double), ("theta_switch", ctypes.c_double),
                ("bulk_format", ctypes.c_int), ("check_every", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("finish_format", ctypes.c_int),
                ("accumulate_g", ctypes.c_int), ("separate_measure", ctypes.c_int),
                ("fixed_links", ctypes.c_int), ("max_sweeps", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("sweep_offset", ctypes.c_uint64)]


class lgf_fix_result(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("sweeps_bulk", ctypes.c_int64),
                ("theta", ctypes.c_double), ("F", ctypes.c_double), ("status", ctypes.c_int),
                ("n_history", ctypes.c_int), ("t_total_ms", ctypes.c_double),
                ("t_sweep_bulk_ms", ctypes.c_double), ("t_sweep_finish_ms", ctypes.c_double),
                ("t_measure_ms", ctypes.c_double), ("t_convert_ms", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class LgfError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


EXPORTS = [
    "lgf_last_error", "lgf_version", "lgf_fix_params_default", "lgf_required_bytes", "lgf_create",
    "lgf_destroy", "lgf_get_info", "lgf_load_links", "lgf_store_links", "lgf_peek_links",
    "lgf_generate_links", "lgf_convert", "lgf_sweep", "lgf_reunitarize", "lgf_measure",
    "lgf_gauge_fix", "lgf_synchronize", "lgf_set_tuning", "lgf_get_tuning", "lgf_autotune",
    "lgf_time_sweeps", "lgf_copy_bandwidth", "lgf_set_fixed_tuning", "lgf_get_fixed_tuning",
    "lgf_autotune_fixed", "lgf_fix_begin", "lgf_fix_chunk", "lgf_fix_end", "lgf_anneal_sweep", "lgf_anneal",
    "lgf_measure_noalloc",
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblgf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1305_3440_amd.build`")
    # PyTorch brings its own HIP runtime and puts it in the global symbol
    # scope.  liblgf.so must bind every HIP call to that same runtime, or the
    # torch streams and device buffers handed across the boundary belong to
    # another runtime than the library's kernels: import torch before the
    # library is loaded (its HIP symbols then all resolve to torch's runtime).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, I, I64, U64, D, SZ = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                             ctypes.c_double, ctypes.c_size_t)
    sig = {
        "lgf_last_error": (ctypes.c_char_p, []),
        "lgf_version": (ctypes.c_char_p, []),
        "lgf_fix_params_default": (I, [P]),
        "lgf_required_bytes": (SZ, [P, I]),
        "lgf_create": (I, [P, I, P, P, SZ, P]),
        "lgf_destroy": (I, [P]),
        "lgf_get_info": (I, [P, P, P]),
        "lgf_load_links": (I, [P, P, SZ]),
        "lgf_store_links": (I, [P, P, SZ]),
        "lgf_peek_links": (I, [P, P, I64, P]),
        "lgf_generate_links": (I, [P, U64, D, I]),
        "lgf_convert": (I, [P, I]),
        "lgf_sweep": (I, [P, I, D, D, U64, U64]),
        "lgf_reunitarize": (I, [P]),
        "lgf_measure": (I, [P, P, P]),
        "lgf_gauge_fix": (I, [P, P, P, P, I]),
        "lgf_synchronize": (I, [P]),
        "lgf_set_tuning": (I, [P, I, P]),
        "lgf_get_tuning": (I, [P, I, P]),
        "lgf_set_fixed_tuning": (I, [P, I, P]),
        "lgf_get_fixed_tuning": (I, [P, I, P]),
        "lgf_autotune_fixed": (I, [P, I, I]),
        "lgf_autotune": (I, [P, I, I]),
        "lgf_time_sweeps": (I, [P, I, D, D, U64, U64, P]),
        "lgf_copy_bandwidth": (I, [SZ, I, P, P]),
        "lgf_fix_begin": (I, [P, I]),
        "lgf_fix_chunk": (I, [P, I, D, D, U64, U64, I, P, P, P]),
        "lgf_fix_end": (I, [P]),
        "lgf_anneal_sweep": (I, [P, I, D, U64, U64, P]),
        "lgf_anneal": (I, [P, I64, D, D, U64, U64, P, P]),
        "lgf_measure_noalloc": (I, [P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, allow=()):
    if status != LGF_OK and status not in allow:
        raise LgfError(status, lgf_last_error())
    return status


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(dims):
    return np.ascontiguousarray(np.asarray(dims, dtype=np.int32).reshape(4))


def _canon(U: np.ndarray) -> np.ndarray:
    if U.dtype != np.complex128 or not U.flags.c_contiguous or U.shape[1:] != (4, 3, 3):
        raise ValueError("links must be a C-contiguous complex128 array of shape (V, 4, 3, 3)")
    return U


# ------------------------------------------------------------------ entry points

def lgf_last_error() -> str:
    return load_library().lgf_last_error().decode()


def lgf_version() -> str:
    return load_library().lgf_version().decode()


def lgf_fix_params_default() -> lgf_fix_params:
    p = lgf_fix_params()
    _check(load_library().lgf_fix_params_default(ctypes.byref(p)))
    return p


def lgf_required_bytes(dims, fmt: int) -> int:
    return int(load_library().lgf_required_bytes(_p(_dims(dims)), fmt))


def _ptr_of(obj):
    if obj is None:
        return None
    if isinstance(obj, int):
        return obj
    if hasattr(obj, "data_ptr"):        # torch tensor
        return obj.data_ptr()
    if hasattr(obj, "cuda_stream"):     # torch stream
        return obj.cuda_stream
    raise TypeError(f"cannot take a device pointer of {type(obj)}")


def lgf_create(dims, fmt: int = LGF_FP64_18, stream=None, device_buf=None, buf_bytes: int = 0):
    """Returns the opaque handle (a c_void_p)."""
    h = ctypes.c_void_p()
    if device_buf is not None and hasattr(device_buf, "numel") and not buf_bytes:
        buf_bytes = device_buf.numel() * device_buf.element_size()
    _check(load_library().lgf_create(_p(_dims(dims)), fmt, _ptr_of(stream), _ptr_of(device_buf),
                                     buf_bytes, ctypes.byref(h)))
    return h


def lgf_destroy(h) -> None:
    _check(load_library().lgf_destroy(h))


def lgf_get_info(h):
    d = np.zeros(4, dtype=np.int32)
    f = ctypes.c_int()
    _check(load_library().lgf_get_info(h, _p(d), ctypes.byref(f)))
    return tuple(int(x) for x in d), int(f.value)


def lgf_load_links(h, U: np.ndarray) -> None:
    _canon(U)
    _check(load_library().lgf_load_links(h, _p(U), U.size * 2))


def lgf_store_links(h, V: int) -> np.ndarray:
    U = np.empty((V, 4, 3, 3), dtype=np.complex128)
    _check(load_library().lgf_store_links(h, _p(U), U.size * 2))
    return U


def lgf_peek_links(h, sites) -> np.ndarray:
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64).reshape(-1))
    out = np.empty((s.size, 4, 3, 3), dtype=np.complex128)
    _check(load_library().lgf_peek_links(h, _p(s), s.size, _p(out)))
    return out


def lgf_generate_links(h, seed: int, eps: float, haar: bool = True) -> None:
    _check(load_library().lgf_generate_links(h, seed, eps, int(haar)))


def lgf_convert(h, fmt: int) -> None:
    _check(load_library().lgf_convert(h, fmt))


def lgf_sweep(h, parity: int, omega: float, p_sr: float = 0.0, seed: int = 0,
              sweep_index: int = 0) -> None:
    _check(load_library().lgf_sweep(h, parity, omega, p_sr, seed, sweep_index))


def lgf_reunitarize(h) -> None:
    _check(load_library().lgf_reunitarize(h))


def lgf_measure(h):
    F = ctypes.c_double()
    th = ctypes.c_double()
    _check(load_library().lgf_measure(h, ctypes.byref(F), ctypes.byref(th)))
    return F.value, th.value


def lgf_gauge_fix(h, params: lgf_fix_params, history_cap: int = 4096):
    """Returns (status, result dict, history array of (sweeps, F, theta))."""
    res = lgf_fix_result()
    hist = np.zeros((max(history_cap, 1), 3))
    st = load_library().lgf_gauge_fix(h, ctypes.byref(params), ctypes.byref(res), _p(hist),
                                      history_cap)
    _check(st, allow=(LGF_ENOTCONV, LGF_ENUMERIC))
    return st, res.as_dict(), hist[: res.n_history].copy()


def lgf_synchronize(h) -> None:
    _check(load_library().lgf_synchronize(h))


class lgf_sweep_tuning(ctypes.Structure):
    _fields_ = [("lanes_per_site", ctypes.c_int), ("sites_per_thread", ctypes.c_int), ("block", ctypes.c_int),
                ("xcd_remap", ctypes.c_int), ("nontemporal", ctypes.c_int), ("schedule", ctypes.c_int)]


TUNING_FIELDS = ("lanes_per_site", "block", "xcd_remap", "nontemporal", "schedule", "sites_per_thread")


def lgf_set_tuning(h, fmt: int, lanes_per_site: int, block: int, xcd_remap: int = 0,
                   nontemporal: int = 1, schedule: int = 0, sites_per_thread: int = 1) -> None:
    t = lgf_sweep_tuning(lanes_per_site=lanes_per_site, sites_per_thread=sites_per_thread, block=block,
                         xcd_remap=xcd_remap, nontemporal=nontemporal, schedule=schedule)
    _check(load_library().lgf_set_tuning(h, fmt, ctypes.byref(t)))


def lgf_get_tuning(h, fmt: int):
    """(lanes_per_site, block, xcd_remap, nontemporal, schedule, sites_per_thread)"""
    t = lgf_sweep_tuning()
    _check(load_library().lgf_get_tuning(h, fmt, ctypes.byref(t)))
    return tuple(getattr(t, k) for k in TUNING_FIELDS)


def lgf_set_fixed_tuning(h, fmt: int, lanes_per_site: int = 2, block: int = 128, xcd_remap: int = 0,
                         layout: int = 0) -> None:
    """xcd_remap is the tile order (0..3), layout the link layout (0 the
    link field, 1 per-site link records) of the fixed-link sweep"""
    t = lgf_sweep_tuning(lanes_per_site=lanes_per_site, sites_per_thread=1, block=block, xcd_remap=xcd_remap,
                         nontemporal=1, schedule=layout)
    _check(load_library().lgf_set_fixed_tuning(h, fmt, ctypes.byref(t)))


def lgf_get_fixed_tuning(h, fmt: int):
    """(lanes_per_site, block, tile order, link layout) of the fixed-link sweep"""
    t = lgf_sweep_tuning()
    _check(load_library().lgf_get_fixed_tuning(h, fmt, ctypes.byref(t)))
    return (t.lanes_per_site, t.block, t.xcd_remap, t.schedule)


def lgf_autotune_fixed(h, fmt: int, trials: int = 4) -> None:
    _check(load_library().lgf_autotune_fixed(h, fmt, trials))


def lgf_autotune(h, fmt: int, trials: int = 4) -> None:
    _check(load_library().lgf_autotune(h, fmt, trials))


def lgf_time_sweeps(h, n: int, omega: float, p_sr: float = 0.0, seed: int = 0,
                    sweep_index: int = 0) -> float:
    ms = ctypes.c_double()
    _check(load_library().lgf_time_sweeps(h, n, omega, p_sr, seed, sweep_index, ctypes.byref(ms)))
    return ms.value


def lgf_measure_noalloc(h, d_out) -> None:
    """d_out: device buffer (e.g. a torch tensor) of 2 doubles; not synchronised."""
    _check(load_library().lgf_measure_noalloc(h, _ptr_of(d_out)))


def lgf_fix_begin(h, fmt: int) -> None:
    _check(load_library().lgf_fix_begin(h, fmt))


def lgf_fix_chunk(h, n: int, omega: float, p_sr: float = 0.0, seed: int = 0, sweep0: int = 0,
                  use_graph: int = 1):
    """Returns (F, theta, sweep_ms) after n sweeps of the open session."""
    F, th, ms = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(load_library().lgf_fix_chunk(h, n, omega, p_sr, seed, sweep0, use_graph, ctypes.byref(F),
                                        ctypes.byref(th), ctypes.byref(ms)))
    return F.value, th.value, ms.value


def lgf_fix_end(h) -> None:
    _check(load_library().lgf_fix_end(h))


def lgf_anneal_sweep(h, parity: int, T: float, seed: int = 0, sweep_index: int = 0, count: bool = True):
    """Returns the accept-reject trials (None when count is False)."""
    n = ctypes.c_uint64()
    _check(load_library().lgf_anneal_sweep(h, parity, T, seed, sweep_index, ctypes.byref(n) if count else None))
    return n.value if count else None


def lgf_anneal(h, n_sweeps: int, T_start: float, T_end: float, seed: int = 0, sweep0: int = 0):
    """Returns (accept-reject trials, ms of the sweeps)."""
    n, ms = ctypes.c_uint64(), ctypes.c_double()
    _check(load_library().lgf_anneal(h, n_sweeps, T_start, T_end, seed, sweep0, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def fix_params(**kw) -> "lgf_fix_params":
    """lgf_fix_params_default() with the named fields replaced (unknown names raise)."""
    p = lgf_fix_params_default()
    names = {f[0] for f in lgf_fix_params._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"lgf_fix_params has no field {k!r}")
        setattr(p, k, v)
    return p


def lgf_copy_bandwidth(nbytes: int, reps: int = 10, stream=None) -> float:
    """Read + write GB/s of a plain device copy of nbytes (the streaming ceiling)."""
    gbs = ctypes.c_double()
    _check(load_library().lgf_copy_bandwidth(nbytes, reps, _ptr_of(stream), ctypes.byref(gbs)))
    return gbs.value


class Lattice:
    """Owns one handle; a convenience around the entry points above."""

    def __init__(self, dims, fmt: int = LGF_FP64_18, stream=None, device_buf=None):
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.h = lgf_create(self.dims, fmt, stream, device_buf)

    @property
    def format(self) -> int:
        return lgf_get_info(self.h)[1]

    def close(self):
        if self.h is not None:
            lgf_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, U):
        lgf_load_links(self.h, U)

    def store(self):
        return lgf_store_links(self.h, self.V)

    def peek(self, sites):
        return lgf_peek_links(self.h, sites)

    def generate(self, seed, eps, haar=True):
        lgf_generate_links(self.h, seed, eps, haar)

    def convert(self, fmt):
        lgf_convert(self.h, fmt)

    def sweep(self, parity, omega, p_sr=0.0, seed=0, sweep_index=0):
        lgf_sweep(self.h, parity, omega, p_sr, seed, sweep_index)

    def reunitarize(self):
        lgf_reunitarize(self.h)

    def measure(self):
        return lgf_measure(self.h)

    def gauge_fix(self, **kw):
        p = fix_params(**kw)
        return lgf_gauge_fix(self.h, p)

    def plaquette(self):
        return lgf_plaquette(self.h)

    def fix_begin(self, fmt):
        lgf_fix_begin(self.h, fmt)

    def fix_chunk(self, n, omega, p_sr=0.0, seed=0, sweep0=0, use_graph=1):
        return lgf_fix_chunk(self.h, n, omega, p_sr, seed, sweep0, use_graph)

    def fix_end(self):
        lgf_fix_end(self.h)

    def anneal_sweep(self, parity, T, seed=0, sweep_index=0, count=True):
        return lgf_anneal_sweep(self.h, parity, T, seed, sweep_index, count)

    def anneal(self, n_sweeps, T_start, T_end, seed=0, sweep0=0):
        return lgf_anneal(self.h, n_sweeps, T_start, T_end, seed, sweep0)

    def sweep_coulomb(self, parity, omega, p_sr=0.0, seed=0, sweep_index=0, slice_active=None):
        lgf_sweep_coulomb(self.h, parity, omega, p_sr, seed, sweep_index, slice_active)

    def measure_coulomb(self):
        return lgf_measure_coulomb(self.h, self.dims[0])

    def coulomb_gauge_fix(self, **kw):
        p = fix_params(**kw)
        return lgf_coulomb_gauge_fix(self.h, p, self.dims[0])


# ------------------------------------------------------------------ ensembles

ENSEMBLE_EXPORTS = [
    "lgf_ensemble_create", "lgf_ensemble_destroy", "lgf_ensemble_generate",
    "lgf_ensemble_load_links", "lgf_ensemble_store_links", "lgf_ensemble_sweep",
    "lgf_ensemble_measure", "lgf_ensemble_gauge_fix", "lgf_ensemble_time_sweeps",
    "lgf_ensemble_time_fixed_sweeps", "lgf_ensemble_set_tuning", "lgf_ensemble_get_tuning",
    "lgf_ensemble_autotune",
]
EXPORTS = EXPORTS + ENSEMBLE_EXPORTS + ["lgf_sweep_coulomb", "lgf_measure_coulomb",
                                        "lgf_coulomb_gauge_fix", "lgf_plaquette"]


def _ens_lib():
    lib = load_library()
    if not getattr(lib, "_lgf_ens_sigs", False):
        P, I, U64, D, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t
        sig = {
            "lgf_ensemble_create": (I, [I, P, I, P, P]),
            "lgf_ensemble_destroy": (I, [P]),
            "lgf_ensemble_generate": (I, [P, I, U64, D, I]),
            "lgf_ensemble_load_links": (I, [P, I, P, SZ]),
            "lgf_ensemble_store_links": (I, [P, I, P, SZ]),
            "lgf_ensemble_sweep": (I, [P, I, D, D, U64, U64]),
            "lgf_ensemble_measure": (I, [P, P, P]),
            "lgf_ensemble_gauge_fix": (I, [P, P, P]),
            "lgf_ensemble_time_sweeps": (I, [P, I, I, D, D, P]),
            "lgf_ensemble_time_fixed_sweeps": (I, [P, I, I, D, D, P]),
            "lgf_ensemble_set_tuning": (I, [P, I, I, I]),
            "lgf_ensemble_get_tuning": (I, [P, P, P, P]),
            "lgf_ensemble_autotune": (I, [P, I, I]),
            "lgf_sweep_coulomb": (I, [P, I, D, D, U64, U64, P]),
            "lgf_measure_coulomb": (I, [P, P, P]),
            "lgf_coulomb_gauge_fix": (I, [P, P, P, P, P, P]),
            "lgf_plaquette": (I, [P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        lib._lgf_ens_sigs = True
    return lib


def lgf_ensemble_set_tuning(e, tile: int = 128, grid_mult: int = 1, nontemporal: int = 1) -> None:
    _check(_ens_lib().lgf_ensemble_set_tuning(e, tile, grid_mult, nontemporal))


def lgf_ensemble_get_tuning(e):
    """(tile, grid_mult, nontemporal)"""
    v = [ctypes.c_int() for _ in range(3)]
    _check(_ens_lib().lgf_ensemble_get_tuning(e, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def lgf_ensemble_autotune(e, fmt: int, trials: int = 2) -> None:
    _check(_ens_lib().lgf_ensemble_autotune(e, fmt, trials))


def lgf_ensemble_create(dims_list, fmt: int = LGF_FP64_18, stream=None):
    d = np.ascontiguousarray(np.asarray(dims_list, dtype=np.int32).reshape(-1, 4))
    e = ctypes.c_void_p()
    _check(_ens_lib().lgf_ensemble_create(d.shape[0], _p(d), fmt, _ptr_of(stream), ctypes.byref(e)))
    return e


def lgf_ensemble_destroy(e) -> None:
    _check(_ens_lib().lgf_ensemble_destroy(e))


def lgf_ensemble_generate(e, i: int, seed: int, eps: float, haar: bool = True) -> None:
    _check(_ens_lib().lgf_ensemble_generate(e, i, seed, eps, int(haar)))


def lgf_ensemble_load_links(e, i: int, U: np.ndarray) -> None:
    _canon(U)
    _check(_ens_lib().lgf_ensemble_load_links(e, i, _p(U), U.size * 2))


def lgf_ensemble_store_links(e, i: int, V: int) -> np.ndarray:
    U = np.empty((V, 4, 3, 3), dtype=np.complex128)
    _check(_ens_lib().lgf_ensemble_store_links(e, i, _p(U), U.size * 2))
    return U


def lgf_ensemble_sweep(e, parity: int, omega: float, p_sr: float = 0.0, seed: int = 0,
                       sweep_index: int = 0) -> None:
    _check(_ens_lib().lgf_ensemble_sweep(e, parity, omega, p_sr, seed, sweep_index))


def lgf_ensemble_measure(e, n: int):
    F = np.zeros(n)
    th = np.zeros(n)
    _check(_ens_lib().lgf_ensemble_measure(e, _p(F), _p(th)))
    return F, th


def lgf_ensemble_gauge_fix(e, params: lgf_fix_params, n: int):
    """Returns (status, list of per-configuration result dicts)."""
    res = (lgf_fix_result * n)()
    st = _ens_lib().lgf_ensemble_gauge_fix(e, ctypes.byref(params), res)
    _check(st, allow=(LGF_ENOTCONV, LGF_ENUMERIC))
    return st, [r.as_dict() for r in res]


def lgf_ensemble_time_sweeps(e, fmt: int, n: int, omega: float, p_sr: float = 0.0) -> float:
    ms = ctypes.c_double()
    _check(_ens_lib().lgf_ensemble_time_sweeps(e, fmt, n, omega, p_sr, ctypes.byref(ms)))
    return ms.value


def lgf_ensemble_time_fixed_sweeps(e, fmt: int, n: int, omega: float, p_sr: float = 0.0) -> float:
    ms = ctypes.c_double()
    _check(_ens_lib().lgf_ensemble_time_fixed_sweeps(e, fmt, n, omega, p_sr, ctypes.byref(ms)))
    return ms.value


def lgf_sweep_coulomb(h, parity: int, omega: float, p_sr: float = 0.0, seed: int = 0,
                      sweep_index: int = 0, slice_active=None) -> None:
    act = None if slice_active is None else np.ascontiguousarray(np.asarray(slice_active, dtype=np.uint8))
    _check(_ens_lib().lgf_sweep_coulomb(h, parity, omega, p_sr, seed, sweep_index,
                                        None if act is None else _p(act)))


def lgf_plaquette(h) -> float:
    P = ctypes.c_double()
    _check(_ens_lib().lgf_plaquette(h, ctypes.byref(P)))
    return P.value


def lgf_measure_coulomb(h, Lt: int):
    F = np.zeros(Lt)
    th = np.zeros(Lt)
    _check(_ens_lib().lgf_measure_coulomb(h, _p(F), _p(th)))
    return F, th


def lgf_coulomb_gauge_fix(h, params: lgf_fix_params, Lt: int):
    """Returns (status, result dict, per-timeslice sweeps, F_C, theta_C)."""
    res = lgf_fix_result()
    sw, F, th = np.zeros(Lt), np.zeros(Lt), np.zeros(Lt)
    st = _ens_lib().lgf_coulomb_gauge_fix(h, ctypes.byref(params), ctypes.byref(res), _p(sw), _p(F), _p(th))
    _check(st, allow=(LGF_ENOTCONV, LGF_ENUMERIC))
    return st, res.as_dict(), sw.astype(np.int64), F, th


class Ensemble:
    """Owns one ensemble handle."""

    def __init__(self, dims_list, fmt: int = LGF_FP64_18, stream=None):
        self.dims = [tuple(int(x) for x in d) for d in dims_list]
        self.n = len(self.dims)
        self.V = [int(np.prod(d)) for d in self.dims]
        self.e = lgf_ensemble_create(self.dims, fmt, stream)

    def close(self):
        if self.e is not None:
            lgf_ensemble_destroy(self.e)
            self.e = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def generate(self, i, seed, eps, haar=True):
        lgf_ensemble_generate(self.e, i, seed, eps, haar)

    def load(self, i, U):
        lgf_ensemble_load_links(self.e, i, U)

    def store(self, i):
        return lgf_ensemble_store_links(self.e, i, self.V[i])

    def sweep(self, parity, omega, p_sr=0.0, seed=0, sweep_index=0):
        lgf_ensemble_sweep(self.e, parity, omega, p_sr, seed, sweep_index)

    def measure(self):
        return lgf_ensemble_measure(self.e, self.n)

    def gauge_fix(self, **kw):
        p = fix_params(**kw)
        return lgf_ensemble_gauge_fix(self.e, p, self.n)

    def time_sweeps(self, fmt, n, omega, p_sr=0.0):
        return lgf_ensemble_time_sweeps(self.e, fmt, n, omega, p_sr)

    def time_fixed_sweeps(self, fmt, n, omega, p_sr=0.0):
        return lgf_ensemble_time_fixed_sweeps(self.e, fmt, n, omega, p_sr)
