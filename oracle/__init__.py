"""Plain FP64 CPU oracle for checkerboard SU(3) Landau gauge fixing.

TEST INFRASTRUCTURE ONLY: the correctness reference for the HIP library.  Only
the test suite, the package smoke check and the CPU-baseline leg of the
benchmark may import it; the library itself never does.  The arithmetic lives
in ``lgf_oracle.c`` (plain C, double precision, no code shared with the HIP
path); this module builds it with gcc and marshals numpy arrays through ctypes.

Links are numpy ``complex128`` arrays of shape ``(V, 4, 3, 3)`` (site, mu, row,
column), which has the memory layout of the C side's double[V][4][3][3][2].
Dimensions are ``(Lt, Lz, Ly, Lx)``; mu = 0 is t, 1 z, 2 y, 3 x; the site index
is ((t*Lz + z)*Ly + y)*Lx + x.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lgf_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblgf_oracle.so")

# Plain IEEE double arithmetic: no FMA contraction, no fast-math; complex
# products without the C99 Annex G inf/nan recovery (values here are finite).
CFLAGS = ["-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared",
          "-ffp-contract=off", "-fcx-limited-range", "-std=gnu11"]

_lib = None


def build() -> str:
    """Compile the oracle into ``oracle/liblgf_oracle.so`` (always recompiles)."""
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    I = ctypes.c_int
    I64 = ctypes.c_int64
    U64 = ctypes.c_uint64
    U32 = ctypes.c_uint32
    D = ctypes.c_double
    P = ctypes.c_void_p
    sig = {
        "orc_volume": (I64, [P]),
        "orc_neighbor": (I64, [P, I64, I, I]),
        "orc_parity": (I, [P, I64]),
        "orc_site_links": (None, [P, I64, P]),
        "orc_philox4x32_10": (None, [P, P, P]),
        "orc_normals4": (None, [U64, P, P]),
        "orc_su3_exp_iH": (None, [P, D, P]),
        "orc_haar_su3": (None, [U64, I64, P]),
        "orc_generated_link": (None, [P, U64, D, I, I64, I, P]),
        "orc_generate_links": (None, [P, U64, D, I, P]),
        "orc_gauge_transform": (None, [P, P, P]),
        "orc_su2_step": (None, [P, D, I, P]),
        "orc_local_update": (None, [P, D, P, P]),
        "orc_sr_decisions": (None, [U64, I64, U64, U32, D, P]),
        "orc_half_sweep": (I, [P, P, I, D, D, U64, U64, U32, P, I64]),
        "orc_sweep": (None, [P, P, D, D, U64, U64, U32]),
        "orc_reunitarize": (None, [I64, P]),
        "orc_measure": (None, [P, P, P, P]),
        "orc_wilson_loop": (D, [P, P, I, I, I, I]),
        "orc_plaquette": (D, [P, P]),
        "orc_gauge_fix": (I, [P, P, D, D, D, I, I, I64, U64, U32, P, P, P, P, I64, P]),
        "orc_num_threads": (I, []),
        "orc_set_num_threads": (None, [I]),
        "orc_local_update_coulomb": (None, [P, D, P, P]),
        "orc_half_sweep_coulomb": (None, [P, P, I, D, D, U64, U64, U32, P]),
        "orc_measure_coulomb": (None, [P, P, P, P]),
        "orc_coulomb_gauge_fix": (I, [P, P, D, D, D, I, I, I64, U64, U32, P, P, P, P]),
        "orc_su2_heatbath": (I, [P, D, U64, I64, U64, U32, I, P]),
        "orc_half_sweep_sa": (I64, [P, P, I, D, U64, U64, U32]),
        "orc_local_update_sa": (I64, [P, D, U64, I64, U64, U32]),
        "orc_anneal_temperature": (D, [I64, I64, D, D]),
        "orc_anneal": (I64, [P, P, I64, D, D, U64, U64, U32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(dims) -> np.ndarray:
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32).reshape(4))
    return d


def _links_arg(U: np.ndarray) -> np.ndarray:
    if U.dtype != np.complex128 or not U.flags.c_contiguous or U.shape[1:] != (4, 3, 3):
        raise ValueError("links must be a C-contiguous complex128 array of shape (V, 4, 3, 3)")
    return U


# ---------------------------------------------------------------- geometry

def volume(dims) -> int:
    return int(_load().orc_volume(_ptr(_dims(dims))))


def neighbor(dims, s: int, mu: int, step: int) -> int:
    return int(_load().orc_neighbor(_ptr(_dims(dims)), s, mu, step))


def parity(dims, s: int) -> int:
    return int(_load().orc_parity(_ptr(_dims(dims)), s))


def site_links(dims, s: int) -> np.ndarray:
    out = np.zeros(8, dtype=np.int64)
    _load().orc_site_links(_ptr(_dims(dims)), s, _ptr(out))
    return out


# ---------------------------------------------------------------- random numbers

def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(4))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def normals4(seed: int, ctr) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(4))
    out = np.zeros(4, dtype=np.float64)
    _load().orc_normals4(seed, _ptr(c), _ptr(out))
    return out


def su3_exp_iH(a, eps: float) -> np.ndarray:
    av = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(8))
    out = np.zeros((3, 3), dtype=np.complex128)
    _load().orc_su3_exp_iH(_ptr(av), eps, _ptr(out))
    return out


def haar_su3(seed: int, s: int) -> np.ndarray:
    out = np.zeros((3, 3), dtype=np.complex128)
    _load().orc_haar_su3(seed, s, _ptr(out))
    return out


def generated_link(dims, seed: int, eps: float, haar: bool, s: int, mu: int) -> np.ndarray:
    out = np.zeros((3, 3), dtype=np.complex128)
    _load().orc_generated_link(_ptr(_dims(dims)), seed, eps, int(haar), s, mu, _ptr(out))
    return out


def generate_links(dims, seed: int, eps: float, haar: bool = True) -> np.ndarray:
    V = volume(dims)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    _load().orc_generate_links(_ptr(_dims(dims)), seed, eps, int(haar), _ptr(U))
    return U


def gauge_transform(dims, U: np.ndarray, g: np.ndarray) -> None:
    _links_arg(U)
    g = np.ascontiguousarray(g, dtype=np.complex128)
    if g.shape != (U.shape[0], 3, 3):
        raise ValueError("g must have shape (V, 3, 3)")
    _load().orc_gauge_transform(_ptr(_dims(dims)), _ptr(U), _ptr(g))


# ---------------------------------------------------------------- the method

def su2_step(w: np.ndarray, omega: float, take_square: bool = False) -> np.ndarray:
    """w: 2x2 complex block; returns the quaternion (r0, r1, r2, r3)."""
    w = np.asarray(w, dtype=np.complex128).reshape(2, 2)
    wv = np.ascontiguousarray(np.array([w[0, 0].real, w[0, 0].imag, w[0, 1].real, w[0, 1].imag,
                                        w[1, 0].real, w[1, 0].imag, w[1, 1].real, w[1, 1].imag]))
    out = np.zeros(4, dtype=np.float64)
    _load().orc_su2_step(_ptr(wv), omega, int(take_square), _ptr(out))
    return out


def local_update(links8: np.ndarray, omega: float, sr=(0, 0, 0)):
    """links8: (8, 3, 3) complex, forward links then backward links.
    Returns (updated links8, G)."""
    L = np.ascontiguousarray(np.array(links8, dtype=np.complex128).reshape(8, 3, 3))
    srv = np.ascontiguousarray(np.asarray(sr, dtype=np.int32).reshape(3))
    G = np.zeros((3, 3), dtype=np.complex128)
    _load().orc_local_update(_ptr(L), omega, _ptr(srv), _ptr(G))
    return L, G


def sr_decisions(seed: int, s: int, sweep: int, instance: int, p: float) -> np.ndarray:
    out = np.zeros(3, dtype=np.int32)
    _load().orc_sr_decisions(seed, s, sweep, instance, p, _ptr(out))
    return out


def half_sweep(dims, U: np.ndarray, parity: int, omega: float, p: float = 0.0,
               seed: int = 0, sweep: int = 0, instance: int = 0, order=None) -> None:
    _links_arg(U)
    if order is None:
        rc = _load().orc_half_sweep(_ptr(_dims(dims)), _ptr(U), parity, omega, p, seed, sweep,
                                    instance, None, 0)
    else:
        o = np.ascontiguousarray(np.asarray(order, dtype=np.int64))
        rc = _load().orc_half_sweep(_ptr(_dims(dims)), _ptr(U), parity, omega, p, seed, sweep,
                                    instance, _ptr(o), o.size)
    if rc != 0:
        raise ValueError("site order lists a site of the other parity")


def sweep(dims, U: np.ndarray, omega: float, p: float = 0.0, seed: int = 0, sweep_index: int = 0,
          instance: int = 0) -> None:
    _links_arg(U)
    _load().orc_sweep(_ptr(_dims(dims)), _ptr(U), omega, p, seed, sweep_index, instance)


def reunitarize(U: np.ndarray) -> None:
    U = np.asarray(U)
    if U.dtype != np.complex128 or not U.flags.c_contiguous or U.shape[-2:] != (3, 3):
        raise ValueError("links must be C-contiguous complex128 (..., 3, 3)")
    _load().orc_reunitarize(U.size // 9, _ptr(U))


def measure(dims, U: np.ndarray):
    """Returns (F, theta) of Eqs. (2), (4), (5)."""
    _links_arg(U)
    F = np.zeros(1)
    th = np.zeros(1)
    _load().orc_measure(_ptr(_dims(dims)), _ptr(U), _ptr(F), _ptr(th))
    return float(F[0]), float(th[0])


def wilson_loop(dims, U: np.ndarray, mu: int, nu: int, R: int, T: int) -> float:
    _links_arg(U)
    return float(_load().orc_wilson_loop(_ptr(_dims(dims)), _ptr(U), mu, nu, R, T))


def plaquette(dims, U: np.ndarray) -> float:
    _links_arg(U)
    return float(_load().orc_plaquette(_ptr(_dims(dims)), _ptr(U)))


def gauge_fix(dims, U: np.ndarray, omega: float, theta_target: float, p: float = 0.0,
              check_every: int = 20, reunitarize: bool = True, max_sweeps: int = 100000,
              seed: int = 0, instance: int = 0, history_cap: int = 100000):
    """Iterate full sweeps until theta < theta_target (measured every
    check_every sweeps, after reunitarizing).  Returns a dict with status
    (0 converged, 1 max_sweeps reached), sweeps, F, theta and the history of
    (sweeps, F, theta) measurements."""
    _links_arg(U)
    sweeps = np.zeros(1, dtype=np.int64)
    F = np.zeros(1)
    th = np.zeros(1)
    hist = np.zeros((history_cap, 3))
    nh = np.zeros(1, dtype=np.int64)
    st = _load().orc_gauge_fix(_ptr(_dims(dims)), _ptr(U), omega, p, theta_target, check_every,
                               int(reunitarize), max_sweeps, seed, instance, _ptr(sweeps), _ptr(F),
                               _ptr(th), _ptr(hist), history_cap, _ptr(nh))
    return {"status": int(st), "sweeps": int(sweeps[0]), "F": float(F[0]), "theta": float(th[0]),
            "history": hist[: int(nh[0])].copy()}


# ---------------------------------------------------------------- Coulomb gauge

def local_update_coulomb(links8: np.ndarray, omega: float, sr=(0, 0, 0)):
    L = np.ascontiguousarray(np.array(links8, dtype=np.complex128).reshape(8, 3, 3))
    srv = np.ascontiguousarray(np.asarray(sr, dtype=np.int32).reshape(3))
    G = np.zeros((3, 3), dtype=np.complex128)
    _load().orc_local_update_coulomb(_ptr(L), omega, _ptr(srv), _ptr(G))
    return L, G


def half_sweep_coulomb(dims, U: np.ndarray, parity: int, omega: float, p: float = 0.0,
                       seed: int = 0, sweep: int = 0, instance: int = 0, slice_active=None) -> None:
    _links_arg(U)
    if slice_active is None:
        act = None
    else:
        act = np.ascontiguousarray(np.asarray(slice_active, dtype=np.uint8).reshape(int(dims[0])))
    _load().orc_half_sweep_coulomb(_ptr(_dims(dims)), _ptr(U), parity, omega, p, seed, sweep,
                                   instance, None if act is None else _ptr(act))


def sweep_coulomb(dims, U: np.ndarray, omega: float, p: float = 0.0, seed: int = 0,
                  sweep_index: int = 0, instance: int = 0, slice_active=None) -> None:
    for parity in (0, 1):
        half_sweep_coulomb(dims, U, parity, omega, p, seed, sweep_index, instance, slice_active)


def measure_coulomb(dims, U: np.ndarray):
    """(F_C(t), theta_C(t)) per timeslice, arrays of length Lt."""
    _links_arg(U)
    Lt = int(dims[0])
    F = np.zeros(Lt)
    th = np.zeros(Lt)
    _load().orc_measure_coulomb(_ptr(_dims(dims)), _ptr(U), _ptr(F), _ptr(th))
    return F, th


def coulomb_gauge_fix(dims, U: np.ndarray, omega: float, theta_target: float, p: float = 0.0,
                      check_every: int = 20, reunitarize: bool = True, max_sweeps: int = 100000,
                      seed: int = 0, instance: int = 0):
    _links_arg(U)
    Lt = int(dims[0])
    sw = np.zeros(Lt)
    F = np.zeros(Lt)
    th = np.zeros(Lt)
    tot = np.zeros(1, dtype=np.int64)
    st = _load().orc_coulomb_gauge_fix(_ptr(_dims(dims)), _ptr(U), omega, p, theta_target,
                                       check_every, int(reunitarize), max_sweeps, seed, instance,
                                       _ptr(sw), _ptr(F), _ptr(th), _ptr(tot))
    return {"status": int(st), "sweeps": int(tot[0]), "sweeps_t": sw.astype(np.int64), "F_t": F,
            "theta_t": th}


# ---------------------------------------------------------------- simulated annealing

def su2_heatbath(w: np.ndarray, T: float, seed: int, s: int, sweep: int, instance: int = 0, k: int = 0):
    """Heat-bath draw for one subgroup block w (2x2 complex) at temperature T,
    from Philox counter (s, sweep, instance, tag of subgroup k).  Returns
    (quaternion r, accept-reject trials used)."""
    w = np.asarray(w, dtype=np.complex128).reshape(2, 2)
    wv = np.ascontiguousarray(np.array([w[0, 0].real, w[0, 0].imag, w[0, 1].real, w[0, 1].imag,
                                        w[1, 0].real, w[1, 0].imag, w[1, 1].real, w[1, 1].imag]))
    out = np.zeros(4, dtype=np.float64)
    n = _load().orc_su2_heatbath(_ptr(wv), T, seed, s, sweep, instance, k, _ptr(out))
    return out, int(n)


def local_update_sa(links8: np.ndarray, T: float, seed: int, s: int, sweep: int, instance: int = 0):
    """Annealing update of the 8 links of site s (forward then backward);
    returns (updated links8, trials)."""
    L = np.ascontiguousarray(np.array(links8, dtype=np.complex128).reshape(8, 3, 3))
    n = _load().orc_local_update_sa(_ptr(L), T, seed, s, sweep, instance)
    return L, int(n)


def half_sweep_sa(dims, U: np.ndarray, parity: int, T: float, seed: int = 0, sweep: int = 0,
                  instance: int = 0) -> int:
    """One annealing half-sweep at temperature T; returns the accept-reject trials."""
    _links_arg(U)
    return int(_load().orc_half_sweep_sa(_ptr(_dims(dims)), _ptr(U), parity, T, seed, sweep, instance))


def anneal_temperature(n: int, n_sweeps: int, T_start: float, T_end: float) -> float:
    return float(_load().orc_anneal_temperature(n, n_sweeps, T_start, T_end))


def anneal(dims, U: np.ndarray, n_sweeps: int, T_start: float, T_end: float, seed: int = 0,
           sweep0: int = 0, instance: int = 0) -> int:
    """n_sweeps annealing sweeps with the linear schedule (reunitarized every 20
    sweeps and at the end); returns the accept-reject trials."""
    _links_arg(U)
    return int(_load().orc_anneal(_ptr(_dims(dims)), _ptr(U), n_sweeps, T_start, T_end, seed, sweep0,
                                  instance))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    _load().orc_set_num_threads(int(n))
