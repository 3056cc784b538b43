"""Degenerate and boundary cases of the method on the GPU, against the FP64
oracle through the C ABI:

* the degenerate SU(2) subproblem (|a| = 0 in Eq. (9)), whose step is the
  identity: a constant field diag(i, i, -1) gives K(x) = diag(0, 0, -8), whose
  (0,1) block has no quaternion part at all;
* omega = 2, the upper end of the overrelaxation range the library accepts
  (Sec. 3.1 gives 1 <= omega < 2);
* a random gauge transformation of the unit field (eps = 0), which the gauge
  fixing must drive back to the global maximum F = 1 with theta -> 0.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import fp32_model as fm
from conftest import gpu_available
from lattice_np import stored_as

pytestmark = pytest.mark.gpu

FP64 = (0, 3)


@pytest.fixture(scope="module")
def lgf():
    if not gpu_available():
        pytest.skip("no GPU visible")
    import paper_1305_3440_amd as pkg
    pkg.load_library()
    return pkg


def announce(*args):
    print("[gpu-case]", *args, flush=True)
    sys.stdout.flush()


def maxabs(a, b) -> float:
    return float(np.abs(np.asarray(a) - np.asarray(b)).max())


def link_errs(A, B):
    d = np.linalg.norm((A - B).reshape(-1, 9), axis=1)
    n = np.linalg.norm(B.reshape(-1, 9), axis=1)
    return d / n


def close(fmt, got, ref, env=None):
    """FP64 storage: 1e-12 per entry; FP32 storage: 2e-6 relative per link
    on 99 % of the links and on every link twice its randomised-rounding
    envelope env (the FP32 bar of the parity tests; exact results need no
    envelope: then every link within u = 2^-24)."""
    if fmt in FP64:
        return maxabs(got, ref) <= 1e-12
    if env is None:
        env = np.zeros(len(link_errs(got, ref)))
    return fm.fp32_bar_ok(got, ref, env)[0]


def constant_field(dims):
    V = int(np.prod(dims))
    U = np.zeros((V, 4, 3, 3), np.complex128)
    U[:, :, 0, 0] = 1j
    U[:, :, 1, 1] = 1j
    U[:, :, 2, 2] = -1.0
    return U


@pytest.mark.parametrize("fmt", [0, 1, 2, 3])
@pytest.mark.parametrize("omega", [1.0, 1.7])
def test_degenerate_block_half_sweep(lgf, orc, fmt, omega):
    """K = diag(0, 0, -8) at every site: subgroup (0,1) is degenerate (|a| = 0,
    identity), (0,2) turns by -1, so every parity-0 site's G is
    diag(-1, 1, -1); the GPU half-sweep equals the oracle's."""
    dims = (4, 4, 6, 8)
    announce("degenerate block", fmt, omega, dims)
    U = constant_field(dims)
    with lgf.Lattice(dims, fmt) as lat:
        lat.load(U)
        lat.sweep(0, omega)
        got = lat.store()
    ref = U.copy()
    orc.half_sweep(dims, ref, 0, omega)
    assert close(fmt, got, ref)
    # the closed form: every link has one parity-0 end, so G U (forward) and
    # U G^dag (backward) make every link diag(-i, i, 1)
    expect = np.broadcast_to(np.diag([-1j, 1j, 1.0]), U.shape)
    assert maxabs(ref, expect) == 0.0
    assert maxabs(got, expect) <= 1e-15


@pytest.mark.parametrize("sweep_fmt", [0, 3, 4, 2])
def test_degenerate_block_fixed_sweep(lgf, orc, sweep_fmt):
    """The same constant field through the fixed-link form (one full sweep,
    g reunitarized as it is stored): the oracle's sweep plus
    reunitarization.  The field is a stationary point already (K is
    Hermitian, theta = 0, though not a maximum), so lgf_gauge_fix would stop
    before sweeping: the sweep runs as one chunk of a stepwise session."""
    dims = (4, 4, 6, 8)
    announce("degenerate block, fixed links", sweep_fmt, dims)
    U = constant_field(dims)
    with lgf.Lattice(dims, 0) as lat:
        lat.load(U)
        assert lat.measure()[1] == 0.0
        lat.fix_begin(sweep_fmt)
        lat.fix_chunk(1, 1.7)
        lat.fix_end()
        got = lat.store()
    ref = U.copy()
    orc.sweep(dims, ref, 1.7)
    orc.reunitarize(ref)
    assert close(0 if sweep_fmt in (0, 3, 4) else 2, got, ref)


@pytest.mark.parametrize("fmt", [0, 1, 2, 3])
@pytest.mark.parametrize("p_sr", [0.0, 0.5])
def test_omega_two_sweep(lgf, orc, fmt, p_sr):
    """One full sweep at omega = 2 (the largest accepted value), each storage
    format, overrelaxation and stochastic relaxation, against the oracle on
    the same (format-rounded) input."""
    dims = (4, 4, 6, 10)
    announce("omega 2", fmt, p_sr, dims)
    U = stored_as(orc.generate_links(dims, 13, 0.3), fmt)
    with lgf.Lattice(dims, fmt) as lat:
        lat.load(U)
        lat.sweep(2, 2.0, p_sr, 5, 3)
        got = lat.store()
    ref = U.copy()
    orc.sweep(dims, ref, 2.0, p_sr, seed=5, sweep_index=3)
    env = None if fmt in FP64 else fm.link_sweep_envelope(orc, dims, U, fmt, ref, 2.0, p_sr, 5, 3)
    assert close(fmt, got, ref, env), (maxabs(got, ref), float(link_errs(got, ref).max()))


@pytest.mark.parametrize("sweep_fmt", [0, 3, 2])
def test_omega_two_fixed_sweep(lgf, orc, sweep_fmt):
    dims = (4, 4, 6, 10)
    announce("omega 2, fixed links", sweep_fmt, dims)
    U = orc.generate_links(dims, 13, 0.3)
    with lgf.Lattice(dims, 0) as lat:
        lat.load(U)
        kw = dict(omega=2.0, theta_target=1e-300, check_every=1, max_sweeps=1, fixed_links=1)
        if sweep_fmt != 0:
            kw.update(bulk_format=sweep_fmt, finish_format=0, theta_switch=1e-300)
        st, res, _ = lat.gauge_fix(**kw)
        assert st == lgf.LGF_ENOTCONV and res["sweeps"] == 1
        got = lat.store()
    ref = U.copy()
    orc.sweep(dims, ref, 2.0)
    orc.reunitarize(ref)
    if sweep_fmt == 2:
        # FP32 sweep of the FP64 input: the oracle on the same input, FP32 bar
        env = fm.fixed_sweep_envelope(orc, dims, U, 2, ref, 2.0)
        ok, info = fm.fp32_bar_ok(got, ref, env)
        assert ok, info
    else:
        assert maxabs(got, ref) <= 1e-12


@pytest.mark.parametrize("mode", ["fp64-18", "mixed", "fixed-split"])
def test_pure_gauge_driven_back_to_F1(lgf, orc, mode):
    """A Haar-random gauge transformation of the unit field (seed 1, eps 0,
    generated on the GPU) is fixed back to the global maximum: the oracle
    measures F >= 1 - 1e-12 and theta < 1e-14 on the links handed back."""
    dims = (4, 4, 4, 4)
    announce("pure gauge", mode, dims)
    with lgf.Lattice(dims, 0) as lat:
        lat.generate(1, 0.0, True)
        start = lat.store()
        kw = dict(omega=1.7, theta_target=1e-14)
        if mode == "mixed":
            kw.update(theta_switch=1e-8, bulk_format=lgf.LGF_FP32_12)
        elif mode == "fixed-split":
            kw.update(theta_switch=1e-8, bulk_format=lgf.LGF_FP32_12, finish_format=lgf.LGF_FP64_12S,
                      fixed_links=1)
        st, res, _ = lat.gauge_fix(**kw)
        got = lat.store()
    F0, th0 = orc.measure(dims, start)
    assert F0 < 0.2 and th0 > 0.1
    assert st == lgf.LGF_OK, res
    F, th = orc.measure(dims, got)
    assert th < 1e-14, th
    assert F >= 1 - 1e-12, F
