"""Simulated annealing on the GPU against the FP64 oracle, through the C ABI.

The heat-bath draws of both sides come from the same Philox words and take
their accept-reject decisions in FP64, so the trial counts must agree
exactly and the links to the FP64 bar of one sweep (1e-12), and to 1e-11
over a whole annealing schedule (45 sweeps with reunitarizations)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from conftest import gpu_available
from lattice_np import stored_as, unitarity_error

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 6, 10), (8, 6, 4, 12)])
@pytest.mark.parametrize("fmt", [0, 3])
@pytest.mark.parametrize("T", [0.2, 1.0, 6.0])
def test_anneal_sweep_matches_oracle(lgf, orc, dims, fmt, T):
    """One half-sweep of each parity and one full sweep: links within 1e-12,
    trial counts equal (every accept-reject decision the same)."""
    announce("anneal sweep", dims, fmt, T)
    U = stored_as(orc.generate_links(dims, 19, 0.3), fmt)
    for parity in (0, 1, 2):
        with lgf.Lattice(dims, fmt) as lat:
            lat.load(U)
            n = lat.anneal_sweep(parity, T, 3, 7)
            got = lat.store()
        ref = U.copy()
        m = 0
        for p in ((0, 1) if parity == 2 else (parity,)):
            m += orc.half_sweep_sa(dims, ref, p, T, 3, 7)
        assert n == m, (parity, n, m)
        assert maxabs(got, ref) <= 1e-12, (parity, maxabs(got, ref))


@pytest.mark.parametrize("fmt", [0, 3])
def test_anneal_schedule_matches_oracle(lgf, orc, fmt):
    """45 sweeps, T from 1.2 down to 0.05, counters from 2: the oracle's
    schedule (reunitarized after 20, 40 and 45 sweeps)."""
    dims = (4, 4, 6, 10)
    announce("anneal schedule", fmt, dims)
    U = stored_as(orc.generate_links(dims, 29, 0.3), fmt)
    with lgf.Lattice(dims, fmt) as lat:
        lat.load(U)
        n, ms = lat.anneal(45, 1.2, 0.05, seed=5, sweep0=2)
        got = lat.store()
    ref = U.copy()
    m = orc.anneal(dims, ref, 45, 1.2, 0.05, seed=5, sweep0=2)
    assert n == m
    assert ms > 0
    assert maxabs(got, ref) <= 1e-11, maxabs(got, ref)
    assert unitarity_error(got) < 1e-13


@pytest.mark.parametrize("fixed", [0, 1])
def test_anneal_then_fix_reaches_the_global_maximum(lgf, orc, fixed):
    """A random gauge transformation of the unit field (4^4, seed 1): 100
    annealing sweeps (T 1 -> 0.02) on the GPU, then overrelaxation to
    theta < 1e-14 -- F = 1 by the oracle's measurement, as in the oracle's
    own run of the same schedule."""
    dims = (4, 4, 4, 4)
    announce("anneal then fix", fixed, dims)
    with lgf.Lattice(dims, 0) as lat:
        lat.generate(1, 0.0, True)
        lat.anneal(100, 1.0, 0.02, seed=7)
        st, res, _ = lat.gauge_fix(omega=1.7, theta_target=1e-14, fixed_links=fixed)
        got = lat.store()
    assert st == lgf.LGF_OK
    F, th = orc.measure(dims, got)
    assert th < 1e-14 and F >= 1 - 1e-12, (F, th)


def test_anneal_64x4_sampled(lgf, orc):
    """The 64^4 workload (seed 3, eps 0.3, Haar gauge): one annealing
    half-sweep of parity 0 at T = 0.5, checked on sampled parity-0 sites
    (edges and wrap-arounds included) against the oracle's update of the
    site from its own generator, and the trial count of the whole sweep is
    plausible (at least one trial per subgroup step)."""
    from test_gpu_parity import gpu_links8, oracle_links8, sample_sites
    dims = (64, 64, 64, 64)
    seed, eps, T = 3, 0.3, 0.5
    announce("anneal 64^4 sampled")
    rng = np.random.default_rng(8)
    with lgf.Lattice(dims, 0) as lat:
        lat.generate(seed, eps, True)
        n = lat.anneal_sweep(0, T, 11, 4)
        for s in sample_sites(orc, dims, 0, 12, rng):
            ref, _ = orc.local_update_sa(oracle_links8(orc, dims, seed, eps, s), T, 11, s, 4)
            assert maxabs(gpu_links8(lat, orc, dims, s), ref) <= 1e-12, s
    V = 64 ** 4
    assert 3 * V // 2 <= n <= 3 * 64 * V // 2


def test_anneal_argument_checks(lgf, orc):
    lib = lgf.load_library()
    dims = (4, 4, 4, 4)
    announce("anneal arguments")
    with lgf.Lattice(dims, lgf.LGF_FP32_12) as lat:
        assert lib.lgf_anneal_sweep(lat.h, 0, 1.0, 0, 0, None) == lgf.LGF_EINVAL
        assert lib.lgf_anneal(lat.h, 10, 1.0, 0.1, 0, 0, None, None) == lgf.LGF_EINVAL
    with lgf.Lattice(dims, 0) as lat:
        assert lib.lgf_anneal_sweep(lat.h, 3, 1.0, 0, 0, None) == lgf.LGF_EINVAL
        assert lib.lgf_anneal_sweep(lat.h, 0, 0.0, 0, 0, None) == lgf.LGF_EINVAL
        assert lib.lgf_anneal_sweep(lat.h, 0, float("inf"), 0, 0, None) == lgf.LGF_EINVAL
        assert lib.lgf_anneal(lat.h, 0, 1.0, 0.1, 0, 0, None, None) == lgf.LGF_EINVAL
        assert lib.lgf_anneal(lat.h, 5, 1.0, -0.1, 0, 0, None, None) == lgf.LGF_EINVAL
    assert lib.lgf_anneal_sweep(None, 0, 1.0, 0, 0, None) == lgf.LGF_EINVAL
