"""Stepwise gauge fixing (lgf_fix_begin / lgf_fix_chunk / lgf_fix_end) and the
driver's handling of the split FP64 finish, through the C ABI.

A session runs the same chunks as lgf_gauge_fix with fixed_links set (Sec. 4:
the parities swept in turn, theta checked every check interval), so its links
and its F, theta must equal that driver's bit for bit; the links it hands back
are compared with the oracle by the fixed-link parity tests.  When the split
finish stops at its own fixed point, whose theta measured on the FP64 links
lies above a very tight target, the driver must go on sweeping (in FP64-12)
rather than give up."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from conftest import gpu_available

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


@pytest.mark.parametrize("fmt", [3, 4, 2])
@pytest.mark.parametrize("p_sr", [0.0, 0.5])
@pytest.mark.parametrize("use_graph", [1, 0])
def test_session_equals_gauge_fix(lgf, orc, fmt, p_sr, use_graph):
    """Three chunks of 20 sweeps of a session = lgf_gauge_fix with the same
    sweep format, 60 sweeps and checks every 20: the same links bit for bit
    and the same F, theta at each check."""
    dims = (4, 4, 6, 10)
    announce("session vs gauge_fix", fmt, p_sr, use_graph, dims)
    U = orc.generate_links(dims, 17, 0.3)
    omega = 1.0 if p_sr > 0 else 1.7
    with lgf.Lattice(dims, 0) as lat:
        lat.load(U)
        lat.fix_begin(fmt)
        seen = [lat.fix_chunk(20, omega, p_sr, 7, 20 * k, use_graph) for k in range(3)]
        lat.fix_end()
        got = lat.store()
    with lgf.Lattice(dims, 0) as lat:
        lat.load(U)
        st, res, hist = lat.gauge_fix(omega=omega, p_sr=p_sr, seed=7, theta_target=1e-300, max_sweeps=60,
                                      check_every=20, fixed_links=1, bulk_format=fmt, finish_format=fmt,
                                      use_graph=use_graph)
        ref = lat.store()
    assert st == lgf.LGF_ENOTCONV and res["sweeps"] == 60
    assert np.array_equal(got, ref)
    for k in range(3):
        assert seen[k][0] == hist[k + 1, 1] and seen[k][1] == hist[k + 1, 2], k
        assert seen[k][2] > 0.0
    assert seen[2][1] < seen[0][1]


def test_session_state_errors(lgf, orc):
    dims = (4, 4, 4, 4)
    announce("session states", dims)
    U = orc.generate_links(dims, 3, 0.3)
    lib = lgf.load_library()
    with lgf.Lattice(dims, 0) as lat:
        lat.load(U)
        assert lib.lgf_fix_chunk(lat.h, 20, 1.7, 0.0, 0, 0, 1, None, None, None) == lgf.LGF_ESTATE
        assert lib.lgf_fix_end(lat.h) == lgf.LGF_ESTATE
        assert lib.lgf_fix_begin(lat.h, 9) == lgf.LGF_EINVAL
        lat.fix_begin(lgf.LGF_FP64_12S)
        assert lib.lgf_fix_chunk(lat.h, 0, 1.7, 0.0, 0, 0, 1, None, None, None) == lgf.LGF_EINVAL
        assert lib.lgf_fix_chunk(lat.h, 1, 2.5, 0.0, 0, 0, 1, None, None, None) == lgf.LGF_EINVAL
        assert lib.lgf_fix_chunk(lat.h, 1, 1.7, 1.5, 0, 0, 1, None, None, None) == lgf.LGF_EINVAL
        lat.fix_chunk(2, 1.7)
        # loading new links closes the session without applying g
        lat.load(U)
        assert lib.lgf_fix_chunk(lat.h, 1, 1.7, 0.0, 0, 0, 1, None, None, None) == lgf.LGF_ESTATE
        assert lib.lgf_fix_end(lat.h) == lgf.LGF_ESTATE
        assert np.array_equal(lat.store(), U)
        # a new fixed-link tuning (here the link layout the session's links
        # are held in) closes the session too
        lat.fix_begin(lgf.LGF_FP64_12)
        lat.fix_chunk(2, 1.7)
        lgf.lgf_set_fixed_tuning(lat.h, lgf.LGF_FP64_12, 2, 128, 2, 1)
        assert lib.lgf_fix_chunk(lat.h, 1, 1.7, 0.0, 0, 0, 1, None, None, None) == lgf.LGF_ESTATE
        assert lib.lgf_fix_end(lat.h) == lgf.LGF_ESTATE
        assert np.array_equal(lat.store(), U)
    with lgf.Lattice(dims, lgf.LGF_FP32_12) as lat:
        lat.load(U)
        assert lib.lgf_fix_begin(lat.h, lgf.LGF_FP32_12) == lgf.LGF_EINVAL


def test_split_finish_goes_on_below_its_fixed_point(lgf, orc):
    """Target 1e-26: the split links (within 2^-41 of the FP64 ones) reach it
    by their own measurement, but the FP64 links at that g sit near 1e-24 (a
    link error of ~5e-13 in each of the 8 terms of K).  The driver then goes
    on in FP64-12 and stops below the target on the FP64 links."""
    dims = (8, 8, 8, 8)
    announce("split finish continues", dims)
    with lgf.Lattice(dims, 0) as lat:
        lat.generate(0, 0.25, True)
        st, res, hist = lat.gauge_fix(omega=1.7, theta_target=1e-26, theta_switch=1e-8,
                                      bulk_format=lgf.LGF_FP32_12, finish_format=lgf.LGF_FP64_12S,
                                      fixed_links=1)
        got = lat.store()
    assert st == lgf.LGF_OK, res
    assert res["theta"] < 1e-26
    # the re-measurement on the FP64 links: same sweep count as the split
    # run's last check, theta above the target, and sweeps went on after it
    k = [i for i in range(1, len(hist)) if hist[i, 0] == hist[i - 1, 0] and hist[i - 1, 2] < 1e-26 <= hist[i, 2]]
    assert len(k) == 1, hist[-6:]
    assert res["sweeps"] > hist[k[0], 0]
    F, th = orc.measure(dims, got)
    # the oracle's theta of the same links: Delta ~ 1e-13 carries a rounding
    # of a few 1e-16, i.e. a few per cent of theta at this level
    assert th < 1.1e-26, th
    assert abs(F - res["F"]) < 1e-14


@pytest.mark.parametrize("bulk,finish", [(3, 4), (4, 3)])
def test_fp64_12_and_split_pair(lgf, orc, bulk, finish):
    """FP64-12 and the split format share one g field: a mixed run from one to
    the other hands g over without a conversion and converges."""
    dims = (4, 4, 6, 10)
    announce("fp64-12 / split pair", bulk, finish, dims)
    U = orc.generate_links(dims, 23, 0.3)
    with lgf.Lattice(dims, 0) as lat:
        lat.load(U)
        st, res, hist = lat.gauge_fix(omega=1.7, theta_target=1e-14, theta_switch=1e-8, bulk_format=bulk,
                                      finish_format=finish, fixed_links=1)
        got = lat.store()
    assert st == lgf.LGF_OK, res
    assert 0 < res["sweeps_bulk"] < res["sweeps"]
    F, th = orc.measure(dims, got)
    assert th < 1e-14 and abs(F - res["F"]) < 1e-14
