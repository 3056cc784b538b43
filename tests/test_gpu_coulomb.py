"""Coulomb-gauge path of the library against the oracle (GPU): one sweep with
and without frozen timeslices, per-timeslice F_C / theta_C, and the
per-timeslice gauge fixing."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import fp32_model as fm
from conftest import gpu_available
from lattice_np import stored_as, unitarity_error

pytestmark = pytest.mark.gpu

DIMS = [(4, 4, 6, 10), (6, 4, 4, 8), (2, 2, 2, 2)]


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


def maxabs(a, b):
    return float(np.abs(a - b).max())


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("omega,p_sr", [(1.7, 0.0), (1.0, 0.5)])
def test_coulomb_sweep_matches_oracle(lgf, orc, dims, omega, p_sr):
    announce("coulomb sweep", dims, omega, p_sr)
    U = orc.generate_links(dims, 31, 0.35)
    Lt = dims[0]
    masks = [None, [1 if t % 2 == 0 else 0 for t in range(Lt)]]
    for mask in masks:
        ref = U.copy()
        orc.sweep_coulomb(dims, ref, omega, p_sr, seed=4, sweep_index=2, slice_active=mask)
        with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
            lat.load(U)
            lat.sweep_coulomb(2, omega, p_sr, seed=4, sweep_index=2, slice_active=mask)
            assert maxabs(lat.store(), ref) < 1e-12, mask


@pytest.mark.parametrize("fmt", [0, 2, 3])
def test_coulomb_measure_matches_oracle(lgf, orc, fmt):
    dims = (6, 4, 4, 8)
    announce("coulomb measure", fmt)
    U = orc.generate_links(dims, 32, 0.35)
    with lgf.Lattice(dims, fmt) as lat:
        lat.load(U)
        F, th = lat.measure_coulomb()
    Fr, thr = orc.measure_coulomb(dims, stored_as(U, fmt))
    # FP32 12-real: row 2 rebuilt with fused multiply-adds on the GPU, without on the host
    tol = 2e-7 if fmt == 2 else 1e-12
    assert np.abs(F - Fr).max() < (2e-7 if fmt == 2 else 1e-14)
    assert np.abs(th - thr).max() < tol * thr.max()


def test_coulomb_gauge_fix_matches_oracle(lgf, orc):
    """FP64 Coulomb gauge fixing with per-timeslice stopping: the same
    per-timeslice sweep counts as the oracle, theta_C(t) below target, and the
    links of the oracle's run."""
    dims = (6, 6, 6, 6)
    announce("coulomb fix")
    U = orc.generate_links(dims, 33, 0.25)
    ref = U.copy()
    r = orc.coulomb_gauge_fix(dims, ref, 1.7, 1e-12)
    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        lat.load(U)
        st, res, sw, F, th = lat.coulomb_gauge_fix(omega=1.7, theta_target=1e-12)
        got = lat.store()
    assert st == lgf.LGF_OK and r["status"] == 0
    assert np.array_equal(sw, r["sweeps_t"])
    assert np.all(th < 1e-12)
    assert maxabs(got, ref) < 1e-9
    assert np.abs(F - r["F_t"]).max() < 1e-12


def test_coulomb_mixed_gauge_fix(lgf, orc):
    dims = (8, 6, 6, 6)
    announce("coulomb mixed")
    U = orc.generate_links(dims, 34, 0.3)
    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        lat.load(U)
        st, res, sw, F, th = lat.coulomb_gauge_fix(omega=1.7, theta_target=1e-14, theta_switch=1e-8,
                                                   bulk_format=lgf.LGF_FP32_12,
                                                   finish_format=lgf.LGF_FP64_12)
        got = lat.store()
    assert st == lgf.LGF_OK and 0 < res["sweeps_bulk"] < res["sweeps"]
    Fo, tho = orc.measure_coulomb(dims, got)
    assert np.all(tho < 1e-14) and unitarity_error(got) < 1e-12
    # gauge invariance: the temporal plaquettes are those of the input
    for nu in (1, 2, 3):
        assert abs(orc.wilson_loop(dims, got, 0, nu, 1, 1) - orc.wilson_loop(dims, U, 0, nu, 1, 1)) < 1e-5


def test_coulomb_accumulated_gauge_keeps_the_orbit(lgf, orc):
    """Mixed Coulomb gauge fixing with the accumulated gauge transformation:
    every timeslice below theta_C < 1e-14, and the links an FP64 gauge
    transformation of the input (temporal and spatial Wilson loops equal the
    input's to 1e-12, where the plain mixed run drifts by far more)."""
    dims = (8, 6, 6, 6)
    announce("coulomb accumulate_g")
    U = orc.generate_links(dims, 34, 0.3)
    loops = lambda V: np.array([orc.wilson_loop(dims, V, mu, nu, R, T) for mu in range(4)
                                for nu in range(mu + 1, 4) for (R, T) in [(1, 1), (1, 2)]])
    L0 = loops(U)
    drift = {}
    for acc in (0, 1):
        with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
            lat.load(U)
            st, res, sw, F, th = lat.coulomb_gauge_fix(omega=1.7, theta_target=1e-14, theta_switch=1e-8,
                                                       bulk_format=lgf.LGF_FP32_12,
                                                       finish_format=lgf.LGF_FP64_12, accumulate_g=acc)
            got = lat.store()
        assert st == lgf.LGF_OK and 0 < res["sweeps_bulk"] < res["sweeps"]
        assert np.all(orc.measure_coulomb(dims, got)[1] < 1e-14) and unitarity_error(got) < 1e-12
        drift[acc] = float(np.abs(loops(got) - L0).max())
    assert drift[1] < 1e-12 and drift[0] > 100 * drift[1], drift


def _links8(orc, dims, seed, eps, s):
    fw = [orc.generated_link(dims, seed, eps, True, s, mu) for mu in range(4)]
    bw = [orc.generated_link(dims, seed, eps, True, orc.neighbor(dims, s, mu, -1), mu) for mu in range(4)]
    return np.array(fw + bw)


def _gpu_links8(lat, orc, dims, s):
    nb = [orc.neighbor(dims, s, mu, -1) for mu in range(4)]
    P = lat.peek([s] + nb)
    return np.array([P[0, mu] for mu in range(4)] + [P[1 + mu, mu] for mu in range(4)])


@pytest.mark.parametrize("fmt", [3, 2])
def test_coulomb_48x3x96_sampled(lgf, orc, fmt):
    """The Coulomb workload at its full size (48^3 x 96, seed 5, eps 0.3, Haar
    gauge), in the formats of its mixed run: one parity-0 half-sweep with every
    other timeslice frozen, checked on sampled sites against the oracle's local
    update from its own generator (active timeslices) and against the
    untouched links (frozen ones); then F_C(t), theta_C(t) of every timeslice
    are finite, and only the relaxed timeslices gained in F_C."""
    dims = (96, 48, 48, 48)
    seed, eps, omega = 5, 0.3, 1.7
    announce("coulomb 48^3x96 sampled", fmt)
    V3 = 48 ** 3
    mask = [1 if t % 2 == 0 else 0 for t in range(dims[0])]
    rng = np.random.default_rng(3)
    V = dims[0] * V3
    cand = [0, 1, 47, V3 - 1, V3, V - 1, V - 2, 95 * V3 + 48] + [int(x) for x in rng.integers(0, V, 200)]
    sites = [s for s in cand if orc.parity(dims, s) == 0][:24]
    checked = []  # FP32: (input links, GPU links, oracle links) of the relaxed sites
    with lgf.Lattice(dims, fmt) as lat:
        lat.generate(seed, eps, True)
        before = {s: _gpu_links8(lat, orc, dims, s) for s in sites}
        lat.sweep_coulomb(0, omega, 0.0, 0, 0, slice_active=mask)
        for s in sites:
            got = _gpu_links8(lat, orc, dims, s)
            if mask[s // V3]:
                L8 = _links8(orc, dims, seed, eps, s)
                ref, _ = orc.local_update_coulomb(L8, omega, [0, 0, 0])
                if fmt == 3:
                    assert maxabs(got, ref) < 1e-12, s
                else:
                    checked.append((L8, got, ref))
            else:
                # a frozen site's spatial links (forward and backward) are only
                # ever written by sites of its own timeslice
                for k in (1, 2, 3, 5, 6, 7):
                    assert np.array_equal(got[k], before[s][k]), (s, k)
        F, th = lat.measure_coulomb()
    assert sum(mask[s // V3] for s in sites) >= 6 and sum(1 - mask[s // V3] for s in sites) >= 6
    if checked:
        # the FP32 bar: twice each link's randomised-rounding envelope (the
        # Coulomb update of the FP32-12 field the generator rounded), 2e-6 on
        # 99 % of the links
        L, got, ref = (np.array(x) for x in zip(*checked))
        env = fm.envelope(lambda R: fm.link_update(R, fm.stored(R, L, fmt), omega, np.zeros((len(L), 3), bool),
                                                   fmt, mu_first=1), ref)
        ok, info = fm.fp32_bar_ok(got, ref, env)
        assert ok, info
    # from a Haar-random gauge F_C(t) starts near 0 (either sign); the relaxed
    # timeslices gained, the frozen ones did not
    act = np.array(mask, dtype=bool)
    assert np.all(np.isfinite(F)) and np.all(np.abs(F) < 1) and np.all(th > 0)
    assert F[act].min() > 100 * np.abs(F[~act]).max()


# ------------------------------------------------------------ fixed-link form

@pytest.mark.parametrize("dims", DIMS + [(8, 8, 8, 16)])
@pytest.mark.parametrize("handle_fmt,sweep_fmt", [(0, 0), (0, 3), (0, 2)])
@pytest.mark.parametrize("omega,p_sr", [(1.7, 0.0), (1.0, 0.5)])
def test_coulomb_fixed_sweep_matches_oracle(lgf, orc, dims, handle_fmt, sweep_fmt, omega, p_sr):
    """One Coulomb sweep of every timeslice with the links fixed (a gauge
    fixing stopped after one sweep hands back g U g^dag, g reunitarized): the
    oracle's Coulomb sweep of the links, then reunitarized, for tunings on the
    link field and on per-site link records (the 12-real formats; one lane per
    site in FP32); the blocked tile order is taken on (8, 8, 8, 16)."""
    announce("coulomb fixed sweep", dims, handle_fmt, sweep_fmt, omega, p_sr)
    U = orc.generate_links(dims, 31, 0.35)
    ref = U.copy()
    orc.sweep_coulomb(dims, ref, omega, p_sr, seed=4, sweep_index=2)
    orc.reunitarize(ref)
    Fr, thr = orc.measure_coulomb(dims, ref)
    env = None
    if sweep_fmt == 2:
        env = fm.fixed_sweep_envelope(orc, dims, U, 2, ref, omega, p_sr, 4, 2, mu_first=1)
    tunes = [(2, 128, 0, 0), (4, 64, 2, 0), (2, 64, 2, 0)]
    if sweep_fmt in (2, 3):
        tunes += [(2, 128, 2, 1), (4, 256, 0, 1)] + ([(1, 64, 3, 1)] if sweep_fmt == 2 else [])
    for tune in tunes:
        with lgf.Lattice(dims, handle_fmt) as lat:
            lgf.lgf_set_fixed_tuning(lat.h, sweep_fmt, *tune)
            lat.load(U)
            kw = dict(omega=omega, p_sr=p_sr, seed=4, sweep_offset=2, theta_target=1e-300, check_every=1,
                      max_sweeps=1, fixed_links=1)
            if sweep_fmt != handle_fmt:
                kw.update(bulk_format=sweep_fmt, finish_format=handle_fmt, theta_switch=1e-300)
            st, res, sw, F, th = lat.coulomb_gauge_fix(**kw)
            got = lat.store()
        assert st == lgf.LGF_ENOTCONV and res["sweeps"] == 1
        assert unitarity_error(got) < 1e-12
        if sweep_fmt == 2:
            ok, info = fm.fp32_bar_ok(got, ref, env)
            assert ok, (tune, info)
        else:
            assert maxabs(got, ref) < 1e-12, (tune, maxabs(got, ref))
            assert np.abs(F - Fr).max() < 1e-13 and np.all(np.abs(th - thr) <= 1e-12 * thr + 1e-15), tune


def test_coulomb_fixed_gauge_fix_matches_link_form(lgf, orc):
    """FP64 Coulomb gauge fixing with per-timeslice stopping, links fixed:
    the oracle's per-timeslice sweep counts, theta_C(t) below target, its F_C(t)
    and links; the Wilson loops of the input kept to 1e-12."""
    dims = (6, 6, 6, 6)
    announce("coulomb fixed fix")
    U = orc.generate_links(dims, 33, 0.25)
    ref = U.copy()
    r = orc.coulomb_gauge_fix(dims, ref, 1.7, 1e-12)
    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        lat.load(U)
        st, res, sw, F, th = lat.coulomb_gauge_fix(omega=1.7, theta_target=1e-12, fixed_links=1)
        got = lat.store()
    assert st == lgf.LGF_OK and r["status"] == 0
    assert np.array_equal(sw, r["sweeps_t"])
    assert np.all(th < 1e-12)
    assert maxabs(got, ref) < 1e-9
    assert np.abs(F - r["F_t"]).max() < 1e-12
    for nu in (1, 2, 3):
        assert abs(orc.wilson_loop(dims, got, 0, nu, 1, 2) - orc.wilson_loop(dims, U, 0, nu, 1, 2)) < 1e-12


@pytest.mark.parametrize("finish", [0, 3])
def test_coulomb_fixed_mixed_keeps_the_orbit(lgf, orc, finish):
    """Mixed Coulomb gauge fixing (FP32-12 bulk, switch at 1e-8) with the links
    fixed: every timeslice below theta_C < 1e-14 on the links handed back, an
    FP64 gauge transformation of the input (temporal and spatial Wilson loops
    to 1e-12), also when stopped inside the bulk."""
    dims = (8, 6, 6, 6)
    announce("coulomb fixed mixed", finish)
    U = orc.generate_links(dims, 34, 0.3)
    loops = lambda V: np.array([orc.wilson_loop(dims, V, mu, nu, R, T) for mu in range(4)
                                for nu in range(mu + 1, 4) for (R, T) in [(1, 1), (1, 2)]])
    L0 = loops(U)
    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        lat.load(U)
        st, res, sw, F, th = lat.coulomb_gauge_fix(omega=1.7, theta_target=1e-14, theta_switch=1e-8,
                                                   bulk_format=lgf.LGF_FP32_12, finish_format=finish,
                                                   fixed_links=1)
        got = lat.store()
    assert st == lgf.LGF_OK and 0 < res["sweeps_bulk"] < res["sweeps"]
    Fo, tho = orc.measure_coulomb(dims, got)
    assert np.all(tho < 1e-14) and np.abs(Fo - F).max() < 1e-13 and unitarity_error(got) < 1e-12
    assert float(np.abs(loops(got) - L0).max()) < 1e-12
    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        lat.load(U)
        st, res, sw, F, th = lat.coulomb_gauge_fix(omega=1.7, theta_target=1e-14, theta_switch=1e-30,
                                                   max_sweeps=30, bulk_format=lgf.LGF_FP32_12,
                                                   finish_format=finish, fixed_links=1)
        got = lat.store()
        assert st == lgf.LGF_ENOTCONV and res["sweeps_bulk"] == 30
        assert float(np.abs(loops(got) - L0).max()) < 1e-12


def test_coulomb_fixed_graph_equals_direct(lgf, orc):
    """Captured chunks of the fixed-link Coulomb sweeps (timeslice flags read
    from the device) give the direct launches' links bit for bit, OR and SR."""
    dims = (6, 4, 4, 8)
    announce("coulomb fixed graph")
    U = orc.generate_links(dims, 35, 0.3)
    for kw in (dict(omega=1.7, theta_target=1e-13), dict(omega=1.0, p_sr=0.5, seed=3, theta_target=1e-30,
                                                         check_every=4, max_sweeps=12)):
        out = []
        for g in (0, 1):
            with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
                lat.load(U)
                st, res, sw, F, th = lat.coulomb_gauge_fix(use_graph=g, fixed_links=1, **kw)
                out.append((st, sw, F, th, lat.store()))
        for a, b in zip(out[0], out[1]):
            assert np.array_equal(np.asarray(a), np.asarray(b)), kw


@pytest.mark.parametrize("fmt", [3, 4])
def test_coulomb_fixed_48x3x96_sampled(lgf, orc, fmt):
    """The Coulomb workload at its full size (48^3 x 96, seed 5, eps 0.3, Haar
    gauge) in the form its benchmark leg runs: one full fixed-link Coulomb
    sweep, the links read from their per-site records (the default at this
    size), FP64-12 or the split links (format 4).  Checked on sampled parity-1
    sites (edges and wrap-arounds included): the oracle redoes the parity-0
    Coulomb updates at the other ends of the site's links, then the site's own
    update; all 8 links move, the temporal ones too.  Bar 1e-12 in FP64-12; on
    the split links the oracle's updates take the split-stored links, whose
    entries differ from the input by at most 2^-40 (rows 0, 1) and 4 x 2^-40
    (row 2), so 9 x 4 x 2^-40 more per entry of g (U - U') g^dag."""
    from lattice_np import SPLIT_UNIT, split_stored
    from test_gpu_parity import gpu_links8, sample_sites
    dims = (96, 48, 48, 48)
    seed, eps, omega = 5, 0.3, 1.7
    announce("coulomb fixed 48^3x96 sampled", fmt)
    rng = np.random.default_rng(4)
    split = fmt == lgf.LGF_FP64_12S
    bar = 1e-12 + (36 * SPLIT_UNIT if split else 0.0)

    def upd(links):
        out, _ = orc.local_update_coulomb(split_stored(links) if split else links, omega, [0, 0, 0])
        return out

    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        assert lgf.lgf_get_fixed_tuning(lat.h, fmt)[3] == 1
        lat.generate(seed, eps, True)
        st, res, sw, F, th = lat.coulomb_gauge_fix(omega=omega, theta_target=1e-300, check_every=1, max_sweeps=1,
                                                   fixed_links=1, bulk_format=fmt, finish_format=fmt)
        assert st == lgf.LGF_ENOTCONV and res["sweeps"] == 1 and np.all(sw == 1)
        ys = sample_sites(orc, dims, 1, 8, rng)
        for y in ys:
            links = np.zeros((8, 3, 3), dtype=np.complex128)
            for mu in range(4):
                links[mu] = upd(_links8(orc, dims, seed, eps, orc.neighbor(dims, y, mu, +1)))[4 + mu]
                links[4 + mu] = upd(_links8(orc, dims, seed, eps, orc.neighbor(dims, y, mu, -1)))[mu]
            ref = upd(links)
            e = maxabs(gpu_links8(lat, orc, dims, y), ref)
            assert e < bar, (y, e, bar)
        assert np.all(np.isfinite(F)) and np.all(np.isfinite(th)) and np.all(th > 0)
    assert len(ys) == 8
