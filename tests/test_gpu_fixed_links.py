"""The fixed-link form of the sweep (lgf_fix_params.fixed_links) against the
FP64 oracle, through the C ABI.  The library keeps the links fixed and
updates the gauge transformation g; what it hands back, g(x) U_mu(x)
g(x+mu)^dag from the input, must be what the oracle's link-rewriting sweeps
produce: after one sweep element by element (1e-12 for FP64 sweeps; the FP32
per-link bound of the other parity tests for FP32 sweeps), and over whole gauge
fixings the same theta history, sweeps and F, with the gauge orbit of the
input kept exactly (Wilson loops to 1e-12) also when the bulk runs in FP32."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import fp32_model as fm
from conftest import gpu_available
from lattice_np import unitarity_error

pytestmark = pytest.mark.gpu

SMALL_DIMS = [(2, 2, 2, 2), (4, 4, 6, 10), (8, 6, 4, 12), (4, 8, 8, 8)]
# (lanes per site, block, tile order); order 2 falls back to 0 where the
# lattice does not split into 8k blocks of t-slices x z-planes of whole tiles
# ((4, 8, 8, 8) takes it, with 32-site tiles)
FIXED_TUNINGS = [(2, 128, 0), (4, 64, 1), (2, 256, 1), (4, 128, 0), (2, 64, 2), (4, 128, 2)]
# (lanes per site, block, tile order, link layout): per-site link records in
# the 12-real formats, one lane per site in the FP32 formats
RECORD_TUNINGS = [(2, 256, 3, 1), (4, 64, 0, 1), (2, 64, 2, 1)]
ONE_LANE_TUNINGS = [(1, 128, 0, 0), (1, 64, 3, 0)]


def tunings_for(fmt):
    return (FIXED_TUNINGS + (RECORD_TUNINGS if fmt in (2, 3) else []) +
            (ONE_LANE_TUNINGS + [(1, 256, 1, 1)] * (fmt == 2) if fmt in (1, 2) else []))


def apply_tune(lgf, h, fmt, tune):
    """set a tuning on one format, leaving out what the format does not take
    (records outside the 12-real and split formats, one lane outside FP32)"""
    lps, block, order, layout = (tuple(tune) + (0,))[:4]
    if fmt not in (2, 3, 4):
        layout = 0
    if lps == 1 and fmt not in (1, 2):
        lps = 2
    lgf.lgf_set_fixed_tuning(h, fmt, lps, block, order, layout)


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


def fp32_ok(got, ref, env):
    """2e-6 relative on 99 % of the links, and on every link twice its
    randomised-rounding envelope (fp32_model) plus u"""
    return fm.fp32_bar_ok(got, ref, env)[0]


def loops(orc, dims, U):
    return np.array([orc.wilson_loop(dims, U, mu, nu, R, T) for mu in range(4) for nu in range(mu + 1, 4)
                     for (R, T) in [(1, 1), (1, 2), (2, 2)]])


def one_fixed_sweep(lgf, dims, U, handle_fmt, sweep_fmt, tune, omega, p_sr, seed, sweep_index):
    """One full sweep in the fixed-link form (a chunk of one sweep stops at
    max_sweeps), the links handed back"""
    with lgf.Lattice(dims, handle_fmt) as lat:
        lgf.lgf_set_fixed_tuning(lat.h, sweep_fmt, *tune)
        lat.load(U)
        kw = dict(omega=omega, p_sr=p_sr, seed=seed, sweep_offset=sweep_index, theta_target=1e-300,
                  check_every=1, max_sweeps=1, fixed_links=1)
        if sweep_fmt != handle_fmt:
            kw.update(bulk_format=sweep_fmt, finish_format=handle_fmt, theta_switch=1e-300)
        st, res, hist = lat.gauge_fix(**kw)
        assert st == lgf.LGF_ENOTCONV and res["sweeps"] == 1, res
        return lat.store(), res, hist


@pytest.mark.parametrize("dims", SMALL_DIMS)
@pytest.mark.parametrize("handle_fmt,sweep_fmt", [(0, 0), (3, 3), (0, 3), (0, 2), (3, 1)])
@pytest.mark.parametrize("omega,p_sr", [(1.0, 0.0), (1.7, 0.0), (1.0, 0.5), (1.8, 0.3)])
def test_fixed_sweep_matches_oracle(lgf, orc, dims, handle_fmt, sweep_fmt, omega, p_sr):
    """One full sweep with the links fixed equals the oracle's sweep of the
    links (then reunitarized), for every tuning; the measured F and theta are
    those of the oracle's links."""
    announce("fixed sweep", dims, handle_fmt, sweep_fmt, omega, p_sr)
    U = orc.generate_links(dims, 7, 0.35)
    ref = U.copy()
    orc.sweep(dims, ref, omega, p_sr, seed=9, sweep_index=3)
    orc.reunitarize(ref)
    F_ref, th_ref = orc.measure(dims, ref)
    env = None
    if sweep_fmt not in (0, 3):
        env = fm.fixed_sweep_envelope(orc, dims, U, sweep_fmt, ref, omega, p_sr, 9, 3)
    for tune in tunings_for(sweep_fmt):
        got, res, hist = one_fixed_sweep(lgf, dims, U, handle_fmt, sweep_fmt, tune, omega, p_sr, 9, 3)
        if sweep_fmt in (0, 3):
            assert maxabs(got, ref) <= 1e-12, (tune, maxabs(got, ref))
            assert abs(res["F"] - F_ref) <= 1e-13 and abs(res["theta"] - th_ref) <= 1e-12 * th_ref + 1e-15, (
                tune, res["F"] - F_ref, res["theta"] / th_ref - 1)
        else:
            assert fp32_ok(got, ref, env), (tune, fm.fp32_bar_ok(got, ref, env)[1])
        assert unitarity_error(got) < 1e-12


def test_fixed_gauge_fix_8x4_matches_oracle_history(lgf, orc):
    """8^4, seed 0, eps 0.25, Haar gauge, omega 1.7 to theta < 1e-12 with the
    links fixed: the oracle's theta history (1e-8 relative while theta >
    1e-10), its number of sweeps, its F, and its final links."""
    dims = (8, 8, 8, 8)
    announce("fixed gauge_fix_8x4")
    U = orc.generate_links(dims, 0, 0.25)
    ref = U.copy()
    r_orc = orc.gauge_fix(dims, ref, 1.7, 1e-12)
    for handle_fmt in (0, 3):
        with lgf.Lattice(dims, handle_fmt) as lat:
            lat.load(U)
            st, res, hist = lat.gauge_fix(omega=1.7, theta_target=1e-12, fixed_links=1)
            got = lat.store()
        assert st == 0 and res["theta"] < 1e-12
        h_orc = r_orc["history"]
        assert res["sweeps"] == r_orc["sweeps"]
        for k in range(min(len(hist), len(h_orc))):
            if h_orc[k, 2] > 1e-10:
                assert abs(hist[k, 2] - h_orc[k, 2]) <= 1e-8 * h_orc[k, 2], (handle_fmt, k)
                assert abs(hist[k, 1] - h_orc[k, 1]) <= 1e-12, (handle_fmt, k)
        assert abs(res["F"] - r_orc["F"]) < 1e-12
        assert maxabs(got, ref) < 1e-9


@pytest.mark.parametrize("finish", [0, 3])
def test_fixed_mixed_keeps_the_orbit(lgf, orc, finish):
    """FP32-12 bulk, switch at theta < 1e-8, FP64 finish, links fixed: theta <
    1e-14 on the links handed back (the oracle measures them), which are an
    exact FP64 gauge transformation of the input (Wilson loops to 1e-12,
    links unitary), the finish running on the input links themselves; the
    same when stopped inside the bulk."""
    dims = (8, 8, 8, 8)
    announce("fixed mixed", finish)
    U = orc.generate_links(dims, 1, 0.25)
    L0 = loops(orc, dims, U)
    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        lat.load(U)
        st, res, hist = lat.gauge_fix(omega=1.7, theta_target=1e-14, theta_switch=1e-8, fixed_links=1,
                                      bulk_format=lgf.LGF_FP32_12, finish_format=finish)
        got = lat.store()
    assert st == 0 and 0 < res["sweeps_bulk"] < res["sweeps"]
    F, th = orc.measure(dims, got)
    assert th < 1e-14 and abs(F - res["F"]) < 1e-13
    assert float(np.abs(loops(orc, dims, got) - L0).max()) < 1e-12
    assert unitarity_error(got) < 1e-12
    # the bulk's last measurement is above the switch, the next one below
    k = int(np.searchsorted(hist[:, 0], res["sweeps_bulk"]))
    assert hist[k, 2] < 1e-8 and hist[k - 1, 2] >= 1e-8
    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        lat.load(U)
        st, res, _ = lat.gauge_fix(omega=1.7, theta_target=1e-14, theta_switch=1e-30, max_sweeps=40,
                                   fixed_links=1, bulk_format=lgf.LGF_FP32_12, finish_format=finish)
        got = lat.store()
        assert st == lgf.LGF_ENOTCONV and res["sweeps_bulk"] == 40
        assert float(np.abs(loops(orc, dims, got) - L0).max()) < 1e-12
        assert unitarity_error(got) < 1e-12


@pytest.mark.parametrize("tune", [(2, 128, 0), (4, 64, 1), (2, 128, 2), (2, 64, 3, 1), (1, 256, 0, 1)])
def test_fixed_fused_measure_equals_separate_passes(lgf, orc, tune):
    """F and theta inside the chunk's last half-sweep (plus one read-only pass
    over parity 0) against two read-only passes: the same g, hence the same
    links bit for bit, and F, theta equal up to the summation order -- plain
    FP64, mixed, stochastic relaxation, and chunks cut short."""
    dims = (8, 8, 8, 16)   # the blocked tile order applies (64-site tiles)
    announce("fixed fused", tune)
    U = orc.generate_links(dims, 51, 0.3)
    runs = [dict(omega=1.7, theta_target=1e-12),
            dict(omega=1.7, theta_target=1e-13, theta_switch=1e-8, bulk_format=lgf.LGF_FP32_12,
                 finish_format=lgf.LGF_FP64_12),
            dict(omega=1.0, p_sr=0.3, seed=5, theta_target=1e-30, check_every=7, max_sweeps=30)]
    for kw in runs:
        out = []
        for sep in (1, 0):
            with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
                for f in range(4):
                    apply_tune(lgf, lat.h, f, tune)
                lat.load(U)
                st, res, hist = lat.gauge_fix(separate_measure=sep, fixed_links=1, **kw)
                out.append((st, res, hist, lat.store()))
        (st1, r1, h1, U1), (st0, r0, h0, U0) = out
        assert st1 == st0 and (st0 == lgf.LGF_OK or kw.get("max_sweeps")), kw
        assert r1["sweeps"] == r0["sweeps"] and r1["sweeps_bulk"] == r0["sweeps_bulk"], kw
        assert np.array_equal(U0, U1), (kw, maxabs(U0, U1))
        assert np.array_equal(h0[:, 0], h1[:, 0])
        assert np.allclose(h0[:, 1], h1[:, 1], rtol=1e-13, atol=0), kw
        dth = np.abs(h0[:, 2] - h1[:, 2])
        assert np.all(dth <= 1e-14 * np.sqrt(h1[:, 2]) + 1e-12 * h1[:, 2]), (kw, float((dth / h1[:, 2]).max()))


def test_fixed_graph_equals_direct(lgf, orc):
    """Chunks replayed from captured hipGraphs give the links and the history
    of direct launches bit for bit, for overrelaxation and for stochastic
    relaxation (whose counter the graph reads from device memory)."""
    dims = (4, 4, 6, 10)
    announce("fixed graph vs direct")
    U = orc.generate_links(dims, 12, 0.3)
    for kw in (dict(omega=1.7, theta_target=1e-13, theta_switch=1e-8, bulk_format=lgf.LGF_FP32_12,
                    finish_format=lgf.LGF_FP64_12),
               dict(omega=1.0, p_sr=0.5, seed=77, sweep_offset=11, theta_target=1e-30, check_every=5,
                    max_sweeps=25)):
        out = []
        for g in (0, 1):
            with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
                lat.load(U)
                st, res, hist = lat.gauge_fix(use_graph=g, fixed_links=1, **kw)
                out.append((st, res["sweeps"], hist, lat.store()))
        assert out[0][0] == out[1][0] and out[0][1] == out[1][1], kw
        assert np.array_equal(out[0][2], out[1][2]), kw
        assert np.array_equal(out[0][3], out[1][3]), kw


def test_fixed_tunings_agree(lgf, orc):
    """Workgroup size and tile order do not change a bit (the blocked order
    is taken on this lattice); 2 and 4 lanes per site sum M in a different
    order, so they agree to rounding."""
    dims = (8, 8, 16, 16)
    announce("fixed tunings")
    U = orc.generate_links(dims, 3, 0.3)
    outs = {}
    for tune in [(2, 64, 0), (2, 256, 1), (2, 128, 2), (4, 128, 0), (4, 64, 1), (4, 256, 2)]:
        got, res, hist = one_fixed_sweep(lgf, dims, U, 0, 0, tune, 1.7, 0.3, 4, 1)
        outs[tune] = (got, res["F"], res["theta"])
    for a, b in [((2, 64, 0), (2, 256, 1)), ((2, 64, 0), (2, 128, 2)), ((4, 128, 0), (4, 64, 1)),
                 ((4, 128, 0), (4, 256, 2))]:
        assert np.array_equal(outs[a][0], outs[b][0]), (a, b)
    assert maxabs(outs[(2, 64, 0)][0], outs[(4, 128, 0)][0]) < 1e-14


def test_fixed_records_and_lockstep_order_change_no_bit(lgf, orc):
    """The per-site link records hold the link field's values and the lockstep
    tile order only reorders the workgroups (each keeps its tile's partial-sum
    slot): the links, F and theta of two chunks are bit for bit those of the
    link field in lexicographic order, for FP64-12 and FP32-12,
    overrelaxation and stochastic relaxation, 1, 2 and 4 lanes per site; the
    lockstep order is taken on this lattice (planes of 8 tiles of 64 sites)."""
    dims = (4, 4, 32, 32)
    announce("fixed records", dims)
    U = orc.generate_links(dims, 17, 0.3)
    for fmt, lanes in [(3, (2, 4)), (2, (1, 2, 4))]:
        for lps in lanes:
            block = 64 * lps
            outs = []
            for order, layout in [(0, 0), (0, 1), (3, 0), (3, 1)]:
                for omega, p_sr in [(1.8, 0.0), (1.0, 0.4)]:
                    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
                        lgf.lgf_set_fixed_tuning(lat.h, fmt, lps, block, order, layout)
                        assert lgf.lgf_get_fixed_tuning(lat.h, fmt) == (lps, block, order, layout)
                        lat.load(U)
                        kw = dict(omega=omega, p_sr=p_sr, seed=3, theta_target=1e-300, check_every=3,
                                  max_sweeps=6, fixed_links=1, bulk_format=fmt, finish_format=fmt)
                        st, res, hist = lat.gauge_fix(**kw)
                        assert st == lgf.LGF_ENOTCONV and res["sweeps"] == 6, res
                        outs.append(((order, layout, omega), lat.store(), hist))
            base = {k[2]: (U1, h1) for k, U1, h1 in outs if k[:2] == (0, 0)}
            for k, U1, h1 in outs:
                U0, h0 = base[k[2]]
                assert np.array_equal(U0, U1), (fmt, lps, k, maxabs(U0, U1))
                assert np.array_equal(h0, h1), (fmt, lps, k)


def test_fixed_autotune_leaves_links_untouched(lgf, orc):
    """The fixed-link autotuner reads the links and writes only the gauge
    transformation: the links come back bit for bit, the pick is a valid
    tuning, and a gauge fixing after it still converges."""
    dims = (8, 8, 16, 16)
    announce("fixed autotune")
    U = orc.generate_links(dims, 45, 0.3)
    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        lat.load(U)
        before = lat.store()
        for fmt in (lgf.LGF_FP64_12, lgf.LGF_FP32_12, lgf.LGF_FP64_18):
            lgf.lgf_autotune_fixed(lat.h, fmt, 1)
            assert np.array_equal(lat.store(), before)
            t = lgf.lgf_get_fixed_tuning(lat.h, fmt)
            lgf.lgf_set_fixed_tuning(lat.h, fmt, *t)
        st, res, _ = lat.gauge_fix(omega=1.7, theta_target=1e-13, theta_switch=1e-8, fixed_links=1,
                                   bulk_format=lgf.LGF_FP32_12, finish_format=lgf.LGF_FP64_12)
        assert st == lgf.LGF_OK and orc.measure(dims, lat.store())[1] < 1e-13


def test_fixed_links_argument_checks(lgf, orc):
    dims = (4, 4, 4, 4)
    announce("fixed checks")
    with lgf.Lattice(dims, lgf.LGF_FP32_12) as lat:
        lat.generate(1, 0.2, True)
        with pytest.raises(lgf.LgfError):
            lat.gauge_fix(omega=1.7, fixed_links=1)   # needs an FP64 handle
    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        # defaults: FP64-12 in the blocked tile order, FP32-12 one lane per
        # site, both on the link field below 2^18 sites, on per-site records
        # from there on
        assert lgf.lgf_get_fixed_tuning(lat.h, 3) == (2, 128, 2, 0)
        assert lgf.lgf_get_fixed_tuning(lat.h, 0) == (2, 64, 2, 0)
        assert lgf.lgf_get_fixed_tuning(lat.h, 2) == (1, 128, 0, 0)
        assert lgf.lgf_get_fixed_tuning(lat.h, 1) == (2, 256, 0, 0)
        with lgf.Lattice((16, 16, 32, 32), lgf.LGF_FP64_18) as big:
            assert lgf.lgf_get_fixed_tuning(big.h, 3) == (2, 128, 2, 1)
            assert lgf.lgf_get_fixed_tuning(big.h, 2) == (1, 128, 0, 1)
        with lgf.Lattice((16, 16, 32, 30), lgf.LGF_FP64_18) as small:
            assert lgf.lgf_get_fixed_tuning(small.h, 3) == (2, 128, 2, 0)
        for bad in [(1, 128, 0), (8, 128, 0), (2, 96, 0), (2, 128, 4), (2, 128, -1), (2, 128, 0, 1),
                    (2, 128, 0, 2)]:
            with pytest.raises(lgf.LgfError):
                lgf.lgf_set_fixed_tuning(lat.h, 0, *bad)
        for fmt, bad in [(3, (1, 128, 0)), (3, (2, 128, 0, 2)), (1, (2, 128, 0, 1)), (4, (2, 64, 2, 2)),
                         (4, (1, 64, 2))]:
            with pytest.raises(lgf.LgfError):
                lgf.lgf_set_fixed_tuning(lat.h, fmt, *bad)
        lgf.lgf_set_fixed_tuning(lat.h, 3, 4, 256, 1)
        assert lgf.lgf_get_fixed_tuning(lat.h, 3) == (4, 256, 1, 0)
        lgf.lgf_set_fixed_tuning(lat.h, 2, 1, 64, 3, 1)
        assert lgf.lgf_get_fixed_tuning(lat.h, 2) == (1, 64, 3, 1)
        lgf.lgf_set_fixed_tuning(lat.h, 1, 1, 128, 0)
        assert lgf.lgf_get_fixed_tuning(lat.h, 1) == (1, 128, 0, 0)


def fixed_links8_model(R, orc, dims, seed, eps, omega, ys, fmt):
    """The randomised-rounding model of one fixed-link FP32 sweep around
    parity-1 sites ys: the parity-0 neighbours' g from their own links (g = 1
    around them), then g(y) from those, and the 8 links of y as the library
    hands them back, g U g^dag in FP64 (forward links then backward)."""
    from test_gpu_parity import oracle_links8
    n = len(ys)
    eye = np.broadcast_to(np.eye(3, dtype=np.complex128), (1, 4, 3, 3))

    def g_new(L8):
        m = L8.shape[0]
        L = fm.stored(R, L8, fmt)
        one = np.broadcast_to(eye, (m, 4, 3, 3))
        return fm.fixed_update(R, L[:, :4], one, L[:, 4:], one, one[:, 0], omega, np.zeros((m, 3), bool), fmt)

    nbf = [orc.neighbor(dims, y, mu, +1) for y in ys for mu in range(4)]
    nbb = [orc.neighbor(dims, y, mu, -1) for y in ys for mu in range(4)]
    gf = g_new(np.array([oracle_links8(orc, dims, seed, eps, s) for s in nbf])).reshape(n, 4, 3, 3)
    gb = g_new(np.array([oracle_links8(orc, dims, seed, eps, s) for s in nbb])).reshape(n, 4, 3, 3)
    Ly = np.array([oracle_links8(orc, dims, seed, eps, y) for y in ys])
    Ls = fm.stored(R, Ly, fmt)
    one = np.broadcast_to(np.eye(3, dtype=np.complex128), (n, 3, 3))
    gy = fm.fixed_update(R, Ls[:, :4], gf, Ls[:, 4:], gb, one, omega, np.zeros((n, 3), bool), fmt)
    gy, gf, gb = fm.reunitarize(gy), fm.reunitarize(gf), fm.reunitarize(gb)
    out = np.empty_like(Ly)
    for mu in range(4):
        out[:, mu] = gy @ Ly[:, mu] @ fm.dag(gf[:, mu])
        out[:, 4 + mu] = gb[:, mu] @ Ly[:, 4 + mu] @ fm.dag(gy)
    return out


@pytest.mark.parametrize("handle_fmt,sweep_fmt,driver", [(0, 3, "gauge_fix"), (0, 2, "gauge_fix"), (0, 3, "session")])
def test_fixed_64x4_sampled(lgf, orc, handle_fmt, sweep_fmt, driver):
    """The 64^4 workload (seed 3, eps 0.3, Haar gauge) at omega 1.8: one full
    sweep with the links fixed, in the formats of the benchmark's step (FP64-12)
    and bulk, checked on sampled parity-1 sites (edges and wrap-arounds
    included): the oracle rebuilds the input links from its own generator,
    redoes the parity-0 updates at the other ends of the site's links, then the
    site's own update.  driver "session": the sweep as the benchmark's step
    runs it, one chunk of a stepwise session (captured in a hipGraph, the
    autotuner's variant)."""
    dims = (64, 64, 64, 64)
    seed, eps, omega = 3, 0.3, 1.8
    announce("fixed 64^4 sampled", handle_fmt, sweep_fmt, driver)
    from test_gpu_parity import gpu_links8, oracle_links8, sample_sites
    rng = np.random.default_rng(2)

    def upd(s):
        out, _ = orc.local_update(oracle_links8(orc, dims, seed, eps, s), omega, [0, 0, 0])
        return out

    with lgf.Lattice(dims, handle_fmt) as lat:
        lat.generate(seed, eps, True)
        if driver == "session":
            lgf.lgf_autotune_fixed(lat.h, sweep_fmt, 2)
            lat.fix_begin(sweep_fmt)
            F, th, _ = lat.fix_chunk(1, omega)
            lat.fix_end()
            res = {"F": F, "theta": th}
        else:
            kw = dict(omega=omega, theta_target=1e-300, check_every=1, max_sweeps=1, fixed_links=1)
            if sweep_fmt != handle_fmt:
                kw.update(bulk_format=sweep_fmt, finish_format=sweep_fmt)
            st, res, _ = lat.gauge_fix(**kw)
            assert st == lgf.LGF_ENOTCONV and res["sweeps"] == 1
        ys, gots, refs = [], [], []
        for y in sample_sites(orc, dims, 1, 8, rng):
            links = np.zeros((8, 3, 3), dtype=np.complex128)
            for mu in range(4):
                links[mu] = upd(orc.neighbor(dims, y, mu, +1))[4 + mu]
                links[4 + mu] = upd(orc.neighbor(dims, y, mu, -1))[mu]
            ref, _ = orc.local_update(links, omega, [0, 0, 0])
            got = gpu_links8(lat, orc, dims, y)
            if sweep_fmt in (0, 3):
                assert maxabs(got, ref) < 1e-12, y
            ys.append(y)
            gots.append(got)
            refs.append(ref)
        if sweep_fmt not in (0, 3):
            env = fm.envelope(lambda R: fixed_links8_model(R, orc, dims, seed, eps, omega, ys, sweep_fmt),
                              np.array(refs))
            ok, info = fm.fp32_bar_ok(np.array(gots), np.array(refs), env)
            assert ok, info
        assert 0 < res["F"] < 1 and np.isfinite(res["theta"])


def test_fixed_large_lattice_beyond_32bit_vector_indices(lgf, orc):
    """64 x 128^3 (134M sites) with FP64-18 links and g: 4.8e9 16-byte link
    vectors, so addresses pass 2^32 vectors.  One fixed-link sweep (fused
    measurement included), checked on sampled parity-1 sites, the last planes
    among them, against the oracle's updates of the neighbourhood."""
    dims = (64, 128, 128, 128)
    seed, eps, omega = 4, 0.3, 1.8
    announce("fixed 64x128^3")
    from test_gpu_parity import gpu_links8, oracle_links8, sample_sites
    rng = np.random.default_rng(5)

    def upd(s):
        out, _ = orc.local_update(oracle_links8(orc, dims, seed, eps, s), omega, [0, 0, 0])
        return out

    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        lat.generate(seed, eps, True)
        st, res, _ = lat.gauge_fix(omega=omega, theta_target=1e-300, check_every=1, max_sweeps=1, fixed_links=1)
        assert st == lgf.LGF_ENOTCONV and res["sweeps"] == 1
        for y in sample_sites(orc, dims, 1, 6, rng):
            links = np.zeros((8, 3, 3), dtype=np.complex128)
            for mu in range(4):
                links[mu] = upd(orc.neighbor(dims, y, mu, +1))[4 + mu]
                links[4 + mu] = upd(orc.neighbor(dims, y, mu, -1))[mu]
            ref, _ = orc.local_update(links, omega, [0, 0, 0])
            assert maxabs(gpu_links8(lat, orc, dims, y), ref) < 1e-12, y
        assert 0 < res["F"] < 1 and np.isfinite(res["theta"])


def test_fixed_records_beyond_32bit_vector_indices(lgf, orc):
    """64 x 128^3 (134M sites) on an FP64-12 handle, the sweeps reading its
    per-site link records (the format's default): 6.4e9 16-byte record
    vectors, parity 1's from 3.2e9 on, so their addresses pass 2^32 vectors.
    One fixed-link sweep checked on sampled parity-1 sites, the last tiles
    among them, against the oracle's updates of the neighbourhood; the
    records stay in use (no fall-back to the link field)."""
    dims = (64, 128, 128, 128)
    seed, eps, omega = 6, 0.3, 1.8
    announce("fixed records 64x128^3")
    from test_gpu_parity import gpu_links8, oracle_links8, sample_sites
    rng = np.random.default_rng(7)

    def upd(s):
        out, _ = orc.local_update(oracle_links8(orc, dims, seed, eps, s), omega, [0, 0, 0])
        return out

    with lgf.Lattice(dims, lgf.LGF_FP64_12) as lat:
        assert lgf.lgf_get_fixed_tuning(lat.h, lgf.LGF_FP64_12)[3] == 1
        lat.generate(seed, eps, True)
        st, res, _ = lat.gauge_fix(omega=omega, theta_target=1e-300, check_every=1, max_sweeps=1, fixed_links=1)
        assert st == lgf.LGF_ENOTCONV and res["sweeps"] == 1
        assert lgf.lgf_get_fixed_tuning(lat.h, lgf.LGF_FP64_12)[3] == 1
        for y in sample_sites(orc, dims, 1, 6, rng):
            links = np.zeros((8, 3, 3), dtype=np.complex128)
            for mu in range(4):
                links[mu] = upd(orc.neighbor(dims, y, mu, +1))[4 + mu]
                links[4 + mu] = upd(orc.neighbor(dims, y, mu, -1))[mu]
            ref, _ = orc.local_update(links, omega, [0, 0, 0])
            assert maxabs(gpu_links8(lat, orc, dims, y), ref) < 1e-12, y
        assert 0 < res["F"] < 1 and np.isfinite(res["theta"])


def test_fixed_records_fall_back_without_memory(lgf, orc):
    """With too little device memory left for the per-site records (twice
    the FP64-12 field), a gauge fixing that asks for them runs on the link
    field instead: the same links and history bit for bit as a run on the
    link field, the tuning switched to the field layout.  The memory is taken
    from the host side by a torch allocation sized to leave room for the
    field, g and the sums but not for the records."""
    import torch
    dims = (48, 48, 48, 48)
    announce("fixed records without memory", dims)
    kw = dict(omega=1.8, theta_target=1e-300, check_every=5, max_sweeps=10, fixed_links=1)
    with lgf.Lattice(dims, lgf.LGF_FP64_12) as lat:
        lat.generate(8, 0.3, True)
        lgf.lgf_set_fixed_tuning(lat.h, lgf.LGF_FP64_12, 2, 128, 2, 0)
        st, res, hist = lat.gauge_fix(**kw)
        ref, ref_hist = lat.store(), hist
    field = 48 ** 4 * 4 * 96
    with lgf.Lattice(dims, lgf.LGF_FP64_12) as lat:
        lat.generate(8, 0.3, True)
        lgf.lgf_set_fixed_tuning(lat.h, lgf.LGF_FP64_12, 2, 128, 2, 1)
        # g and the partial sums of a first run on the field, then the block
        lgf.lgf_set_fixed_tuning(lat.h, lgf.LGF_FP64_12, 2, 128, 2, 0)
        lat.gauge_fix(omega=1.8, theta_target=1e-300, check_every=1, max_sweeps=1, fixed_links=1)
        lat.generate(8, 0.3, True)
        lgf.lgf_set_fixed_tuning(lat.h, lgf.LGF_FP64_12, 2, 128, 2, 1)
        # leave about one field's worth free (the records need two), taken in
        # pieces of at most 8 GiB
        block = []
        free, _ = torch.cuda.mem_get_info()
        while free > field + (64 << 20):
            block.append(torch.empty(min(free - field, 8 << 30), dtype=torch.uint8, device="cuda"))
            free, _ = torch.cuda.mem_get_info()
        try:
            st1, res1, hist1 = lat.gauge_fix(**kw)
            got = lat.store()
            assert lgf.lgf_get_fixed_tuning(lat.h, lgf.LGF_FP64_12)[3] == 0
        finally:
            del block
            torch.cuda.empty_cache()
    assert st1 == st and res1["sweeps"] == res["sweeps"] == 10
    assert np.array_equal(got, ref)
    assert np.array_equal(hist1, ref_hist)


def _random_cases():
    """Seeded lattice shapes (even extents 2..12), formats and tunings, plus
    shapes on which the blocked tile order is taken (with 2 and 4 t-z blocks)."""
    rng = np.random.default_rng(2026)
    cases = []
    for k in range(12):
        dims = tuple(int(2 * rng.integers(1, 7)) for _ in range(4))
        tune = (int(rng.choice([2, 4])), int(rng.choice([64, 128, 256])), int(rng.integers(0, 3)))
        fmt = int(rng.choice([0, 3, 2, 1]))
        cases.append((dims, tune, fmt) + [(1.7, 0.0), (1.0, 0.5), (1.9, 0.2)][k % 3])
    cases += [((8, 8, 16, 8), (2, 64, 2), 3, 1.7, 0.0), ((16, 8, 4, 16), (4, 128, 2), 0, 1.0, 0.5),
              ((16, 16, 8, 16), (2, 128, 2), 2, 1.8, 0.0), ((8, 8, 8, 16), (4, 256, 2), 3, 1.9, 0.2)]
    # per-site link records (a last partial tile of records on the 6^4 and
    # 6 x 4 x 2 x 10 lattices), the lockstep tile order (taken on the last two)
    # and one lane per site
    cases += [((6, 6, 6, 6), (2, 128, 0, 1), 3, 1.9, 0.2), ((6, 4, 2, 10), (1, 64, 0, 1), 2, 1.0, 0.5),
              ((4, 8, 16, 32), (2, 64, 3, 1), 3, 1.7, 0.0), ((4, 4, 32, 32), (1, 64, 3, 1), 2, 1.8, 0.0)]
    return cases


@pytest.mark.parametrize("dims,tune,fmt,omega,p_sr", _random_cases())
def test_fixed_sweep_random_shapes(lgf, orc, dims, tune, fmt, omega, p_sr):
    """One fixed-link sweep on seeded random lattice shapes, formats and
    tunings (tile orders included) against the oracle's sweep of the links."""
    announce("fixed random", dims, tune, fmt, omega, p_sr)
    U = orc.generate_links(dims, 61, 0.35)
    ref = U.copy()
    orc.sweep(dims, ref, omega, p_sr, seed=12, sweep_index=7)
    orc.reunitarize(ref)
    handle = 0 if fmt in (1, 2) else fmt
    got, res, _ = one_fixed_sweep(lgf, dims, U, handle, fmt, tune, omega, p_sr, 12, 7)
    if fmt in (0, 3):
        assert maxabs(got, ref) <= 1e-12, maxabs(got, ref)
    else:
        env = fm.fixed_sweep_envelope(orc, dims, U, fmt, ref, omega, p_sr, 12, 7)
        assert fp32_ok(got, ref, env), fm.fp32_bar_ok(got, ref, env)[1]
    assert unitarity_error(got) < 1e-12
