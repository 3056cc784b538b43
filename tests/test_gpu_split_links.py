"""Fixed-link sweeps in LGF_FP64_12S (FP64 arithmetic, g in FP64-12, the
read-only links held split as fl32 + a 16-bit remainder in units of 2^-40)
against the FP64 oracle, through the C ABI.

The split copy holds every real entry of rows 0 and 1 within 2^-40 of the
input.  For element-wise parity the tests hand both sides links already on
that grid (split_stored: the library's copy of them is then exact, row 2
rebuilt from rows 0 and 1 as in FP64-12), and the bar is the FP64 one, 1e-12.
Gauge fixings of ordinary inputs are checked by what the result must satisfy:
theta < 1e-14 measured by the oracle on the links handed back, an exact gauge
transformation of the input (Wilson loops to 1e-12), and the F of the same
run with FP64-12 links."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from conftest import gpu_available
from lattice_np import SPLIT_UNIT, split_stored, unitarity_error

pytestmark = pytest.mark.gpu

DIMS = [(2, 2, 2, 2), (4, 4, 6, 10), (8, 6, 4, 12), (4, 8, 8, 8)]
# (lanes per site, block, tile order[, link layout]): the last three read
# the links from per-site records ((2, 2, 2, 2) has a partial last tile)
TUNINGS = [(2, 64, 2), (2, 128, 0), (4, 64, 1), (4, 128, 2), (2, 64, 2, 1), (2, 256, 3, 1), (4, 128, 0, 1)]


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


def loops(orc, dims, U):
    return np.array([orc.wilson_loop(dims, U, mu, nu, R, T) for mu in range(4) for nu in range(mu + 1, 4)
                     for (R, T) in [(1, 1), (1, 2), (2, 2)]])


def fixed_sweep(lgf, dims, U, handle_fmt, sweep_fmt, tune, omega, p_sr):
    with lgf.Lattice(dims, handle_fmt) as lat:
        lgf.lgf_set_fixed_tuning(lat.h, sweep_fmt, *tune)
        lat.load(U)
        st, res, _ = lat.gauge_fix(omega=omega, p_sr=p_sr, seed=9, sweep_offset=3, theta_target=1e-300,
                                   check_every=1, max_sweeps=1, fixed_links=1, bulk_format=sweep_fmt,
                                   finish_format=sweep_fmt)
        assert st == lgf.LGF_ENOTCONV and res["sweeps"] == 1, res
        return lat.store(), res


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("handle_fmt", [0, 3])
@pytest.mark.parametrize("omega,p_sr", [(1.0, 0.0), (1.7, 0.0), (1.8, 0.3)])
def test_split_sweep_matches_fp64_12_and_oracle(lgf, orc, dims, handle_fmt, omega, p_sr):
    """One full sweep on links the split copy stores exactly, for every
    tuning: (a) the same links as the FP64-12 sweep of them to 1e-15 (the
    same 12-real arithmetic on the same values; FP64-12 is checked against
    the oracle at 1e-12 on SU(3) links elsewhere); (b) the oracle's sweep of
    them within 1e-12 + 2 delta, delta the input's distance from SU(3)
    (max |U U^dag - 1|, |det U - 1|, ~2e-12 on the grid): the 12-real
    products rebuild row 2 as conj(row0 x row1), exact for SU(3) operands and
    off by about delta otherwise; (c) the reported F and theta those of the
    links handed back (one more FP64 measurement of them).  The oracle's
    links are compared as its sweep leaves them: a reunitarization would
    also project away the input's own deviation, which g U g^dag keeps."""
    announce("split sweep", dims, handle_fmt, omega, p_sr)
    U = split_stored(orc.generate_links(dims, 7, 0.35))
    bar = 1e-12 + 2 * unitarity_error(U)
    ref = U.copy()
    orc.sweep(dims, ref, omega, p_sr, seed=9, sweep_index=3)
    for tune in TUNINGS:
        got, res = fixed_sweep(lgf, dims, U, handle_fmt, lgf.LGF_FP64_12S, tune, omega, p_sr)
        got12, _ = fixed_sweep(lgf, dims, U, handle_fmt, lgf.LGF_FP64_12, tune, omega, p_sr)
        assert maxabs(got, got12) <= 1e-15, (tune, maxabs(got, got12))
        assert maxabs(got, ref) <= bar, (tune, maxabs(got, ref), bar)
        F, th = orc.measure(dims, got)
        assert abs(res["F"] - F) <= 1e-13 and abs(res["theta"] - th) <= 1e-12 * th + 1e-15, (
            tune, res["F"] - F, res["theta"] / th - 1)
        assert unitarity_error(got) < 1e-11   # that of the grid input


@pytest.mark.parametrize("dims", [(4, 4, 6, 10), (8, 6, 4, 12), (4, 8, 8, 8)])
@pytest.mark.parametrize("omega,p_sr", [(1.7, 0.0), (1.8, 0.3)])
def test_split_sweep_on_ordinary_links(lgf, orc, dims, omega, p_sr):
    """One split sweep of ordinary FP64 links (not on the split grid) against
    the oracle's sweep of those very links.  The library decides g from its
    split copy U' = split_stored(U) and applies it to U itself, so per entry
    |g U g^dag - ref| <= |g U' g^dag - ref'| + |g (U - U') g^dag| + |ref' - ref|,
    with ref and ref' the oracle's sweeps of U and U':
      * the first term is the parity of the grid test, 1e-12 + 2 delta;
      * the second is at most 3 max|U - U'| (Frobenius norm of the difference,
        kept by the unitary g);
      * the third is the update's own sensitivity to the 2^-41 perturbation
        (large where the SU(2) subproblem is ill conditioned), computed by the
        oracle.
    The bar is their sum; the worst |g U g^dag - ref| is printed next to the
    FP64 bar of 1e-12, which this format does not promise on every link."""
    announce("split sweep, ordinary links", dims, omega, p_sr)
    U = orc.generate_links(dims, 7, 0.35)
    Us = split_stored(U)
    ref = U.copy()
    orc.sweep(dims, ref, omega, p_sr, seed=9, sweep_index=3)
    ref_s = Us.copy()
    orc.sweep(dims, ref_s, omega, p_sr, seed=9, sweep_index=3)
    sens, din = maxabs(ref_s, ref), maxabs(Us, U)
    bar = 1e-12 + 2 * unitarity_error(Us) + 3 * din + sens
    got, res = fixed_sweep(lgf, dims, U, 0, lgf.LGF_FP64_12S, TUNINGS[0], omega, p_sr)
    err = maxabs(got, ref)
    announce(f"split ordinary {dims} omega {omega} p {p_sr}: |gpu - oracle| {err:.3e} (FP64 bar 1e-12), "
             f"sensitivity {sens:.3e}, input rounding {din:.3e}, bar {bar:.3e}")
    # the storage's definition: rows 0 and 1 within 2^-40 (row 2 is rebuilt)
    assert maxabs(Us[..., :2, :], U[..., :2, :]) <= SPLIT_UNIT
    assert err <= bar, (err, bar)
    # the per-site records hold the same split values: the same bits
    got_rec, _ = fixed_sweep(lgf, dims, U, 0, lgf.LGF_FP64_12S, (2, 64, 2, 1), omega, p_sr)
    assert np.array_equal(got_rec, got)


def test_split_history_matches_oracle(lgf, orc):
    """8^4 FP64 gauge fixing to theta < 1e-12 on grid links: the measured
    theta history (1e-8 relative while theta > 1e-10) and F follow the
    oracle's gauge fixing of the same links, with the same number of sweeps
    and its final links; the reported F and theta are those of the links
    handed back."""
    dims = (8, 8, 8, 8)
    announce("split history")
    U = split_stored(orc.generate_links(dims, 0, 0.25))
    ref = U.copy()
    r_orc = orc.gauge_fix(dims, ref, 1.7, 1e-12)
    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        lat.load(U)
        st, res, hist = lat.gauge_fix(omega=1.7, theta_target=1e-12, fixed_links=1,
                                      bulk_format=lgf.LGF_FP64_12S, finish_format=lgf.LGF_FP64_12S)
        got = lat.store()
    assert st == 0 and res["theta"] < 1e-12
    h_orc = r_orc["history"]
    assert res["sweeps"] == r_orc["sweeps"]
    for k in range(min(len(hist), len(h_orc))):
        if h_orc[k, 2] > 1e-10:
            assert abs(hist[k, 2] - h_orc[k, 2]) <= 1e-8 * h_orc[k, 2], k
            assert abs(hist[k, 1] - h_orc[k, 1]) <= 1e-12, k
    assert abs(res["F"] - r_orc["F"]) < 1e-12
    assert maxabs(got, ref) < 1e-9
    Fg, thg = orc.measure(dims, got)
    assert abs(res["F"] - Fg) <= 1e-13 and abs(res["theta"] - thg) <= 1e-8 * thg + 1e-20


@pytest.mark.parametrize("handle_fmt", [0, 3])
def test_split_mixed_reaches_target_on_the_orbit(lgf, orc, handle_fmt):
    """FP32-12 bulk, switch at theta < 1e-8, split FP64 finish, on ordinary
    (not grid) links: theta < 1e-14 measured by the oracle on the links handed
    back, equal to the reported theta; the input's gauge orbit kept exactly;
    the same sweeps as the run with FP64-12 links and F within 1e-12 of it."""
    dims = (8, 8, 8, 8)
    announce("split mixed", handle_fmt)
    U = orc.generate_links(dims, 1, 0.25)
    L0 = loops(orc, dims, U)
    out = {}
    for finish in (lgf.LGF_FP64_12, lgf.LGF_FP64_12S):
        with lgf.Lattice(dims, handle_fmt) as lat:
            lat.load(U)
            st, res, hist = lat.gauge_fix(omega=1.7, theta_target=1e-14, theta_switch=1e-8, fixed_links=1,
                                          bulk_format=lgf.LGF_FP32_12, finish_format=finish)
            out[finish] = (st, res, hist, lat.store())
    st, res, hist, got = out[lgf.LGF_FP64_12S]
    assert st == 0 and 0 < res["sweeps_bulk"] < res["sweeps"]
    F, th = orc.measure(dims, got)
    assert th < 1e-14 and abs(F - res["F"]) < 1e-13 and abs(th - res["theta"]) <= 1e-8 * th + 1e-20
    assert float(np.abs(loops(orc, dims, got) - L0).max()) < 1e-12
    assert unitarity_error(got) < 1e-12
    st4, res4, _, got4 = out[lgf.LGF_FP64_12]
    assert st4 == 0 and res4["sweeps_bulk"] == res["sweeps_bulk"]
    assert abs(res4["sweeps"] - res["sweeps"]) <= 20
    assert abs(res4["F"] - res["F"]) < 1e-12, res4["F"] - res["F"]


def test_split_graph_and_fused_agree(lgf, orc):
    """Chunks replayed from hipGraphs equal direct launches bit for bit; the
    measurement fused into the chunk's last half-sweep gives the same links
    and F, theta up to the summation order."""
    dims = (8, 8, 8, 16)
    announce("split graph / fused")
    U = orc.generate_links(dims, 12, 0.3)
    kw = dict(omega=1.7, theta_target=1e-13, theta_switch=1e-8, bulk_format=lgf.LGF_FP32_12,
              finish_format=lgf.LGF_FP64_12S, fixed_links=1)
    out = {}
    for g, sep in ((0, 0), (1, 0), (1, 1)):
        with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
            lat.load(U)
            st, res, hist = lat.gauge_fix(use_graph=g, separate_measure=sep, **kw)
            out[(g, sep)] = (st, res, hist, lat.store())
    (s0, r0, h0, U0), (s1, r1, h1, U1) = out[(0, 0)], out[(1, 0)]
    assert s0 == s1 == 0 and r0["sweeps"] == r1["sweeps"]
    assert np.array_equal(h0, h1) and np.array_equal(U0, U1)
    s2, r2, h2, U2 = out[(1, 1)]
    assert s2 == 0 and r2["sweeps"] == r1["sweeps"] and np.array_equal(U2, U1)
    assert np.allclose(h2[:, 1], h1[:, 1], rtol=1e-13, atol=0)
    dth = np.abs(h2[:, 2] - h1[:, 2])
    assert np.all(dth <= 1e-14 * np.sqrt(h1[:, 2]) + 1e-12 * h1[:, 2])


def test_split_64x4_sampled(lgf, orc):
    """The 64^4 workload (seed 3, eps 0.3, Haar gauge) at omega 1.8: one full
    split sweep, checked on sampled parity-1 sites against the oracle's
    updates of the neighbourhood on the split-stored input links.  The
    library's links after the sweep are g U g^dag of the unsplit input, the
    oracle's g' U' g'^dag of the stored U', whose entries differ by at most
    2^-40 in rows 0 and 1 and 4 x 2^-40 in row 2 (two products of entries of
    modulus <= 1): each entry of g (U - U') g^dag is a sum of 9 such terms,
    so the bar is 9 x 4 x 2^-40 plus the FP64 bar, 1e-12.  (The oracle builds
    the input from its own generator, equal to the library's to ~1e-16.)"""
    dims = (64, 64, 64, 64)
    seed, eps, omega = 3, 0.3, 1.8
    announce("split 64^4 sampled")
    from test_gpu_parity import gpu_links8, oracle_links8, sample_sites
    rng = np.random.default_rng(2)
    bar = 36 * SPLIT_UNIT + 1e-12

    def upd(s, split=True):
        links = oracle_links8(orc, dims, seed, eps, s)
        out, _ = orc.local_update(split_stored(links) if split else links, omega, [0, 0, 0])
        return out

    def around(y, split):
        links = np.zeros((8, 3, 3), dtype=np.complex128)
        for mu in range(4):
            links[mu] = upd(orc.neighbor(dims, y, mu, +1), split)[4 + mu]
            links[4 + mu] = upd(orc.neighbor(dims, y, mu, -1), split)[mu]
        ref, _ = orc.local_update(split_stored(links) if split else links, omega, [0, 0, 0])
        return ref

    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        lat.generate(seed, eps, True)
        st, res, _ = lat.gauge_fix(omega=omega, theta_target=1e-300, check_every=1, max_sweeps=1, fixed_links=1,
                                   bulk_format=lgf.LGF_FP64_12S, finish_format=lgf.LGF_FP64_12S)
        assert st == lgf.LGF_ENOTCONV and res["sweeps"] == 1
        worst = worst_plain = 0.0
        for y in sample_sites(orc, dims, 1, 8, rng):
            got = gpu_links8(lat, orc, dims, y)
            ref = around(y, True)
            e = maxabs(got, ref)
            worst = max(worst, e)
            assert e < bar, (y, e)
            # against the oracle's updates of the unsplit links: the bar plus
            # the updates' own sensitivity to the split copy's rounding
            ref_plain = around(y, False)
            e_plain = maxabs(got, ref_plain)
            worst_plain = max(worst_plain, e_plain)
            assert e_plain < bar + maxabs(ref, ref_plain), (y, e_plain)
        announce("split 64^4 worst", worst, "against the unsplit links", worst_plain)
        assert 0 < res["F"] < 1 and np.isfinite(res["theta"])


def test_split_large_lattice_beyond_32bit_vector_indices(lgf, orc):
    """64 x 128^3 (134M sites): the split copy's residual planes start 24 Vh
    16-byte vectors into it (3.2e9), so its addresses pass 2^32 vectors.  One
    split sweep checked on sampled parity-1 sites, the last planes among
    them, with the bar of the 64^4 sampled test; the same sweep on the
    per-site records (77 GB) and on the split field gives the same bits."""
    dims = (64, 128, 128, 128)
    seed, eps, omega = 4, 0.3, 1.8
    announce("split 64x128^3")
    from test_gpu_parity import gpu_links8, oracle_links8, sample_sites
    rng = np.random.default_rng(5)
    bar = 36 * SPLIT_UNIT + 1e-12

    def upd(s):
        out, _ = orc.local_update(split_stored(oracle_links8(orc, dims, seed, eps, s)), omega, [0, 0, 0])
        return out

    ys = sample_sites(orc, dims, 1, 6, rng)
    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        # per-site records (the default at this size; their addresses pass
        # 2^32 bytes many times over), then the split field itself
        assert lgf.lgf_get_fixed_tuning(lat.h, lgf.LGF_FP64_12S)[3] == 1
        seen = []
        for layout in (1, 0):
            lgf.lgf_set_fixed_tuning(lat.h, lgf.LGF_FP64_12S, 2, 128, 2, layout)
            lat.generate(seed, eps, True)
            st, res, _ = lat.gauge_fix(omega=omega, theta_target=1e-300, check_every=1, max_sweeps=1,
                                       fixed_links=1, bulk_format=lgf.LGF_FP64_12S,
                                       finish_format=lgf.LGF_FP64_12S)
            assert st == lgf.LGF_ENOTCONV and res["sweeps"] == 1
            seen.append(([gpu_links8(lat, orc, dims, y) for y in ys], res["F"], res["theta"]))
            assert 0 < res["F"] < 1 and np.isfinite(res["theta"])
        for k, y in enumerate(ys):
            links = np.zeros((8, 3, 3), dtype=np.complex128)
            for mu in range(4):
                links[mu] = upd(orc.neighbor(dims, y, mu, +1))[4 + mu]
                links[4 + mu] = upd(orc.neighbor(dims, y, mu, -1))[mu]
            ref, _ = orc.local_update(split_stored(links), omega, [0, 0, 0])
            assert maxabs(seen[0][0][k], ref) < bar, y
            assert np.array_equal(seen[1][0][k], seen[0][0][k]), y
        assert seen[0][1:] == seen[1][1:]


def test_split_argument_checks(lgf, orc):
    """LGF_FP64_12S is a sweep format of the fixed-link form only: not a
    handle's format, not for the link-rewriting sweeps (Landau, Coulomb,
    ensembles) or the link-sweep tuning; an ensemble takes it as the finish
    after an FP32-12 bulk or alone."""
    dims = (4, 4, 4, 4)
    announce("split checks")
    with pytest.raises(lgf.LgfError):
        lgf.Lattice(dims, lgf.LGF_FP64_12S)
    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        lat.generate(1, 0.2, True)
        with pytest.raises(lgf.LgfError):
            lat.gauge_fix(omega=1.7, finish_format=lgf.LGF_FP64_12S)
        with pytest.raises(lgf.LgfError):
            lat.coulomb_gauge_fix(omega=1.7, finish_format=lgf.LGF_FP64_12S)   # link-rewriting form
        with pytest.raises(lgf.LgfError):
            lgf.lgf_set_tuning(lat.h, lgf.LGF_FP64_12S, 1, 128)
        # default: as FP64-12, per-site records from 2^18 sites on
        assert lgf.lgf_get_fixed_tuning(lat.h, lgf.LGF_FP64_12S) == (2, 128, 2, 0)
        with lgf.Lattice((16, 16, 32, 32), lgf.LGF_FP64_18) as big:
            assert lgf.lgf_get_fixed_tuning(big.h, lgf.LGF_FP64_12S) == (2, 128, 2, 1)
        lgf.lgf_set_fixed_tuning(lat.h, lgf.LGF_FP64_12S, 4, 128, 1)
        assert lgf.lgf_get_fixed_tuning(lat.h, lgf.LGF_FP64_12S) == (4, 128, 1, 0)
        lgf.lgf_set_fixed_tuning(lat.h, lgf.LGF_FP64_12S, 2, 64, 3, 1)
        assert lgf.lgf_get_fixed_tuning(lat.h, lgf.LGF_FP64_12S) == (2, 64, 3, 1)
        for bad in [(1, 128, 0), (2, 128, 0, 2)]:
            with pytest.raises(lgf.LgfError):
                lgf.lgf_set_fixed_tuning(lat.h, lgf.LGF_FP64_12S, *bad)
        lgf.lgf_autotune_fixed(lat.h, lgf.LGF_FP64_12S, 1)
        st, res, _ = lat.gauge_fix(omega=1.7, theta_target=1e-13, fixed_links=1,
                                   bulk_format=lgf.LGF_FP64_12S, finish_format=lgf.LGF_FP64_12S)
        assert st == 0 and res["theta"] < 1e-13
    with lgf.Ensemble([dims, dims], lgf.LGF_FP64_18) as ens:
        with pytest.raises(lgf.LgfError):   # link-rewriting form
            ens.gauge_fix(omega=1.7, bulk_format=lgf.LGF_FP64_12S, finish_format=lgf.LGF_FP64_12S)
        with pytest.raises(lgf.LgfError):   # split bulk before an FP32 finish: no such pair
            ens.gauge_fix(omega=1.7, fixed_links=1, theta_switch=1e-8, bulk_format=lgf.LGF_FP64_12S,
                          finish_format=lgf.LGF_FP32_12)


# ------------------------------------------------------------ Coulomb gauge

@pytest.mark.parametrize("dims", DIMS + [(8, 8, 8, 16)])
@pytest.mark.parametrize("omega,p_sr", [(1.7, 0.0), (1.0, 0.5)])
def test_split_coulomb_sweep_matches_fp64_12_and_oracle(lgf, orc, dims, omega, p_sr):
    """One Coulomb sweep of every timeslice on grid links with the split
    finish: the FP64-12 fixed-link Coulomb sweep of the same links to 1e-15,
    the oracle's Coulomb sweep within 1e-12 + 2 delta (as for the Landau
    sweep), and per-timeslice F_C, theta_C of the links handed back."""
    announce("split coulomb sweep", dims, omega, p_sr)
    U = split_stored(orc.generate_links(dims, 31, 0.35))
    bar = 1e-12 + 2 * unitarity_error(U)
    ref = U.copy()
    orc.sweep_coulomb(dims, ref, omega, p_sr, seed=4, sweep_index=2)
    for tune in [(2, 128, 0), (4, 64, 2), (2, 64, 2), (2, 128, 3, 1)]:
        out = {}
        for fmt in (lgf.LGF_FP64_12S, lgf.LGF_FP64_12):
            with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
                lgf.lgf_set_fixed_tuning(lat.h, fmt, *tune)
                lat.load(U)
                st, res, sw, F, th = lat.coulomb_gauge_fix(omega=omega, p_sr=p_sr, seed=4, sweep_offset=2,
                                                           theta_target=1e-300, check_every=1, max_sweeps=1,
                                                           fixed_links=1, bulk_format=fmt, finish_format=fmt)
                assert st == lgf.LGF_ENOTCONV and res["sweeps"] == 1
                out[fmt] = (lat.store(), F, th)
        got, F, th = out[lgf.LGF_FP64_12S]
        assert maxabs(got, out[lgf.LGF_FP64_12][0]) <= 1e-15, tune
        assert maxabs(got, ref) <= bar, (tune, maxabs(got, ref), bar)
        Fo, tho = orc.measure_coulomb(dims, got)
        assert np.abs(F - Fo).max() < 1e-13 and np.all(np.abs(th - tho) <= 1e-12 * tho + 1e-15), tune


def test_split_coulomb_mixed_keeps_the_orbit(lgf, orc):
    """Mixed Coulomb gauge fixing (FP32-12 bulk, switch at 1e-8, split
    finish) on ordinary links: every timeslice below theta_C < 1e-14 by the
    oracle on the links handed back, equal to the reported F_C, theta_C; the
    input's Wilson loops to 1e-12; the per-timeslice sweeps of the FP64-12
    finish and F_C within 1e-12 of it."""
    dims = (8, 6, 6, 6)
    announce("split coulomb mixed")
    U = orc.generate_links(dims, 34, 0.3)
    L0 = loops(orc, dims, U)
    out = {}
    for finish in (lgf.LGF_FP64_12, lgf.LGF_FP64_12S):
        with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
            lat.load(U)
            out[finish] = lat.coulomb_gauge_fix(omega=1.7, theta_target=1e-14, theta_switch=1e-8,
                                                bulk_format=lgf.LGF_FP32_12, finish_format=finish,
                                                fixed_links=1) + (lat.store(),)
    st, res, sw, F, th, got = out[lgf.LGF_FP64_12S]
    assert st == lgf.LGF_OK and 0 < res["sweeps_bulk"] < res["sweeps"]
    Fo, tho = orc.measure_coulomb(dims, got)
    assert np.all(tho < 1e-14) and np.abs(Fo - F).max() < 1e-13
    assert np.all(np.abs(tho - th) <= 1e-8 * tho + 1e-20)
    assert float(np.abs(loops(orc, dims, got) - L0).max()) < 1e-12 and unitarity_error(got) < 1e-12
    st4, res4, sw4, F4, th4, _ = out[lgf.LGF_FP64_12]
    assert st4 == lgf.LGF_OK and res4["sweeps_bulk"] == res["sweeps_bulk"]
    assert np.abs(sw4 - sw).max() <= 20
    assert np.abs(F4 - F).max() < 1e-12


def test_split_session_on_records_equals_link_field(lgf, orc):
    """A stepwise session on the split format's per-site records (two chunks
    of 10 sweeps, a partial last tile on this lattice) against lgf_gauge_fix
    reading the split field: the same links and the same F and theta at each
    check, bit for bit."""
    dims = (6, 6, 6, 6)
    announce("split session on records", dims)
    U = orc.generate_links(dims, 29, 0.3)
    with lgf.Lattice(dims, 0) as lat:
        lgf.lgf_set_fixed_tuning(lat.h, lgf.LGF_FP64_12S, 2, 128, 0, 1)
        lat.load(U)
        lat.fix_begin(lgf.LGF_FP64_12S)
        seen = [lat.fix_chunk(10, 1.8, 0.0, 5, 10 * k, 1) for k in range(2)]
        lat.fix_end()
        got = lat.store()
    with lgf.Lattice(dims, 0) as lat:
        lgf.lgf_set_fixed_tuning(lat.h, lgf.LGF_FP64_12S, 2, 128, 0, 0)
        lat.load(U)
        st, res, hist = lat.gauge_fix(omega=1.8, seed=5, theta_target=1e-300, max_sweeps=20, check_every=10,
                                      fixed_links=1, bulk_format=lgf.LGF_FP64_12S,
                                      finish_format=lgf.LGF_FP64_12S)
        ref = lat.store()
    assert st == lgf.LGF_ENOTCONV and res["sweeps"] == 20
    assert np.array_equal(got, ref)
    for k in range(2):
        assert seen[k][0] == hist[k + 1, 1] and seen[k][1] == hist[k + 1, 2], k
