"""Parity of the gfx950 library with the FP64 oracle, through the C ABI.

Small lattices (several workgroups and a ragged tail) are compared element by
element on identical input links; the full 64^4 workload is compared on
sampled sites, which the oracle rebuilds from its own generator.  Tolerances:
1e-12 absolute per entry for FP64 formats; for FP32 formats 2e-6 relative
(Frobenius) per link on 99% of the links, and on every link twice the largest
error of 16 randomised-rounding runs of the same FP32 steps (fp32_model), all
against the oracle run on the FP32-rounded input (see tol_ok)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from conftest import gpu_available
import fp32_model as fm
from lattice_np import dag, parity_grid, stored_as, unitarity_error

pytestmark = pytest.mark.gpu

FP64 = (0, 3)      # LGF_FP64_18, LGF_FP64_12
ALL_FORMATS = (0, 1, 2, 3)
SMALL_DIMS = [(2, 2, 2, 2), (4, 4, 6, 10), (8, 6, 4, 12)]


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


def maxabs(A, B) -> float:
    return float(np.abs(np.asarray(A) - np.asarray(B)).max())


def link_rel_err(A, B):
    """max over links of ||A - B||_F / ||B||_F"""
    d = np.linalg.norm((A - B).reshape(-1, 9), axis=1)
    n = np.linalg.norm(B.reshape(-1, 9), axis=1)
    return float((d / n).max())


def link_errs(A, B):
    d = np.linalg.norm((A - B).reshape(-1, 9), axis=1)
    n = np.linalg.norm(B.reshape(-1, 9), axis=1)
    return d / n


def tol_ok(fmt, got, ref, env=None):
    """FP64: 1e-12 per entry.  FP32: 2e-6 relative per link for 99% of the
    links, and on every link at most twice its randomised-rounding envelope
    env plus u = 2^-24 -- exact IEEE FP32 arithmetic of the same steps exceeds
    2e-6 on the few sites whose SU(2) subproblem is ill conditioned (small
    quaternion projection |a| against |W|), which the stochastic square
    doubles; the envelope is that amplification, link by link."""
    if fmt in FP64:
        return float(maxabs(got, ref)) <= 1e-12
    return fm.fp32_bar_ok(got, ref, env)[0]


# ------------------------------------------------------------ boundary

@pytest.mark.parametrize("fmt", ALL_FORMATS)
def test_load_store_round_trip(lgf, orc, fmt):
    dims = (4, 4, 6, 10)
    announce("load_store", fmt, dims)
    U = orc.generate_links(dims, 5, 0.3)
    with lgf.Lattice(dims, fmt) as lat:
        lat.load(U)
        got = lat.store()
    if fmt == 0:
        assert np.array_equal(got, U)
    elif fmt == 3:
        # row 2 rebuilt as conj(row0 x row1): exact up to the input's own
        # distance from SU(3) (a few 1e-15 after the Haar transform)
        assert maxabs(got, U) < 2e-14
    else:
        assert maxabs(got, U) < 5e-7
        assert unitarity_error(got) < 2e-6


@pytest.mark.parametrize("fmt", ALL_FORMATS)
@pytest.mark.parametrize("haar", [False, True])
def test_generator_matches_oracle(lgf, orc, fmt, haar):
    dims = (4, 4, 6, 10)
    announce("generate", fmt, haar, dims)
    ref = orc.generate_links(dims, 11, 0.27, haar=haar)
    with lgf.Lattice(dims, fmt) as lat:
        lat.generate(11, 0.27, haar)
        got = lat.store()
    if fmt in FP64:
        assert maxabs(got, ref) < 1e-13
    else:
        assert maxabs(got, ref) < 5e-7


def test_peek_matches_store(lgf, orc):
    dims = (8, 6, 4, 12)
    announce("peek", dims)
    with lgf.Lattice(dims, 0) as lat:
        lat.generate(4, 0.3)
        full = lat.store()
        sites = [0, 1, 17, 1151, 600, 3]
        assert np.array_equal(lat.peek(sites), full[sites])
        with pytest.raises(lgf.LgfError):
            lat.peek([len(full)])


# ------------------------------------------------------------ one sweep

# (lanes per site, block, XCD remap, non-temporal, schedule: 0 in place,
# 1 t-slice pipeline, 2 out of place[, sites per thread])
TUNINGS = [(1, 128, 0, 1, 0), (2, 128, 1, 1, 1), (4, 64, 0, 1, 0), (4, 256, 1, 0, 1), (1, 64, 1, 1, 1),
           (2, 256, 0, 0, 0), (1, 128, 0, 1, 1), (1, 128, 0, 1, 2), (2, 64, 1, 1, 2), (4, 256, 0, 1, 2),
           (1, 128, 0, 1, 0, 2), (2, 64, 1, 1, 2, 4), (4, 64, 0, 0, 0, 2), (1, 64, 1, 1, 0, 4)]


@pytest.mark.parametrize("fmt", ALL_FORMATS)
@pytest.mark.parametrize("dims", SMALL_DIMS)
@pytest.mark.parametrize("omega,p_sr", [(1.0, 0.0), (1.7, 0.0), (1.0, 0.5), (1.8, 0.3)])
def test_half_and_full_sweep_match_oracle(lgf, orc, fmt, dims, omega, p_sr):
    """After one half-sweep and after one full sweep (both parities, either as
    two calls or as one parity-2 call), on the same input links."""
    announce("sweep", fmt, dims, omega, p_sr)
    U = orc.generate_links(dims, 7, 0.35)
    U0 = stored_as(U, fmt)   # the field a load of U in this format holds (up to its row-2 rounding)
    ref_half = U0.copy()
    orc.half_sweep(dims, ref_half, 0, omega, p_sr, seed=9, sweep=3)
    ref_full = ref_half.copy()
    orc.half_sweep(dims, ref_full, 1, omega, p_sr, seed=9, sweep=3)
    env_half = env_full = None
    if fmt not in FP64:
        env_half = fm.link_sweep_envelope(orc, dims, U0, fmt, ref_half, omega, p_sr, 9, 3, parities=(0,))
        env_full = fm.link_sweep_envelope(orc, dims, U0, fmt, ref_full, omega, p_sr, 9, 3)
    for tune in TUNINGS:
        with lgf.Lattice(dims, fmt) as lat:
            lgf.lgf_set_tuning(lat.h, fmt, *tune)
            lat.load(U)
            lat.sweep(0, omega, p_sr, seed=9, sweep_index=3)
            got = lat.store()
            assert tol_ok(fmt, got, ref_half, env_half), ("half", tune, maxabs(got, ref_half),
                                                link_rel_err(got, ref_half),
                                                float(np.quantile(link_errs(got, ref_half), 0.99)))
            lat.sweep(1, omega, p_sr, seed=9, sweep_index=3)
            got = lat.store()
            assert tol_ok(fmt, got, ref_full, env_full), ("full", tune, maxabs(got, ref_full),
                                                link_rel_err(got, ref_full),
                                                float(np.quantile(link_errs(got, ref_full), 0.99)))
            lat.load(U)
            lat.sweep(2, omega, p_sr, seed=9, sweep_index=3)
            got2 = lat.store()
            assert np.array_equal(got2, got), ("parity-2 call differs from two half-sweeps", tune)


def test_sr_decisions_bitwise(lgf, orc):
    """p = 1 squares every subgroup: after one half-sweep at omega = 1 the GPU
    and the oracle agree to rounding, which they could not if any coin differed;
    with p = 0.5 the per-site updates agree only when every coin matches."""
    dims = (8, 6, 4, 12)
    announce("sr_bits", dims)
    U = orc.generate_links(dims, 13, 0.4)
    for p in (0.5, 0.25, 1.0):
        ref = U.copy()
        with lgf.Lattice(dims, 0) as lat:
            lat.load(U)
            lat.sweep(0, 1.0, p, seed=2**40 + 77, sweep_index=123456)
            got = lat.store()
        orc.half_sweep(dims, ref, 0, 1.0, p, seed=2**40 + 77, sweep=123456)
        assert maxabs(got, ref) < 1e-12


# ------------------------------------------------------------ reunitarize, measure

@pytest.mark.parametrize("fmt", ALL_FORMATS)
def test_measure_matches_oracle(lgf, orc, fmt):
    dims = (8, 6, 4, 12)
    announce("measure", fmt, dims)
    U = orc.generate_links(dims, 3, 0.4)
    F_ref, th_ref = orc.measure(dims, stored_as(U, fmt))
    with lgf.Lattice(dims, fmt) as lat:
        lat.load(U)
        F, th = lat.measure()
    # FP32 12-real: the GPU rebuilds row 2 with fused multiply-adds, the host
    # without, so its entries may differ by an FP32 rounding unit
    ftol, thtol = (2e-7, 2e-7) if fmt == 2 else (1e-14, 1e-12)
    assert abs(F - F_ref) < ftol * abs(F_ref) + 1e-15
    assert abs(th - th_ref) < thtol * th_ref


@pytest.mark.parametrize("fmt", ALL_FORMATS)
def test_reunitarize_matches_oracle(lgf, orc, fmt):
    dims = (4, 4, 6, 10)
    announce("reunit", fmt, dims)
    rng = np.random.default_rng(0)
    U = orc.generate_links(dims, 3, 0.4)
    noisy = U + 1e-4 * (rng.normal(size=U.shape) + 1j * rng.normal(size=U.shape))
    ref = stored_as(noisy, fmt)
    orc.reunitarize(ref)
    with lgf.Lattice(dims, fmt) as lat:
        lat.load(noisy)
        lat.reunitarize()
        got = lat.store()
    if fmt in FP64:
        assert maxabs(got, ref) < 1e-14
    else:
        assert maxabs(got, ref) < 5e-7


# ------------------------------------------------------------ gauge fixing

def test_gauge_fix_8x4_matches_oracle_history(lgf, orc):
    """8^4, seed 0, eps 0.25, Haar gauge, omega 1.7 to theta < 1e-12: the GPU
    FP64 run has the oracle's theta history (1e-8 relative while theta >
    1e-10) and the same number of sweeps."""
    dims = (8, 8, 8, 8)
    announce("gauge_fix_8x4")
    U = orc.generate_links(dims, 0, 0.25)
    ref = U.copy()
    r_orc = orc.gauge_fix(dims, ref, 1.7, 1e-12)
    with lgf.Lattice(dims, 0) as lat:
        lat.load(U)
        st, res, hist = lat.gauge_fix(omega=1.7, theta_target=1e-12)
        got = lat.store()
    assert st == 0 and res["theta"] < 1e-12
    h_orc = r_orc["history"]
    assert res["sweeps"] == r_orc["sweeps"]
    n = min(len(hist), len(h_orc))
    for k in range(n):
        if h_orc[k, 2] > 1e-10:
            assert abs(hist[k, 2] - h_orc[k, 2]) <= 1e-8 * h_orc[k, 2], k
            assert abs(hist[k, 1] - h_orc[k, 1]) <= 1e-12
    assert abs(res["F"] - r_orc["F"]) < 1e-12
    assert maxabs(got, ref) < 1e-9


@pytest.mark.parametrize("bulk,finish", [(1, -1), (2, -1), (2, 3)])
def test_mixed_gauge_fix_reaches_target(lgf, orc, bulk, finish):
    """FP32 bulk sweeps, FP64 reunitarization every 20 sweeps, switch below
    theta = 1e-8, FP64 finish (18 or 12 reals): converges to theta < 1e-14
    like the plain run, to the same F within the FP32 orbit drift."""
    dims = (8, 8, 8, 8)
    announce("mixed", bulk, finish)
    U = orc.generate_links(dims, 1, 0.25)
    ref = U.copy()
    r_orc = orc.gauge_fix(dims, ref, 1.7, 1e-14)
    with lgf.Lattice(dims, 0) as lat:
        lat.load(U)
        st, res, hist = lat.gauge_fix(omega=1.7, theta_target=1e-14, theta_switch=1e-8,
                                      bulk_format=bulk, finish_format=finish)
        got = lat.store()
    assert st == 0 and res["theta"] < 1e-14
    assert 0 < res["sweeps_bulk"] < res["sweeps"]
    assert abs(res["F"] - r_orc["F"]) < 1e-5
    assert unitarity_error(got) < 1e-12
    # the FP64 finish: theta recomputed by the oracle on the returned links
    assert orc.measure(dims, got)[1] < 1e-14


def test_gauge_fix_graph_equals_direct(lgf, orc):
    """Chunks replayed from captured graphs (each replay followed by the
    eager measurement that reads the partial sums the graph's last launch
    wrote) against direct launches: the same links and the same F, theta at
    every check, plain, mixed, and stochastic relaxation (whose replays read
    the chunk's first counter from the device)."""
    dims = (8, 6, 4, 12)
    announce("graph_vs_direct")
    U = orc.generate_links(dims, 2, 0.3)
    for kw in (dict(omega=1.6, theta_target=1e-12),
               dict(omega=1.6, theta_target=1e-13, theta_switch=1e-8, bulk_format=lgf.LGF_FP32_12,
                    finish_format=lgf.LGF_FP64_12),
               dict(omega=1.0, p_sr=0.5, seed=3, theta_target=1e-11, sweep_offset=1000)):
        outs = []
        for use_graph in (0, 1, 1):
            with lgf.Lattice(dims, 0) as lat:
                lat.load(U)
                st, res, hist = lat.gauge_fix(use_graph=use_graph, **kw)
                assert st == lgf.LGF_OK and hist.shape[0] > 5
                outs.append((lat.store(), hist))
        for got, hist in outs[1:]:
            assert np.array_equal(got, outs[0][0]) and np.array_equal(hist, outs[0][1]), kw


def test_sweep_schedules_are_bitwise_identical(lgf, orc):
    """The t-slice pipelined and the out-of-place full sweeps perform every
    site update on the same links as the two in-place launches: identical
    bits after a gauge fixing (mixed, graph-captured chunks)."""
    dims = (8, 6, 4, 12)
    announce("schedules")
    U = orc.generate_links(dims, 21, 0.3)
    outs = []
    for fmt in (lgf.LGF_FP64_18, lgf.LGF_FP32_12):
        for pipe in (0, 1, 2):
            with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
                lgf.lgf_set_tuning(lat.h, fmt, 1, 128, 0, 1, pipe)
                lgf.lgf_set_tuning(lat.h, lgf.LGF_FP64_12, 1, 128, 0, 1, pipe)
                lat.load(U)
                st, res, _ = lat.gauge_fix(omega=1.7, theta_target=1e-12, theta_switch=1e-8,
                                           bulk_format=fmt, finish_format=lgf.LGF_FP64_12)
                outs.append((lat.store(), res["sweeps"]))
        for k in (-1, -2):
            assert np.array_equal(outs[k][0], outs[-3][0]) and outs[k][1] == outs[-3][1]


def test_sr_gauge_fix_converges(lgf, orc):
    dims = (8, 6, 4, 12)
    announce("sr_fix")
    U = orc.generate_links(dims, 2, 0.3)
    ref = U.copy()
    r_orc = orc.gauge_fix(dims, ref, 1.0, 1e-12, p=0.5, seed=5)
    with lgf.Lattice(dims, 0) as lat:
        lat.load(U)
        st, res, _ = lat.gauge_fix(omega=1.0, p_sr=0.5, seed=5, theta_target=1e-12)
        got = lat.store()
    assert st == 0 and res["sweeps"] == r_orc["sweeps"]
    assert maxabs(got, ref) < 1e-9


def test_status_codes(lgf, orc):
    dims = (4, 4, 4, 4)
    announce("status")
    with lgf.Lattice(dims, 0) as lat:
        lat.generate(0, 0.3)
        with pytest.raises(lgf.LgfError) as e:
            lat.sweep(0, 2.5)
        assert e.value.status == lgf.LGF_EINVAL
        with pytest.raises(lgf.LgfError) as e:
            lat.sweep(3, 1.5)
        assert e.value.status == lgf.LGF_EINVAL
        with pytest.raises(lgf.LgfError) as e:
            lat.sweep(0, 1.5, p_sr=1.5)
        assert e.value.status == lgf.LGF_EINVAL
        st, res, hist = lat.gauge_fix(omega=1.7, theta_target=1e-30, max_sweeps=40)
        assert st == lgf.LGF_ENOTCONV and res["sweeps"] == 40 and len(hist) == 3
        U = lat.store()
        U[5, 2, 1, 1] = np.nan
        lat.load(U)
        st, res, hist = lat.gauge_fix(omega=1.7, theta_target=1e-12)
        assert st == lgf.LGF_ENUMERIC


def test_determinism(lgf, orc):
    dims = (8, 8, 8, 8)
    announce("determinism")
    outs = []
    for _ in range(2):
        with lgf.Lattice(dims, 2) as lat:
            lat.generate(3, 0.3)
            for k in range(5):
                lat.sweep(2, 1.8, 0.0, 0, k)
                lat.sweep(2, 1.0, 0.5, 1, k)
            outs.append((lat.store(), lat.measure()))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]


# ------------------------------------------------------------ full size, sampled

def oracle_links8(orc, dims, seed, eps, s):
    fw = [orc.generated_link(dims, seed, eps, True, s, mu) for mu in range(4)]
    bw = [orc.generated_link(dims, seed, eps, True, orc.neighbor(dims, s, mu, -1), mu)
          for mu in range(4)]
    return np.array(fw + bw)


def gpu_links8(lat, orc, dims, s):
    nb = [orc.neighbor(dims, s, mu, -1) for mu in range(4)]
    P = lat.peek([s] + nb)
    return np.array([P[0, mu] for mu in range(4)] + [P[1 + mu, mu] for mu in range(4)])


def sample_sites(orc, dims, parity, n, rng):
    V = int(np.prod(dims))
    Lt, Lz, Ly, Lx = dims
    edge = [0, 1, Lx - 1, Lx, V - 1, V - 2, V - Lx, (Lt - 1) * Lz * Ly * Lx, Lz * Ly * Lx - 1]
    cand = list(edge) + list(rng.integers(0, V, 4 * n))
    out = []
    for s in cand:
        if orc.parity(dims, int(s)) == parity and int(s) not in out:
            out.append(int(s))
        if len(out) >= n:
            break
    return out


@pytest.mark.parametrize("fmt,omega,p_sr", [(0, 1.8, 0.0), (2, 1.8, 0.0), (3, 1.8, 0.0), (0, 1.0, 0.5)])
def test_64x4_sampled_sweep(lgf, orc, fmt, omega, p_sr):
    """The 64^4 workload (seed 3, eps 0.3, Haar gauge) in the launch
    configuration the benchmark times (the autotuner's pick): one half-sweep
    of parity 0, checked on sampled parity-0 sites, and, on a fresh field, one
    full sweep, checked on sampled parity-1 sites (edges and wrap-arounds
    included), with the oracle rebuilding every input link from its own
    generator."""
    dims = (64, 64, 64, 64)
    seed, eps, sr_seed, sweep = 3, 0.3, 17, 5
    announce("64^4 sampled", fmt, omega, p_sr)
    rng = np.random.default_rng(0)
    fp32 = fmt not in FP64
    checked = []   # FP32: (sites, GPU links, oracle links) per stage, bounded below

    def check(got, ref, where):
        if fmt in FP64:
            assert maxabs(got, ref) < 1e-12, where

    def srd(s):
        return orc.sr_decisions(sr_seed, s, sweep, 0, p_sr)

    def upd(s):
        out, _ = orc.local_update(oracle_links8(orc, dims, seed, eps, s), omega,
                                  orc.sr_decisions(sr_seed, s, sweep, 0, p_sr))
        return out

    with lgf.Lattice(dims, fmt) as lat:
        lat.generate(seed, eps, True)
        lgf.lgf_autotune(lat.h, fmt, 1)
        announce("tuning", lgf.lgf_get_tuning(lat.h, fmt))
        sites0 = sample_sites(orc, dims, 0, 24, rng)
        for s in sites0[:6]:
            got = gpu_links8(lat, orc, dims, s)
            ref = oracle_links8(orc, dims, seed, eps, s)
            assert (maxabs(got, ref) < 1e-13) if fmt in FP64 else (link_rel_err(got, ref) < 5e-7)
        lat.sweep(0, omega, p_sr, sr_seed, sweep)
        got0 = np.array([gpu_links8(lat, orc, dims, s) for s in sites0])
        ref0 = np.array([upd(s) for s in sites0])
        for s, got, ref in zip(sites0, got0, ref0):
            check(got, ref, s)
        # parity 1 after a full sweep: each of its 8 links was last changed by
        # the parity-0 site at its other end; the oracle redoes those first
        lat.generate(seed, eps, True)
        lat.sweep(2, omega, p_sr, sr_seed, sweep)
        sites1 = sample_sites(orc, dims, 1, 8, rng)
        for y in sites1:
            links = np.zeros((8, 3, 3), dtype=np.complex128)
            for mu in range(4):
                links[mu] = upd(orc.neighbor(dims, y, mu, +1))[4 + mu]   # U_mu(y): backward link of y+mu
                links[4 + mu] = upd(orc.neighbor(dims, y, mu, -1))[mu]   # U_mu(y-mu): forward link of y-mu
            ref, _ = orc.local_update(links, omega, srd(y))
            got = gpu_links8(lat, orc, dims, y)
            check(got, ref, y)
            checked.append((y, got, ref))
        if fp32:
            # the FP32 bar: each sampled site's links against twice their
            # randomised-rounding envelope; the model starts from the oracle's
            # FP64 links rounded to the format, as the GPU's field holds them
            L0 = np.array([oracle_links8(orc, dims, seed, eps, s) for s in sites0])
            sr0 = np.array([srd(s) for s in sites0], dtype=bool)
            env0 = fm.envelope(lambda R: fm.link_update(R, fm.stored(R, L0, fmt), omega, sr0, fmt), ref0)
            _, info0 = fm.fp32_bar_ok(got0, ref0, env0)
            ys = [c[0] for c in checked]
            nbf = [orc.neighbor(dims, y, mu, +1) for y in ys for mu in range(4)]
            nbb = [orc.neighbor(dims, y, mu, -1) for y in ys for mu in range(4)]
            LF = np.array([oracle_links8(orc, dims, seed, eps, s) for s in nbf])
            LB = np.array([oracle_links8(orc, dims, seed, eps, s) for s in nbb])
            srf = np.array([srd(s) for s in nbf], dtype=bool)
            srb = np.array([srd(s) for s in nbb], dtype=bool)
            sr1 = np.array([srd(y) for y in ys], dtype=bool)
            n1 = len(ys)

            def run1(R):
                of = fm.link_update(R, fm.stored(R, LF, fmt), omega, srf, fmt).reshape(n1, 4, 8, 3, 3)
                ob = fm.link_update(R, fm.stored(R, LB, fmt), omega, srb, fmt).reshape(n1, 4, 8, 3, 3)
                links = np.stack([of[:, mu, 4 + mu] for mu in range(4)] + [ob[:, mu, mu] for mu in range(4)], 1)
                return fm.link_update(R, links, omega, sr1, fmt)

            ref1 = np.array([c[2] for c in checked])
            _, info1 = fm.fp32_bar_ok(np.array([c[1] for c in checked]), ref1, fm.envelope(run1, ref1))
            # 2e-6 on 99 % of all the sampled links, the envelope on every one
            e = np.concatenate([fm.link_errs(got0, ref0), fm.link_errs(np.array([c[1] for c in checked]), ref1)])
            assert float(np.quantile(e, 0.99)) <= 2e-6, float(np.quantile(e, 0.99))
            assert info0["worst_ratio"] <= 1 and info1["worst_ratio"] <= 1, (info0, info1)
        F, th = lat.measure()
        assert np.isfinite(F) and np.isfinite(th) and 0 < F < 1


def test_large_lattice_beyond_32bit_vector_indices(lgf, orc):
    """64 x 128^3 (134M sites) in FP64-18: 4.8e9 16-byte vectors, so link
    addresses pass 2^32 vectors (and 2^36 bytes).  One half-sweep of parity 0
    checked on sampled sites (the last planes included), then F and theta of
    the whole field."""
    dims = (64, 128, 128, 128)
    seed, eps = 4, 0.3
    announce("64x128^3 fp64-18")
    rng = np.random.default_rng(1)
    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        lat.generate(seed, eps, True)
        sites = sample_sites(orc, dims, 0, 10, rng)
        for s in sites[:3]:
            assert maxabs(gpu_links8(lat, orc, dims, s), oracle_links8(orc, dims, seed, eps, s)) < 1e-13, s
        lat.sweep(0, 1.8, 0.0, 0, 0)
        for s in sites:
            ref, _ = orc.local_update(oracle_links8(orc, dims, seed, eps, s), 1.8, [0, 0, 0])
            assert maxabs(gpu_links8(lat, orc, dims, s), ref) < 1e-12, s
        F, th = lat.measure()
        assert np.isfinite(F) and np.isfinite(th) and 0 < F < 1


# ------------------------------------------------------------ observables, exact mixed precision

@pytest.mark.parametrize("fmt", ALL_FORMATS)
def test_plaquette_matches_oracle(lgf, orc, fmt):
    dims = (8, 6, 4, 12)
    announce("plaquette", fmt)
    U = orc.generate_links(dims, 14, 0.4)
    with lgf.Lattice(dims, fmt) as lat:
        lat.load(U)
        P = lat.plaquette()
    # FP32 12-real: row 2 rebuilt with fused multiply-adds on the GPU, without on the host
    assert abs(P - orc.plaquette(dims, stored_as(U, fmt))) < (2e-7 if fmt == 2 else 1e-14)


def _loops(orc, dims, U):
    return np.array([orc.wilson_loop(dims, U, mu, nu, R, T) for mu in range(4) for nu in range(mu + 1, 4)
                     for (R, T) in [(1, 1), (1, 2), (2, 2)]])


def test_accumulated_gauge_keeps_the_orbit(lgf, orc):
    """Mixed FP32-12 bulk with the accumulated gauge transformation: the links
    handed back are an FP64 gauge transformation of the input (plaquette and
    Wilson loops unchanged to 1e-12, unlike the plain mixed run, whose FP32
    bulk drifts off the orbit) and reach theta < 1e-14."""
    dims = (8, 8, 8, 8)
    announce("accumulate_g")
    U = orc.generate_links(dims, 1, 0.25)
    L0 = _loops(orc, dims, U)
    out = {}
    for acc in (0, 1):
        with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
            lat.load(U)
            st, res, _ = lat.gauge_fix(omega=1.7, theta_target=1e-14, theta_switch=1e-8,
                                       bulk_format=lgf.LGF_FP32_12, finish_format=lgf.LGF_FP64_12,
                                       accumulate_g=acc)
            got = lat.store()
        assert st == 0 and orc.measure(dims, got)[1] < 1e-14
        out[acc] = float(np.abs(_loops(orc, dims, got) - L0).max())
    assert out[1] < 1e-12
    assert out[0] > 100 * out[1]
    # stopped inside the bulk: the exact transformation is handed back too
    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        lat.load(U)
        st, res, _ = lat.gauge_fix(omega=1.7, theta_target=1e-14, theta_switch=1e-30, max_sweeps=40,
                                   bulk_format=lgf.LGF_FP32_12, finish_format=lgf.LGF_FP64_12,
                                   accumulate_g=1)
        got = lat.store()
        assert st == lgf.LGF_ENOTCONV and res["sweeps_bulk"] == 40
        assert float(np.abs(_loops(orc, dims, got) - L0).max()) < 1e-12
        assert unitarity_error(got) < 1e-12
        with pytest.raises(lgf.LgfError):
            lat.gauge_fix(omega=1.7, accumulate_g=1)   # no FP32 bulk: rejected


def test_copy_bandwidth(lgf):
    """The copy-ceiling utility runs and reports a plausible HBM rate."""
    announce("copy bandwidth")
    gbs = lgf.lgf_copy_bandwidth(256 << 20, 4)
    assert 500.0 < gbs < 10000.0


def test_autotune_leaves_links_untouched(lgf, orc):
    """The autotuner sweeps the handle's own field (saved and restored) or its
    working copy in another format: the links come back bit for bit, and the
    picked variant is one the library accepts."""
    dims = (8, 6, 4, 12)
    announce("autotune restore")
    U = orc.generate_links(dims, 44, 0.3)
    with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
        lat.load(U)
        before = lat.store()
        for fmt in (lgf.LGF_FP64_18, lgf.LGF_FP32_12):
            lgf.lgf_autotune(lat.h, fmt, 1)
            assert np.array_equal(lat.store(), before)
            t = lgf.lgf_get_tuning(lat.h, fmt)
            lgf.lgf_set_tuning(lat.h, fmt, *t)
        st, res, _ = lat.gauge_fix(omega=1.7, theta_target=1e-12, theta_switch=1e-8,
                                   bulk_format=lgf.LGF_FP32_12, finish_format=lgf.LGF_FP64_12)
        assert st == lgf.LGF_OK and orc.measure(dims, lat.store())[1] < 1e-12


@pytest.mark.parametrize("dims,tune", [((8, 6, 4, 12), (1, 128, 0, 1, 0, 1)), ((8, 6, 4, 12), (2, 64, 1, 1, 2, 1)),
                                       ((8, 6, 4, 12), (4, 256, 0, 1, 0, 2)), ((8, 6, 4, 12), (1, 64, 0, 1, 2, 4)),
                                       ((4, 4, 6, 10), (1, 64, 1, 1, 0, 2)), ((2, 2, 2, 2), (2, 64, 0, 1, 2, 1))])
def test_fused_measure_equals_separate_passes(lgf, orc, dims, tune):
    """Reunitarize + measure inside the chunk's last half-sweep (plus one
    read-only pass over parity 0) against the separate passes: the same
    sweeps, the same links, and F, theta equal up to the summation order --
    plain FP64-18, mixed FP32-12 / FP64-12, and mixed with the accumulated
    gauge transformation; and chunks cut short by max_sweeps."""
    announce("fused measure", dims, tune)
    U = orc.generate_links(dims, 51, 0.3)
    runs = [dict(omega=1.7, theta_target=1e-12),
            dict(omega=1.7, theta_target=1e-13, theta_switch=1e-8, bulk_format=lgf.LGF_FP32_12,
                 finish_format=lgf.LGF_FP64_12),
            dict(omega=1.7, theta_target=1e-13, theta_switch=1e-8, bulk_format=lgf.LGF_FP32_12,
                 finish_format=lgf.LGF_FP64_12, accumulate_g=1),
            dict(omega=1.6, theta_target=1e-30, check_every=7, max_sweeps=30)]
    for kw in runs:
        out = []
        for sep in (1, 0):
            with lgf.Lattice(dims, lgf.LGF_FP64_18) as lat:
                for f in ALL_FORMATS:
                    lgf.lgf_set_tuning(lat.h, f, *tune)
                lat.load(U)
                st, res, hist = lat.gauge_fix(separate_measure=sep, **kw)
                out.append((st, res, hist, lat.store()))
        (st1, r1, h1, U1), (st0, r0, h0, U0) = out
        assert st1 == st0 and st0 in (lgf.LGF_OK, lgf.LGF_ENOTCONV), kw
        assert st0 == lgf.LGF_OK or kw.get("max_sweeps"), kw
        assert r1["sweeps"] == r0["sweeps"] and r1["sweeps_bulk"] == r0["sweeps_bulk"], kw
        assert np.array_equal(U0, U1), (kw, maxabs(U0, U1))
        assert np.array_equal(h0[:, 0], h1[:, 0])
        assert np.allclose(h0[:, 1], h1[:, 1], rtol=1e-13, atol=0), kw
        # theta sums |Delta|^2 with Delta = (K - K^dag)/2i of O(1) entries: a
        # different summation order of K moves theta by ~eps |K| |Delta| per site
        dth = np.abs(h0[:, 2] - h1[:, 2])
        assert np.all(dth <= 1e-14 * np.sqrt(h1[:, 2]) + 1e-12 * h1[:, 2]), (kw, float((dth / h1[:, 2]).max()))
        th_orc = orc.measure(dims, U0)[1]
        assert th_orc < kw["theta_target"] if st0 == lgf.LGF_OK else abs(th_orc - r0["theta"]) <= 1e-9 * th_orc + 1e-28
