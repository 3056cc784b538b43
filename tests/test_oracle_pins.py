"""Pins of the FP64 oracle to things other than itself: closed forms,
invariants, special cases that reduce to a textbook or library routine, and
brute force on tiny lattices (CPU only)."""
from __future__ import annotations

import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.linalg

from lattice_np import (GELLMANN, K_field, as_grid, backward, dag, expm_hermitian,
                        parity_grid, quat_matrix, random_su2, random_su3, unitarity_error)

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------- Philox

@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("rocrand") / "rocrand_philox_ref")
    subprocess.run([hipcc, "-O1", os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_ref):
    """Oracle Philox4x32-10 == rocRAND's philox4x32_10 engine, bit for bit."""
    rng = np.random.default_rng(7)
    qs = []
    for i in range(400):
        k = rng.integers(0, 2**32, 2)
        c = rng.integers(0, 2**32, 4)
        c[1] %= 2**30  # rocRAND reaches counter word 1 through a 64-bit offset of 4 per counter
        if i % 5 == 0:
            c[1:] = [i % 4, 0, 1]
        qs.append((k, c))
    qs.append((np.array([0, 0]), np.array([0, 0, 0, 0])))
    qs.append((np.array([2**32 - 1, 2**32 - 1]), np.array([2**32 - 1, 0, 2**32 - 1, 2**32 - 1])))
    inp = "\n".join(" ".join(str(int(x)) for x in list(k) + list(c)) for k, c in qs)
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for (k, c), line in zip(qs, out):
        ref = [int(x) for x in line.split()]
        assert list(orc.philox4x32_10(c, k)) == ref, (k, c)


def test_philox_uniform_bits(orc):
    words = np.concatenate([orc.philox4x32_10([i, 3, 7, 1], [11, 0]) for i in range(4096)])
    # every bit is set with probability 1/2
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(np.float64)
    frac = bits.mean(axis=0)
    sigma = 0.5 / np.sqrt(words.size)
    assert np.all(np.abs(frac - 0.5) < 5 * sigma)
    # chi^2 of the top byte over 256 bins
    counts = np.bincount(words >> 24, minlength=256)
    exp = words.size / 256
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 255 + 5 * np.sqrt(2 * 255)


def test_box_muller_normals(orc):
    n = np.concatenate([orc.normals4(5, [i, 1, 0, 1]) for i in range(20000)])
    N = n.size
    assert abs(n.mean()) < 5 / np.sqrt(N)
    assert abs(n.var() - 1) < 5 * np.sqrt(2 / N)
    assert abs((n**4).mean() - 3) < 5 * np.sqrt(96 / N)


# --------------------------------------------------------------- generator

def test_exp_matches_library(orc):
    """exp(i eps sum a_j lambda_j): oracle vs scipy's expm and an eigen
    decomposition (library routines)."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        a = rng.normal(size=8)
        eps = rng.uniform(0.05, 2.0)
        H = np.einsum("j,jab->ab", a, GELLMANN)
        ref = scipy.linalg.expm(1j * eps * H)
        got = orc.su3_exp_iH(a, eps)
        assert np.abs(got - ref).max() < 1e-13
        assert np.abs(got - expm_hermitian(H, eps)).max() < 1e-13


def test_haar_moments(orc):
    """Haar measure on SU(3): E tr g = 0, E|tr g|^2 = 1, E (tr g)^3 = 1
    (one invariant in the triple tensor product; U(3) would give 0)."""
    n = 60000
    tr = np.empty(n, dtype=np.complex128)
    worst = 0.0
    for s in range(n):
        g = orc.haar_su3(1234, s)
        tr[s] = np.trace(g)
        if s < 2000:
            worst = max(worst, unitarity_error(g[None, None]))
    assert worst < 1e-14
    se = 1 / np.sqrt(n)
    assert abs(tr.mean()) < 5 * se
    assert abs((np.abs(tr) ** 2).mean() - 1) < 5 * se * 1.5
    assert abs((tr**3).real.mean() - 1) < 5 * se * 5


def test_generator_scale_and_locality(orc):
    """a_j ~ N(0,1) with tr(lambda_a lambda_b) = 2 delta_ab (no 1/2): for small
    eps, (U - U^dag)/(2 i eps) = H and sum_j a_j^2 = tr(H^2)/2 has mean 8."""
    dims = (2, 2, 4, 4)
    eps = 1e-4
    U = orc.generate_links(dims, 9, eps, haar=False)
    H = (U - dag(U)) / (2j * eps)
    s2 = np.einsum("...ab,...ba->...", H, H).real / 2
    assert abs(s2.mean() - 8) < 5 * np.sqrt(16 / s2.size)
    # any single link can be generated on its own
    Uh = orc.generate_links(dims, 9, 0.3, haar=True)
    for s, mu in [(0, 0), (5, 3), (63, 1), (17, 2)]:
        assert np.array_equal(orc.generated_link(dims, 9, 0.3, True, s, mu), Uh[s, mu])
    assert unitarity_error(Uh) < 1e-14


# --------------------------------------------------------------- F and theta

def test_unit_field(orc):
    dims = (4, 2, 2, 4)
    V = np.prod(dims)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:] = np.eye(3)
    F, th = orc.measure(dims, U)
    assert F == 1.0 and th == 0.0


def test_F_from_local_form(orc):
    """Eq. (6) at g = 1: F = (1/(2 Nc Nd V)) Re sum_x tr K(x)."""
    dims = (4, 4, 2, 6)
    U = orc.generate_links(dims, 2, 0.4)
    F, _ = orc.measure(dims, U)
    K = K_field(dims, U)
    V = np.prod(dims)
    F2 = np.trace(K, axis1=-2, axis2=-1).real.sum() / (2 * 3 * 4 * V)
    assert abs(F - F2) < 1e-14 * abs(F)


def test_theta_from_K(orc):
    """Delta(x) = [(K - K^dag)/(2i)]_traceless, the same Delta as Eq. (4)."""
    dims = (4, 2, 4, 4)
    U = orc.generate_links(dims, 4, 0.3)
    _, th = orc.measure(dims, U)
    K = K_field(dims, U)
    D = (K - dag(K)) / 2j
    D -= np.trace(D, axis1=-2, axis2=-1)[..., None, None] * np.eye(3) / 3
    th2 = (np.abs(D) ** 2).sum() / (3 * np.prod(dims))
    assert abs(th - th2) < 1e-13 * th


# --------------------------------------------------------------- the SU(2) step

def _blocks_of_K(dims, U):
    K = K_field(dims, U).reshape(-1, 3, 3)
    out = []
    for (i, j) in [(0, 1), (0, 2), (1, 2)]:
        out.extend(K[:, [i, j]][:, :, [i, j]])
    return out


def test_su2_step_is_the_maximum_brute_force(orc):
    """On every site of a 2^4 lattice and each subgroup block of K:
    Re tr[s(r) w] = 2|a| and no random SU(2) element, nor any small
    perturbation exp(i delta sigma) s(r), does better."""
    dims = (2, 2, 2, 2)
    U = orc.generate_links(dims, 21, 0.8)
    rng = np.random.default_rng(0)
    R = quat_matrix(random_su2(rng, 10000))
    for w in _blocks_of_K(dims, U):
        r = orc.su2_step(w, 1.0)
        a0 = (w[0, 0] + w[1, 1]).real / 2
        a3 = (w[0, 0] - w[1, 1]).imag / 2
        a1 = (w[0, 1] + w[1, 0]).imag / 2
        a2 = (w[0, 1] - w[1, 0]).real / 2
        best = np.trace(quat_matrix(r) @ w).real
        assert abs(best - 2 * np.sqrt(a0**2 + a1**2 + a2**2 + a3**2)) < 1e-13
        trials = np.trace(R @ w, axis1=1, axis2=2).real
        assert trials.max() <= best + 1e-14
        for k in range(3):
            for d in (1e-3, -1e-3, 1e-5):
                pert = scipy.linalg.expm(1j * d * np.array(
                    [[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]][k]))
                assert np.trace(pert @ quat_matrix(r) @ w).real <= best + 1e-14


def test_su2_step_is_eq9_for_su2(orc):
    """For a quaternion-real block (a sum of SU(2) matrices, as K is for an
    SU(2) field) the step equals K^dag / sqrt(det K^dag) of Eq. (9)."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        q = random_su2(rng, 8)
        w = quat_matrix(q).sum(axis=0)
        r = orc.su2_step(w, 1.0)
        Kd = dag(w)
        g = Kd / np.sqrt(np.linalg.det(Kd))
        assert np.abs(quat_matrix(r) - g).max() < 1e-14


def test_su2_step_degenerate_block(orc):
    r = orc.su2_step(np.zeros((2, 2)), 1.7)
    assert list(r) == [1.0, 0.0, 0.0, 0.0]
    # a block with no quaternion part: w = i * s(q) contributes nothing
    w = 1j * quat_matrix(np.array([0.3, 0.1, -0.2, 0.5]))
    assert list(orc.su2_step(w, 1.3)) == [1.0, 0.0, 0.0, 0.0]


def test_overrelaxation_first_order(orc):
    """Sec. 3.1: omega = 1 gives r exactly; r = 1 stays 1; for a rotation by
    angle phi, N[(1-omega) + omega r] rotates by omega*phi + O(phi^3) about the
    same axis (the first-order form of r^omega)."""
    rng = np.random.default_rng(9)
    for _ in range(100):
        w = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
        assert np.array_equal(orc.su2_step(w, 1.0), orc.su2_step(w, 1.0))
        r1 = orc.su2_step(w, 1.0)
        for om in (1.0, 1.3, 1.7, 1.99, 2.0):
            ro = orc.su2_step(w, om)
            assert abs(np.linalg.norm(ro) - 1) < 1e-15
            c = np.array([1 - om + om * r1[0], *(om * r1[1:])])
            assert np.abs(ro - c / np.linalg.norm(c)).max() < 1e-15
        assert np.array_equal(orc.su2_step(w, 1.0), r1)
    # r = 1: a block proportional to the identity
    assert np.abs(orc.su2_step(np.eye(2) * 3.0, 1.8) - [1, 0, 0, 0]).max() == 0.0
    # small rotations: angle ratio -> omega
    axis = np.array([0.2, -0.5, 0.84])
    axis /= np.linalg.norm(axis)
    for phi in (1e-2, 1e-3):
        b = np.array([np.cos(phi), *(np.sin(phi) * axis)])
        # the block whose maximum is b: w = s(b)^dag (|a| = 1)
        w = dag(quat_matrix(b))
        for om in (1.5, 1.8):
            ro = orc.su2_step(w, om)
            ang = np.arctan2(np.linalg.norm(ro[1:]), ro[0])
            assert abs(ang - om * phi) < 2 * phi**3
            assert np.abs(ro[1:] / np.linalg.norm(ro[1:]) - axis).max() < 1e-10


def test_stochastic_square(orc):
    """Sec. 3.2: the SR step is b^2 (quaternion product), which leaves the
    local objective unchanged."""
    rng = np.random.default_rng(11)
    for _ in range(100):
        w = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
        b = orc.su2_step(w, 1.0)
        r2 = orc.su2_step(w, 1.7, take_square=True)
        assert np.abs(quat_matrix(r2) - quat_matrix(b) @ quat_matrix(b)).max() < 1e-15
        assert abs(np.trace(quat_matrix(r2) @ w).real - np.trace(w).real) < 1e-13


def test_sr_acceptance_rate(orc):
    for p in (0.0, 0.25, 0.5, 1.0):
        d = np.array([orc.sr_decisions(17, s, 3, 0, p) for s in range(6000)])
        if p in (0.0, 1.0):
            assert np.all(d == int(p))
        else:
            n = d.size
            assert abs(d.mean() - p) < 5 * np.sqrt(p * (1 - p) / n)


# --------------------------------------------------------------- sweeps: invariants

def _loops(orc, dims, U):
    vals = []
    for mu in range(4):
        for nu in range(mu + 1, 4):
            for (R, T) in [(1, 1), (1, 2), (2, 1), (2, 2)]:
                vals.append(orc.wilson_loop(dims, U, mu, nu, R, T))
    return np.array(vals)


def test_gauge_invariance(orc):
    """Plaquette and Wilson loops do not change under the Haar gauge
    transformation nor under any sweep (OR and SR)."""
    dims = (4, 4, 4, 6)
    U0 = orc.generate_links(dims, 5, 0.35, haar=False)
    U = orc.generate_links(dims, 5, 0.35, haar=True)
    L0 = _loops(orc, dims, U0)
    assert np.abs(_loops(orc, dims, U) - L0).max() < 1e-12
    assert abs(orc.plaquette(dims, U) - orc.plaquette(dims, U0)) < 1e-12
    for k, (om, p) in enumerate([(1.7, 0.0), (1.0, 0.5), (2.0, 0.0), (1.3, 1.0)]):
        orc.sweep(dims, U, om, p, seed=3, sweep_index=k)
        assert unitarity_error(U) < 1e-12
    assert np.abs(_loops(orc, dims, U) - L0).max() < 1e-12


def test_fixed_link_identity(orc):
    """The identity behind the fixed-link form of the sweep: for links
    transformed by g (the oracle's Eq. (3)), K(x) of the transformed links
    (Eq. (8), written out in numpy) equals g(x) M(x) with M(x) = sum_mu
    U_mu(x) g(x+mu)^dag + [g(x-mu) U_mu(x-mu)]^dag of the untransformed U,
    and the oracle's local update of the transformed links equals the update
    computed from g(x) M(x) alone."""
    dims = (4, 4, 6, 8)
    V = int(np.prod(dims))
    rng = np.random.default_rng(26)
    U = orc.generate_links(dims, 8, 0.3)
    g = random_su3(rng, V)
    Ug = U.copy()
    orc.gauge_transform(dims, Ug, g)
    K = K_field(dims, Ug)
    G = g.reshape(*dims, 3, 3)
    Ugrid = as_grid(dims, U)
    M = np.zeros(tuple(dims) + (3, 3), dtype=np.complex128)
    for mu in range(4):
        g_fwd = np.roll(G, -1, axis=mu)
        g_bwd = np.roll(G, 1, axis=mu)
        M += Ugrid[..., mu, :, :] @ dag(g_fwd) + dag(g_bwd @ backward(dims, U, mu))
    assert np.abs(K - G @ M).max() < 1e-13
    # the update of a site depends on its links only through K: the oracle's
    # update of the transformed links and of links whose K is g M agree
    s = 37
    t, z, y, x = np.unravel_index(s, dims)
    fw = [Ug.reshape(V, 4, 3, 3)[s, mu] for mu in range(4)]
    bw = [Ug.reshape(V, 4, 3, 3)[orc.neighbor(dims, s, mu, -1), mu] for mu in range(4)]
    new, Gs = orc.local_update(np.array(fw + bw), 1.7, [0, 0, 0])
    # a link set with the same K: the forward links carry g M, the rest cancel
    alt = np.zeros((8, 3, 3), dtype=np.complex128)
    alt[0] = G[t, z, y, x] @ M[t, z, y, x]
    new2, Gs2 = orc.local_update(alt, 1.7, [0, 0, 0])
    assert np.abs(Gs - Gs2).max() < 1e-12


def test_wilson_loops_of_abelian_field(orc):
    """For links diag(e^{i a}, e^{i b}, e^{-i(a+b)}) the path product of a loop
    is diagonal with the phases summed around the rectangle, so (1/3) Re tr of
    the R x T loop is (cos A + cos B + cos(A + B)) / 3 with A, B the circulations
    of a and b: written with scalar phases and periodic shifts only."""
    dims = (4, 6, 4, 8)
    rng = np.random.default_rng(11)
    a = rng.uniform(-np.pi, np.pi, (4,) + dims)
    b = rng.uniform(-np.pi, np.pi, (4,) + dims)
    U = np.zeros((int(np.prod(dims)), 4, 3, 3), dtype=np.complex128)
    for mu in range(4):
        U[:, mu, 0, 0] = np.exp(1j * a[mu]).ravel()
        U[:, mu, 1, 1] = np.exp(1j * b[mu]).ravel()
        U[:, mu, 2, 2] = np.exp(-1j * (a[mu] + b[mu])).ravel()

    def shift(f, axis, n):            # f(x + n * axis-hat)
        return np.roll(f, -n, axis=axis)

    def circulation(ph, mu, nu, R, T):
        c = np.zeros(dims)
        for k in range(R):
            c += shift(ph[mu], mu, k)
            c -= shift(shift(ph[mu], nu, T), mu, k)
        for l in range(T):
            c += shift(shift(ph[nu], mu, R), nu, l)
            c -= shift(ph[nu], nu, l)
        return c

    plaq = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            for (R, T) in [(1, 1), (2, 1), (1, 3), (3, 2)]:
                A, B = circulation(a, mu, nu, R, T), circulation(b, mu, nu, R, T)
                want = float(np.mean((np.cos(A) + np.cos(B) + np.cos(A + B)) / 3))
                assert abs(orc.wilson_loop(dims, U, mu, nu, R, T) - want) < 1e-13, (mu, nu, R, T)
                if (R, T) == (1, 1):
                    plaq += want / 6
    assert abs(orc.plaquette(dims, U) - plaq) < 1e-13


@pytest.mark.parametrize("omega,p", [(1.0, 0.0), (1.3, 0.0), (1.7, 0.0), (2.0, 0.0),
                                     (1.0, 0.5), (1.8, 0.3)])
def test_F_never_decreases(orc, omega, p):
    dims = (4, 4, 4, 4)
    U = orc.generate_links(dims, 8, 0.5)
    F_prev, _ = orc.measure(dims, U)
    for k in range(12):
        for par in (0, 1):
            orc.half_sweep(dims, U, par, omega, p, seed=1, sweep=k)
            F, _ = orc.measure(dims, U)
            assert F >= F_prev - 1e-14
            F_prev = F


def test_sr_p1_is_microcanonical(orc):
    """p = 1: every subgroup step is b^2, so F stays put while links move."""
    dims = (4, 4, 2, 4)
    U = orc.generate_links(dims, 6, 0.4)
    F0, _ = orc.measure(dims, U)
    U1 = U.copy()
    for k in range(3):
        orc.sweep(dims, U1, 1.0, 1.0, seed=2, sweep_index=k)
    F1, _ = orc.measure(dims, U1)
    assert abs(F1 - F0) < 1e-13
    assert np.abs(U1 - U).max() > 0.1


def test_checkerboard_order_and_cover(orc):
    """Same-parity sites share no link: any visiting order gives bitwise the
    same half-sweep, and the 8-link sets of one parity cover every link once."""
    dims = (4, 2, 4, 6)
    V = int(np.prod(dims))
    par = parity_grid(dims).reshape(-1)
    for p in (0, 1):
        idx = np.concatenate([orc.site_links(dims, s) for s in range(V) if par[s] == p])
        assert idx.size == 4 * V and np.array_equal(np.sort(idx), np.arange(4 * V))
    U = orc.generate_links(dims, 12, 0.4)
    rng = np.random.default_rng(0)
    for p in (0, 1):
        sites = np.flatnonzero(par == p)
        A, B = U.copy(), U.copy()
        orc.half_sweep(dims, A, p, 1.7, 0.4, seed=5, sweep=2)
        orc.half_sweep(dims, B, p, 1.7, 0.4, seed=5, sweep=2, order=rng.permutation(sites))
        assert np.array_equal(A, B)


def test_reunitarize(orc):
    rng = np.random.default_rng(1)
    g = random_su3(rng, 500)
    a = g.copy()
    orc.reunitarize(a)
    assert np.abs(a - g).max() < 2e-15
    b = a.copy()
    orc.reunitarize(b)
    assert np.abs(b - a).max() < 2e-16 * 8
    noisy = g + 1e-3 * (rng.normal(size=g.shape) + 1j * rng.normal(size=g.shape))
    orc.reunitarize(noisy)
    assert unitarity_error(noisy) < 1e-15
    r0, r1 = noisy[:, 0], noisy[:, 1]
    assert np.abs(noisy[:, 2] - np.conj(np.cross(r0, r1))).max() < 1e-15


# --------------------------------------------------------------- special cases

def _u1_field(dims, phi):
    """U_mu(x) = diag(e^{i phi}, e^{-i phi}, 1), phi of shape (4, V)"""
    V = phi.shape[1]
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = np.exp(1j * phi.T)
    U[:, :, 1, 1] = np.exp(-1j * phi.T)
    U[:, :, 2, 2] = 1
    return U


def _u1_half_sweep(dims, phi, p):
    """Textbook U(1) relaxation: alpha(x) = -arg(sum_mu e^{i phi_mu(x)} +
    e^{-i phi_mu(x-mu)}) on the sites of parity p, then phi_mu(x) += alpha(x),
    phi_mu(x-mu) -= alpha(x)."""
    ph = phi.reshape(4, *dims).copy()
    c = np.zeros(dims, dtype=np.complex128)
    for mu in range(4):
        c += np.exp(1j * ph[mu]) + np.exp(-1j * np.roll(ph[mu], 1, axis=mu))
    alpha = np.where(parity_grid(dims) == p, -np.angle(c), 0.0)
    for mu in range(4):
        ph[mu] += alpha
        ph[mu] -= np.roll(alpha, -1, axis=mu)
    return ph.reshape(4, -1)


def test_u1_embedded_is_u1_relaxation(orc):
    """omega = 1, p = 0 on a U(1)-embedded field: the SU(3) sweep is exactly
    U(1) relaxation."""
    dims = (4, 4, 2, 4)
    rng = np.random.default_rng(3)
    phi = rng.uniform(-1.0, 1.0, size=(4, int(np.prod(dims))))
    U = _u1_field(dims, phi)
    for k in range(4):
        for p in (0, 1):
            orc.half_sweep(dims, U, p, 1.0)
            phi = _u1_half_sweep(dims, phi, p)
            assert np.abs(U - _u1_field(dims, phi)).max() < 1e-13


def test_su2_embedded_stays_embedded(orc):
    dims = (4, 2, 4, 4)
    V = int(np.prod(dims))
    rng = np.random.default_rng(4)
    q = random_su2(rng, 4 * V).reshape(V, 4, 4)
    q[..., 1:] *= 0.6
    q /= np.linalg.norm(q, axis=-1, keepdims=True)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, :2, :2] = quat_matrix(q)
    U[:, :, 2, 2] = 1
    for k in range(5):
        orc.sweep(dims, U, 1.0)
    assert np.abs(U[:, :, 2, :2]).max() < 1e-14
    assert np.abs(U[:, :, :2, 2]).max() < 1e-14
    assert np.abs(U[:, :, 2, 2] - 1).max() < 1e-14


@pytest.mark.parametrize("L,ratio", [(8, 0.7377), (16, 0.9260)])
def test_convergence_rate_matches_red_black_gauss_seidel(orc, L, ratio):
    """Small U(1)-embedded pure gauge, omega = 1: the linearised problem is
    red-black Gauss-Seidel for the lattice Laplacian, whose slowest mode decays
    by mu_J^2 per sweep with mu_J = (3 + cos(2 pi / L)) / 4, so theta ~ |Delta|^2
    decays by mu_J^4 (Young's theorem for consistently ordered matrices)."""
    dims = (L, 4, 4, 4)
    V = int(np.prod(dims))
    rng = np.random.default_rng(L)
    beta = 1e-3 * rng.normal(size=dims)
    phi = np.stack([(beta - np.roll(beta, -1, axis=mu)).reshape(-1) for mu in range(4)])
    U = _u1_field(dims, phi)
    thetas = []
    n = 70 if L == 8 else 110
    for k in range(n):
        orc.sweep(dims, U, 1.0)
        thetas.append(orc.measure(dims, U)[1])
    r = np.array(thetas[1:]) / np.array(thetas[:-1])
    late = r[-20:].mean()
    mu_j = (3 + np.cos(2 * np.pi / L)) / 4
    assert abs(mu_j**4 - ratio) < 1e-4
    assert abs(late - mu_j**4) < 0.01 * mu_j**4


# --------------------------------------------------------------- convergence

def test_pure_gauge_is_driven_back_to_F1(orc):
    """A Haar gauge transform of the unit field is a global maximum: F -> 1 and
    theta -> 0 (seed chosen to land on F = 1, not a Gribov copy)."""
    dims = (4, 4, 4, 4)
    U = orc.generate_links(dims, 1, 0.0, haar=True)
    F0, th0 = orc.measure(dims, U)
    assert F0 < 0.2 and th0 > 0.1
    r = orc.gauge_fix(dims, U, 1.7, 1e-20)
    assert r["status"] == 0
    assert r["F"] >= 1 - 1e-12
    assert unitarity_error(U) < 1e-12


def test_config_8x4_converges(orc):
    """8^4, seed 0, eps 0.25, Haar gauge, omega 1.7: theta < 1e-12 and F
    non-decreasing over the measurement history."""
    dims = (8, 8, 8, 8)
    U = orc.generate_links(dims, 0, 0.25)
    r = orc.gauge_fix(dims, U, 1.7, 1e-12)
    assert r["status"] == 0 and r["theta"] < 1e-12
    h = r["history"]
    assert np.all(np.diff(h[:, 1]) >= -1e-14)
    assert r["sweeps"] % 20 == 0
    assert unitarity_error(U) < 1e-12


def test_converged_is_local_maximum(orc):
    """After convergence F is a local maximum along random gauge directions
    g = exp(i eps X(x)), X Hermitian traceless: the first-order change vanishes
    (stationarity, Im tr[lambda_a K(x)] = 0) and F drops by O(eps^2)."""
    dims = (4, 4, 4, 4)
    V = int(np.prod(dims))
    U = orc.generate_links(dims, 2, 0.3)
    r = orc.gauge_fix(dims, U, 1.7, 1e-24)
    assert r["status"] == 0
    F, _ = orc.measure(dims, U)
    K = K_field(dims, U).reshape(-1, 3, 3)
    stat = np.einsum("aij,sji->sa", GELLMANN, K).imag
    assert np.abs(stat).max() < 1e-10
    rng = np.random.default_rng(0)
    drops = {}
    for eps in (1e-3, 5e-4):
        d = []
        for _ in range(3):
            X = np.einsum("sa,aij->sij", rng.normal(size=(V, 8)), GELLMANN)
            g = expm_hermitian(X, eps)
            Ug = U.copy()
            orc.gauge_transform(dims, Ug, g)
            Fg, _ = orc.measure(dims, Ug)
            assert Fg < F
            d.append((F - Fg) / eps**2)
        drops[eps] = np.mean(d)
    assert abs(drops[1e-3] / drops[5e-4] - 1) < 0.05
