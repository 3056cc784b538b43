"""Pins of the oracle's simulated annealing (CPU only).

The paper names simulated annealing among the supported methods (Sec. 1)
without its details.  The reading: the SU(2) step of each Cabibbo-Marinari
subgroup draws r with weight exp(Re tr[s(r) w] / T) against the Haar measure
of SU(2), i.e. r = x b with b the maximum of Eq. (9) and x0 = <r, b> of
density sqrt(1 - x0^2) exp(alpha x0), alpha = 2|a|/T; the direction of
(x1, x2, x3) is uniform.  These tests pin it to what the mathematics fixes:
T -> 0 gives Eq. (9); the x0 histogram follows the closed-form density (its
CDF by quadrature, its mean I_2(alpha)/I_1(alpha)); the directions are
isotropic; w = 0 gives the Haar measure; the accept-reject loop accepts at
the closed-form rates; annealing is a gauge transformation; the schedule is
linear; and annealing then overrelaxation drives a pure gauge back to F = 1.
"""
from __future__ import annotations

import numpy as np
import pytest
from scipy import integrate, special

from lattice_np import quat_matrix, unitarity_error

N_DRAWS = 20000


def draws(orc, w, T, n=N_DRAWS, seed=11, k=0):
    rs = np.zeros((n, 4))
    trials = np.zeros(n, dtype=np.int64)
    for i in range(n):
        rs[i], trials[i] = orc.su2_heatbath(w, T, seed, i, 3, 0, k)
    return rs, trials


def x0_cdf(alpha):
    """CDF of sqrt(1 - x^2) exp(alpha x) on [-1, 1] by quadrature on a grid
    (dense near the ends, where the density has square-root edges)."""
    th = np.linspace(np.pi, 0.0, 20001)
    x = np.cos(th)
    # x = cos(theta): sqrt(1 - x^2) dx = sin^2(theta) dtheta (up to sign)
    f = np.sin(th) ** 2 * np.exp(alpha * x)
    c = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * np.diff(-th))])
    z = np.pi * special.iv(1, alpha) / alpha
    assert abs(c[-1] / z - 1) < 1e-6
    return lambda q: np.interp(q, x, c / c[-1])


def ks_pvalue(samples, cdf):
    from scipy import stats
    return stats.kstest(samples, cdf).pvalue


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_zero_temperature_is_the_eq9_maximum(orc, seed):
    """T -> 0: alpha -> infinity, x0 = 1 and x = 1, so r is the maximum b of
    Eq. (9), which su2_step gives at omega = 1."""
    rng = np.random.default_rng(seed)
    for _ in range(50):
        w = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
        r, n = orc.su2_heatbath(w, 1e-300, 5, int(rng.integers(1 << 20)), 0)
        assert n == 1
        assert np.abs(r - orc.su2_step(w, 1.0)).max() <= 1e-15


@pytest.mark.parametrize("alpha", [0.2, 0.69, 0.71, 2.0, 8.0])
def test_x0_follows_the_boltzmann_density(orc, alpha):
    """w = (alpha/2) 1 at T = 1: b = 1, r = x; x0 against the closed-form
    density (both samplers, either side of their switch at alpha = 0.7)."""
    rs, _ = draws(orc, 0.5 * alpha * np.eye(2), 1.0)
    x0 = rs[:, 0]
    assert ks_pvalue(x0, x0_cdf(alpha)) > 1e-4
    mean = special.iv(2, alpha) / special.iv(1, alpha)
    assert abs(x0.mean() - mean) < 5 * x0.std() / np.sqrt(len(x0))


def test_directions_are_isotropic(orc):
    rs, _ = draws(orc, 0.5 * 1.3 * np.eye(2), 1.0)
    v = rs[:, 1:]
    n = len(v)
    assert np.all(np.abs(v.mean(axis=0)) < 5 * v.std(axis=0) / np.sqrt(n))
    expect = (1 - (rs[:, 0] ** 2).mean()) / 3
    m2 = (v ** 2).mean(axis=0)
    assert np.all(np.abs(m2 - expect) < 5 * (v ** 2).std(axis=0) / np.sqrt(n))
    c = (v[:, 0] * v[:, 1]).mean(), (v[:, 0] * v[:, 2]).mean(), (v[:, 1] * v[:, 2]).mean()
    assert np.all(np.abs(c) < 5 * expect / np.sqrt(n) * 2)


def test_rotated_to_the_maximum(orc):
    """A general block: r is a unit quaternion and <r, b> (b of Eq. (9)) has
    the density of x0 at alpha = 2|a|/T."""
    rng = np.random.default_rng(4)
    w = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    T = 0.8
    b = orc.su2_step(w, 1.0)
    a = np.array([(w[0, 0] + w[1, 1]).real, (w[0, 1] + w[1, 0]).imag, (w[0, 1] - w[1, 0]).real,
                  (w[0, 0] - w[1, 1]).imag]) / 2
    alpha = 2 * np.linalg.norm(a) / T
    rs, _ = draws(orc, w, T, n=10000)
    assert np.abs(np.linalg.norm(rs, axis=1) - 1).max() < 1e-14
    assert ks_pvalue(rs @ b, x0_cdf(alpha)) > 1e-4
    # the weight is the subgroup functional: Re tr[s(r) w] = 2 |a| <r, b>
    f = np.array([np.trace(quat_matrix(r) @ w).real for r in rs[:50]])
    assert np.abs(f - 2 * np.linalg.norm(a) * (rs[:50] @ b)).max() < 1e-12


def test_degenerate_block_gives_the_haar_measure(orc):
    """w = 0: alpha = 0 and r is Haar distributed on SU(2) = S^3:
    E r0 = 0, E r0^2 = 1/4, E |tr s(r)|^2 = 1."""
    rs, _ = draws(orc, np.zeros((2, 2)), 1.0)
    n = len(rs)
    assert abs(rs[:, 0].mean()) < 5 * 0.5 / np.sqrt(n)
    assert abs((rs[:, 0] ** 2).mean() - 0.25) < 5 * np.sqrt(1 / 8 - 1 / 16) / np.sqrt(n)
    assert abs(((2 * rs[:, 0]) ** 2).mean() - 1.0) < 5 * np.sqrt(2.0 - 1.0) / np.sqrt(n)


@pytest.mark.parametrize("alpha", [0.3, 0.69, 0.71, 3.0])
def test_acceptance_rates(orc, alpha):
    """Mean trials per draw = 1 / acceptance probability, the closed forms of
    the two samplers: uniform proposal (1/2) int sqrt(1-x^2) e^{alpha(x-1)} dx,
    Kennedy-Pendleton E[sqrt(1 - l); l < 1] for l ~ Gamma(3/2, rate 2 alpha)."""
    _, trials = draws(orc, 0.5 * alpha * np.eye(2), 1.0, n=10000)
    if alpha < 0.7:
        acc = 0.5 * integrate.quad(lambda x: np.sqrt(1 - x * x) * np.exp(alpha * (x - 1)), -1, 1)[0]
    else:
        acc = integrate.quad(lambda l: np.sqrt(1 - l) * (2 * alpha) ** 1.5 * np.sqrt(l) * np.exp(-2 * alpha * l)
                             / special.gamma(1.5), 0, 1)[0]
    mean, sd = 1 / acc, np.sqrt(1 - acc) / acc
    assert abs(trials.mean() - mean) < 5 * sd / np.sqrt(len(trials))
    assert trials.max() <= 64


def test_schedule_is_linear(orc):
    assert orc.anneal_temperature(0, 100, 1.5, 0.05) == 1.5
    assert orc.anneal_temperature(99, 100, 1.5, 0.05) == 0.05
    assert abs(orc.anneal_temperature(33, 100, 1.5, 0.05) - (1.5 + (0.05 - 1.5) * 33 / 99)) < 1e-15
    T = [orc.anneal_temperature(n, 100, 1.5, 0.05) for n in range(100)]
    assert np.abs(np.diff(T) - (0.05 - 1.5) / 99).max() < 1e-15
    assert orc.anneal_temperature(0, 1, 0.7, 0.1) == 0.7


def test_annealing_is_a_gauge_transformation(orc):
    """Annealing sweeps transform every link by g(x) . g(x+mu)^dag: plaquette
    and Wilson loops are unchanged (1e-12) and the links stay in SU(3)."""
    dims = (4, 4, 4, 6)
    U = orc.generate_links(dims, 8, 0.3)
    before = [orc.wilson_loop(dims, U, mu, nu, R, T) for mu in range(4) for nu in range(mu + 1, 4)
              for (R, T) in [(1, 1), (1, 2), (2, 2)]]
    n = orc.anneal(dims, U, 30, 1.2, 0.1, seed=3)
    assert n >= 30 * 3 * U.shape[0]
    after = [orc.wilson_loop(dims, U, mu, nu, R, T) for mu in range(4) for nu in range(mu + 1, 4)
             for (R, T) in [(1, 1), (1, 2), (2, 2)]]
    assert np.abs(np.array(after) - np.array(before)).max() < 1e-12
    assert unitarity_error(U) < 1e-13


def test_high_temperature_scrambles_and_low_temperature_orders(orc):
    """At high T the heat bath randomises the gauge (F of a fixed field drops
    towards 0); at low T it raises F like relaxation."""
    dims = (4, 4, 4, 4)
    U = orc.generate_links(dims, 2, 0.0, haar=False)   # the unit field, F = 1
    orc.anneal(dims, U, 5, 50.0, 50.0, seed=1)
    F_hot, _ = orc.measure(dims, U)
    assert abs(F_hot) < 0.1
    orc.anneal(dims, U, 60, 0.05, 0.05, seed=1, sweep0=5)
    F_cold, _ = orc.measure(dims, U)
    assert F_cold > 0.9


def test_annealing_then_overrelaxation_reaches_the_global_maximum(orc):
    """A random gauge transformation of the unit field (4^4, seed 1): 100
    annealing sweeps from T = 1 to 0.02, then overrelaxation to theta < 1e-14:
    F = 1, the global maximum."""
    dims = (4, 4, 4, 4)
    U = orc.generate_links(dims, 1, 0.0, haar=True)
    orc.anneal(dims, U, 100, 1.0, 0.02, seed=7)
    r = orc.gauge_fix(dims, U, 1.7, 1e-14)
    assert r["status"] == 0
    assert r["F"] >= 1 - 1e-12
