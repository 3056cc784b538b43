"""Pins of the oracle's Coulomb-gauge functions (CPU): the functional is the
spatial links of each timeslice, the gauge transformation still acts on the
temporal links, and the timeslices are independent problems."""
from __future__ import annotations

import numpy as np
import pytest

from lattice_np import GELLMANN, as_grid, dag, unitarity_error


def K_spatial(dims, U):
    G = as_grid(dims, U)
    K = np.zeros(tuple(dims) + (3, 3), dtype=np.complex128)
    for mu in (1, 2, 3):
        K += G[..., mu, :, :] + dag(np.roll(G[..., mu, :, :], 1, axis=mu))
    return K


def test_coulomb_measure_two_ways(orc):
    """theta_C(t) from the A_i differences (oracle) equals the K form over the
    spatial links; F_C(t) is the spatial trace average of each timeslice."""
    dims = (4, 4, 6, 4)
    U = orc.generate_links(dims, 3, 0.4)
    F, th = orc.measure_coulomb(dims, U)
    K = K_spatial(dims, U)
    D = (K - dag(K)) / 2j
    D -= np.trace(D, axis1=-2, axis2=-1)[..., None, None] * np.eye(3) / 3
    th2 = (np.abs(D) ** 2).sum(axis=(1, 2, 3, 4, 5)) / (3 * np.prod(dims[1:]))
    G = as_grid(dims, U)
    F2 = np.trace(G[..., 1:, :, :], axis1=-2, axis2=-1).real.sum(axis=(1, 2, 3, 4)) / (9 * np.prod(dims[1:]))
    assert np.abs(th - th2).max() < 1e-13 * th.max()
    assert np.abs(F - F2).max() < 1e-14


def test_coulomb_pure_gauge_driven_to_F1(orc):
    dims = (4, 6, 6, 6)
    U = orc.generate_links(dims, 5, 0.0, True)
    r = orc.coulomb_gauge_fix(dims, U, 1.7, 1e-20)
    assert r["status"] == 0
    assert np.all(r["F_t"] > 1 - 1e-12) and np.all(r["theta_t"] < 1e-20)
    assert unitarity_error(U) < 1e-12


def test_coulomb_gauge_invariance_includes_temporal_links(orc):
    """Plaquettes and Wilson loops in all six planes, temporal ones included,
    are unchanged: the update is a full gauge transformation of every link."""
    dims = (4, 4, 4, 6)
    U = orc.generate_links(dims, 8, 0.35)
    loops0 = [orc.wilson_loop(dims, U, mu, nu, R, T) for mu in range(4) for nu in range(mu + 1, 4)
              for (R, T) in [(1, 1), (2, 1)]]
    for k in range(4):
        orc.sweep_coulomb(dims, U, 1.7, 0.3 if k == 2 else 0.0, seed=1, sweep_index=k)
    loops1 = [orc.wilson_loop(dims, U, mu, nu, R, T) for mu in range(4) for nu in range(mu + 1, 4)
              for (R, T) in [(1, 1), (2, 1)]]
    assert np.abs(np.array(loops1) - np.array(loops0)).max() < 1e-12


@pytest.mark.parametrize("omega", [1.0, 1.5, 1.9])
def test_coulomb_functional_never_decreases_per_slice(orc, omega):
    dims = (4, 4, 4, 4)
    U = orc.generate_links(dims, 9, 0.5)
    F0, _ = orc.measure_coulomb(dims, U)
    for k in range(6):
        for parity in (0, 1):
            orc.half_sweep_coulomb(dims, U, parity, omega)
            F1, _ = orc.measure_coulomb(dims, U)
            assert np.all(F1 >= F0 - 1e-14)
            F0 = F1


def test_timeslices_are_independent(orc):
    """The spatial links of a timeslice evolve the same, bit for bit, whatever
    the other timeslices and the temporal links hold; a frozen timeslice keeps
    its spatial links."""
    dims = (4, 4, 4, 6)
    A = orc.generate_links(dims, 1, 0.4)
    B = orc.generate_links(dims, 2, 0.4)
    GA, GB = as_grid(dims, A), as_grid(dims, B)
    GB[1, ..., 1:, :, :] = GA[1, ..., 1:, :, :]          # same spatial links in slice 1
    for k in range(3):
        orc.sweep_coulomb(dims, A, 1.7)
        orc.sweep_coulomb(dims, B, 1.7)
    assert np.array_equal(GA[1, ..., 1:, :, :], GB[1, ..., 1:, :, :])
    C = orc.generate_links(dims, 4, 0.4)
    GC = as_grid(dims, C)
    before = GC[2, ..., 1:, :, :].copy()
    orc.sweep_coulomb(dims, C, 1.7, slice_active=[1, 1, 0, 1])
    assert np.array_equal(GC[2, ..., 1:, :, :], before)
    assert not np.array_equal(GC[1, ..., 1:, :, :], as_grid(dims, orc.generate_links(dims, 4, 0.4))[1, ..., 1:, :, :])


def test_coulomb_converged_is_stationary(orc):
    """At convergence Im tr[lambda_a K_C(x)] = 0 on every site (first-order
    optimality of each timeslice's functional)."""
    dims = (4, 4, 4, 4)
    U = orc.generate_links(dims, 6, 0.3)
    r = orc.coulomb_gauge_fix(dims, U, 1.7, 1e-24)
    assert r["status"] == 0
    K = K_spatial(dims, U).reshape(-1, 3, 3)
    stat = np.einsum("aij,sji->sa", GELLMANN, K).imag
    assert np.abs(stat).max() < 1e-10
    assert np.all(r["sweeps_t"] > 0) and r["sweeps_t"].max() == r["sweeps"]
