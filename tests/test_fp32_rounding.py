"""Where the FP32 parity bar comes from (CPU only).

Exact IEEE single-precision evaluations of one sweep (numpy float32, every
operation rounded to FP32, the same steps as the method: K summed link by
link, the three SU(2) subgroup steps, G applied to the 8 links) are compared
with the FP64 oracle on the FP32-rounded input links, in two operation
orders: every operation rounded (as written), and every dot product and
multiply-add rounded once (as fused multiply-adds do).  Their worst links
exceed 2e-6 relative error: those sites' SU(2) subproblem is ill conditioned
(quaternion projection |a| small against |W|, so the rounding of W is
amplified by |W|/|a|), and the stochastic-relaxation square doubles the angle
error.  The two orders also differ from each other by more than a factor 2
on single links, so no fixed ratio to one emulation bounds another rounding
order.  The GPU tests therefore take the bar link by link from a
randomised-rounding model of the same steps (fp32_model: the largest error of
16 runs with every operation perturbed by up to 2^-24, times 2, plus 2^-24),
and keep 2e-6 on 99 % of the links.  These tests check that both exact
orders stay within that bar on every link."""
from __future__ import annotations

import numpy as np
import pytest

import fp32_model as fm
from lattice_np import stored_as

f32 = np.float32


def _site_update_fp32(L, omega, squares):
    Lr = L.real.astype(f32)
    Li = L.imag.astype(f32)
    Kr = np.zeros((3, 3), f32)
    Ki = np.zeros((3, 3), f32)
    for m in range(4):
        Kr = Kr + Lr[m] + Lr[4 + m].T
        Ki = Ki + Li[m] - Li[4 + m].T
    Gr, Gi = np.eye(3, dtype=f32), np.zeros((3, 3), f32)
    Wr, Wi = Kr.copy(), Ki.copy()
    for k, (i, j) in enumerate([(0, 1), (0, 2), (1, 2)]):
        a0 = Wr[i, i] + Wr[j, j]
        a3 = Wi[i, i] - Wi[j, j]
        a1 = Wi[i, j] + Wi[j, i]
        a2 = Wr[i, j] - Wr[j, i]
        inv = f32(1) / np.sqrt(f32(a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3))
        b = np.array([a0 * inv, -a1 * inv, -a2 * inv, -a3 * inv], dtype=f32)
        if squares[k]:
            b = np.array([b[0] * b[0] - (b[1] * b[1] + b[2] * b[2] + b[3] * b[3]),
                          f32(2) * b[0] * b[1], f32(2) * b[0] * b[2], f32(2) * b[0] * b[3]], dtype=f32)
        elif omega != 1.0:
            c = np.array([f32(1 - omega) + f32(omega) * b[0], f32(omega) * b[1], f32(omega) * b[2],
                          f32(omega) * b[3]], dtype=f32)
            b = (c * (f32(1) / np.sqrt(f32((c * c).sum())))).astype(f32)
        Rr, Ri = np.eye(3, dtype=f32), np.zeros((3, 3), f32)
        Rr[i, i], Ri[i, i], Rr[i, j], Ri[i, j] = b[0], b[3], b[2], b[1]
        Rr[j, i], Ri[j, i], Rr[j, j], Ri[j, j] = -b[2], b[1], b[0], -b[3]
        Gr, Gi = (Rr @ Gr - Ri @ Gi).astype(f32), (Rr @ Gi + Ri @ Gr).astype(f32)
        Wr, Wi = (Rr @ Wr - Ri @ Wi).astype(f32), (Rr @ Wi + Ri @ Wr).astype(f32)
    G = (Gr + 1j * Gi).astype(np.complex64)
    out = L.astype(np.complex64).copy()
    for m in range(4):
        out[m] = G @ out[m]
        out[4 + m] = out[4 + m] @ G.conj().T
    return out


def _site_update_fp32_fused(L, omega, squares):
    """The same steps with every dot product and multiply-add rounded once."""
    Lr = L.real.astype(f32).astype(np.float64)
    Li = L.imag.astype(f32).astype(np.float64)

    def r(x):
        return np.asarray(x).astype(f32).astype(np.float64)

    Kr, Ki = np.zeros((3, 3)), np.zeros((3, 3))
    for m in range(4):
        Kr = r(r(Kr + Lr[m]) + Lr[4 + m].T)
        Ki = r(r(Ki + Li[m]) - Li[4 + m].T)
    Gr, Gi = np.eye(3), np.zeros((3, 3))
    Wr, Wi = Kr.copy(), Ki.copy()
    for k, (i, j) in enumerate([(0, 1), (0, 2), (1, 2)]):
        a0, a3 = r(Wr[i, i] + Wr[j, j]), r(Wi[i, i] - Wi[j, j])
        a1, a2 = r(Wi[i, j] + Wi[j, i]), r(Wr[i, j] - Wr[j, i])
        inv = r(1.0 / r(np.sqrt(r(a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3))))
        b = r(np.array([a0, -a1, -a2, -a3]) * inv)
        if squares[k]:
            b = r(np.array([b[0] * b[0] - (b[1] ** 2 + b[2] ** 2 + b[3] ** 2), 2 * b[0] * b[1],
                            2 * b[0] * b[2], 2 * b[0] * b[3]]))
        elif omega != 1.0:
            c = r(np.array([(1 - omega) + omega * b[0], omega * b[1], omega * b[2], omega * b[3]]))
            b = r(c * r(1.0 / r(np.sqrt((c * c).sum()))))
        Rr, Ri = np.eye(3), np.zeros((3, 3))
        Rr[i, i], Ri[i, i], Rr[i, j], Ri[i, j] = b[0], b[3], b[2], b[1]
        Rr[j, i], Ri[j, i], Rr[j, j], Ri[j, j] = -b[2], b[1], b[0], -b[3]
        Gr, Gi = r(Rr @ Gr - Ri @ Gi), r(Rr @ Gi + Ri @ Gr)
        Wr, Wi = r(Rr @ Wr - Ri @ Wi), r(Rr @ Wi + Ri @ Wr)
    G = Gr + 1j * Gi
    out = L.astype(np.complex64).astype(np.complex128).copy()
    for m in range(4):
        o = G @ out[m]
        out[m] = r(o.real) + 1j * r(o.imag)
        o = out[4 + m] @ G.conj().T
        out[4 + m] = r(o.real) + 1j * r(o.imag)
    return out


def _sweep_fp32(orc, dims, U32, update, omega, p, seed, sweep, instance=0):
    """one full sweep (parity 0, then 1) with an exact FP32 site update"""
    W = U32.astype(np.complex128).copy()
    for par in (0, 1):
        for s in range(W.shape[0]):
            if orc.parity(dims, s) != par:
                continue
            nb = [orc.neighbor(dims, s, mu, -1) for mu in range(4)]
            L = np.array([W[s, mu] for mu in range(4)] + [W[nb[mu], mu] for mu in range(4)])
            out = update(L, omega, orc.sr_decisions(seed, s, sweep, instance, p)).astype(np.complex128)
            for mu in range(4):
                W[s, mu] = out[mu]
                W[nb[mu], mu] = out[4 + mu]
    return W


def _rebuild_row2(W):
    W = W.copy()
    W[..., 2, :] = np.conj(np.cross(W[..., 0, :].astype(np.complex64), W[..., 1, :].astype(np.complex64)))
    return W


def test_exact_fp32_misses_2e6_on_ill_conditioned_links(orc):
    dims = (4, 4, 6, 10)
    omega, p, seed, sweep = 1.0, 0.5, 9, 3
    U32 = orc.generate_links(dims, 7, 0.35).astype(np.complex64)
    ref = U32.astype(np.complex128)
    orc.sweep(dims, ref, omega, p, seed=seed, sweep_index=sweep)
    W = _sweep_fp32(orc, dims, U32, _site_update_fp32, omega, p, seed, sweep)
    e = fm.link_errs(W, ref)
    assert e.max() > 2e-6                        # exact FP32 misses 2e-6 on some links ...
    assert np.quantile(e, 0.99) <= 2e-6          # ... but not on 99% of them


@pytest.mark.parametrize("dims,omega,p,fmt,useed", [((4, 4, 6, 10), 1.0, 0.5, 1, 7), ((4, 4, 6, 10), 1.7, 0.0, 2, 7),
                                                    ((8, 6, 4, 12), 1.8, 0.3, 1, 7), ((6, 4, 4, 8), 1.0, 0.5, 2, 7),
                                                    ((4, 4, 6, 10), 1.0, 0.5, 1, 8), ((4, 4, 6, 10), 2.0, 0.0, 2, 9)])
def test_envelope_bounds_exact_fp32_in_two_orders(orc, dims, omega, p, fmt, useed):
    """Both exact FP32 orders are within twice the randomised-rounding
    envelope (plus u) on every link; the orders themselves disagree by more
    than the factor 2 of the suggestion 'GPU <= 2 x emulation + c' on some
    case, which is why the bar comes from the envelope."""
    U0 = stored_as(orc.generate_links(dims, useed, 0.35), fmt)
    ref = U0.copy()
    orc.sweep(dims, ref, omega, p, seed=9, sweep_index=3)
    env = fm.link_sweep_envelope(orc, dims, U0, fmt, ref, omega, p, 9, 3)
    U32 = U0.astype(np.complex64)
    for update in (_site_update_fp32, _site_update_fp32_fused):
        W = _sweep_fp32(orc, dims, U32, update, omega, p, 9, 3)
        if fmt == 2:
            W = _rebuild_row2(W)
        ok, info = fm.fp32_bar_ok(W, ref, env)
        assert ok, (update.__name__, info)


def test_two_exact_orders_differ_by_more_than_twice(orc):
    """On this case the plain order's worst link is 1.6 times 2 x (fused
    order's error) + 4e-7: a bar of 'twice another rounding sequence' fails."""
    dims = (4, 4, 6, 10)
    U32 = orc.generate_links(dims, 7, 0.35).astype(np.complex64)
    ref = U32.astype(np.complex128)
    orc.sweep(dims, ref, 1.0, 0.5, seed=9, sweep_index=3)
    A = _sweep_fp32(orc, dims, U32, _site_update_fp32, 1.0, 0.5, 9, 3)
    B = _sweep_fp32(orc, dims, U32, _site_update_fp32_fused, 1.0, 0.5, 9, 3)
    eA, eB = fm.link_errs(A, ref), fm.link_errs(B, ref)
    assert np.max(eA / (2 * eB + 4e-7)) > 1.0


def test_envelope_on_a_12x4_ensemble_configuration(orc):
    """A 12^4 configuration of the 48-lattice workload (index 2: seed 102,
    Haar gauge; FP32 12-real input), one full stochastic-relaxation sweep:
    82944 links, the worst of exact FP32 near 1e-5, all within the bar."""
    import json
    import os
    man = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                      "ensemble48_manifest.json")))["configs"]
    c = man[2]
    d, i = tuple(c["dims"]), c["index"]
    U0 = stored_as(orc.generate_links(d, c["seed"], c["eps"], True), 2)
    ref = U0.copy()
    orc.sweep(d, ref, 1.0, 0.5, seed=5, sweep_index=0, instance=i)
    env = fm.link_sweep_envelope(orc, d, U0, 2, ref, 1.0, 0.5, 5, 0, instance=i)
    W = _rebuild_row2(_sweep_fp32(orc, d, U0.astype(np.complex64), _site_update_fp32, 1.0, 0.5, 5, 0, i))
    e = fm.link_errs(W, ref)
    assert np.quantile(e, 0.99) <= 2e-6 and 5e-6 < e.max()
    ok, info = fm.fp32_bar_ok(W, ref, env)
    assert ok, info
