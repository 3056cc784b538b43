"""Where the FP32 parity tolerance comes from (CPU only).

A plain IEEE single-precision emulation of one site update (numpy float32,
every operation rounded to FP32, the same steps as the method: K summed link by
link, the three SU(2) subgroup steps, G applied to the 8 links) is compared with
the FP64 oracle on the FP32-rounded input links.  The worst links exceed
2e-6 relative error: their SU(2) subproblem is ill conditioned (quaternion
projection |a| small against |W|, so the rounding of W is amplified by
|W|/|a|), and the stochastic-relaxation square doubles the angle error.  The
GPU parity tests therefore bound FP32 sweeps by 2e-6 on 99% of links and
2e-5 on all, the distribution exact FP32 arithmetic itself produces: its worst
link grows with the number of links (2.4e-6..1e-5 on a 4x4x6x10 lattice, 9e-6
on the 12^4 lattice of the 48-configuration workload, 82944 links)."""
from __future__ import annotations

import numpy as np

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


def test_fp32_tolerance_is_arithmetic(orc):
    dims = (4, 4, 6, 10)
    omega, p, seed, sweep = 1.0, 0.5, 9, 3
    U = orc.generate_links(dims, 7, 0.35)
    U32 = U.astype(np.complex64)
    ref = U32.astype(np.complex128)
    orc.half_sweep(dims, ref, 0, omega, p, seed=seed, sweep=sweep)
    orc.half_sweep(dims, ref, 1, omega, p, seed=seed, sweep=sweep)
    W = U32.copy()
    V = W.shape[0]
    for par in (0, 1):
        for s in range(V):
            if orc.parity(dims, s) != par:
                continue
            nb = [orc.neighbor(dims, s, mu, -1) for mu in range(4)]
            L = np.array([W[s, mu] for mu in range(4)] + [W[nb[mu], mu] for mu in range(4)])
            out = _site_update_fp32(L, omega, orc.sr_decisions(seed, s, sweep, 0, p))
            for mu in range(4):
                W[s, mu] = out[mu]
                W[nb[mu], mu] = out[4 + mu]
    e = np.linalg.norm((W.astype(np.complex128) - ref).reshape(-1, 9), axis=1) / np.sqrt(3)
    assert e.max() > 2e-6                        # exact FP32 misses 2e-6 on some links ...
    assert np.quantile(e, 0.99) <= 2e-6          # ... but not on 99% of them
    assert e.max() <= 2e-5


def test_fp32_tail_grows_with_the_lattice(orc):
    """The same emulation on a 12^4 configuration of the 48-lattice workload
    (index 2: seed 102, eps 0.332797, Haar gauge; FP32 12-real input), one full
    stochastic-relaxation sweep: the worst of its 82944 links is near 1e-5."""
    import json
    import os
    man = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                      "ensemble48_manifest.json")))["configs"]
    c = man[2]
    d, i = tuple(c["dims"]), c["index"]
    U32 = orc.generate_links(d, c["seed"], c["eps"], True).astype(np.complex64)
    U32[..., 2, :] = np.conj(np.cross(U32[..., 0, :], U32[..., 1, :]))
    ref = U32.astype(np.complex128)
    orc.sweep(d, ref, 1.0, 0.5, seed=5, sweep_index=0, instance=i)
    W = U32.copy()
    for par in (0, 1):
        for s in range(W.shape[0]):
            if orc.parity(d, s) != par:
                continue
            nb = [orc.neighbor(d, s, mu, -1) for mu in range(4)]
            L = np.array([W[s, mu] for mu in range(4)] + [W[nb[mu], mu] for mu in range(4)])
            out = _site_update_fp32(L, 1.0, orc.sr_decisions(5, s, 0, i, 0.5))
            for mu in range(4):
                W[s, mu] = out[mu]
                W[nb[mu], mu] = out[4 + mu]
    W[..., 2, :] = np.conj(np.cross(W[..., 0, :], W[..., 1, :]))
    e = np.linalg.norm((W.astype(np.complex128) - ref).reshape(-1, 9), axis=1) / np.sqrt(3)
    assert np.quantile(e, 0.99) <= 2e-6
    assert 5e-6 < e.max() <= 2e-5
