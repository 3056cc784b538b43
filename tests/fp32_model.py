"""A randomised-rounding model of the library's FP32 site updates, from which
the GPU tests derive their per-link FP32 bar (test helper; CPU only).

Every FP32 operation of an update rounds its result to the nearest float, a
relative error of at most u = 2^-24.  The model runs the update's steps in
FP64 and multiplies the result of every operation by (1 + d), d uniform in
[-u, u] and independent per operation (Monte Carlo arithmetic, D. S. Parker,
"Monte Carlo arithmetic: exploiting randomness in floating-point arithmetic",
1997).  A run of the GPU is one such sequence of roundings, a fixed rather
than a random one; how far a link can move under them is set by the link's
conditioning (an SU(2) subproblem with |a| small against |W| amplifies the
rounding of W by |W|/|a|).  The envelope of a link is the largest error of
N independent runs; the bar on a link is twice that, plus one unit u, and
the stated 2e-6 still holds for 99 % of the links.  The CPU tests check
that exact IEEE FP32 evaluations of the same steps in two different operation
orders stay within the bar on every link.

The steps follow the library's updates (reading them is what makes the
model a model of the GPU's arithmetic, not of the oracle's):
  link-rewriting form: K = sum_mu U_mu(x) + U_mu(x-mu)^dag summed in
  direction order, the three SU(2) steps (Eq. (9), OR / SR), G U_mu(x) and
  U_mu(x-mu) G^dag; 12-real storage keeps rows 0 and 1 and rebuilds row 2 as
  conj(row0 x row1) in FP32;
  fixed-link form: M = sum_mu U_mu(x) g(x+mu)^dag + [g(x-mu) U_mu(x-mu)]^dag
  (rows 0 and 1 of every product, row 2 rebuilt), K = g(x) M, the same SU(2)
  steps on G = g(x), the new g reunitarized in FP64 and stored in FP32-12,
  and the links handed back as g(x) U_mu(x) g(x+mu)^dag in FP64.
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24
SUBGROUPS = ((0, 1), (0, 2), (1, 2))


class Rounding:
    """x -> x (1 + d), d ~ U[-u, u], one draw per element and operation."""

    def __init__(self, rng: np.random.Generator, u: float = U32):
        self.rng, self.u = rng, u

    def __call__(self, x):
        x = np.asarray(x, dtype=np.float64)
        return x * (1.0 + self.u * self.rng.uniform(-1.0, 1.0, x.shape))

    def c(self, z):
        z = np.asarray(z, dtype=np.complex128)
        return self(z.real) + 1j * self(z.imag)


def cmul(R, a, b):
    """complex product, each real product and sum rounded"""
    return (R(R(a.real * b.real) - R(a.imag * b.imag))
            + 1j * R(R(a.real * b.imag) + R(a.imag * b.real)))


def matmul(R, A, B, rows=3):
    """rows [0, rows) of A B for stacks of 3x3 matrices, the three terms of
    each entry summed in index order"""
    A = A[..., :rows, :]
    out = cmul(R, A[..., :, 0:1], B[..., 0:1, :])
    for k in (1, 2):
        out = R.c(out + cmul(R, A[..., :, k:k + 1], B[..., k:k + 1, :]))
    return out


def dag(A):
    return np.conj(np.swapaxes(A, -1, -2))


def with_row2(R, A2):
    """rows 0 and 1 of A2, row 2 = conj(row0 x row1) in rounded arithmetic"""
    r0, r1 = A2[..., 0, :], A2[..., 1, :]
    row2 = np.stack([R.c(cmul(R, r0[..., (k + 1) % 3], r1[..., (k + 2) % 3])
                         - cmul(R, r0[..., (k + 2) % 3], r1[..., (k + 1) % 3])) for k in range(3)], axis=-1)
    return np.concatenate([A2[..., :2, :], np.conj(row2)[..., None, :]], axis=-2)


def stored(R, A, fmt):
    """A as the FP32 storage format holds it: every entry rounded (FP32-18,
    fmt 1), or rows 0 and 1 rounded and row 2 rebuilt (FP32-12, fmt 2)"""
    if fmt == 1:
        return R.c(A)
    return with_row2(R, R.c(A[..., :2, :]))


def su2_steps(R, K, omega, sr, G0=None):
    """G = R3 R2 R1 G0 (G0 = 1 by default) from the three subgroup steps on
    W = K (Eq. (9); OR r = N[(1 - omega) + omega b], SR r = b^2 where
    sr[:, k]), each R applied to G and W in turn"""
    n = K.shape[0]
    W = K.copy()
    G = np.broadcast_to(np.eye(3, dtype=np.complex128), (n, 3, 3)).copy() if G0 is None else G0.copy()
    for k, (i, j) in enumerate(SUBGROUPS):
        a0 = R(W[:, i, i].real + W[:, j, j].real)
        a3 = R(W[:, i, i].imag - W[:, j, j].imag)
        a1 = R(W[:, i, j].imag + W[:, j, i].imag)
        a2 = R(W[:, i, j].real - W[:, j, i].real)
        n2 = R(R(R(R(a0 * a0) + R(a1 * a1)) + R(a2 * a2)) + R(a3 * a3))
        ok = n2 > 0
        inv = np.where(ok, R(1.0 / R(np.sqrt(np.where(ok, n2, 1.0)))), 0.0)
        b = [R(a0 * inv), R(-a1 * inv), R(-a2 * inv), R(-a3 * inv)]
        sq = R(b[0] * b[0] - R(R(R(b[1] * b[1]) + R(b[2] * b[2])) + R(b[3] * b[3])))
        bs = [sq, R(2 * b[0] * b[1]), R(2 * b[0] * b[2]), R(2 * b[0] * b[3])]
        if omega != 1.0:
            c = [R(R(1.0 - omega) + R(omega * b[0])), R(omega * b[1]), R(omega * b[2]), R(omega * b[3])]
            ic = R(1.0 / R(np.sqrt(R(R(R(R(c[0] * c[0]) + R(c[1] * c[1])) + R(c[2] * c[2])) + R(c[3] * c[3])))))
            bo = [R(x * ic) for x in c]
        else:
            bo = b
        r = [np.where(sr[:, k], bs[m], bo[m]) for m in range(4)]
        r = [np.where(ok, r[0], 1.0)] + [np.where(ok, r[m], 0.0) for m in (1, 2, 3)]
        s00, s01 = r[0] + 1j * r[3], r[2] + 1j * r[1]
        s10, s11 = -r[2] + 1j * r[1], r[0] - 1j * r[3]
        for M in ((G, W) if k < 2 else (G,)):
            mi, mj = M[:, i, :].copy(), M[:, j, :].copy()
            M[:, i, :] = R.c(cmul(R, s00[:, None], mi) + cmul(R, s01[:, None], mj))
            M[:, j, :] = R.c(cmul(R, s10[:, None], mi) + cmul(R, s11[:, None], mj))
    return G


def link_update(R, links8, omega, sr, fmt, mu_first=0):
    """The link-rewriting update of a stack of sites (n, 8, 3, 3): forward
    links then backward links as the sweep reads them; returns them updated
    and read back in format fmt (1 FP32-18, 2 FP32-12)."""
    K = np.zeros(links8.shape[:1] + (3, 3), np.complex128)
    for mu in range(mu_first, 4):
        K = R.c(K + links8[:, mu])
        K = R.c(K + dag(links8[:, 4 + mu]))
    G = su2_steps(R, K, omega, sr)
    rows = 3 if fmt == 1 else 2
    out = np.empty_like(links8)
    for mu in range(4):
        f = matmul(R, G, links8[:, mu], rows)
        b = matmul(R, links8[:, 4 + mu], dag(G), rows)
        out[:, mu] = f if rows == 3 else with_row2(R, f)
        out[:, 4 + mu] = b if rows == 3 else with_row2(R, b)
    return out


def reunitarize(A):
    """Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1) (FP64)"""
    r0 = A[..., 0, :] / np.linalg.norm(A[..., 0, :], axis=-1, keepdims=True)
    r1 = A[..., 1, :] - np.sum(np.conj(r0) * A[..., 1, :], axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    return np.stack([r0, r1, np.conj(np.cross(r0, r1))], axis=-2)


def fixed_update(R, u_f, g_f, u_b, g_b, g_x, omega, sr, fmt=2, mu_first=0):
    """The fixed-link update in FP32 of a stack of sites: u_f, g_f the 4
    forward links and the g at x+mu, u_b, g_b the 4 backward links and the g
    at x-mu, g_x the site's own g, all (n, 4 or -, 3, 3) as held in format
    fmt (FP32-12: rows 0 and 1 meaningful, products on rows 0 and 1 with row 2
    rebuilt; FP32-18: full products).  Lanes: directions mu and mu+2 are
    summed on two lanes, then added.  Returns the new g(x), reunitarized in
    FP64 and rounded to the format."""
    n = u_f.shape[0]
    full = (fmt == 1)
    rows = 3 if full else 2
    own = (lambda A: A) if full else (lambda A: with_row2(R, A[..., :2, :]))
    fin = (lambda A: A) if full else (lambda A: with_row2(R, A))
    lane = [np.zeros((n, 3, 3), np.complex128) for _ in range(2)]
    for mu in range(mu_first, 4):
        y = own(g_f[:, mu])
        p = fin(matmul(R, u_f[:, mu], dag(y), rows))
        lane[mu % 2] = R.c(lane[mu % 2] + p)
        ub = own(u_b[:, mu])
        p = fin(matmul(R, g_b[:, mu], ub, rows))
        lane[mu % 2] = R.c(lane[mu % 2] + dag(p))
    M = R.c(lane[0] + lane[1])
    G0 = own(g_x)
    K = matmul(R, G0, M)
    G = su2_steps(R, K, omega, sr, G0)
    return stored(R, reunitarize(G), fmt)


# ----------------------------------------------------------------- lattices

def neighbours(dims):
    """back[mu][s], fwd[mu][s]: the sites s -/+ mu (lexicographic, x fastest)"""
    V = int(np.prod(dims))
    coords = np.array(np.unravel_index(np.arange(V), dims))
    back, fwd = [], []
    for mu in range(4):
        for step, out in ((-1, back), (1, fwd)):
            c = coords.copy()
            c[mu] = (c[mu] + step) % dims[mu]
            out.append(np.ravel_multi_index(tuple(c), dims))
    return back, fwd, coords.sum(axis=0) % 2


def link_sweep(dims, U, omega, sr_of, fmt, R, parities=(0, 1), mu_first=0, active=None):
    """Half-sweeps of the link-rewriting form on U (V, 4, 3, 3) as the GPU
    holds it; sr_of(sites) -> (n, 3) bool; active: per-site flags (Coulomb
    masks)."""
    back, _, par = neighbours(dims)
    W = U.copy()
    for p in parities:
        sites = np.nonzero((par == p) & (True if active is None else active))[0]
        L = np.concatenate([W[sites][:, :4]] + [W[back[mu][sites], mu][:, None] for mu in range(4)], axis=1)
        out = link_update(R, L, omega, sr_of(sites), fmt, mu_first)
        W[sites, :4] = out[:, :4]
        for mu in range(4):
            W[back[mu][sites], mu] = out[:, 4 + mu]
    return W


def fixed_sweep(dims, U, omega, sr_of, R, fmt=2, mu_first=0):
    """One full sweep of the fixed-link form (FP32 sweeps in format fmt of the
    FP64 links U, g from 1), the links handed back as g U g^dag in FP64"""
    back, fwd, par = neighbours(dims)
    V = U.shape[0]
    U32 = stored(R, U, fmt)
    g = np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 3, 3)).copy()
    for p in (0, 1):
        s = np.nonzero(par == p)[0]
        u_f = U32[s]
        g_f = np.stack([g[fwd[mu][s]] for mu in range(4)], axis=1)
        u_b = np.stack([U32[back[mu][s], mu] for mu in range(4)], axis=1)
        g_b = np.stack([g[back[mu][s]] for mu in range(4)], axis=1)
        g[s] = fixed_update(R, u_f, g_f, u_b, g_b, g[s], omega, sr_of(s), fmt, mu_first)
    gr = reunitarize(g)
    out = np.empty_like(U)
    for mu in range(4):
        out[:, mu] = gr @ U[:, mu] @ dag(gr[fwd[mu]])
    return out


def sr_of(orc, seed, sweep, p, instance=0):
    """per-site stochastic-relaxation decisions, (n, 3) bool, from the
    oracle's Philox stream (all False for p = 0)"""
    def f(sites):
        if p <= 0:
            return np.zeros((len(sites), 3), dtype=bool)
        return np.array([orc.sr_decisions(seed, int(s), sweep, instance, p) for s in sites], dtype=bool)
    return f


def held(R, U0, fmt):
    """the field a load of U0 (already rounded to fmt on the host) holds on
    the GPU: FP32-12 rebuilds row 2 itself"""
    return with_row2(R, U0[..., :2, :]) if fmt == 2 else U0


def link_sweep_envelope(orc, dims, U0, fmt, ref, omega, p=0.0, seed=0, sweep=0, instance=0, parities=(0, 1),
                        mu_first=0, active=None, n=16):
    """per-link envelope of the link-rewriting half-sweeps `parities` of the
    field U0 as stored in fmt, against ref"""
    srf = sr_of(orc, seed, sweep, p, instance)
    return envelope(lambda R: link_sweep(dims, held(R, U0, fmt), omega, srf, fmt, R, parities, mu_first, active),
                    ref, n=n)


def fixed_sweep_envelope(orc, dims, U, fmt, ref, omega, p=0.0, seed=0, sweep=0, mu_first=0, n=16):
    """per-link envelope of one fixed-link sweep in FP32 format fmt of the
    FP64 links U, against ref"""
    srf = sr_of(orc, seed, sweep, p)
    return envelope(lambda R: fixed_sweep(dims, U, omega, srf, R, fmt, mu_first), ref, n=n)


def link_errs(A, B):
    d = np.linalg.norm((A - B).reshape(-1, 9), axis=1)
    return d / np.linalg.norm(B.reshape(-1, 9), axis=1)


def envelope(run, ref, n=16, seed=0):
    """largest per-link relative error of n randomised-rounding runs of
    run(R) against ref"""
    rng = np.random.default_rng(seed)
    return np.max([link_errs(run(Rounding(rng)), ref) for _ in range(n)], axis=0)


def fp32_bar_ok(got, ref, env):
    """the FP32 bar: 2e-6 relative on 99 % of the links, and on every link at
    most twice its envelope plus u"""
    e = link_errs(got, ref)
    bad = np.nonzero(e > 2.0 * env + U32)[0]
    return (float(np.quantile(e, 0.99)) <= 2e-6 and bad.size == 0,
            {"q99": float(np.quantile(e, 0.99)), "max": float(e.max()),
             "worst_ratio": float(np.max(e / (2.0 * env + U32)))})
