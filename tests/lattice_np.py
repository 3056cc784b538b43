"""Small numpy helpers the tests use to check the oracle and the HIP library
from outside: lattice reshapes, K(x), unitarity, Gell-Mann matrices, random
SU(2)/SU(3) elements.  Nothing here is called by either implementation."""
from __future__ import annotations

import numpy as np

SQ3 = np.sqrt(3.0)

# Gell-Mann matrices, tr(l_a l_b) = 2 delta_ab
GELLMANN = np.zeros((8, 3, 3), dtype=np.complex128)
GELLMANN[0][0, 1] = GELLMANN[0][1, 0] = 1
GELLMANN[1][0, 1] = -1j
GELLMANN[1][1, 0] = 1j
GELLMANN[2][0, 0] = 1
GELLMANN[2][1, 1] = -1
GELLMANN[3][0, 2] = GELLMANN[3][2, 0] = 1
GELLMANN[4][0, 2] = -1j
GELLMANN[4][2, 0] = 1j
GELLMANN[5][1, 2] = GELLMANN[5][2, 1] = 1
GELLMANN[6][1, 2] = -1j
GELLMANN[6][2, 1] = 1j
GELLMANN[7] = np.diag([1, 1, -2]) / SQ3

PAULI = np.array([[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]], dtype=np.complex128)


def dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def as_grid(dims, U):
    """(V, 4, 3, 3) -> (Lt, Lz, Ly, Lx, 4, 3, 3) view"""
    return U.reshape(*dims, 4, 3, 3)


def backward(dims, U, mu):
    """U_mu(x - mu) for every x, as a (Lt, Lz, Ly, Lx, 3, 3) array"""
    G = as_grid(dims, U)
    return np.roll(G[..., mu, :, :], 1, axis=mu)


def K_field(dims, U):
    """K(x) = sum_mu U_mu(x) + U_mu(x - mu)^dag on every site"""
    G = as_grid(dims, U)
    K = np.zeros(tuple(dims) + (3, 3), dtype=np.complex128)
    for mu in range(4):
        K += G[..., mu, :, :] + dag(backward(dims, U, mu))
    return K


def unitarity_error(U):
    M = U.reshape(-1, 3, 3)
    e1 = np.abs(M @ dag(M) - np.eye(3)).max()
    e2 = np.abs(np.linalg.det(M) - 1.0).max()
    return max(e1, e2)


def parity_grid(dims):
    t, z, y, x = np.meshgrid(*[np.arange(L) for L in dims], indexing="ij")
    return (t + z + y + x) % 2


def random_su2(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def quat_matrix(q):
    """s(q) = q0 + i q.sigma as 2x2 matrices, q of shape (..., 4)"""
    q = np.asarray(q)
    m = np.zeros(q.shape[:-1] + (2, 2), dtype=np.complex128)
    m[..., 0, 0] = q[..., 0] + 1j * q[..., 3]
    m[..., 0, 1] = q[..., 2] + 1j * q[..., 1]
    m[..., 1, 0] = -q[..., 2] + 1j * q[..., 1]
    m[..., 1, 1] = q[..., 0] - 1j * q[..., 3]
    return m


def random_su3(rng, n):
    Z = (rng.normal(size=(n, 3, 3)) + 1j * rng.normal(size=(n, 3, 3))) / np.sqrt(2)
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=1, axis2=2)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    return Q * (det ** (-1.0 / 3.0))[:, None, None]


def expm_hermitian(H, eps):
    """exp(i eps H) for Hermitian H via its eigendecomposition"""
    w, v = np.linalg.eigh(H)
    return (v * np.exp(1j * eps * w)[..., None, :]) @ dag(v)


def stored_as(U, fmt):
    """U as a field in storage format fmt holds it, computed on the host: the
    FP32 formats (1 FP32-18, 2 FP32-12) round every entry to single precision,
    the 12-real formats (2, 3 FP64-12) keep rows 0 and 1 and rebuild row 2 as
    conj(row0 x row1) in the storage precision; format 0 (FP64-18) is U."""
    W = U.astype(np.complex64) if fmt in (1, 2) else U.copy()
    if fmt in (2, 3):
        W[..., 2, :] = np.conj(np.cross(W[..., 0, :], W[..., 1, :]))
    return W.astype(np.complex128)


SPLIT_UNIT = 2.0 ** -40


def split_entry(x):
    """The split FP64 storage of one real array: hi = fl32(x) (nearest, ties
    to even) and q = round((x - hi) / 2^-40) clipped to +-32767; returns (hi
    as float32, q as int16)."""
    x = np.asarray(x, dtype=np.float64)
    hi = x.astype(np.float32)
    q = np.clip(np.rint((x - hi.astype(np.float64)) / SPLIT_UNIT), -32767, 32767).astype(np.int16)
    return hi, q


def split_stored(U):
    """Links as the split storage reads them back: every real entry of rows
    0 and 1 as hi + q 2^-40, row 2 rebuilt as conj(row0 x row1)."""
    U = np.asarray(U, dtype=np.complex128)
    out = U.copy()

    def back(x):
        hi, q = split_entry(x)
        return hi.astype(np.float64) + q.astype(np.float64) * SPLIT_UNIT

    r01 = U[..., :2, :]
    out[..., :2, :] = back(r01.real) + 1j * back(r01.imag)
    out[..., 2, :] = np.conj(np.cross(out[..., 0, :], out[..., 1, :]))
    return out
