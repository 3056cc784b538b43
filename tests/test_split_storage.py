"""The split FP64 storage of read-only links (format LGF_FP64_12S) as the
tests define it: every real entry x of rows 0 and 1 held as hi = fl32(x) plus
a 16-bit q = round((x - hi) 2^40).  Checked here from its definition: the
entry read back is within 2^-40 of x for |x| <= 1, x - hi is exact in FP64,
and storing an entry already on that grid gives it back bit for bit (so a
parity test may hand the oracle and the library the same stored links)."""
from __future__ import annotations

import numpy as np

from lattice_np import SPLIT_UNIT, split_entry, split_stored, unitarity_error


def _cases():
    rng = np.random.default_rng(11)
    f = rng.uniform(0.5, 1.0, 20000).astype(np.float32).astype(np.float64)
    return np.concatenate([rng.uniform(-1, 1, 200000), rng.uniform(-1e-3, 1e-3, 20000),
                           f + 2.0 ** -25, f - 2.0 ** -25, f / 2 + 2.0 ** -26,   # exact ties
                           [0.0, 1.0, -1.0, 0.5, 2.0 ** -60, 1 - 2.0 ** -30]])


def test_split_entry_error_bound():
    x = _cases()
    hi, q = split_entry(x)
    back = hi.astype(np.float64) + q.astype(np.float64) * SPLIT_UNIT
    assert float(np.abs(back - x).max()) <= SPLIT_UNIT
    # below the clip the rounding of q alone: half a unit
    free = np.abs(q) < 32767
    assert float(np.abs(back - x)[free].max()) <= SPLIT_UNIT / 2
    # x - hi is exact in FP64 (hi is x rounded to 24 bits)
    d = x - hi.astype(np.float64)
    assert np.array_equal(hi.astype(np.float64) + d, x)


def test_split_entry_is_idempotent_on_its_grid():
    x = _cases()
    hi, q = split_entry(x)
    back = hi.astype(np.float64) + q.astype(np.float64) * SPLIT_UNIT
    hi2, q2 = split_entry(back)
    assert np.array_equal(hi2.astype(np.float64) + q2.astype(np.float64) * SPLIT_UNIT, back)


def test_split_stored_links(orc):
    """stored links stay within the bound of SU(3): unitary to ~1e-12, rows 0
    and 1 within 2^-40 per real entry of the input, and storing them again
    changes nothing."""
    U = orc.generate_links((4, 4, 4, 4), 3, 0.4)
    S = split_stored(U)
    assert float(np.abs((S - U)[..., :2, :].real).max()) <= SPLIT_UNIT
    assert float(np.abs((S - U)[..., :2, :].imag).max()) <= SPLIT_UNIT
    assert unitarity_error(S) < 1e-11
    assert np.array_equal(split_stored(S)[..., :2, :], S[..., :2, :])
