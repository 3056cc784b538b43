"""Checkpoint / resume and buffer ownership through the C ABI (GPU).

Resume: the random numbers of stochastic relaxation are keyed by (seed, site,
sweep counter), so a gauge fixing stopped after N sweeps, stored to the host,
loaded into a fresh handle and continued with the counter at N must end in
the same bits as 2N sweeps in one call.  Ownership: a handle on a borrowed
device buffer (a torch tensor) works in it and never frees it."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("kw", [dict(omega=1.0, p_sr=0.5, seed=13), dict(omega=1.7), dict(omega=1.8, use_graph=0)])
def test_resume_is_bitwise(lgf, orc, kw):
    """40 sweeps in one call = 20 sweeps, store, load into a new handle, 20
    more from sweep counter 20 (the checks every 20 sweeps fall on the same
    sweeps, so the reunitarizations match too)."""
    dims = (4, 4, 6, 10)
    announce("resume", kw)
    U = orc.generate_links(dims, 41, 0.3)
    common = dict(theta_target=1e-300, check_every=20, **kw)
    with lgf.Lattice(dims, 0) as lat:
        lat.load(U)
        st, res, hist = lat.gauge_fix(max_sweeps=40, **common)
        whole = lat.store()
    assert st == lgf.LGF_ENOTCONV and res["sweeps"] == 40
    with lgf.Lattice(dims, 0) as lat:
        lat.load(U)
        lat.gauge_fix(max_sweeps=20, **common)
        half = lat.store()
    with lgf.Lattice(dims, 0) as lat:
        lat.load(half)
        st2, res2, hist2 = lat.gauge_fix(max_sweeps=20, sweep_offset=20, **common)
        resumed = lat.store()
    assert np.array_equal(resumed, whole)
    assert res2["F"] == res["F"] and res2["theta"] == res["theta"]
    assert hist2[-1, 1] == hist[-1, 1] and hist2[-1, 2] == hist[-1, 2]


def test_borrowed_buffer_is_used_and_never_freed(lgf, orc):
    import torch
    dims = (4, 4, 6, 8)
    announce("borrowed buffer", dims)
    U = orc.generate_links(dims, 43, 0.3)
    n = lgf.lgf_required_bytes(dims, lgf.LGF_FP64_18)
    buf = torch.zeros(n, dtype=torch.uint8, device="cuda")
    with lgf.Lattice(dims, lgf.LGF_FP64_18, device_buf=buf) as lat:
        lat.load(U)
        lat.sweep(2, 1.7)
        swept = lat.store()
    torch.cuda.synchronize()
    # the handle is gone, the tensor still holds the field the sweep wrote
    assert int(buf.count_nonzero()) > 0
    with lgf.Lattice(dims, lgf.LGF_FP64_18, device_buf=buf) as lat:
        assert np.array_equal(lat.store(), swept)
    ref = U.copy()
    orc.sweep(dims, ref, 1.7)
    assert float(np.abs(swept - ref).max()) <= 1e-12
    # a buffer one byte short is refused before anything is written
    small = torch.zeros(n - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(lgf.LgfError) as e:
        lgf.lgf_create(dims, lgf.LGF_FP64_18, None, small)
    assert e.value.status == lgf.LGF_EINVAL
    assert int(small.count_nonzero()) == 0
