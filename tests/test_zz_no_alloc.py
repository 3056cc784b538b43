"""The allocation-free measurement (lgf_measure_noalloc) through the C ABI:
its F and theta, written to device memory, are the bits lgf_measure returns,
on two calls in a row (the second on a smaller lattice, so the partial sums
of the first are still in the library's scratch array), and lattices beyond
its limit are refused before any GPU work."""
from __future__ import annotations

import ctypes
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


def test_measure_noalloc_equals_measure(lgf, orc):
    import torch
    lib = lgf.load_library()
    stream = torch.cuda.current_stream()
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    cases = [((8, 8, 8, 12), lgf.LGF_FP64_18, 31), ((4, 4, 6, 8), lgf.LGF_FP32_12, 32),
             ((2, 2, 2, 2), lgf.LGF_FP64_12, 33)]
    for dims, fmt, seed in cases:
        print("[gpu-case] measure_noalloc", dims, fmt, flush=True)
        sys.stdout.flush()
        with lgf.Lattice(dims, fmt, stream=stream) as lat:
            lat.generate(seed, 0.3, True)
            F, th = lat.measure()
            out.fill_(float("nan"))
            assert lib.lgf_measure_noalloc(lat.h, ctypes.c_void_p(out.data_ptr())) == lgf.LGF_OK
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            assert got[0] == F and got[1] == th, (got, F, th)
            if fmt == lgf.LGF_FP64_18:
                F_ref, th_ref = orc.measure(dims, lat.store())
                assert abs(F - F_ref) <= 1e-14 and abs(th - th_ref) <= 1e-12 * th_ref


def test_measure_noalloc_rejects_what_does_not_fit(lgf):
    import torch
    lib = lgf.load_library()
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    assert lib.lgf_measure_noalloc(None, ctypes.c_void_p(out.data_ptr())) == lgf.LGF_EINVAL
    # 2^26 + 2^21 sites (FP32-12, 13 GB): beyond the 2^26 sites of the scratch array
    dims = (66, 64, 64, 64 * 4)
    assert int(np.prod(dims)) > 1 << 26
    with lgf.Lattice(dims, lgf.LGF_FP32_12) as lat:
        assert lib.lgf_measure_noalloc(lat.h, ctypes.c_void_p(out.data_ptr())) == lgf.LGF_EINVAL
        assert "2^26" in lgf.lgf_last_error()
        assert lib.lgf_measure_noalloc(lat.h, None) == lgf.LGF_EINVAL
    # the largest lattice it serves: 2^26 sites exactly
    dims = (64, 64, 64, 256)
    with lgf.Lattice(dims, lgf.LGF_FP32_12) as lat:
        lat.generate(3, 0.3, True)
        F, th = lat.measure()
        assert lib.lgf_measure_noalloc(lat.h, ctypes.c_void_p(out.data_ptr())) == lgf.LGF_OK
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert got[0] == F and got[1] == th
