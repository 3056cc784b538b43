"""The C-ABI library loads, exports every symbol include/lgf.h declares, and
validates arguments on the host before touching a GPU (CPU only)."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lgf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lgf_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lgf():
    import paper_1305_3440_amd as pkg
    pkg.load_library()
    return pkg


def test_library_exports_every_declared_symbol(lgf):
    names = declared_functions()
    assert len(names) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", lgf.lgf.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = lgf.load_library()
    for n in names:
        assert hasattr(lib, n)
    assert sorted(lgf.lgf.EXPORTS) == names


def test_struct_layouts_match_header(lgf):
    """The ctypes mirrors have the C structs' sizes (checked by compiling a
    probe against the header)."""
    src = ('#include "lgf.h"\n#include <stdio.h>\n#include <stddef.h>\nint main(void){'
           'printf("%zu %zu %zu %zu\\n", sizeof(lgf_fix_params), sizeof(lgf_fix_result),'
           ' sizeof(lgf_sweep_tuning), offsetof(lgf_sweep_tuning, schedule));return 0;}\n')
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        a, b, c, d = (int(x) for x in subprocess.run([exe], capture_output=True, text=True,
                                                     check=True).stdout.split())
    assert ctypes.sizeof(lgf.lgf_fix_params) == a
    assert ctypes.sizeof(lgf.lgf_fix_result) == b
    assert ctypes.sizeof(lgf.lgf_sweep_tuning) == c
    assert lgf.lgf_sweep_tuning.schedule.offset == d


def test_required_bytes(lgf):
    V = 8 * 8 * 8 * 8
    assert lgf.lgf_required_bytes((8, 8, 8, 8), lgf.LGF_FP64_18) == V * 4 * 144
    assert lgf.lgf_required_bytes((8, 8, 8, 8), lgf.LGF_FP32_18) == V * 4 * 72
    assert lgf.lgf_required_bytes((8, 8, 8, 8), lgf.LGF_FP32_12) == V * 4 * 48
    assert lgf.lgf_required_bytes((8, 8, 8, 8), lgf.LGF_FP64_12) == V * 4 * 96
    assert lgf.lgf_required_bytes((64, 64, 64, 64), lgf.LGF_FP64_18) == 9663676416
    assert lgf.lgf_required_bytes((8, 8, 8, 7), lgf.LGF_FP64_18) == 0
    assert lgf.lgf_required_bytes((8, 8, 8, 8), 9) == 0


@pytest.mark.parametrize("dims", [(8, 8, 8, 7), (0, 8, 8, 8), (8, 8, 8, -2), (2, 2, 2, 1),
                                  (65536, 65536, 2, 2)])
def test_create_rejects_bad_dims_without_gpu(lgf, dims):
    with pytest.raises(lgf.LgfError) as e:
        lgf.lgf_create(dims, lgf.LGF_FP64_18)
    assert e.value.status == lgf.LGF_EINVAL
    assert "even" in lgf.lgf_last_error()


def test_format_codes_match_header(lgf):
    """The binding's format constants are the header's enum values; the split
    FP64 sweep format of the fixed-link form is no storage format."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef enum \{([^}]*)\} lgf_format;", text).group(1)
    enum = {k: int(v) for k, v in re.findall(r"(LGF_FP\w+)\s*=\s*(\d+)", body)}
    assert enum == {k: getattr(lgf, k) for k in enum}
    assert set(enum) == {"LGF_FP64_18", "LGF_FP32_18", "LGF_FP32_12", "LGF_FP64_12", "LGF_FP64_12S"}
    assert lgf.lgf_required_bytes((8, 8, 8, 8), lgf.LGF_FP64_12S) == 0
    with pytest.raises(lgf.LgfError) as e:
        lgf.lgf_create((4, 4, 4, 4), lgf.LGF_FP64_12S)
    assert e.value.status == lgf.LGF_EINVAL


def test_create_rejects_bad_format_and_small_buffer(lgf):
    with pytest.raises(lgf.LgfError) as e:
        lgf.lgf_create((4, 4, 4, 4), 7)
    assert e.value.status == lgf.LGF_EINVAL
    with pytest.raises(lgf.LgfError) as e:
        lgf.lgf_create((4, 4, 4, 4), lgf.LGF_FP64_18, device_buf=0x1000, buf_bytes=100)
    assert e.value.status == lgf.LGF_EINVAL


def test_null_handles(lgf):
    lib = lgf.load_library()
    assert lib.lgf_destroy(None) == lgf.LGF_OK
    assert lib.lgf_sweep(None, 0, 1.5, 0.0, 0, 0) == lgf.LGF_EINVAL
    assert lib.lgf_measure(None, None, None) == lgf.LGF_EINVAL
    assert lib.lgf_create(None, 0, None, None, 0, None) == lgf.LGF_EINVAL
    assert lib.lgf_gauge_fix(None, None, None, None, 0) == lgf.LGF_EINVAL


def test_copy_bandwidth_rejects_bad_arguments_without_gpu(lgf):
    import ctypes
    lib = lgf.load_library()
    out = ctypes.c_double()
    assert lib.lgf_copy_bandwidth(0, 1, None, ctypes.byref(out)) == lgf.LGF_EINVAL
    assert lib.lgf_copy_bandwidth(17, 1, None, ctypes.byref(out)) == lgf.LGF_EINVAL
    assert lib.lgf_copy_bandwidth(1 << 20, 0, None, ctypes.byref(out)) == lgf.LGF_EINVAL
    assert lib.lgf_copy_bandwidth(1 << 20, 1, None, None) == lgf.LGF_EINVAL


def test_ensemble_tuning_null_and_bad_args_without_gpu(lgf):
    lib = lgf.lgf._ens_lib()
    assert lib.lgf_ensemble_set_tuning(None, 128, 1, 1) == lgf.LGF_EINVAL
    assert lib.lgf_ensemble_get_tuning(None, None, None, None) == lgf.LGF_EINVAL
    assert lib.lgf_ensemble_autotune(None, 0, 1) == lgf.LGF_EINVAL
    assert lib.lgf_set_tuning(None, 0, None) == lgf.LGF_EINVAL
    assert lib.lgf_get_tuning(None, 0, None) == lgf.LGF_EINVAL


def test_fix_params_default(lgf):
    p = lgf.lgf_fix_params_default()
    assert p.omega == 1.7 and p.p_sr == 0.0 and p.theta_target == 1e-14
    assert p.check_every == 20 and p.max_sweeps == 100000 and p.bulk_format == -1
    assert p.use_graph == 1 and p.theta_switch == 0.0 and p.finish_format == -1
    assert p.accumulate_g == 0


def test_binding_holds_no_arithmetic():
    """The Python binding only marshals arguments: no numpy arithmetic on links."""
    src = open(os.path.join(ROOT, "paper_1305_3440_amd", "lgf.py")).read()
    for forbidden in ("np.linalg", "np.einsum", "@ ", "np.exp", "import oracle", "from oracle"):
        assert forbidden not in src, forbidden


def test_fix_params_rejects_unknown_fields(lgf):
    p = lgf.fix_params(omega=1.5, separate_measure=1)
    assert p.omega == 1.5 and p.separate_measure == 1 and p.check_every == 20
    with pytest.raises(TypeError):
        lgf.fix_params(omgea=1.5)


def _abi_client():
    exe = os.path.join(ROOT, "tests", "abi_client")
    if not os.path.exists(exe):
        import __graft_entry__
        __graft_entry__.build_abi_client()
    return exe


def test_c_program_links_through_the_header(lgf):
    """A C program built against include/lgf.h alone links liblgf.so and gets
    the documented status codes for bad arguments (no GPU needed)."""
    out = subprocess.run([_abi_client(), "check"], capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "check ok"
    libs = subprocess.run(["ldd", _abi_client()], capture_output=True, text=True, check=True).stdout
    assert "liblgf.so" in libs


@pytest.mark.gpu
def test_c_program_sweep_matches_oracle(lgf, orc, tmp_path):
    """create / load / sweep / measure / store / destroy from C: the links
    after one full sweep and their F, theta match the oracle (1e-12)."""
    from conftest import gpu_available
    if not gpu_available():
        pytest.skip("no GPU visible")
    dims = (4, 4, 6, 8)
    U = orc.generate_links(dims, 21, 0.3, True)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    U.tofile(fin)
    print("[gpu-case] abi_client run", dims, flush=True)
    out = subprocess.run([_abi_client(), "run", *map(str, dims), "1.7", str(fin), str(fout)],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    F, theta = (float(x) for x in out.stdout.split())
    got = np.fromfile(fout, dtype=np.complex128).reshape(U.shape)
    ref = U.copy()
    orc.sweep(dims, ref, 1.7)
    F_ref, th_ref = orc.measure(dims, ref)
    assert float(np.abs(got - ref).max()) <= 1e-12
    assert abs(F - F_ref) <= 1e-13 and abs(theta - th_ref) <= 1e-12 * th_ref
