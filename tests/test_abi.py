"""Host-side checks of the C ABI: the library loads, exports every symbol
include/lbk.h declares, and rejects bad descriptions without a GPU."""
import ctypes
import os
import re

import pytest

from paper_1411_7051_amd import _lib
from paper_1411_7051_amd.lattice import make_desc, workspace_bytes

HEADER = os.path.join(os.path.dirname(__file__), "..", "include", "lbk.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbk3?_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared() == sorted(_lib.symbols())


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in declared():
        assert hasattr(lib, name), name


def test_desc_struct_layout():
    # 8 int32, 9 doubles, 3 int32: 32 + 72 + 12 bytes, 4 of tail padding
    assert ctypes.sizeof(_lib.Desc) == 120
    assert _lib.Desc.slip_b.offset == 96 and _lib.Desc.correlation.offset == 104
    assert _lib.Desc.band.offset == 112


def test_workspace_size_scales_with_lattice():
    small = workspace_bytes(make_desc(64, 32))
    big = workspace_bytes(make_desc(128, 64))
    assert big > 3 * small
    f16 = workspace_bytes(make_desc(1024, 512, storage="f16"))
    f32 = workspace_bytes(make_desc(1024, 512, storage="f32"))
    assert f16 < f32


@pytest.mark.parametrize("kw,msg", [
    (dict(tau=0.5), "tau"),
    (dict(tau=float("nan")), "tau"),
    (dict(bc_x=3), "bc_x"),
    (dict(bc_y=2), "bc_y"),
    (dict(storage=7), "storage"),
    (dict(bc_x=2, rho_in=-1.0), "rho_in"),
    (dict(init=1, rho_out=0.0), "rho_in"),
    (dict(init=5), "init"),
    (dict(rho_ref=0.0), "rho_ref"),
    (dict(check_every=-1), "check_every"),
    (dict(f_eps=-1.0), "f_eps"),
    (dict(correlation=3), "correlation"),
    (dict(slip_b=0.5), "slip_b"),
    (dict(pass_mode=4), "pass_mode"),
    (dict(pass_mode=-1), "pass_mode"),
    (dict(band=-1), "band"),
    (dict(band=1025), "band"),
])
def test_invalid_descriptions_rejected(kw, msg):
    d = make_desc(16, 8, **kw)
    with pytest.raises(_lib.LbkError) as e:
        workspace_bytes(d)
    assert e.value.status == -1 and msg in str(e.value)


@pytest.mark.parametrize("nx,ny", [(0, 8), (8, 0), (0, 0), (-3, 4)])
def test_empty_lattice_rejected(nx, ny):
    with pytest.raises(_lib.LbkError) as e:
        workspace_bytes(make_desc(nx, ny))
    assert e.value.status == -1 and "nx, ny" in str(e.value)


def test_empty_lattice3_rejected():
    from paper_1411_7051_amd.lattice3 import make_desc3, workspace_bytes3
    for n in [(0, 4, 4), (4, 0, 4), (4, 4, 0)]:
        with pytest.raises(_lib.LbkError) as e:
            workspace_bytes3(make_desc3(*n))
        assert e.value.status == -1


def test_pressure_needs_three_columns():
    with pytest.raises(_lib.LbkError):
        workspace_bytes(make_desc(2, 8, bc_x=2))


def test_too_large_rejected():
    with pytest.raises(_lib.LbkError) as e:
        workspace_bytes(make_desc(65536, 65536))
    assert e.value.status == -5


def test_size_limit_is_exact():
    """2^30 padded nodes is the largest lattice: 32768 x 32768 (and any nx
    whose pitch is 32768) is accepted, one more row is not; FP32 needs
    about 108 GB of workspace there."""
    n = workspace_bytes(make_desc(32768, 32768))
    assert 100e9 < n < 112e9
    workspace_bytes(make_desc(32705, 32768))  # pitch 32768
    for nx, ny in [(32768, 32769), (32769, 32768)]:
        with pytest.raises(_lib.LbkError) as e:
            workspace_bytes(make_desc(nx, ny))
        assert e.value.status == -5


def test_size_limit_3d():
    from paper_1411_7051_amd.lattice3 import make_desc3, workspace_bytes3
    workspace_bytes3(make_desc3(1024, 1024, 1024))  # 2^30 nodes
    for n in [(1024, 1024, 1025), (64, 4096, 4097)]:
        with pytest.raises(_lib.LbkError) as e:
            workspace_bytes3(make_desc3(*n))
        assert e.value.status == -5


def test_row_width_limit():
    """Kernels address each row block with 32-bit buffer offsets, so a row's
    widest form (FP32 state, 40 B per node in 2-D, 80 B in 3-D) must stay
    under 4 GiB: the widest accepted rows are 107,374,144 and 53,687,040
    nodes (pitch a multiple of 64), whatever the storage type."""
    from paper_1411_7051_amd.lattice3 import make_desc3, workspace_bytes3
    for storage in ("f32", "f16"):
        workspace_bytes(make_desc(107374144, 1, storage=storage))
        with pytest.raises(_lib.LbkError) as e:
            workspace_bytes(make_desc(107374145, 1, storage=storage))
        assert e.value.status == -5
        workspace_bytes3(make_desc3(53687040, 1, 1, storage=storage))
        with pytest.raises(_lib.LbkError) as e:
            workspace_bytes3(make_desc3(53687041, 1, 1, storage=storage))
        assert e.value.status == -5


def test_null_arguments_rejected():
    lib = _lib.load()
    assert lib.lbk_step(None, 1) == -1
    assert lib.lbk_destroy(None) == 0
    out = ctypes.c_void_p()
    d = make_desc(16, 8)
    # missing fields are rejected before any device work
    assert lib.lbk_create(ctypes.byref(d), None, None, None, None, 0, None,
                          ctypes.byref(out)) == -1
    assert out.value is None
    assert b"eps and k" in lib.lbk_last_error()


def test_create_without_gpu_reports_device_error():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import numpy as np
    lib = _lib.load()
    d = make_desc(16, 8)
    n = workspace_bytes(d)
    buf = np.zeros(n + 256, dtype=np.uint8)
    base = buf.ctypes.data
    ws = (base + 255) // 256 * 256
    f = np.ones((8, 16), dtype=np.float32)
    out = ctypes.c_void_p()
    st = lib.lbk_create(ctypes.byref(d), f.ctypes.data, f.ctypes.data, None, ws, n, None,
                        ctypes.byref(out))
    assert st == -2 and out.value is None


def test_batch_null_arguments_rejected():
    lib = _lib.load()
    out = ctypes.c_void_p()
    n = ctypes.c_size_t()
    assert lib.lbk_batch_workspace_size(None, 1, ctypes.byref(n)) == -1
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.lbk_batch_workspace_size(arr, 1, ctypes.byref(n)) == -1
    assert b"lats[0] is NULL" in lib.lbk_last_error()
    assert lib.lbk_batch_workspace_size(arr, 0, ctypes.byref(n)) == -1
    assert lib.lbk_batch_create(arr, 1, None, 0, ctypes.byref(out)) == -1
    assert out.value is None
    assert lib.lbk_batch_step(None, 1) == -1
    assert lib.lbk_batch_set_launch(None, 256, 1, 0, 0) == -1
    assert lib.lbk_batch_autotune(None, 1, None) == -1
    assert lib.lbk_batch_apparent_permeability(None, None) == -1
    assert lib.lbk_batch_check(None) == -1
    assert lib.lbk_batch_destroy(None) == 0


def test_batch_gradient_null_arguments_rejected():
    lib = _lib.load()
    n = ctypes.c_size_t()
    h = ctypes.c_int64()
    assert lib.lbk_batch_adjoint_workspace_size(None, 10, 5, 5, ctypes.byref(n)) == -1
    assert lib.lbk_batch_adjoint_plan(None, 10, 5, 1 << 30, ctypes.byref(h), None) == -1
    J = ctypes.c_double()
    assert lib.lbk_batch_adjoint_forward(None, 0, 10, 5, 5, None, 0, ctypes.byref(J)) == -1
    assert lib.lbk_batch_adjoint_backward(None, None, 0, None, None) == -1
    assert lib.lbk_adjoint_plan(None, 10, 5, 1 << 30, ctypes.byref(h), None) == -1
