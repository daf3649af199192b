"""The C-ABI library loads and exports every entry point include/gsr.h
declares, and the binding declares each of them (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsr.h")
LIB = os.path.join(ROOT, "paper_2512_08498_amd", "libgsr.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsr_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("gsr_create", "gsr_destroy", "gsr_plan", "gsr_render_forward", "gsr_render_backward",
                     "gsr_l1_loss", "gsr_adam_step", "gsr_render_backward_adam", "gsr_debug_binning",
                     "gsr_check", "gsr_required_capacity", "gsr_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgsr.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_declares_every_symbol():
    from paper_2512_08498_amd import _lib
    assert set(_lib.EXPORTED) == set(declared_functions())


def test_camera_struct_layout_matches_rows():
    import numpy as np
    from paper_2512_08498_amd import _lib, camera_rows
    from workloads import make_config
    _, cams = make_config(3, scale=0.0001)
    rows = camera_rows(cams)
    assert ctypes.sizeof(_lib.Camera) == 72 == rows.shape[1] * 4
    arr = (_lib.Camera * len(cams))()
    ctypes.memmove(arr, rows.ctypes.data, rows.nbytes)
    for c, a in zip(cams, arr):
        assert a.width == c.width and a.height == c.height
        assert np.allclose(list(a.R), np.asarray(c.R).reshape(-1)) and a.fx == np.float32(c.fx)


def test_binding_rejects_tensors_the_entry_points_would_misread():
    """The binding checks dtype, device, contiguity and size before handing a
    pointer to the C ABI, which cannot check them itself."""
    import torch

    from paper_2512_08498_amd.rasterizer import _check_flat, _check_param

    cpu = torch.device("cpu")
    ok = torch.zeros(12, dtype=torch.float32)
    _check_flat("x", ok, 12, cpu)
    _check_flat("x", ok.view(3, 4), 12, cpu)
    _check_param("x", ok.view(3, 4), (3, 4), cpu)
    for bad in (ok.double(), ok[:11], ok.view(3, 4).t(), torch.zeros(13)):
        with pytest.raises(ValueError):
            _check_flat("x", bad, 12, cpu)
    with pytest.raises(ValueError):
        _check_param("x", ok.view(4, 3), (3, 4), cpu)
