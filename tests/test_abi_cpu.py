"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/lego_raster.h declares, and its host-only calls
behave as documented."""
import ctypes as C
import os
import re

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lego_raster.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lgs_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lgs_forward", "lgs_backward", "lgs_graph_create", "lgs_graph_launch",
                 "lgs_autotune", "lgs_context_create"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2511_16144_amd as P
    lib = P.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(P.EXPORTS)


def test_default_settings_and_status_strings():
    import paper_2511_16144_amd as P
    lib = P.lib()
    s = lib.lgs_default_settings()
    assert (s.tile, s.chunk) == (16, 4)
    assert abs(s.alpha_min - 1 / 255) < 1e-9 and s.alpha_max == pytest.approx(0.99)
    assert s.T_eps == pytest.approx(1e-4) and s.cutoff2 == 9.0 and s.z_near == pytest.approx(0.2)
    for code, name in enumerate(["LGS_OK", "LGS_ERR_INVALID_ARG", "LGS_ERR_HIP", "LGS_ERR_CAPACITY",
                                 "LGS_ERR_UNSUPPORTED", "LGS_ERR_STATE"]):
        assert lib.lgs_status_string(code).decode() == name


def test_null_arguments_are_rejected_without_touching_the_device():
    import paper_2511_16144_amd as P
    lib = P.lib()
    assert lib.lgs_context_create(0, None) == P.binding.LGS_ERR_INVALID_ARG
    assert lib.lgs_forward(None, None, None, 1, None, None, None, None) == P.binding.LGS_ERR_INVALID_ARG
    assert lib.lgs_backward(None, None, None, None, None, None) == P.binding.LGS_ERR_INVALID_ARG
    assert lib.lgs_last_error(None).decode() == "NULL context"


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-GPU error path")
def test_context_create_without_gpu_reports_hip_error():
    import paper_2511_16144_amd as P
    h = C.c_void_p()
    assert P.lib().lgs_context_create(0, C.byref(h)) == P.binding.LGS_ERR_HIP
