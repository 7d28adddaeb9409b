"""The C-ABI library loads and exports every entry point include/mpmlite.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpmlite.h")
LIB = os.path.join(ROOT, "paper_2602_07853_amd", "libmpmlite.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"(?:mpl_status|void|const char\s*\*)\s+(mpl_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for required in ("mpl_create", "mpl_destroy", "mpl_step", "mpl_unload", "mpl_reconstruct_stretch",
                     "mpl_energy_grad", "mpl_build_tangent", "mpl_hv", "mpl_pcg", "mpl_solve",
                     "mpl_load", "mpl_last_error", "mpl_export_field", "mpl_precond_param_count",
                     "mpl_precond_set_weights", "mpl_precond_get_weights", "mpl_nn_forward",
                     "mpl_nn_backward", "mpl_precond_train_step", "mpl_precond_apply",
                     "mpl_precond_reserve", "mpl_precond_collect", "mpl_precond_sample_count",
                     "mpl_precond_train", "mpl_precond_online", "mpl_precond_online_stats"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (mpl_\w+)", out))
    assert set(declared()) <= exported
    # and nothing is exported that the header does not document
    assert exported <= set(declared()), sorted(exported - set(declared()))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_version_string_and_argument_checks():
    lib = ctypes.CDLL(LIB)
    lib.mpl_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.mpl_version()
    # invalid arguments are rejected before any device work
    assert lib.mpl_create(None, None, 0, None, None, None) != 0
    out = ctypes.c_void_p()
    assert lib.mpl_create(None, None, 0, None, None, ctypes.byref(out)) != 0
    assert out.value is None
