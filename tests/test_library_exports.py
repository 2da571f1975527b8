"""The C-ABI library loads and exports every function its header declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "evlbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(evlbm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("evlbm_create", "evlbm_set_eos", "evlbm_set_relaxation", "evlbm_init_fields", "evlbm_step",
                     "evlbm_read_moments", "evlbm_global_sums", "evlbm_measure", "evlbm_batch_create",
                     "evlbm_batch_autotune", "evlbm_mlp_train", "evlbm_mlp_grad", "evlbm_init_droplet"):
        assert required in names, required


def test_library_exports_every_declared_symbol():
    from paper_2508_00577_amd import LIB_PATH, build
    if not os.path.exists(LIB_PATH):
        build.build()
    lib = ctypes.CDLL(LIB_PATH)
    names = declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert len(names) >= 40


def test_version_string_without_gpu():
    from paper_2508_00577_amd import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB_PATH)
    lib.evlbm_version.restype = ctypes.c_char_p
    assert lib.evlbm_version().decode().startswith("evlbm")
