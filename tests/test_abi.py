"""The C-ABI library builds, loads and exports every declared entry point
(no GPU needed)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fpeps.h")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(fpeps_[a-z_]+)\s*\(", src)))


def test_header_declares_the_four_calls_and_context():
    names = declared()
    for n in ("fpeps_env_absorb", "fpeps_rsvd_truncate", "fpeps_cbe_expand", "fpeps_expect",
              "fpeps_create", "fpeps_destroy", "fpeps_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2511_01039_amd as pkg
    lib = pkg.load()
    for n in declared():
        assert hasattr(lib, n), n
    assert sorted(pkg.exported_symbols()) == declared()
    assert lib.fpeps_version().decode().startswith("fpeps-gfx950")


def test_library_is_built_for_gfx950_only():
    """The offload bundle of the library built here names one device target."""
    import paper_2511_01039_amd as pkg
    blob = open(pkg.LIB_PATH, "rb").read()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa--(gfx[0-9a-f]+)", blob))
    assert targets == {b"gfx950"}, targets


def test_create_reports_no_device_without_gpu():
    import ctypes as C
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_2511_01039_amd as pkg
    lib = pkg.load()
    h = C.c_void_p()
    rc = lib.fpeps_create(C.byref(h), 0, None)
    assert rc == -9
    assert h.value is None
    # null arguments are rejected without a context
    assert lib.fpeps_create(None, 0, None) == -1
    assert lib.fpeps_destroy(None) == -1
    assert lib.fpeps_last_error(None) == b"null context"
