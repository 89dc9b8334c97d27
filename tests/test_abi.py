"""The C-ABI library loads and exports every entry point include/tfmm.h declares (CPU only).

No compute call is made here: without a GPU, context creation must fail cleanly
with TFMM_ERR_NO_DEVICE (the library has no CPU fallback).
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tfmm.h")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:tfmm_status|const char\*)\s+(tfmm_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_2010_00520_amd as P

    if not os.path.exists(P.tfmm.LIB_PATH):
        pytest.fail("libtfmm.so is not built (run __graft_entry__.build())")
    return P.load()


def test_header_declares_the_documented_entry_points():
    names = declared()
    for n in ("tfmm_setup_compressed", "tfmm_translate", "tfmm_submit", "tfmm_poll", "tfmm_op_import",
              "tfmm_op_export", "tfmm_ctx_create", "tfmm_ctx_destroy"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", lib._name], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(tfmm_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    for n in declared():
        assert hasattr(lib, n)


def test_binding_covers_every_symbol():
    import paper_2010_00520_amd as P

    bound = {name for name, _, _ in P.SIGNATURES}
    assert bound == set(declared())


def test_status_strings(lib):
    assert lib.tfmm_status_str(0) == b"ok"
    assert lib.tfmm_status_str(10) == b"no HIP device"


def test_no_device_fails_cleanly_without_gpu():
    import torch

    import paper_2010_00520_amd as P

    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(P.TfmmError) as e:
        P.Context(0)
    assert e.value.status == 10
