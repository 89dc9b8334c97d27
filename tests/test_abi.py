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


def _c_layout(struct, fields):
    """offsetof / sizeof of a tfmm.h struct, from a C program compiled with gcc."""
    import tempfile

    body = "".join(f'  printf("%s %zu\\n", "{f}", offsetof({struct}, {f}));\n' for f in fields)
    src = ("#include <stddef.h>\n#include <stdio.h>\n#include \"tfmm.h\"\nint main(void) {\n" + body +
           f'  printf("sizeof %zu\\n", sizeof({struct}));\n  return 0;\n}}\n')
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    return {k: int(v) for k, v in (line.split() for line in out.splitlines())}


@pytest.mark.parametrize("struct,cls", [("tfmm_problem", "Problem"), ("tfmm_op_info", "OpInfo")])
def test_binding_structs_match_the_header(struct, cls):
    """The ctypes mirrors of tfmm_problem and tfmm_op_info have the header's field
    offsets and size (a field added to one side only shifts every field after it)."""
    import paper_2010_00520_amd as P

    C = getattr(P.tfmm, cls)
    names = [f for f, _ in C._fields_]
    lay = _c_layout(struct, names)
    assert lay.pop("sizeof") == ctypes.sizeof(C)
    assert lay == {f: getattr(C, f).offset for f in names}


def test_problem_fields_from_keywords():
    """Complex wavenumber and explicit directions reach the C struct."""
    import numpy as np

    import paper_2010_00520_amd as P

    d = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    p = P.make_problem((4, 4, 4), k=2 * np.pi * (1.4 - 0.3j), dirs=d, fmt="tt4d")
    assert p.k_re == pytest.approx(2 * np.pi * 1.4) and p.k_im == pytest.approx(-2 * np.pi * 0.3)
    assert p.n_dir == 2 and [p.dirs[i] for i in range(6)] == [0.0, 0.0, 1.0, 1.0, 0.0, 0.0]
    assert p.fmt == P.FORMATS["tt4d"]
