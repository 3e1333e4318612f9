"""The C-ABI library loads and exports every entry point the public header
declares; the binding declares the same set (no device is touched)."""
import ctypes
import os
import re

import pytest

from paper_1309_5796_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    with open(os.path.join(ROOT, "include", "mmsd.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(mmsd_[a-z_0-9]+)\s*\(", text))
    return names - {"mmsd_alloc_fn", "mmsd_free_fn"}


def test_header_declares_the_expected_entry_points():
    names = header_functions()
    assert {"mmsd_minimize", "mmsd_hysteresis", "mmsd_minimize_batch", "mmsd_submit", "mmsd_poll"} <= names
    assert len(names) == 42


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libmmsd.so is not built (python -m paper_1309_5796_amd.build)")
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in sorted(header_functions()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_exactly_the_header_set():
    assert {s[0] for s in binding.SIGNATURES} == header_functions()
    binding.load_library()


def test_options_default_and_struct_layout():
    lib = binding.load_library()
    o = binding.OptionsC()
    lib.mmsd_options_default(ctypes.byref(o))
    assert o.tol_torque == 1e-6 and o.max_evals == 100000 and o.terms == 15 and o.nonmono_M == 20
    assert ctypes.sizeof(binding.OptionsC) == 56
    assert ctypes.sizeof(binding.ResultC) == 8 * 17


def test_ctypes_structs_match_the_c_layout(tmp_path):
    """Compile a probe against the header with gcc and compare every field
    offset of the ABI structs with the binding's ctypes mirrors."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"mmsd_mesh": binding.MeshC, "mmsd_material": binding.MaterialC,
               "mmsd_options": binding.OptionsC, "mmsd_result": binding.ResultC}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mmsd.h"', "int main(void){"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
