"""The C-ABI library builds, loads and exports every entry point that
include/cdhip.h declares (CPU only: no compute calls)."""
import ctypes
import os

import pytest

from paper_1104_3516_amd import binding


def test_header_declares_the_boundary():
    names = binding.declared_symbols()
    for required in ("cd_create", "cd_destroy", "cd_set_particles", "cd_set_external",
                     "cd_set_walls", "cd_set_box", "cd_step", "cd_get_state",
                     "cd_get_contacts", "cd_get_tree", "cd_get_timing", "cd_status_string",
                     "cd_last_error", "cd_num_contacts", "cd_get_walls", "cd_set_timing",
                     "cd_set_solve_mode", "cd_set_launch", "cd_solve_contacts"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libcdhip.so is not built (run __graft_entry__.build())")
    L = binding.lib()
    for name in binding.declared_symbols():
        assert hasattr(L, name), name
    # status strings need no device
    assert L.cd_status_string(0) == b"ok"
    assert L.cd_status_string(1).startswith(b"sweep cap")


def test_struct_layouts_match_header(tmp_path):
    # the ctypes mirrors have the sizes and field offsets the C compiler gives
    # the header structs
    import subprocess
    structs = {"cd_params": binding.Params, "cd_result": binding.Result,
               "cd_timing": binding.Timing, "cd_batch_timing": binding.BatchTiming}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "cdhip.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(py, fname).offset, (cname, fname)


def test_product_package_does_not_import_the_oracle():
    import re

    import paper_1104_3516_amd
    root = os.path.dirname(paper_1104_3516_amd.__file__)
    for dirpath, _, files in os.walk(root):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", text, re.M), f
                assert "cdref" not in text, f
