"""The ctypes mirrors of the C ABI's structs have the header's layout: a C program built
against include/eifp.h with the host compiler prints every struct's size and each
field's offset, and the Python binding's structures must agree field by field (a field
added to one side only, or reordered, would silently corrupt every call that passes the
struct)."""
import ctypes
import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = ("eifp_domain", "eifp_invariant_set", "eifp_invariant_ext_set", "eifp_request", "eifp_event",
           "eifp_server_stat_set")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_struct_layouts_match_the_header(tmp_path):
    from paper_2210_06232_amd import eifp as m  # loads the library lazily: no GPU needed
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "eifp.h"', "int main(void) {", 'printf("{");']
    first = True
    for name in STRUCTS:
        cls = getattr(m, name)
        fields = [f for f, _ in cls._fields_]
        parts = [f'\\"size\\": %zu'] + [f'\\"{f}\\": %zu' for f in fields]
        args = [f"sizeof({name})"] + [f"offsetof({name}, {f})" for f in fields]
        sep = "" if first else ", "
        first = False
        lines.append(f'printf("{sep}\\"{name}\\": {{{", ".join(parts)}}}", {", ".join(args)});')
    lines += ['printf("}\\n");', "return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True,
                   capture_output=True, text=True)
    c = json.loads(subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout)
    for name in STRUCTS:
        cls = getattr(m, name)
        assert c[name]["size"] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert c[name][f] == getattr(cls, f).offset, (name, f)
