"""The ctypes mirrors of the C-ABI structs (paper_2007_00324_amd/gdp2d.py)
must have the size and field offsets the header gives them: a C program
compiled from include/gdp2d.h with the host compiler prints sizeof and
offsetof of every field, and each mirror is compared with it."""
import ctypes as C
import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ["gdp_pslg", "gdp_job_times", "gdp_params", "gdp_kernel_prof", "gdp_mesh_info", "gdp_device_views",
           "gdp_round_stats"]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    from paper_2007_00324_amd import gdp2d
    d = tmp_path_factory.mktemp("abi")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gdp2d.h"', "int main(void) {", 'printf("{");']
    for k, name in enumerate(STRUCTS):
        fields = [f[0] for f in getattr(gdp2d, name)._fields_]
        parts = [f'printf("\\"{name}\\": {{\\"size\\": %zu", sizeof({name}));']
        for f in fields:
            parts.append(f'printf(", \\"{f}\\": %zu", offsetof({name}, {f}));')
        parts.append('printf("}");' if k == len(STRUCTS) - 1 else 'printf("}, ");')
        lines += parts
    lines += ['printf("}\\n");', "return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines))
    exe = d / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    return json.loads(subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout)


@pytest.mark.parametrize("name", STRUCTS)
def test_ctypes_mirror_matches_header(c_layout, name):
    from paper_2007_00324_amd import gdp2d
    cls = getattr(gdp2d, name)
    want = c_layout[name]
    assert C.sizeof(cls) == want["size"], (name, C.sizeof(cls), want["size"])
    for f, _ in cls._fields_:
        assert getattr(cls, f).offset == want[f], (name, f, getattr(cls, f).offset, want[f])
