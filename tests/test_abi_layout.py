"""The binding's ctypes mirrors of the C-ABI structs against the header: a
small C program built with the host compiler prints every struct's size and
each field's offset as the header lays them out, and every constant the
binding restates; the mirrors must agree field by field. Runs on the CPU."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from paper_2606_08469_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

STRUCTS = {"oo_disparity": binding._Disparity, "oo_tree": binding._Tree, "oo_mlp": binding._MLP,
           "oo_residual_batch": binding._Batch, "oo_adam_config": binding._AdamCfg,
           "oo_adam_segment": binding._AdamSeg}
CONSTANTS = {"OO_MAX_LEVELS": binding.MAX_LEVELS, "OO_MAX_LAYERS": binding.MAX_LAYERS,
             "OO_HASH_MAX_LEVELS": binding.HASH_MAX_LEVELS, "OO_INTERP_NODE_BILINEAR": binding.INTERP_NODE_BILINEAR,
             "OO_INTERP_PAPER": binding.INTERP_PAPER, "OO_F32": binding.F32, "OO_F16": binding.F16,
             "OO_BF16": binding.BF16}


@pytest.fixture(scope="module")
def header_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None or not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime_api.h")):
        pytest.skip("needs a host C compiler and the HIP runtime headers")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "octaoctree.h"', 'int main(void) {']
    for name, mirror in STRUCTS.items():
        lines.append(f'  printf("size {name} %zu\\n", sizeof({name}));')
        for field, _ in mirror._fields_:
            lines.append(f'  printf("off {name}.{field} %zu\\n", offsetof({name}, {field}));')
    for name in CONSTANTS:
        lines.append(f'  printf("const {name} %lld\\n", (long long)({name}));')
    lines += ["  return 0;", "}"]
    d = tmp_path_factory.mktemp("abi")
    src, exe = d / "layout.c", d / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run([cc, "-std=c99", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROOT, "include"),
                    "-I" + os.path.join(ROCM, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {k: int(v) for _, k, v in (line.split() for line in out.splitlines())}


@pytest.mark.parametrize("name", sorted(STRUCTS))
def test_struct_mirrors_header(header_layout, name):
    mirror = STRUCTS[name]
    assert C.sizeof(mirror) == header_layout[name], (name, C.sizeof(mirror), header_layout[name])
    for field, _ in mirror._fields_:
        assert getattr(mirror, field).offset == header_layout[f"{name}.{field}"], (name, field)


def test_constants_mirror_header(header_layout):
    for name, value in CONSTANTS.items():
        assert header_layout[name] == value, name
