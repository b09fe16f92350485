"""The C-ABI library loads and exports every entry point declared in
include/ocm.h, and the binding's ctypes layouts match the C structs.  No
compute calls: these tests run without a GPU."""

import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ocm.h")


@pytest.fixture(scope="module")
def libpath():
    from paper_1111_0627_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return build.LIB


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ocm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("ocm_min", "ocm_max", "ocm_workspace_size", "ocm_default_options",
              "ocm_phase_sweep", "ocm_phase_cycles", "ocm_phase_select",
              "ocm_phase_connect", "ocm_phase_values", "ocm_status_string",
              "ocm_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol(libpath):
    lib = C.CDLL(libpath)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_status_strings_and_defaults(libpath):
    from paper_1111_0627_amd import ocm
    L = ocm.lib()
    for code in range(-9, 1):
        assert L.ocm_status_string(code)
    o = ocm.Options()
    L.ocm_default_options(C.byref(o))
    assert (o.max_iters, o.validate, o.schedule, o.tie_check, o.fast_path) == (0, 1, 0, 1, 1)


def test_workspace_size_rejects_bad_graphs(libpath):
    from paper_1111_0627_amd import ocm
    L = ocm.lib()
    g = ocm.Graph(0, 5, 8, 8, 8, 0)
    assert L.ocm_workspace_size(C.byref(g), None) == 0
    g = ocm.Graph(10, 20, 8, 8, 8, 0)
    assert L.ocm_workspace_size(C.byref(g), None) >= 10 * 80


def test_struct_layouts_match_header(tmp_path, libpath):
    from paper_1111_0627_amd import ocm
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "ocm.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(ocm_graph), sizeof(ocm_result), sizeof(ocm_options), sizeof(ocm_profile));
  printf("%zu %zu %zu %zu %zu %zu\n", offsetof(ocm_result, flags), offsetof(ocm_result, W), offsetof(ocm_result, tight_edges), offsetof(ocm_options, profile), offsetof(ocm_options, int128_values), offsetof(ocm_options, multichain));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    sizes = [int(x) for x in out]
    assert sizes[:4] == [C.sizeof(ocm.Graph), C.sizeof(ocm._Result), C.sizeof(ocm.Options),
                         C.sizeof(ocm.Profile)]
    assert sizes[4:] == [ocm._Result.flags.offset, ocm._Result.W.offset,
                         ocm._Result.tight_edges.offset, ocm.Options.profile.offset,
                         ocm.Options.int128_values.offset, ocm.Options.multichain.offset]


def test_product_path_has_no_oracle_dependency():
    """The library sources and the binding never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_1111_0627_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower() or f == "synth.py", f
