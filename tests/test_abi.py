"""The C-ABI library loads on a host without a GPU and exports every function
that include/lbm.h declares.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header: str) -> list[str]:
    src = open(header).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s+([a-z][a-z_0-9]*)\s*\(", src, flags=re.M)))


def all_headers() -> list[str]:
    d = os.path.join(ROOT, "include")
    return [os.path.join(d, f) for f in sorted(os.listdir(d)) if f.endswith(".h")]


def test_header_declares_the_boundary():
    names = declared_functions(os.path.join(ROOT, "include", "lbm.h"))
    for core in ("lbm_init", "lbm_step", "lbm_fields", "lbm_diagnostics"):
        assert core in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol():
    from paper_2306_11320_amd import lbm
    if not os.path.exists(lbm.LIB_PATH):
        pytest.fail("HIP library not built: run `python -m paper_2306_11320_amd.build`")
    L = ctypes.CDLL(lbm.LIB_PATH)
    names = [n for h in all_headers() for n in declared_functions(h)]
    assert any(n.startswith("sur_") for n in names) and any(n.startswith("lbm_") for n in names)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(lbm.EXPORTED) <= set(names)


def test_binding_struct_sizes_match_header():
    """The ctypes structs must have the layout of the C structs: compile a
    probe with the host compiler that prints sizeof/offsetof."""
    import subprocess
    import tempfile
    from paper_2306_11320_amd import lbm
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "lbm.h"
int main(void){
  printf("%zu %zu %zu %zu %zu\n", sizeof(lbm_params), sizeof(lbm_diag),
         offsetof(lbm_params, rho_l), offsetof(lbm_params, bubble_y), offsetof(lbm_diag, bub_sum));
  return 0;
}'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    got = [int(x) for x in out]
    want = [ctypes.sizeof(lbm.Params), ctypes.sizeof(lbm.Diag), lbm.Params.rho_l.offset,
            lbm.Params.bubble_y.offset, lbm.Diag.bub_sum.offset]
    assert got == want
