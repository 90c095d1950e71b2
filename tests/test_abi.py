"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, its struct layouts match the C compiler's, and argument
validation happens on the host (no compute call is made here)."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_2111_11538_amd import pf
from paper_2111_11538_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pf.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[A-Za-z_][\w \*]*?[\s\*])(pf_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pf.LIB_PATH):
        from paper_2111_11538_amd import build
        build.build()
    return pf.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert set(names) == set(pf.EXPORTS), names
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layouts_match_the_header(lib):
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "pf.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(pf_config), sizeof(pf_params), sizeof(pf_step_stats),
         offsetof(pf_config, ledger_tol), offsetof(pf_params, m_form), offsetof(pf_step_stats, nonfinite));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        exe = os.path.join(d, "s")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, c])
        out = [int(v) for v in subprocess.check_output([exe]).split()]
    assert out == [C.sizeof(pf.pf_config), C.sizeof(pf.pf_params), C.sizeof(pf.pf_step_stats),
                   pf.pf_config.ledger_tol.offset, pf.pf_params.m_form.offset, pf.pf_step_stats.nonfinite.offset]


def test_workspace_size_and_validation(lib):
    cfg = pf.make_config(2, (64, 64), I.H_DEFAULT, 1e-8)
    n64 = lib.pf_workspace_bytes(C.byref(cfg))
    assert n64 > 0 and n64 % 256 == 0
    cfg32 = pf.make_config(2, (64, 64), I.H_DEFAULT, 1e-8, precision="mixed")
    assert 0 < lib.pf_workspace_bytes(C.byref(cfg32)) < n64
    bad = pf.make_config(2, (64, 64), I.H_DEFAULT, 1e-8)
    bad.nz = 3
    assert lib.pf_workspace_bytes(C.byref(bad)) == 0
    bad = pf.make_config(3, (4, 4, 4), I.H_DEFAULT, -1.0)
    assert lib.pf_workspace_bytes(C.byref(bad)) == 0
    ctx = C.c_void_p()
    prm = pf.make_params(I.Params())
    rc = lib.pf_init(C.byref(cfg), C.byref(prm), None, 0, None, C.byref(ctx))
    assert rc == pf.PF_ERR_INVALID_ARG and not ctx.value
    assert b"workspace" in lib.pf_last_error(None)
    rc = lib.pf_init(C.byref(cfg), C.byref(prm), C.c_void_p(256), 16, None, C.byref(ctx))
    assert rc == pf.PF_ERR_OOM
    assert lib.pf_step(None, 1, None) == pf.PF_ERR_INVALID_ARG
