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
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(pf_config), sizeof(pf_params), sizeof(pf_step_stats),
         offsetof(pf_config, ledger_tol), offsetof(pf_params, m_form), offsetof(pf_step_stats, nonfinite),
         sizeof(pf_fs_config), offsetof(pf_fs_config, cg_rtol), sizeof(pf_fs_stats), offsetof(pf_fs_stats, yielded),
         offsetof(pf_config, cg_precond));
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
                   pf.pf_config.ledger_tol.offset, pf.pf_params.m_form.offset, pf.pf_step_stats.nonfinite.offset,
                   C.sizeof(pf.pf_fs_config), pf.pf_fs_config.cg_rtol.offset, C.sizeof(pf.pf_fs_stats),
                   pf.pf_fs_stats.yielded.offset, pf.pf_config.cg_precond.offset]


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


def test_multigrid_workspace_and_validation(lib):
    """The multigrid preconditioner adds its levels to the workspace (3D: two
    more fine vectors and 17 arrays per coarse level, 1/8 of the cells each,
    and in FP32 the sweeps' bf16 copies of K, G and D^-1 on every level; 2D:
    12 arrays per coarse level, 1/4 of the cells each); batches and unknown
    preconditioner codes are refused."""
    sz = lambda c: lib.pf_workspace_bytes(C.byref(c))
    for prec in ("fp64", "mixed"):
        jac = pf.make_config(3, (32, 32, 32), I.H_DEFAULT, 1e-8, precision=prec)
        mg = pf.make_config(3, (32, 32, 32), I.H_DEFAULT, 1e-8, precision=prec, cg_precond="mg")
        es = 8 if prec == "fp64" else 4
        fine = 32 * 32 * 32 * es
        extra = sz(mg) - sz(jac)
        # level 0: 6 vectors; levels 16^3 and 8^3: 17 arrays each; alignment and stagger slack
        want = 6 * fine + 17 * (fine // 8 + fine // 64)
        if prec == "mixed":       # 5 bf16 arrays per level (the 8^3 rows padded to 16)
            want += 5 * 2 * (32 ** 3 + 16 ** 3 + 16 * 8 * 8)
        assert want <= extra <= want + 64 * 8192, (prec, extra, want)
    odd = pf.make_config(3, (9, 12, 16), I.H_DEFAULT, 1e-8, cg_precond="mg")
    assert sz(odd) > sz(pf.make_config(3, (9, 12, 16), I.H_DEFAULT, 1e-8))   # levels 16x12x9 and 8x6x5
    jac2 = pf.make_config(2, (64, 64), I.H_DEFAULT, 1e-8)
    mg2 = pf.make_config(2, (64, 64), I.H_DEFAULT, 1e-8, cg_precond="mg")
    fine2 = 64 * 64 * 8
    want2 = 4 * fine2 + 12 * (fine2 // 4 + fine2 // 16 + fine2 // 64)     # levels 32^2, 16^2, 8^2
    assert want2 <= sz(mg2) - sz(jac2) <= want2 + 64 * 8192
    ext = (pf.pf_extent * 1)()
    ext[0].nx, ext[0].ny, ext[0].nz = 64, 64, 1
    assert lib.pf_batch_workspace_bytes(C.byref(jac2), ext, 1) > 0
    assert lib.pf_batch_workspace_bytes(C.byref(mg2), ext, 1) == 0
    bad = pf.make_config(3, (32, 32, 32), I.H_DEFAULT, 1e-8)
    bad.cg_precond = 2
    assert sz(bad) == 0


def test_batch_workspace_validation(lib):
    """Batch sizing on the host: 1..256 instances, 2D only, mechanics on, the
    previous-step start, non-empty extents; the workspace grows with the
    instances and is 0 for every invalid request."""
    def ext_of(shapes):
        e = (pf.pf_extent * max(1, len(shapes)))()
        for k, (ny, nx) in enumerate(shapes):
            e[k].nx, e[k].ny, e[k].nz = nx, ny, 1
        return e

    cfg = pf.make_config(2, (8, 8), I.H_DEFAULT, 1e-8, precision="mixed", plasticity=True)
    one = lib.pf_batch_workspace_bytes(C.byref(cfg), ext_of([(8, 8)]), 1)
    full = lib.pf_batch_workspace_bytes(C.byref(cfg), ext_of([(8, 8)] * 256), 256)
    assert 0 < one < full
    wide = lib.pf_batch_workspace_bytes(C.byref(cfg), ext_of([(8, 8), (40, 130)]), 2)
    assert lib.pf_batch_workspace_bytes(C.byref(cfg), ext_of([(8, 8)] * 2), 2) < wide
    assert lib.pf_batch_workspace_bytes(C.byref(cfg), ext_of([(8, 8)] * 257), 257) == 0
    assert lib.pf_batch_workspace_bytes(C.byref(cfg), ext_of([]), 0) == 0
    assert lib.pf_batch_workspace_bytes(C.byref(cfg), ext_of([(0, 8)]), 1) == 0
    assert lib.pf_batch_workspace_bytes(C.byref(cfg), ext_of([(8, 0)]), 1) == 0
    for kw in ({"mechanics": False}, {"warm": "learned"}):
        bad = pf.make_config(2, (8, 8), I.H_DEFAULT, 1e-8, precision="mixed", **kw)
        assert lib.pf_batch_workspace_bytes(C.byref(bad), ext_of([(8, 8)]), 1) == 0, kw
    bad3 = pf.make_config(3, (8, 8, 8), I.H_DEFAULT, 1e-8, precision="mixed")
    assert lib.pf_batch_workspace_bytes(C.byref(bad3), ext_of([(8, 8)]), 1) == 0
    b = C.c_void_p()
    prm = pf.make_params(I.Params())
    rc = lib.pf_batch_init(C.byref(cfg), C.byref(prm), ext_of([(8, 8)] * 257), 257, None, 0, None, C.byref(b))
    assert rc == pf.PF_ERR_INVALID_ARG and not b.value
    assert b"count" in lib.pf_batch_last_error(None)


def test_network_workspace_size(lib):
    """pf_nn_workspace_bytes is host arithmetic: it grows with the capacity
    (about 224 bytes per voxel, 384 with training buffers) and is 0 for an
    invalid configuration."""
    from paper_2111_11538_amd import pf
    c = pf.pf_nn_config()
    c.max_voxels, c.training = 0, 0
    assert lib.pf_nn_workspace_bytes(C.byref(c)) == 0
    sizes = {}
    for tr in (0, 1):
        for cap in (4096, 8192):
            c.max_voxels, c.training = cap, tr
            sizes[tr, cap] = lib.pf_nn_workspace_bytes(C.byref(c))
    assert 220 * 4096 <= sizes[0, 8192] - sizes[0, 4096] <= 230 * 4096
    assert 380 * 4096 <= sizes[1, 8192] - sizes[1, 4096] <= 390 * 4096
    assert all(v % 256 == 0 for v in sizes.values())


def test_finite_strain_workspace_and_validation(lib):
    cfg = pf.make_fs_config(2, (8, 10), 1e-7)
    n2 = lib.pf_fs_workspace_bytes(C.byref(cfg))
    assert n2 > 0 and n2 % 256 == 0
    cfg3 = pf.make_fs_config(3, (8, 8, 10), 1e-7)
    assert lib.pf_fs_workspace_bytes(C.byref(cfg3)) > n2
    for field, value in (("nz", 2), ("h", 0.0), ("newton_rtol", -1.0), ("cg_max_iter", 0), ("dim", 4)):
        bad = pf.make_fs_config(2, (8, 10), 1e-7)
        setattr(bad, field, value)
        assert lib.pf_fs_workspace_bytes(C.byref(bad)) == 0, field
    fs = C.c_void_p()
    prm = pf.make_params(I.Params())
    assert lib.pf_fs_init(C.byref(cfg), C.byref(prm), None, n2, None, C.byref(fs)) == pf.PF_ERR_INVALID_ARG
    assert b"workspace" in lib.pf_fs_last_error(None)
    # a misaligned workspace is rejected before any HIP call
    assert lib.pf_fs_init(C.byref(cfg), C.byref(prm), C.c_void_p(257 * 256 + 8), n2, None,
                          C.byref(fs)) == pf.PF_ERR_INVALID_ARG
    assert lib.pf_fs_init(C.byref(cfg), C.byref(prm), C.c_void_p(256), 16, None, C.byref(fs)) == pf.PF_ERR_OOM
    assert not fs.value
    assert lib.pf_fs_solve(None, None) == pf.PF_ERR_INVALID_ARG
    assert lib.pf_fs_fields(None, 0, 0, None, 0, 0) == pf.PF_ERR_INVALID_ARG
