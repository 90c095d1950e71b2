"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The FP64 oracle is built with gcc and -fsanitize=address,undefined and runs
a few coupled steps of every mode it has (2D and 3D, plasticity, the closed
box, both implicit species modes, a lone mechanics solve, the energies); the
host pass of ``libpf.so`` is built with the same sanitizers (the device code
is not instrumented) and the ABI tests run against it: workspace sizing of
every context kind and the argument checks made before any HIP call.  Each
runs in a child process with the sanitizer runtime preloaded; a sanitizer
report, or any failure, fails the test.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

ORACLE_RUN = r'''
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
from paper_2111_11538_amd import inputs as I
from oracle import oracle as O
assert O.LIB_PATH.endswith("liboracle_san.so"), O.LIB_PATH
wl = I.workload("core_shell_2d", n=24)
o = O.OracleSim(2, wl.shape, wl.h, wl.dt, wl.params, wl.fields, plasticity=True, cg_rtol=1e-10)
for _ in range(3):
    o.step()
o.energy(); o.elastic_energy(); o.fields()
c = O.OracleSim(2, wl.shape, wl.h, wl.dt, wl.params, wl.fields, plasticity=True, dirichlet=False)
c.step(); c.mech_solve()
shape = (10, 12, 9)
f = I.ic_core_shell(shape, r_core=3.5, r_shell=4.3, noise_seed=I.SEED_BASE + 2)
p = I.Params()
o3 = O.OracleSim(3, shape, I.H_DEFAULT, I.stable_dt(p, I.H_DEFAULT, 3), p, f, plasticity=True, cg_rtol=1e-10)
o3.step(); o3.step()
for mode in (1, 2):
    s = O.OracleSim(2, wl.shape, wl.h, 20 * wl.dt, wl.params, wl.fields, plasticity=False, implicit=mode)
    s.step(); s.step()
print("oracle ok", flush=True)
'''


def _instrumented(lib):
    syms = subprocess.check_output(["nm", "-D", lib], text=True)
    assert "__asan_report" in syms and "__ubsan_handle" in syms, lib


def _run(cmd, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    r = subprocess.run(cmd, env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    return out


def test_oracle_under_asan_and_ubsan(tmp_path):
    from oracle import oracle as O
    lib = O.build(out=str(tmp_path / "liboracle_san.so"),
                  extra=("-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                         "-fno-sanitize-recover=undefined"))
    _instrumented(lib)
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    script = tmp_path / "run_oracle.py"
    script.write_text(ORACLE_RUN)
    out = _run([sys.executable, str(script), ROOT],
               {"PF_ORACLE_LIBRARY": lib, "LD_PRELOAD": asan, "ASAN_OPTIONS": "detect_leaks=0",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1", "OMP_NUM_THREADS": "2"})
    assert "oracle ok" in out


def test_host_library_under_asan_and_ubsan(tmp_path):
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("the ROCm clang AddressSanitizer runtime is not installed")
    from paper_2111_11538_amd import build as B
    lib = B.build(out=str(tmp_path / "libpf_san.so"),
                  extra=("-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                         "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                         "-Xarch_host", "-g"))
    _instrumented(lib)
    # the layout test compiles and runs a C program, which the preloaded
    # runtime would instrument as well; the other ABI tests load the library
    out = _run([sys.executable, "-m", "pytest", "tests/test_abi.py", "-q", "-p", "no:cacheprovider",
                "-k", "not struct_layouts"],
               {"PF_LIBRARY": lib, "LD_PRELOAD": rt[-1], "ASAN_OPTIONS": "detect_leaks=0",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    assert " passed" in out and " failed" not in out
