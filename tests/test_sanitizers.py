"""CPU hygiene: the oracle and the library's host-side mechanism compiler
run under AddressSanitizer and UndefinedBehaviorSanitizer (gcc builds;
no GPU involved)."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2501_00011_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined", "-g", "-O1"]
ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _libasan():
    return subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()


@pytest.mark.slow
def test_oracle_pins_under_sanitizers(tmp_path):
    """The oracle's own pins (f/J, controller, warm start, reverse mode, the
    BDF closed forms) with the oracle built with ASan + UBSan."""
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", *SAN, "-std=c11", "-fopenmp", "-shared", "-fPIC", "-o", str(lib),
                    os.path.join(ROOT, "oracle", "oracle.c"), "-lm"], check=True)
    env = dict(os.environ, LD_PRELOAD=_libasan(), MCC_ORACLE_LIB=str(lib), **ENV)
    tests = ["tests/test_oracle_fj.py", "tests/test_oracle_controller.py", "tests/test_oracle_warm_start.py",
             "tests/test_oracle_adjoint.py", "tests/test_oracle_multicell.py", "tests/test_oracle_bdf.py"]
    # the Radau comparisons add minutes of scipy and nothing of the oracle's own code
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-k", "not radau",
                        *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode in (0, 5), r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout


def _write_mech(m, path):
    with open(path, "wb") as f:
        np.array([m.n_species, m.n_reactions, len(m.reac_idx), len(m.prod_idx)], dtype=np.int32).tofile(f)
        for a, dt in ((m.rxn_type, np.int32), (m.reac_ptr, np.int32), (m.reac_idx, np.int32), (m.prod_ptr, np.int32),
                      (m.prod_idx, np.int32), (m.prod_yield, np.float64), (m.A, np.float64), (m.theta, np.float64)):
            np.ascontiguousarray(a, dtype=dt).tofile(f)


@pytest.mark.slow
def test_host_tables_under_sanitizers(tmp_path):
    """The mechanism compiler, the host emulation of the solver and f/J
    tables and the kernel-source generator, built with ASan + UBSan (g++),
    on the 20-, 72- and 150-species mechanisms at every dense-tail size and
    for the transposed system: no sanitizer finding, no table violation."""
    csrc = os.path.join(ROOT, "paper_2501_00011_amd", "csrc")
    exe = tmp_path / "host_tables"
    subprocess.run(["g++", *SAN, "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I" + os.path.join(ROOT, "include"), "-o", str(exe),
                    os.path.join(ROOT, "tests", "sanitize_host_tables.cpp"),
                    os.path.join(csrc, "mech_compile.cpp"), os.path.join(csrc, "mech_emulate.cpp"),
                    os.path.join(csrc, "fj_codegen.cpp"), "-L/opt/rocm/lib", "-lhiprtc",
                    "-Wl,-rpath,/opt/rocm/lib"], check=True)
    env = dict(os.environ, **ENV)
    for mech in (synth.mech_small_thermal(), synth.mech_medium(), synth.mech_large()):
        path = tmp_path / f"mech{mech.n_species}.bin"
        _write_mech(mech, path)
        r = subprocess.run([str(exe), str(path)], env=env, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-3000:]
        assert "violations" in r.stdout
