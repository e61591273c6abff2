"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only): a set of its pins runs in a child process against that
build, so an out-of-bounds index, a use of freed memory or undefined integer
arithmetic in hlb_oracle.c ends the run with a sanitizer report instead of
passing silently."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hlb_oracle.c")

# a coupled run of each LB model and coupling, the stencils, the pins that
# read every routine of the library
PINS = [
    "tests/test_oracle_pins.py::test_mass_conservation_coupled",
    "tests/test_oracle_pins.py::test_momentum_conservation_with_stress",
    "tests/test_oracle_pins.py::test_q_stays_symmetric_traceless",
    "tests/test_oracle_pins.py::test_init_then_readout",
    "tests/test_oracle_pins.py::test_cholesteric_helix_is_stationary",
    "tests/test_oracle_split.py",
    "tests/test_oracle_d3q15.py",
]


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True, check=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_pins_under_address_and_ub_sanitizers(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp",
                           "-fPIC", "-shared", "-std=c11", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-o", lib, SRC, "-lm"])
    env = dict(os.environ)
    env.update(HLB_ORACLE_LIB=lib, LD_PRELOAD=asan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    report = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, report
    assert "ERROR: AddressSanitizer" not in report and "runtime error" not in report, report
