"""The oracle's pins once more, on an AddressSanitizer + UndefinedBehavior-
Sanitizer build of the oracle (CPU only): any out-of-bounds access, use of
freed memory, signed overflow, bad shift or misaligned access in
lbm_oracle.c aborts the run.  The sanitized library is built with gcc into a
temporary directory and loaded by a child interpreter with the ASan runtime
preloaded (ORACLE_LIB selects it)."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbm_oracle.c")
PINS = ["test_oracle_lattice.py", "test_oracle_streaming.py", "test_oracle_switches.py",
        "test_oracle_walls.py", "test_oracle_adjoint.py", "test_oracle_dynamics.py",
        "test_oracle_incompressible.py"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan():
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "liboracle_san.so")
        subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                        "-fopenmp", "-fPIC", "-shared", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", "-o", lib, SRC, "-lm"], check=True)
        log = os.path.join(d, "san")
        env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=asan, OMP_NUM_THREADS="2",
                   ASAN_OPTIONS=f"detect_leaks=0:log_path={log}",
                   UBSAN_OPTIONS=f"print_stacktrace=1:halt_on_error=1:log_path={log}")
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"]
                           + [os.path.join(ROOT, "tests", t) for t in PINS],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
        reports = "".join(open(os.path.join(d, f)).read() for f in sorted(os.listdir(d))
                          if f.startswith("san"))
        tail = (r.stdout + r.stderr)[-2000:] + reports[-4000:]
        assert r.returncode == 0 and not reports, tail
        assert "passed" in r.stdout, tail
