"""The oracle's C code under the host sanitizers (CPU only): every entry
point, on every lattice, ragged and degenerate boxes and the argument
checks, built once with AddressSanitizer and UndefinedBehaviorSanitizer
(errors abort) and once plainly; the sanitized run must report nothing and
print exactly the plain run's checksums.  The oracle is the reference every
parity test trusts, so an out-of-bounds access or an undefined operation in
it would make those tests compare against garbage."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = [os.path.join(ROOT, "oracle", "cmflb_oracle.c"),
           os.path.join(ROOT, "tests", "oracle_sanitize_driver.c")]
FLAGS = ["-std=gnu11", "-O2", "-g", "-fopenmp", "-Wall"]
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _build(tmp_path, name, extra):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / name)
    subprocess.run([gcc, *FLAGS, *extra, *SOURCES, "-lm", "-o", exe], check=True, capture_output=True)
    return exe


def _run(exe):
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    return subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)


def test_oracle_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    plain = _run(_build(tmp_path, "plain", []))
    assert plain.returncode == 0, plain.stdout + plain.stderr
    try:
        sanitized_exe = _build(tmp_path, "sanitized", SANITIZE)
    except subprocess.CalledProcessError as e:  # no sanitizer runtime in this toolchain
        pytest.skip(f"sanitizer build unavailable: {e.stderr[-200:]!r}")
    san = _run(sanitized_exe)
    assert "runtime error" not in san.stderr, san.stderr[-4000:]
    assert "AddressSanitizer" not in san.stderr, san.stderr[-4000:]
    assert "LeakSanitizer" not in san.stderr, san.stderr[-4000:]
    assert san.returncode == 0, san.stdout[-2000:] + san.stderr[-4000:]
    assert san.stdout == plain.stdout
    assert "failures 0" in san.stdout
    assert san.stdout.count("\n") > 60  # every entry point reported
