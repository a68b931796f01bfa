"""The oracle's pins run against a build of the oracle instrumented with
AddressSanitizer and UndefinedBehaviorSanitizer: no out-of-bounds access, use
after free or undefined operation anywhere on the paths the pins exercise
(every local-step model, aperture kind, the gain sheets, the roughness, free
propagation, the spectrum and every FFT length).  CPU only."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    try:
        path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                              check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.timeout(1200)
def test_oracle_pins_under_asan_and_ubsan():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime for gcc")
    env = dict(os.environ)
    env.update(ORC_SANITIZE="1", LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_oracle.py", "-q", "-x", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1100)
    out = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out
