"""The host side of the library (validation, site tables and thresholds,
Pauli-frame tables, tiled schedules, lightcone networks with slicing and
merged steps, gate-by-gate groups, the job server's argument checks) under
AddressSanitizer and UndefinedBehaviorSanitizer: the host-only checks of
test_abi_host.py run in a child process against a build whose host sources
are instrumented (device code is built as usual and never launched here).
Any sanitizer report fails the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.timeout(900)
def test_host_code_under_address_and_undefined_behaviour_sanitizers():
    import shutil
    if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not available")
    sys.path.insert(0, ROOT)
    from paper_2210_15874_amd.build import build_sanitized_library, sanitizer_runtime
    lib = build_sanitized_library()
    env = dict(os.environ)
    env.update(LD_PRELOAD=sanitizer_runtime(), STN_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0:exitcode=99",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=98")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_host.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=850)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out, out[-2000:]
