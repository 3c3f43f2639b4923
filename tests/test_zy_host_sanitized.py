"""The CPU checks of the C-ABI library (tests/test_abi.py) rerun against the
host-sanitised build (AddressSanitizer + UndefinedBehaviorSanitizer on the
host code, `python paper_2101_06354_amd/build_lib.py --sanitize-host`), in a
child process that preloads clang's ASan runtime.  Any sanitizer report ends
the child with a failure.  Skipped when that build is absent."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2101_06354_amd"))
import build_lib  # noqa: E402

pytestmark = pytest.mark.slow


@pytest.mark.skipif(not os.path.exists(build_lib.SAN_LIB),
                    reason="host-sanitised library not built (build_lib.py --sanitize-host)")
def test_abi_checks_under_host_sanitizers():
    srcs = build_lib.sources() + [os.path.join(ROOT, "include", "ssimx.h")]
    if max(os.path.getmtime(s) for s in srcs) > os.path.getmtime(build_lib.SAN_LIB):
        pytest.skip("host-sanitised library older than the sources; rebuild it")
    env = dict(os.environ, LD_PRELOAD=build_lib.sanitizer_runtime(), SSIMX_LIBRARY=build_lib.SAN_LIB,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
