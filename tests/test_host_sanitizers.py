"""The host code of the library (planner, C ABI, launch set-up) under
AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

build.build_host_sanitized() compiles every source with the sanitizers on
the host side only (the device code as usual); the ABI, binding, tuning and
descriptor-fuzz tests then run in a child process that loads that library
(FOCK_LIBRARY) with the ASan runtime preloaded, stopping at the first report
(output not captured, so that a report printed just before the exit is kept).
The build is reused while the sources are unchanged (about two minutes
otherwise)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = ["tests/test_abi.py", "tests/test_binding.py", "tests/test_autotune.py", "tests/test_descriptor_fuzz.py"]


@pytest.mark.slow
def test_host_code_is_clean_under_asan_and_ubsan():
    from paper_1111_0716_amd import build

    try:
        build.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    if not shutil.which(build.hipcc()) and not os.path.exists(build.hipcc()):
        pytest.skip("hipcc not available")
    lib = build.build_host_sanitized()
    env = dict(os.environ)
    env.update(
        FOCK_LIBRARY=lib,
        LD_PRELOAD=build.asan_runtime(),
        ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
        UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
        CUDA_VISIBLE_DEVICES="",
        HIP_VISIBLE_DEVICES="",
    )
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider", "-m", "not gpu", *TESTS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "Sanitizer" not in out, out[-6000:]
    assert " passed" in out
