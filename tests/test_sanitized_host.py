"""The host C++ of the library (assembly, boundary rule, p-transfers,
aggregation, host CSR objects, argument checks of the C ABI) under
AddressSanitizer and UndefinedBehaviorSanitizer: the library is rebuilt with
both sanitizers on its host code and the CPU tests of the host stages and of
the C ABI run against it in a subprocess with the sanitizer runtime
preloaded; any report aborts that run.  No GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_stages_under_address_and_undefined_behavior_sanitizers():
    sys.path.insert(0, ROOT)
    from paper_2512_15121_amd import build
    lib = build.build_sanitized()
    env = dict(os.environ,
               LD_PRELOAD=build.sanitizer_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               GIAMG_TEST_LIBRARY=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_host_setup.py"),
                        os.path.join(ROOT, "tests", "test_abi.py"),
                        os.path.join(ROOT, "tests", "test_binding_checks.py"),
                        "-k", "not layouts"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "passed" in r.stdout
    assert "AddressSanitizer" not in out and "runtime error" not in out
