"""The oracle's C code under AddressSanitizer and UBSan: its pin tests run in
a child process against a sanitized build (gcc -fsanitize=address,undefined,
UB fatal), with the ASan runtime preloaded into the interpreter.  Any invalid
access, leak-free use-after-free, overflow or undefined behaviour in
shadow_oracle.c aborts the child, and the test fails.

The host side of the HIP library's C ABI (argument checks, layouts, node
tables) is checked the same way, by tests/test_abi.py run against a build
of the library whose host code carries the sanitizers; that build takes
several minutes, so it is not made here."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_pins_under_asan_ubsan():
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"]).decode().strip()
    env = dict(os.environ, ORACLE_SANITIZE="1", LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               OMP_NUM_THREADS="4")
    subprocess.check_call([sys.executable, "-c", "import oracle; oracle.build(force=True)"], cwd=ROOT, env=env)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests/test_oracle_pins.py", "tests/test_oracle_energy.py", "tests/test_oracle_vce.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in tail and "runtime error" not in tail, tail
