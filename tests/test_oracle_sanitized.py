"""The CPU oracle under the sanitizers: rb_oracle.c built with
UndefinedBehaviorSanitizer (and AddressSanitizer where this host's ASan
actually detects a heap overflow), and the oracle's pin tests run against
that build in a child interpreter.  Any sanitizer report fails the test."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROBE = r"""
#include <stdio.h>
#include <stdlib.h>
int main(int argc, char **argv) {
  (void)argv;
  int *a = malloc(40);
  a[argc + 20] = 1;
  printf("%d\n", a[argc + 20]);
  free(a);
  return 0;
}
"""


def _gcc_file(name):
    return subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()


def _asan_works():
    """True if a heap overflow built with -fsanitize=address is reported here."""
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "p.c"), os.path.join(d, "p")
        open(src, "w").write(PROBE)
        if subprocess.run(["gcc", "-O1", "-g", "-fsanitize=address", src, "-o", exe]).returncode != 0:
            return False
        r = subprocess.run([exe], capture_output=True, text=True, env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
        return "heap-buffer-overflow" in r.stderr


def test_oracle_pins_under_sanitizers(tmp_path):
    if subprocess.run(["gcc", "--version"], capture_output=True).returncode != 0:
        pytest.skip("gcc not available")
    asan = _asan_works()
    lib = tmp_path / "liboracle_san.so"
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=undefined", "-fno-sanitize-recover=undefined"]
    if asan:
        flags[3] = "-fsanitize=address,undefined"
    subprocess.run(["gcc", *flags, "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-o", str(lib),
                    os.path.join(ROOT, "oracle", "rb_oracle.c"), "-lm"], check=True)
    # the oracle package loads liboracle_san.so from its own folder
    dst = os.path.join(ROOT, "oracle", "liboracle_san.so")
    os.replace(str(lib), dst)
    env = dict(os.environ, RB_ORACLE_SANITIZE="1", OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    if asan:
        pre = _gcc_file("libasan.so") + " " + _gcc_file("libubsan.so")
        env["LD_PRELOAD"] = pre + (" " + os.environ["LD_PRELOAD"] if os.environ.get("LD_PRELOAD") else "")
    tests = ["tests/test_oracle_pins.py", "tests/test_oracle_next.py", "tests/test_golden.py",
             "tests/test_oracle_mlp.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *tests], cwd=ROOT,
                       env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    print("sanitizers: %s" % ("address,undefined" if asan else "undefined (ASan inactive on this host)"))
    print(out[-2000:])
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out
