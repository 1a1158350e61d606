"""The CPU test suite under AddressSanitizer and UndefinedBehaviorSanitizer:
once with the library's host code (api.cpp: argument checks, pass plans,
batch and pipeline plan images) built with clang's sanitizers, once with the
oracle (oracle.c, lbm.c) built with gcc's.  Each run is a child process that
preloads the matching sanitizer runtime; any report aborts it.  A planted
heap overflow, compiled the same way, shows that the set-up catches errors."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OPTIONS = {"ASAN_OPTIONS": "detect_leaks=0:new_delete_type_mismatch=0:detect_odr_violation=0:"
                           "halt_on_error=1",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}

RUNNER = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r})
    if {which!r} == "jacobi":
        import paper_0912_4506_amd._lib as L
        L.LIB_PATH = {lib!r}
        assert L.load()._name == {lib!r}
    else:
        import oracle
        oracle._LIB_PATH = {lib!r}
        assert oracle._load()._name == {lib!r}
    import pytest
    sys.exit(pytest.main(["-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider", {tests!r},
                          "--ignore", {me!r}]))
""")

pytestmark = pytest.mark.slow


def run_suite(which, lib, preload):
    env = dict(os.environ, LD_PRELOAD=" ".join(preload), **OPTIONS)
    code = RUNNER.format(root=ROOT, which=which, lib=lib, tests=os.path.join(ROOT, "tests"),
                         me=os.path.abspath(__file__))
    return subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True,
                          text=True, timeout=900)


def test_library_host_code_under_asan_ubsan():
    from paper_0912_4506_amd.csrc import build
    lib = build.build_sanitized()
    r = run_suite("jacobi", lib, [build.asan_runtime()])
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert " passed" in r.stdout


def test_oracle_under_asan_ubsan():
    from oracle import build
    lib = build.build_sanitized()
    r = run_suite("oracle", lib, build.sanitizer_runtimes())
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert " passed" in r.stdout


def test_planted_overflow_is_caught(tmp_path):
    """Positive control: an off-by-one heap write in a library built with the
    oracle's sanitizer flags aborts the child process with a report."""
    from oracle import build
    src = tmp_path / "bad.c"
    src.write_text("#include <stdlib.h>\nint bad(int n) { int *p = malloc(n * sizeof(int));"
                   " p[n] = 1; int v = p[0]; free(p); return v; }\n")
    lib = str(tmp_path / "libbad.so")
    subprocess.run(["gcc", "-shared", "-fPIC", "-g", "-fsanitize=address,undefined", str(src),
                    "-o", lib], check=True)
    code = f"import ctypes; ctypes.CDLL({lib!r}).bad(4)"
    env = dict(os.environ, LD_PRELOAD=" ".join(build.sanitizer_runtimes()), **OPTIONS)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr
