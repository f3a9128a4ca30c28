"""The CPU suite under AddressSanitizer and UndefinedBehaviorSanitizer.

The library's host code (planner, Overlap Tree, cache policies, cost fit,
argument checks of every entry point, the C-ABI) and the oracle are rebuilt
with -fsanitize=address,undefined (clang, one shared runtime preloaded into
the Python process; device code is not instrumented), and every other
-m "not gpu" test runs in a child process against those builds.  A planted
out-of-bounds read in a throw-away C file shows that the set-up reports
errors rather than passing silently."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.slow


def _sources_digest() -> str:
    h = hashlib.sha256()
    for d, names in (("paper_2201_04058_amd/csrc", None), ("oracle", ["oracle.c"]), ("include", None)):
        path = os.path.join(ROOT, d)
        for n in sorted(names or os.listdir(path)):
            with open(os.path.join(path, n), "rb") as f:
                h.update(n.encode() + f.read())
    return h.hexdigest()[:16]


@pytest.fixture(scope="module")
def sanitized():
    """(environment for a child process, directory) with sanitizer builds,
    rebuilt when a source changes."""
    from paper_2201_04058_amd import build as b
    import oracle
    d = os.path.join("/tmp", "atp_san_" + _sources_digest())
    lib, orc = os.path.join(d, "libatrapos.so"), os.path.join(d, "liboracle.so")
    if not (os.path.exists(lib) and os.path.exists(orc)):
        os.makedirs(d, exist_ok=True)
        b.build(sanitize=True, out=lib)
        oracle.build_sanitized(orc)
    env = dict(os.environ)
    env.update({"LD_PRELOAD": b.asan_runtime(), "ATP_LIBRARY": lib, "ATP_ORACLE_LIBRARY": orc,
                "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    return env, d


def test_planted_out_of_bounds_read_is_reported(sanitized):
    env, d = sanitized
    src, so = os.path.join(d, "planted.c"), os.path.join(d, "planted.so")
    with open(src, "w") as f:
        f.write("#include <stdlib.h>\nint planted(int i) { int *p = malloc(4 * sizeof(int)); int v = p[i]; "
                "free(p); return v; }\n")
    subprocess.check_call(["/opt/rocm/llvm/bin/clang", "-shared", "-fPIC", "-g", "-fsanitize=address", src, "-o", so])
    code = f"import ctypes; ctypes.CDLL({so!r}).planted(4)"
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr


def test_cpu_suite_passes_under_sanitizers(sanitized):
    env, d = sanitized
    probe = ("import ctypes, paper_2201_04058_amd as atp, oracle; atp.lib(); oracle._load(); "
             "print(atp.LIB_PATH, oracle._LIB, hasattr(ctypes.CDLL(None), '__asan_report_load8'))")
    r = subprocess.run([sys.executable, "-c", probe], env=env, cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.split() == [env["ATP_LIBRARY"], env["ATP_ORACLE_LIBRARY"], "True"]
    tests = sorted(f for f in os.listdir(os.path.join(ROOT, "tests"))
                   if f.startswith("test_") and f.endswith(".py") and f != os.path.basename(__file__))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        *[os.path.join("tests", f) for f in tests]],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert " passed" in r.stdout and "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail
