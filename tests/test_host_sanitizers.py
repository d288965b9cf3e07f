"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no GPU).

Two builds of the repository's host code with both sanitizers, each exercised by tests that
already exist:
  - the oracle (g++), run through the oracle test files;
  - the C ABI library (hipcc: the sanitizers apply to the host pass only, the gfx950 device
    code is built as usual and never runs here), run through the argument-check and export
    tests, which reach every entry point's validation path without launching anything.
The Python interpreter is not instrumented, so each run preloads the compiler's ASan runtime
(which also carries the UBSan handlers) in a child process; leak detection is off because the
interpreter's own allocations would be reported.  Any sanitizer report aborts the child
(halt_on_error, -fno-sanitize-recover), so a clean exit means a clean run.  A planted heap
overflow and a planted signed overflow show that each toolchain's runtime does report."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def gcc_asan_runtime():
    try:
        p = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True,
                           text=True, check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def run_child(code, args, runtime, timeout):
    env = dict(os.environ, LD_PRELOAD=runtime, **SAN_ENV)
    return subprocess.run([sys.executable, "-c", code] + args, cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=timeout)


ORACLE_CHILD = """
import sys
sys.path.insert(0, {root!r})
from oracle import build
build.LIB = sys.argv[1]
import pytest
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + sys.argv[2:]))
"""

ABI_CHILD = """
import sys
sys.path.insert(0, {root!r})
from paper_2004_07954_amd import _lib
_lib.LIB_PATH = sys.argv[1]
import pytest
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider"] + sys.argv[2:]))
"""

PLANTED = {
    # (sanitizer, source, what its report names)
    "asan": ("address", r"""
#include <cstdio>
#include <cstdlib>
int main(int argc, char**) {
  double* a = (double*)std::malloc(4 * sizeof(double));
  for (int i = 0; i < 4; ++i) a[i] = i;
  std::printf("%f\n", a[3 + argc]);  // one past the end
  std::free(a);
  return 0;
}
""", "heap-buffer-overflow"),
    "ubsan": ("undefined", r"""
#include <climits>
#include <cstdio>
int main(int argc, char**) {
  int x = INT_MAX - 1;
  x += argc + 1;  // signed overflow
  std::printf("%d\n", x);
  return 0;
}
""", "signed integer overflow"),
}


@pytest.mark.slow
def test_planted_errors_are_reported(tmp_path):
    """The harness itself: a heap overflow and a signed overflow, built with each toolchain's
    sanitizer flags, must be reported (and end the run)."""
    compilers = [("g++", gcc_asan_runtime())]
    if os.path.exists("/opt/rocm/lib/llvm/bin/clang++"):
        compilers.append(("/opt/rocm/lib/llvm/bin/clang++", clang_asan_runtime()))
    ran = 0
    for cxx, rt in compilers:
        if rt is None:
            continue
        for name, (san, code, report) in PLANTED.items():
            src = tmp_path / (name + ".cpp")
            src.write_text(code)
            exe = tmp_path / (name + "_" + os.path.basename(cxx).replace("+", "p"))
            subprocess.run([cxx, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=" + san,
                            "-fno-sanitize-recover=all", str(src), "-o", str(exe)],
                           check=True, timeout=120)
            r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60,
                               env=dict(os.environ, **SAN_ENV))
            assert r.returncode != 0, (cxx, name, r.stdout)
            assert report in r.stderr, (cxx, name, r.stderr[-2000:])
            ran += 1
    if not ran:
        pytest.skip("no sanitizer runtime found")


@pytest.mark.slow
def test_oracle_under_asan_ubsan(tmp_path):
    rt = gcc_asan_runtime()
    if rt is None:
        pytest.skip("g++ has no AddressSanitizer runtime here")
    lib = tmp_path / "liboracle_san.so"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-o", str(lib),
           os.path.join(ROOT, "oracle", "wenozn_oracle.cpp"), "-lquadmath"]
    subprocess.run(cmd, check=True, timeout=300)
    tests = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    r = run_child(ORACLE_CHILD.format(root=ROOT), [str(lib)] + tests, rt, timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert " passed" in r.stdout


@pytest.mark.slow
def test_abi_host_code_under_asan_ubsan(tmp_path):
    rt = clang_asan_runtime()
    clangxx = "/opt/rocm/lib/llvm/bin/clang++"
    if rt is None or not os.path.exists(clangxx):
        pytest.skip("no clang AddressSanitizer runtime here")
    sys.path.insert(0, ROOT)
    from paper_2004_07954_amd import build as B
    flags = [f for f in B.HIP_FLAGS if f != "-O3"] + [
        "-O1", "-g", "-fno-omit-frame-pointer",
        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
        "-Xarch_host", "-fno-sanitize-recover=all"]
    objs, procs = [], []
    for src in B.sources():
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen(["hipcc", *flags, "-c", src, "-o", obj],
                                      stdout=subprocess.DEVNULL, stderr=subprocess.PIPE))
    for p in procs:
        _, err = p.communicate(timeout=900)
        assert p.returncode == 0, err.decode()[-3000:]
    lib = str(tmp_path / "libwenozn_san.so")
    # host link with clang++: the HIP runtime plus the sanitizer runtimes' shared form
    subprocess.run([clangxx, "-shared", "-fPIC", *objs, "-L/opt/rocm/lib", "-lamdhip64",
                    "-fsanitize=address,undefined", "-shared-libsan", "-o", lib],
                   check=True, timeout=300)
    tests = [os.path.join(ROOT, "tests", "test_abi_args.py"),
             os.path.join(ROOT, "tests", "test_abi_exports.py")]
    r = run_child(ABI_CHILD.format(root=ROOT), [lib] + tests, rt, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert " passed" in r.stdout
