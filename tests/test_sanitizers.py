"""Sanitizer runs of the host code (CPU only, no GPU needed).

* The oracle (oracle/cams_oracle.c) built with gcc's AddressSanitizer and
  UndefinedBehaviorSanitizer, no recovery, runs small cases through every C
  entry point (tests/sanitize_oracle_cases.py: both restrictions, the four
  smoothers, C-AMS, Newton, histories, the conservative sweep, basis types
  B1-B3, boundary faces).
* The library built with clang's sanitizers on the host side only
  (-Xarch_host; device code as in the normal build) runs the ABI tests that
  need no GPU (tests/test_abi_cpu.py: validation, tables, workspace sizes,
  batch validation).

Each runs in a child process with the sanitizer runtime preloaded (the
interpreter itself is not instrumented) and leak detection off (the
interpreter's own allocations); a report ends the child with an error.  A
third test checks that the harness catches a heap overflow planted in a
four-line C file of its own.
"""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_SRC = os.path.join(ROOT, "oracle", "cams_oracle.c")
CASES = os.path.join(ROOT, "tests", "sanitize_oracle_cases.py")
GCC_SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def _gcc_runtime():
    return subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()


def _env(preload):
    env = dict(os.environ)
    env["LD_PRELOAD"] = preload
    env["ASAN_OPTIONS"] = "detect_leaks=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return env


def _clean(r):
    return r.returncode == 0 and "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_harness_catches_a_planted_overflow(tmp_path):
    src = tmp_path / "overflow.c"
    src.write_text("#include <stdlib.h>\nint main(void) {\n    int *a = malloc(4 * sizeof(int));\n"
                   "    a[4] = 1;\n    return a[0];\n}\n")
    exe = tmp_path / "overflow"
    subprocess.check_call(["gcc", "-O1", *GCC_SAN, str(src), "-o", str(exe)])
    r = subprocess.run([str(exe)], env=_env(""), capture_output=True, text=True, timeout=60)
    # UndefinedBehaviorSanitizer's object-size check or AddressSanitizer's
    # shadow check, whichever sees the store first
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr or "insufficient space" in r.stderr, r.stderr[-2000:]


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
                           "-Wno-alloc-size-larger-than", *GCC_SAN, ORACLE_SRC, "-o", str(lib), "-lm"])
    r = subprocess.run([sys.executable, CASES, str(lib)], env=_env(_gcc_runtime()), capture_output=True,
                       text=True, timeout=900, cwd=ROOT)
    assert _clean(r), r.stdout[-2000:] + r.stderr[-6000:]
    assert "oracle cases done" in r.stdout


def _clang_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_library_host_code_under_sanitizers(tmp_path):
    from paper_1705_05783_amd import build as B
    runtime = _clang_runtime()
    if runtime is None or not os.path.exists(B.HIPCC):
        pytest.skip("hipcc or clang's sanitizer runtime not installed")
    host_san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer", "-g"):
        host_san += ["-Xarch_host", f]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", B.CSRC]
    procs, objs = [], []
    for src in B.sources():
        obj = str(tmp_path / (os.path.splitext(os.path.basename(src))[0] + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([B.HIPCC, *[f for f in B.FLAGS if f != "-shared"], *host_san, *inc, "-c",
                                       src, "-o", obj], stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                      text=True))
    for p in procs:
        out, _ = p.communicate(timeout=900)
        assert p.returncode == 0, out[-4000:]
    lib = str(tmp_path / "libcams_san.so")
    subprocess.check_call([B.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                           "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", *objs, "-o", lib])
    child = ("import sys\n"
             f"sys.path.insert(0, {ROOT!r})\n"
             "import paper_1705_05783_amd._cams as C\n"
             f"C.LIB_PATH = {lib!r}\n"
             "import pytest\n"
             f"sys.exit(pytest.main(['-q', '-p', 'no:cacheprovider', {os.path.join(ROOT, 'tests', 'test_abi_cpu.py')!r}]))\n")
    r = subprocess.run([sys.executable, "-c", child], env=_env(runtime), capture_output=True, text=True,
                       timeout=900, cwd=ROOT)
    assert _clean(r), r.stdout[-4000:] + r.stderr[-6000:]
    assert " passed" in r.stdout and "failed" not in r.stdout and "error" not in r.stdout.lower()
