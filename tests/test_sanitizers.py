"""CPU hardening: the C oracle and the host side of the HIP library, built
with AddressSanitizer and UndefinedBehaviorSanitizer, run their CPU tests.

* oracle.c is built with gcc's ASan/UBSan (any UBSan finding aborts) and the
  oracle pins run against it (ORACLE_LIB names the build).
* libsgr is built with ASan/UBSan on host code only (device code is built as
  usual): the argument validation, workspace planning and launch set-up of
  the C ABI.  The ABI and binding host tests run against it (SGR_LIB names
  the build); they call every entry point with valid and invalid arguments,
  and with no GPU nothing is launched.

Each run is a child process with the matching sanitizer runtime preloaded
(Python itself is not instrumented) and leak detection off (the interpreter
keeps its allocations until exit).  A planted out-of-bounds read in a tiny
program built the same way checks that the sanitizer reports at all.
"""
import glob
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_00225_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
GCC_SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
# host-only sanitizers for hipcc: each flag goes to the host compilation
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _gcc_runtime(name):
    return subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()


def _clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.fixture(scope="module")
def tmp():
    with tempfile.TemporaryDirectory(prefix="sgr_san_") as d:
        yield d


def _run(env_extra, args, timeout=900):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env.setdefault("OMP_NUM_THREADS", "4")
    return subprocess.run([sys.executable, *args], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=timeout)


def test_sanitizer_reports_a_planted_overflow(tmp):
    src = os.path.join(tmp, "planted.c")
    with open(src, "w") as f:
        f.write("#include <stdlib.h>\nint main(int c, char **v) { int *a = malloc(4 * sizeof(int));"
                " int r = a[c + 3]; free(a); return r; }\n")
    exe = os.path.join(tmp, "planted")
    subprocess.check_call(["gcc", *GCC_SAN, "-o", exe, src])
    r = subprocess.run([exe], capture_output=True, text=True, env={**os.environ, "ASAN_OPTIONS": "detect_leaks=0"})
    # ASan (heap-buffer-overflow) or UBSan's object-size check (runtime error) reports it
    assert r.returncode != 0 and ("heap-buffer-overflow" in r.stderr or "runtime error" in r.stderr), r.stderr


def test_oracle_pins_under_asan_ubsan(tmp):
    lib = os.path.join(tmp, "liboracle_san.so")
    subprocess.check_call(["gcc", *GCC_SAN, "-fopenmp", "-fPIC", "-shared", "-std=c11", "-fno-fast-math",
                           "-ffp-contract=off", "-o", lib, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    pre = ":".join([_gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")])
    r = _run({"LD_PRELOAD": pre, "ORACLE_LIB": lib},
             ["-c", "from oracle import oracle as O; O.lib(); print(O._LIB)"])
    assert r.returncode == 0 and r.stdout.strip() == lib, r.stderr[-2000:]
    r = _run({"LD_PRELOAD": pre, "ORACLE_LIB": lib},
             ["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "tests/test_oracle_pins.py",
              "tests/test_oracle_branch_pins.py", "tests/test_compare_host.py"])
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])


def test_abi_host_layer_under_asan_ubsan(tmp):
    rt = _clang_asan_runtime()
    if rt is None or not os.path.exists(HIPCC):
        pytest.skip("no hipcc / clang ASan runtime")
    objs, procs = [], []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        obj = os.path.join(tmp, os.path.basename(src) + ".o")
        cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
               "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC, *HOST_SAN,
               "-c", src, "-o", obj]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE))
        objs.append(obj)
    for p in procs:
        _, err = p.communicate(timeout=900)
        assert p.returncode == 0, err[-2000:]
    lib = os.path.join(tmp, "libsgr_san.so")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib, *objs])
    r = _run({"LD_PRELOAD": rt, "SGR_LIB": lib},
             ["-c", "from paper_2506_00225_amd import _lib; _lib.lib(); print(_lib.LIB_PATH)"])
    assert r.returncode == 0 and r.stdout.strip() == lib, r.stderr[-2000:]
    r = _run({"LD_PRELOAD": rt, "SGR_LIB": lib},
             ["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "tests/test_abi_host.py",
              "tests/test_binding_host.py"])
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "passed" in r.stdout
