"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (oracle.c) and the input generator (synth.c), rebuilt with
  gcc -fsanitize=address,undefined, run the oracle pins and the generator,
  volume and owner-grouping host tests in a child process.
* The C-ABI library's host code (argument checks, plan handles, variant and
  shape rules), rebuilt with -fsanitize=address,undefined on the host pass
  only (the device code is the ordinary build), runs the ABI tests.
* A positive control: a planted heap overflow in a throwaway C library must
  make the same harness fail, so the harness cannot pass by being deaf.

Python itself is not instrumented, so each child preloads the sanitizer
runtime that matches the compiler (gcc's libasan, clang's for hipcc); leak
checking is off (the interpreter keeps its allocations at exit).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer", "-g", "-O1"]
ENV_SAN = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _runtime(cmd):
    try:
        p = subprocess.run(cmd, capture_output=True, text=True, check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _gcc_runtimes():
    a = _runtime(["gcc", "-print-file-name=libasan.so"])
    u = _runtime(["gcc", "-print-file-name=libubsan.so"])
    if not (a and u):
        pytest.skip("gcc's sanitizer runtimes are not installed")
    return f"{a}:{u}"


def _child(args, preload, extra_env, timeout=900):
    env = dict(os.environ, LD_PRELOAD=preload, **ENV_SAN, **extra_env)
    return subprocess.run([sys.executable, *args], cwd=ROOT, env=env, capture_output=True,
                          text=True, timeout=timeout)


@pytest.fixture(scope="module")
def gcc_libs(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    oracle_so = str(d / "liboracle_san.so")
    synth_so = str(d / "libsynth_san.so")
    subprocess.run(["gcc", *SAN, "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
                    "-fno-fast-math", os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o",
                    oracle_so], check=True)
    subprocess.run(["gcc", *SAN, "-fPIC", "-shared", "-fopenmp", "-std=c11",
                    os.path.join(ROOT, "paper_2404_19638_amd", "synth", "synth.c"), "-o",
                    synth_so], check=True)
    return d, oracle_so, synth_so


def test_positive_control_catches_a_heap_overflow(gcc_libs):
    d, _, _ = gcc_libs
    src = d / "planted.c"
    src.write_text("#include <stdlib.h>\n"
                   "int planted(int n) { int* a = malloc(n * sizeof(int));\n"
                   "  a[n] = 1; int r = a[0]; free(a); return r; }\n")
    so = str(d / "libplanted.so")
    subprocess.run(["gcc", *SAN, "-fPIC", "-shared", str(src), "-o", so], check=True)
    r = _child(["-c", f"import ctypes; ctypes.CDLL({so!r}).planted(8)"], _gcc_runtimes(), {})
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr, r.stderr[-2000:]


def test_oracle_and_generator_pins_under_asan_ubsan(gcc_libs):
    _, oracle_so, synth_so = gcc_libs
    check = ("import oracle, paper_2404_19638_amd.synth as s; "
             f"assert oracle._SO == {oracle_so!r} and s._SO == {synth_so!r}")
    env = {"ORACLE_SO": oracle_so, "SYNTH_SO": synth_so}
    r = _child(["-c", check], _gcc_runtimes(), env)
    assert r.returncode == 0, r.stderr[-2000:]
    # the 2^32-pattern bfloat16 sweep is left out (minutes under ASan)
    r = _child(["-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                "-k", "not all_fp32_patterns", "tests/test_oracle_pins.py",
                "tests/test_synth.py", "tests/test_volume_host.py", "tests/test_grouped_host.py",
                "tests/test_selector_oracle.py"], _gcc_runtimes(), env)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "Sanitizer" not in r.stderr, tail
    assert " passed" in r.stdout


def test_library_host_code_under_asan_ubsan(tmp_path_factory):
    """The C ABI's host-side validation: every ABI test against the library
    built with -Xarch_host -fsanitize=address,undefined."""
    from paper_2404_19638_amd import build as hipbuild
    rt = _runtime([os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang"),
                   "-print-file-name=libclang_rt.asan-x86_64.so"])
    if rt is None:
        pytest.skip("clang's ASan runtime is not installed")
    d = tmp_path_factory.mktemp("san_hip")
    so = str(d / "libspc3d_san.so")
    flags = []
    for f in SAN:
        flags += ["-Xarch_host", f]
    hipbuild.build(so=so, build_dir=str(d / "build"), extra=flags)
    r = _child(["-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "tests/test_abi.py"], rt,
               {"SPC3D_LIB": so})
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "Sanitizer" not in r.stderr, tail
    assert " passed" in r.stdout
