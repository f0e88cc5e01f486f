"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code (CPU).

* The C ABI's CPU checks (tests/test_abi_cpu.py: validation, error paths,
  host helpers, refused foreign handles) run against libtpcf_san.so, whose host
  code is instrumented (every -fsanitize= behind -Xarch_host; device code as
  usual), with clang's ASan runtime preloaded.
* The oracle's pins run against liboracle_san.so (gcc, -fsanitize=address,
  undefined), with gcc's ASan runtime preloaded.

Undefined behaviour aborts (-fno-sanitize-recover) and an ASan report exits
non-zero, so either fails the child pytest run and this test. The two builds
run in separate processes: the two compilers' ASan runtimes cannot share one.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))


def _stale(out, srcs):
    return not os.path.exists(out) or any(os.path.getmtime(out) < os.path.getmtime(s) for s in srcs)


def _run(env_extra, tests):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    # the runtime really is loaded (a child without it would pass vacuously)
    probe = subprocess.run([sys.executable, "-c", "import ctypes; ctypes.CDLL(None)['__asan_report_load1']"],
                           env=env, capture_output=True, text=True, timeout=120)
    assert probe.returncode == 0, probe.stderr[-2000:]
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"]
                         + [os.path.join(HERE, t) for t in tests],
                         env=env, capture_output=True, text=True, timeout=900, cwd=ROOT)
    tail = (res.stdout + res.stderr)[-4000:]
    assert res.returncode == 0, tail
    assert "passed" in res.stdout, tail
    return tail


def _exports_asan(lib):
    out = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    return "__asan_" in out and "__ubsan_" in out


def test_abi_under_asan_ubsan():
    from paper_2408_03036_amd import build as B
    csrc = os.path.join(ROOT, "paper_2408_03036_amd", "csrc")
    srcs = [os.path.join(csrc, f) for f in os.listdir(csrc)]
    if _stale(B.OUT_SAN, srcs):
        B.build(sanitize=True)
    assert _exports_asan(B.OUT_SAN), "libtpcf_san.so is not instrumented"
    _run({"LD_PRELOAD": B.asan_runtime(), "TPCF_LIBRARY": B.OUT_SAN}, ["test_abi_cpu.py"])


def test_oracle_pins_under_asan_ubsan():
    from oracle import oracle as O
    lib = O.build(sanitize=True)
    assert _exports_asan(lib), "liboracle_san.so is not instrumented"
    gcc_asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(gcc_asan):
        pytest.skip("gcc's libasan is not installed")
    _run({"LD_PRELOAD": gcc_asan, "ORACLE_LIBRARY": lib},
         ["test_oracle_pins.py", "test_xi_oracle_pins.py", "test_edge_oracle_pins.py", "test_cov_oracle_pins.py"])
