"""Host sanitizers over the CPU tests (no GPU needed).

* The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (g++) runs
  every oracle pin test.
* The library's host code built with both sanitizers (hipcc, sanitizers on the host
  compilation only; device code unchanged) runs the ABI and binding tests, which
  call every entry point's argument checks and the context set-up.

Each runs in a child process that preloads the sanitizer runtime; a report of either
sanitizer fails the test (UBSan is built not to recover).
"""

import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.slow

REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _child(env_extra: dict, argv: list, timeout: int) -> subprocess.CompletedProcess:
    env = dict(os.environ)
    env.update(env_extra)
    return subprocess.run([sys.executable, *argv], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=timeout)


def _check(r: subprocess.CompletedProcess):
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    for rep in REPORTS:
        assert rep not in out, out[-4000:]


def _gcc_runtime(name: str) -> str:
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"gcc's {name} is not installed")
    return path


def test_oracle_under_asan_and_ubsan(oracle_mod):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    oracle_mod.build(sanitize=True)
    env = {"LD_PRELOAD": f"{_gcc_runtime('libasan.so')} {_gcc_runtime('libubsan.so')}",
           "GS2D_ORACLE_SANITIZED": "1", "ASAN_OPTIONS": "detect_leaks=0",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}
    probe = _child(env, ["-c", "import oracle; print(oracle._load()._name)"], 120)
    _check(probe)
    assert probe.stdout.strip().endswith("liboracle_san.so"), probe.stdout
    files = sorted(os.path.relpath(f, ROOT) for f in glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py"))
                   if not f.endswith("test_oracle_mutations.py"))
    _check(_child(env, ["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *files], 900))


def test_library_host_code_under_asan_and_ubsan():
    from paper_2506_00970_amd import build as b

    try:
        b.hipcc()
    except RuntimeError:
        pytest.skip("no hipcc")
    lib = b.build(variant="sanitize_host")
    out = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in out and "__ubsan_handle" in out, "host code is not instrumented"
    env = {"LD_PRELOAD": b.asan_runtime(), "GS2D_LIB": lib, "ASAN_OPTIONS": "detect_leaks=0",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}
    probe = _child(env, ["-c", "from paper_2506_00970_amd import _lib; _lib.load(); print(_lib.LIB_PATH)"], 120)
    _check(probe)
    assert probe.stdout.strip() == lib, probe.stdout
    _check(_child(env, ["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "tests/test_abi.py",
                        "tests/test_map_binding.py"], 600))
