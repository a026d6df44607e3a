"""The oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only): the oracle's pins run against an
instrumented build of the oracle, and the host-side validation tests run
against a build of the library whose host code is instrumented (the device
code is unchanged and never runs here).  Any sanitizer report aborts the
child process, which fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(env_extra, test_file):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1",
               OMP_NUM_THREADS="2", **env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", test_file)], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]


def test_oracle_pins_under_asan_ubsan():
    import oracle
    so = oracle.build_sanitized()
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.isabs(asan):
        pytest.skip("gcc's ASan runtime not found")
    _run({"NNDTW_ORACLE_LIB": so, "LD_PRELOAD": asan}, "test_oracle_pins.py")


def test_host_validation_under_asan_ubsan(tmp_path):
    from paper_1808_09617_amd import build as hipbuild
    so = hipbuild.build_host_sanitized(str(tmp_path / "libnndtw_san.so"))
    rt = subprocess.check_output([hipbuild.HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        import glob
        found = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        if not found:
            pytest.skip("clang's ASan runtime not found")
        rt = found[0]
    _run({"NNDTW_LIB": so, "LD_PRELOAD": rt}, "test_abi_cpu.py")
