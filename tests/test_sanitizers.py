"""AddressSanitizer and UBSan over the host code: the C oracle (rebuilt with
both sanitizers and driven by the oracle's own tests), and the host side of
the C ABI (libspx_hostsan.so: host code instrumented, gfx950 code as usual)
driven by tests/sanitize/abi_driver.cpp. The host-only checks run here; the
server's pool, worker thread and request bookkeeping run on the GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "sanitize", "abi_driver_hostsan")
ORACLE_TESTS = ["test_oracle_spmv.py", "test_oracle_formats.py", "test_oracle_solvers.py", "test_oracle_sellp.py",
                "test_oracle_block_jacobi.py", "test_oracle_bicg_pipecg.py", "test_oracle_omp.py"]
FINDINGS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _gcc_lib(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                          check=True).stdout.strip()


def _no_findings(out):
    for f in FINDINGS:
        assert f not in out, out[-6000:]


def test_oracle_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "oracle_asan.so")
    src = [os.path.join(ROOT, "oracle", f) for f in ("spx_oracle.c", "spx_oracle_omp.c")]
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
                    "-fno-fast-math", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-o", lib, *src, "-lm"], check=True)
    env = dict(os.environ)
    env.update(LD_PRELOAD=f"{_gcc_lib('libasan.so')}:{_gcc_lib('libubsan.so')}", SPX_ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        *[os.path.join(ROOT, "tests", t) for t in ORACLE_TESTS]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    _no_findings(out)
    assert " passed" in out


def _run_driver(mode, timeout):
    if not os.path.exists(DRIVER):
        pytest.fail("tests/sanitize/abi_driver_hostsan is not built (build() builds it)")
    env = dict(os.environ)
    # the HIP runtime keeps allocations until exit; leaks are not what is checked
    env.update(ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    print(f"case abi_driver {mode}", flush=True)
    r = subprocess.run([DRIVER, mode], env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert r.returncode == 0, out[-6000:]
    _no_findings(out)
    assert "abi_driver ok" in out
    return out


def test_abi_host_checks_under_asan_ubsan():
    out = _run_driver("host", 120)
    assert "validate_csr_host: repeated column" in out


@pytest.mark.gpu
def test_serve_host_side_under_asan_ubsan():
    out = _run_driver("serve", 300)
    assert "served results checked on the host" in out
