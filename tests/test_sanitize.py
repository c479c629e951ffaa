"""Host code under the address and undefined-behaviour sanitizers (CPU only):
the oracle, driven through every entry point on random small pairs, and the
device-pool bookkeeping of the serving front end.  Any invalid access, leak
or undefined operation aborts the program and fails the test."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd_build, exe, token):
    subprocess.check_call(cmd_build)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert out.returncode == 0, out.stdout[-2000:] + out.stderr[-4000:]
    assert token in out.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=c99", "-pthread"] + SAN + [os.path.join(ROOT, "tests", "native", "oracle_driver.c"),
                                                  os.path.join(ROOT, "oracle", "sw_oracle.c"), "-o", exe],
         exe, "oracle sanitize ok")


def test_pool_allocator_under_sanitizers(tmp_path):
    exe = str(tmp_path / "pool_test")
    _run(["g++", "-std=c++17"] + SAN + ["-I", os.path.join(ROOT, "paper_2208_12350_amd", "csrc"),
                                        os.path.join(ROOT, "tests", "native", "pool_test.cpp"), "-o", exe],
         exe, "pool ok")
