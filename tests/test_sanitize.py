"""The host half of libtsf (host.cpp) and the oracle (oracle.c) built with
AddressSanitizer and UndefinedBehaviorSanitizer, each driven through all of
its operations by a small program (tests/sanitize/); any finding aborts the
program with a report.  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _build_and_run(tmp_path, cmd, exe):
    subprocess.check_call(cmd + ["-o", str(exe)], cwd=ROOT)
    env = dict(ENV)
    env.pop("LD_PRELOAD", None)
    proc = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert proc.returncode == 0, proc.stdout[-2000:] + proc.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in proc.stderr
    assert "runtime error" not in proc.stderr
    return proc.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_library_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, ["g++", "-std=c++17"] + SAN + [
        os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
        os.path.join(ROOT, "paper_2511_20317_amd", "csrc", "host.cpp")], tmp_path / "host_san")
    assert "host driver ok" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, ["gcc", "-std=c11"] + SAN + [
        os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
        os.path.join(ROOT, "oracle", "oracle.c"), "-lpthread"], tmp_path / "oracle_san")
    assert "oracle driver ok" in out
