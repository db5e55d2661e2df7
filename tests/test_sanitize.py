"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU): the
oracle, the server's scheduling core and the tile schedule, built with g++/gcc
(no device code) and run as a separate program."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                    reason="needs the host compilers")
def test_host_code_is_clean_under_sanitizers(tmp_path):
    obj = str(tmp_path / "oracle.o")
    exe = str(tmp_path / "sanitize_main")
    subprocess.run(["gcc", "-std=c11", "-c", *SAN, os.path.join(ROOT, "oracle", "ktau_oracle.c"),
                    "-o", obj], check=True)
    subprocess.run(["g++", "-std=c++17", *SAN,
                    "-I", os.path.join(ROOT, "paper_1704_03767_amd", "csrc"),
                    "-I", os.path.join(ROOT, "tests", "native"),
                    os.path.join(ROOT, "tests", "native", "sanitize_main.cpp"), obj, "-o", exe],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "passed" in r.stdout
