"""The request server's host bookkeeping (pool allocator, ticket board),
built with g++ and the address and undefined-behaviour sanitizers and run on
the host: no GPU involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_server_book_under_sanitizers(tmp_path):
    exe = tmp_path / "server_book_test"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=address,undefined",
           "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "paper_2203_02798_amd", "csrc"),
           os.path.join(ROOT, "tests", "server_book_test.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1")
    p = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "server_book ok" in p.stdout
