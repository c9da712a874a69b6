"""Host code under the address and undefined-behaviour sanitizers (CPU only): the checkpoint
format and the normalisation check of the learned closure (csrc/kcf_checkpoint.h), driven by
tests/sanitize_checkpoint.cpp with corrupted, truncated, oversized and garbage inputs."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2605_19796_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_checkpoint_parser_under_sanitizers(tmp_path):
    exe = tmp_path / "sanitize_checkpoint"
    build = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-I", CSRC, os.path.join(HERE, "sanitize_checkpoint.cpp"), "-o", str(exe)]
    subprocess.run(build, check=True, capture_output=True, text=True)
    # the sanitizer runtime need not be first in the library list of the process
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "ok: 0 failure(s)" in res.stdout
