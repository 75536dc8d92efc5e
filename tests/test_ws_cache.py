"""The library-cached workspace policy (csrc/ws_cache.h), checked on the host
with a stand-in device: a caller's lease keeps the buffer alive until its
launches are enqueued, a request that grows the buffer waits for the lease and
for the device before freeing, and each device has its own buffer."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1710_08471_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_workspace_cache_policy(tmp_path):
    exe = tmp_path / "ws_cache_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-pthread", "-I", CSRC,
                    os.path.join(HERE, "host", "ws_cache_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
