"""The host planner's thread pool and parallel loop (msdd.cpp: HostPool, parallel_for),
built on the CPU with ThreadSanitizer and driven by tests/host/pool_driver.cpp: every index
visited exactly once for 2000 loops of varied sizes and thread counts, an MsddError from a
worker rethrown on the caller, and two threads planning at once (one on the pool, the
other on threads of its own).  Any data race reported by the sanitizer fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "paper_2106_06404_amd", "csrc", "msdd.cpp")


def _pool_source():
    s = open(SRC).read()
    a = s.index("class HostPool {")
    b = s.index("// An element group (a subdomain or a patch)")
    return s[a:s.rindex("// ----", a, b)]


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host compiler")
def test_planner_pool_under_thread_sanitizer(tmp_path):
    driver = open(os.path.join(HERE, "host", "pool_driver.cpp")).read()
    src = tmp_path / "pool.cpp"
    src.write_text(driver.replace("// @@POOL@@\n", _pool_source()))
    exe = tmp_path / "pool"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
                           str(src), "-o", str(exe)])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:exitcode=66")
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok"), out.stdout
