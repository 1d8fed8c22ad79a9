"""Host logic of the library tested on the CPU: the stack-memory pool
(first-fit chunks with merging, an exact-size cache of freed regions),
built with the host compiler under AddressSanitizer and run with a
malloc-backed allocator; the host worker threads under ThreadSanitizer."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_region_pool(tmp_path):
    exe = str(tmp_path / "pool_test")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-I", os.path.join(ROOT, "paper_2404_01585_amd", "csrc"),
                           os.path.join(HERE, "host_pool_test.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "ok"


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
@pytest.mark.parametrize("sanitizer", ["thread", "address,undefined"])
def test_host_workers(tmp_path, sanitizer):
    exe = str(tmp_path / "workers_test")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={sanitizer}", "-pthread",
                           "-I", os.path.join(ROOT, "paper_2404_01585_amd", "csrc"),
                           os.path.join(HERE, "host_workers_test.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "ok"


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_step_checks(tmp_path):
    """The host-side checks of a step's segment table and tile map (the
    check_steps tunable) accept a well-formed step and catch every way one
    could index outside its buffers."""
    exe = str(tmp_path / "check_test")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-I", os.path.join(ROOT, "paper_2404_01585_amd", "csrc"),
                           os.path.join(HERE, "host_check_test.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "ok"
