"""The batched runtime's launch schedule (which pipeline runs each batch,
and the fork / join / fold order of the streams) is plain host code: it is
built with g++ and the address and undefined-behaviour sanitizers and driven
over plan shapes including more pipelines than batches, single-batch
replicas, empty plans and zero replicas."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1503_01725_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_schedule_under_sanitizers(tmp_path):
    exe = str(tmp_path / "schedule_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", f"-I{CSRC}",
           os.path.join(HERE, "schedule_driver.cpp"), os.path.join(CSRC, "schedule.cpp"),
           "-o", exe]
    subprocess.check_call(cmd)
    # a library preloaded into every process may load ahead of the sanitizer
    # runtime; the link-order check would then refuse to start
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
