"""Host logic of the translation step (rrq_consts.cpp, build_order_tables): the term lists
of every (l, m) split into 1, 2 or 4 pieces on aligned adjacent slots, the packed operand
offsets vq_rec(n) << 8 | r and the coefficients in 4-term chunks, zero-padded.  A small C++
checker (tests/host/order_tables_check.cpp) is compiled with g++ against the host source and
run; it needs no GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_translation_slot_tables(tmp_path):
    exe = tmp_path / "order_tables_check"
    src = [os.path.join(HERE, "host", "order_tables_check.cpp"),
           os.path.join(ROOT, "paper_2411_08342_amd", "csrc", "rrq_consts.cpp")]
    # the header's __host__ __device__ qualifiers are empty for the host compiler
    cmd = ["g++", "-std=c++17", "-O1", "-D__host__=", "-D__device__=",
           "-I", os.path.join(ROOT, "paper_2411_08342_amd", "csrc")] + src + ["-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True)
    print(res.stdout)
    assert res.returncode == 0, res.stdout + res.stderr
    lines = {l.split()[0]: dict(kv.split("=") for kv in l.split()[1:])
             for l in res.stdout.splitlines() if l.startswith("q=")}
    assert set(lines) == {"q=4", "q=5", "q=6", "q=8", "q=10"}
    # order 8 (the benchmark): 36 lists, 574 terms, 60 slots of at most 16 terms, one pass of
    # a 256-lane workgroup for 4 targets
    o8 = lines["q=8"]
    assert (o8["lists"], o8["terms"], o8["slots"], o8["longest"], o8["chunks"], o8["passes_T4"]) == \
        ("36", "574", "60", "16", "4", "1")
