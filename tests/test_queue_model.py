"""CPU model of the persistent batched launch's work queue
(paper_1109_6885_amd/csrc/queue.hpp): host threads run the kernel's
protocol (one ticket counter, the kernel's decode, the same wait targets,
relaxed atomics and fences) on random plans with 1 to 16 workers and random
delays; every item must run once, after everything it depends on, and every
run must end.  A copy with a planted off-by-one wait target must fail."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "queue_model.cpp")
INC = os.path.join(ROOT, "paper_1109_6885_amd", "csrc")


def _build(tmp_path, text=None, name="queue_model"):
    src = SRC
    if text is not None:
        src = str(tmp_path / (name + ".cpp"))
        with open(src, "w") as f:
            f.write(text)
    exe = str(tmp_path / name)
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-pthread", "-Wall", "-I", INC, "-o", exe,
                           src])
    return exe


def test_queue_protocol_model(tmp_path):
    exe = _build(tmp_path)
    res = subprocess.run([exe, "7", "30"], capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "0 failures" in res.stdout


def test_queue_model_catches_a_planted_wait_target(tmp_path):
    """The model has teeth: waiting for one item less than the column's
    earlier items lets items start before their inputs are done."""
    text = open(SRC).read()
    good = "ok = wait_ge(R.col_done[it.col], P.cum[(size_t)it.col * kNumPhases + it.phase]);"
    assert good in text
    bad = ("{ const uint32_t c = P.cum[(size_t)it.col * kNumPhases + it.phase]; "
           "ok = wait_ge(R.col_done[it.col], c ? c - 1 : 0); }")
    exe = _build(tmp_path, text.replace(good, bad), "queue_model_planted")
    res = subprocess.run([exe, "3", "8"], capture_output=True, text=True, timeout=600)
    assert res.returncode != 0, res.stdout
