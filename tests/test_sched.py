"""The request server's admission code (csrc/rc_sched.hpp) on a simulated
executor, on the CPU: admission in arrival order with backfill, the budget and
the ray cap of a round, refusal of requests larger than the budget, bounded
overtaking of the oldest request, latency accounting, and the first-fit arena
that holds library-allocated outputs.  The simulation is built with the
address and undefined-behaviour sanitizers (host code only, g++)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2503_01471_amd", "csrc")
SIM = os.path.join(ROOT, "tests", "sched_sim.cpp")


def _build(tmp_path, sanitize):
    exe = str(tmp_path / ("sim_san" if sanitize else "sim"))
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror", "-I", CSRC, SIM, "-o", exe]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    subprocess.check_call(cmd)
    return exe


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert p.returncode == 0, p.stdout + p.stderr
    assert p.stdout.strip().endswith("ALL OK"), p.stdout
    return {m.group(1): dict(kv.split("=") for kv in m.group(2).split())
            for m in re.finditer(r"^(\w+) (.*)$", p.stdout, re.M) if m.group(1) != "ALL"}


@pytest.mark.parametrize("sanitize", [False, True], ids=["plain", "asan_ubsan"])
def test_admission_simulation(tmp_path, sanitize):
    res = _run(_build(tmp_path, sanitize))
    # arrival order where nothing forces backfill
    assert res["plain_fifo"]["inversions"] == "0"
    assert res["batched_roomy_fifo"]["inversions"] == "0"
    # a tight budget makes later requests fill in ahead of earlier ones, boundedly
    assert int(res["batched_tight_budget"]["inversions"]) > 0
    assert int(res["batched_large_heads"]["max_bypass"]) <= 8
    assert int(res["batched_refusals"]["refused"]) == 100
    # the stated arrival rate is above the executor's throughput: latency is backlog
    assert float(res["batched_stated_rate"]["p99_ms"]) > float(res["batched_roomy_fifo"]["p99_ms"])
