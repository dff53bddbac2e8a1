"""The request server's policy (ct_sched.h) on the host: the arena allocator
against a granule bitmap (first fit, coalescing, exact byte accounting) and
the scheduler under a simulated clock -- first come, first served admission,
batch and slot limits, footprint admission with least-recently-used
eviction of complete layers only, checks that verify a complete layer of
their shape or run as tag generation, rejection of layers larger than the
arena, and no deadlock (every request completes exactly once)."""
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_sim(tmp_path):
    exe = str(tmp_path / "sched_sim")
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-Wall", "-Wextra", "-Werror",
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2311_04406_amd", "csrc"),
                           "-o", exe, os.path.join(ROOT, "tests", "sched_sim.cpp")])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr + r.stdout
    out = {}
    for line in r.stdout.splitlines():
        m = re.match(r"ok sched (\w+) (.*)", line)
        if m:
            out[m.group(1)] = {k: int(v) for k, v in (kv.split("=") for kv in m.group(2).split())}
    return r.stdout, out


def test_scheduler_simulation(tmp_path):
    text, s = run_sim(tmp_path)
    assert text.count("ok arena") == 3
    assert set(s) == {"roomy", "tight", "small", "serial", "dupes", "prep"}
    # preprocessing ahead of a TAG: the TAG runs the online phase only
    assert s["prep"] == {"prepared": 3, "online_only": 2}
    # ids of resident layers are refused, never taken over
    assert s["dupes"] == {"refused": 3, "resident": 2}
    # overload with room to spare: batches fill to the limit, every slot in use, nothing evicted
    assert s["roomy"]["max_batch"] == 8 and s["roomy"]["concurrent"] == 3 and s["roomy"]["evictions"] == 0
    assert s["roomy"]["multi"] > 0
    # a tight arena evicts complete layers; checks of evicted shapes run as tag generation
    assert s["tight"]["evictions"] > 0 and s["tight"]["converted"] > 0 and s["tight"]["rejected"] == 0
    assert s["tight"]["peak"] <= 900 << 20
    # layers larger than the arena are rejected, the others served
    assert s["small"]["rejected"] > 0 and s["small"]["peak"] <= 200 << 20
    # one slot, batch limit one: a plain queue
    assert s["serial"]["max_batch"] == 1 and s["serial"]["concurrent"] == 1
