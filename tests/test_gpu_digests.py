"""Bit-exact parity of every benchmark configuration at full size, in both
protocols, against digests the oracle wrote (tests/golden/make_digests.py):
every dealt share and tag of every party, the opened E, U, D, the output
shares and tags of every party (and the truncated outputs), the compact-tag
vectors, and the exact check values of every party -- from the fused check
records of a captured plan (the launch configuration bench.py times) and from
the standalone verification.  No value crosses from the GPU path into the
expected results: the digests were computed by the oracle alone.

Canonical bytes of an array: row-major elements as little-endian 64-bit
limbs, (lo, hi) for k = s = 64 and lo alone for k = s = 32 -- the layout of
the library's buffers -- and a digest is the first 32 hex digits of SHA-256."""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import json
import os

import pytest
import torch

from gpu_util import free, say

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "digests")
CASES = sorted(f[:-5] for f in os.listdir(GOLD) if f.endswith(".json")) if os.path.isdir(GOLD) else []
MODE_IDS = {"spdz2k": 0, "compact": 1}
# configurations also run as one persistent launch (two parties, matrix-core
# layers only, nothing compressed along M)
PERSISTENT_CASES = ("batched", "transformer")
_POOL = cf.ThreadPoolExecutor(max_workers=16)


def _sha(buf) -> str:
    return hashlib.sha256(buf).hexdigest()[:32]


def digests(named):
    """{name: digest} of device tensors; copies run one at a time, the hashing
    on a thread pool (hashlib releases the interpreter lock)."""
    futs = {}
    for name, t in named:
        host = t.detach().contiguous().cpu().numpy()
        futs[name] = _POOL.submit(_sha, host)
    return {n: f.result() for n, f in futs.items()}


def dealt_tensors(gl, f):
    names = ["X", "tX", "A", "tA", "Y", "tY", "B", "tB", "C", "tC", "R", "tR"] + (["Rf", "tRf"] if f else [])
    return [(f"{n}/{p}", gl[n][p]) for n in names for p in range(gl.parties)]


def online_tensors(gl, mode_name, f, along_m):
    out = [("E", gl["E"]), ("U", gl["U"]), ("D", gl["D"])]
    for n in ["Z", "tZ"] + (["Zf", "tZf"] if f else []):
        out += [(f"{n}/{p}", gl[n][p]) for p in range(gl.parties)]
    if mode_name == "compact":
        parts = gl.cvec_parts()
        single = ["Ec", "Dc", "EUc"] if along_m else ["Uc", "Dc", "EUc"]
        per = ["tAc", "tCc", "tRc", "tZc", "tDc"] if along_m else ["tBc", "tCc", "tRc", "tZc", "tDc"]
        out += [(f"cvec/{n}", parts[n]) for n in single]
        out += [(f"cvec/{n}/{p}", parts[f"{n}{p}"]) for n in per for p in range(gl.parties)]
    return out


def compare(got: dict, want: dict, what: str):
    assert set(got) == set(want), (what, sorted(set(got) ^ set(want)))
    bad = sorted(n for n in want if got[n] != want[n])
    assert not bad, f"{what}: {len(bad)} arrays differ from the oracle: {bad[:8]}"


def check_records(res, want_cs, parties, what):
    for w in range(3):
        for p in range(parties):
            assert res.cs[w][p] == int(want_cs[w][p], 16), f"{what}: check value W={w} party {p}"
    assert res.accept, f"{what}: honest run rejected"


@pytest.mark.parametrize("case", CASES)
def test_config_digests(case):
    from paper_2311_04406_amd import Context
    from paper_2311_04406_amd.binding import RESULT_WORDS

    g = json.load(open(os.path.join(GOLD, case + ".json")))
    kbits, f, parties, lays = g["kbits"], g["f"], g["parties"], g["layers"]
    say(f"[digests] {case}: {len(lays)} layers, k={kbits}, f={f}, parties={parties}, modes {g['modes']}")
    ctx = Context(device=0, key_seed=g["key_seed"], max_layers=max(256, len(lays)), kbits=kbits, parties=parties)
    try:
        layers = [ctx.layer(l["M"], l["K"], l["N"], l["seed"], l["layer_id"], f=f, compress=g["compress_setting"],
                            conv=tuple(l["conv"]) if l["conv"] else None) for l in lays]
        ctx.gen_triple_tags(layers)
        torch.cuda.synchronize()
        for gl, l in zip(layers, lays):
            compare(digests(dealt_tensors(gl, f)), l["dealt"], f"{case} {l['name']} dealt")
        say(f"  dealt arrays of {len(lays)} layers match")
        for mname in g["modes"]:
            mode = MODE_IDS[mname]
            out = torch.zeros(RESULT_WORDS * len(layers), dtype=torch.int64, device="cuda:0")
            if g["config"] == "batched":
                ctx.autotune(mode, layers)   # the launch configuration bench.py chooses
            plan = ctx.plan(mode, layers, out)   # the captured step bench.py times
            plan.launch()
            torch.cuda.synchronize()
            plan.close()
            fused = Context.decode_results(out, len(layers), parties)
            for gl, l, r in zip(layers, lays, fused):
                along_m = mname == "compact" and l["compress"][mname] == 1
                assert gl.along_m == along_m or mname != "compact", (case, l["name"], "compressed dimension")
                compare(digests(online_tensors(gl, mname, f, along_m)), l["online"][mname],
                        f"{case} {l['name']} {mname}")
                check_records(r, l["cs"][mname], parties, f"{case} {l['name']} {mname} fused")
            if case in PERSISTENT_CASES:
                # the same step as one persistent launch, into cleared outputs
                from paper_2311_04406_amd.binding import LAUNCH_PERSISTENT, LAUNCH_STAGED
                for gl in layers:
                    for n, t in online_tensors(gl, mname, f, False):
                        t.zero_()
                    gl["cvec"].zero_()
                out.zero_()
                ctx.set_launch(LAUNCH_PERSISTENT)
                try:
                    plan = ctx.plan(mode, layers, out)
                finally:
                    ctx.set_launch(LAUNCH_STAGED)
                plan.launch()
                torch.cuda.synchronize()
                plan.close()
                fused = Context.decode_results(out, len(layers), parties)
                for gl, l, r in zip(layers, lays, fused):
                    compare(digests(online_tensors(gl, mname, f, False)), l["online"][mname],
                            f"{case} {l['name']} {mname} persistent")
                    check_records(r, l["cs"][mname], parties, f"{case} {l['name']} {mname} persistent")
                say(f"  {mname}: the persistent launch matches too")
            st, res = ctx.mac_check(mode, layers)
            assert st == 0, (case, mname, "standalone check rejected")
            for l, r in zip(lays, res):
                check_records(r, l["cs"][mname], parties, f"{case} {l['name']} {mname} standalone")
            say(f"  {mname}: every output array and check value matches")
        del layers
    finally:
        ctx.close()
        free()
