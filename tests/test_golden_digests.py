"""The stored full-size digests (tests/golden/digests/) are the oracle's: the
smallest layer of every case is recomputed with the oracle now and must give
the stored digests and check values; the small FC case is recomputed whole.
Also: the stored check values of every layer pass the check (their per-party
shares sum to zero), and every case covers the arrays the GPU test compares."""
import importlib.util
import json
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "digests")


def _maker():
    spec = importlib.util.spec_from_file_location("make_digests", os.path.join(HERE, "golden", "make_digests.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


MD = _maker()
CASES = sorted(f[:-5] for f in os.listdir(GOLD) if f.endswith(".json"))


def load(case):
    return json.load(open(os.path.join(GOLD, case + ".json")))


def test_every_case_is_stored():
    assert set(CASES) == set(MD.CASES), sorted(set(CASES) ^ set(MD.CASES))


@pytest.mark.parametrize("case", CASES)
def test_stored_checks_accept_and_cover(case):
    g = load(case)
    mask = (1 << (2 * g["kbits"])) - 1
    P = g["parties"]
    for l in g["layers"]:
        assert len(l["dealt"]) == P * (12 + (2 if g["f"] else 0)), l["name"]
        for m in g["modes"]:
            for w in range(3):
                assert sum(int(v, 16) for v in l["cs"][m][w]) & mask == 0, (l["name"], m, w)
            n_out = 3 + P * (2 + (2 if g["f"] else 0))
            if m == "compact":
                n_out += 3 + 5 * P
            assert len(l["online"][m]) == n_out, (l["name"], m)


@pytest.mark.parametrize("case", CASES)
def test_smallest_layer_recomputed_by_oracle(case):
    g = load(case)
    config = MD.CASES[case][0]
    specs = MD.W.CONFIGS[config]()
    small = min(range(len(specs)), key=lambda i: specs[i].mkn * (1 + specs[i].K))
    only = {small} if case != "fc_small" else None
    rec = MD.run_case(case, threads=4, only=only)
    stored = {l["name"]: l for l in g["layers"]}
    for l in rec["layers"]:
        s = stored[l["name"]]
        for key in ("M", "K", "N", "seed", "layer_id", "conv", "compress", "dealt", "online", "cs"):
            assert l[key] == s[key], (case, l["name"], key)
