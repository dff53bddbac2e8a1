#!/usr/bin/env python3
"""Writes the expected results of the benchmark configurations at full size,
computed by the oracle alone: SHA-256 digests of every array of every layer
(the dealt shares and tags of each party, the opened E, U, D, the output
shares and tags Z, tZ of each party, the truncated outputs, the compact-tag
vectors) and the exact check values of every party, for each protocol.

    python3 tests/golden/make_digests.py [case ...] [--threads N]

One JSON file per case under tests/golden/digests/.  Nothing here comes from
the GPU library: the script loads only the oracle (and the workload module
for the layer shapes and seeds).  Each layer runs as row ranges of the M
dimension on a thread pool (the oracle's row ranges compose to the full
run, a pinned property); the digests are taken over the ranges in order.

Canonical bytes of an array: its elements row-major, each as little-endian
64-bit limbs -- (lo, hi) for k = s = 64, lo alone for k = s = 32 (whose high
limb is zero).  A digest is the first 32 hex digits of SHA-256 over them.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import importlib.util
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402


def _workloads():
    """The shape/seed module, loaded by path (no GPU binding is imported)."""
    path = os.path.join(ROOT, "paper_2311_04406_amd", "workloads.py")
    spec = importlib.util.spec_from_file_location("ct_workloads", path)
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod
    spec.loader.exec_module(mod)
    return mod


W = _workloads()
OUT_DIR = os.path.join(HERE, "digests")
DIGEST_HEX = 32
MODES = (("spdz2k", O.MODE_SPDZ2K), ("compact", O.MODE_COMPACT))

# case -> (configuration, k = s, f, parties, implicit convolutions, compress, protocols)
CASES = {
    "fc_small": ("fc_small", 64, 0, 2, True, 0, ("spdz2k", "compact")),
    "cnn": ("cnn", 64, 0, 2, True, 0, ("spdz2k", "compact")),
    "transformer": ("transformer", 64, 0, 2, True, 0, ("spdz2k", "compact")),
    "batched": ("batched", 64, 0, 2, True, 0, ("spdz2k", "compact")),
    "training": ("training", 64, 0, 2, True, 0, ("spdz2k", "compact")),
    "cnn_k32": ("cnn", 32, 0, 2, True, 0, ("spdz2k", "compact")),
    "transformer_k32": ("transformer", 32, 0, 2, True, 0, ("spdz2k", "compact")),
    "batched_k32": ("batched", 32, 0, 2, True, 0, ("spdz2k", "compact")),
    "cnn_f13": ("cnn", 64, 13, 2, True, 0, ("spdz2k", "compact")),
    "cnn_auto": ("cnn", 64, 0, 2, True, 2, ("compact",)),
    "cnn_p3": ("cnn", 64, 0, 3, False, 0, ("spdz2k", "compact")),
    "cnn_p4": ("cnn", 64, 0, 4, False, 0, ("spdz2k", "compact")),
    "cnn_p5": ("cnn", 64, 0, 5, False, 0, ("spdz2k", "compact")),
    "transformer_p3": ("transformer", 64, 0, 3, True, 0, ("spdz2k", "compact")),
    "transformer_p5": ("transformer", 64, 0, 5, True, 0, ("spdz2k", "compact")),
}

# Arrays of a layer by the dimension that indexes their rows.
DEALT_MK = ("X", "tX", "A", "tA")
DEALT_KN = ("Y", "tY", "B", "tB")
DEALT_MN = ("C", "tC", "R", "tR")
TRUNC_DEALT = ("Rf", "tRf")
TRUNC_OUT = ("Zf", "tZf")


def canon(a: np.ndarray, kbits: int):
    """Canonical bytes (a buffer) of an oracle array (..., 2 limbs)."""
    if kbits == 64:
        return np.ascontiguousarray(a)
    if a[..., 1].any():
        raise AssertionError("k = s = 32: a high limb is not zero")
    return np.ascontiguousarray(a[..., 0])


def compress_of(spec, setting: int) -> int:
    return O.cheaper_compress(spec.M, spec.K, spec.N) if setting == 2 else setting


def chunk_rows(spec, along_m: bool) -> int:
    """Rows of one task: about 2^26 products and at most 2^21 M x K elements."""
    if along_m:
        return spec.M
    by_work = (1 << 26) // max(1, spec.K * spec.N)
    by_mem = (1 << 21) // max(1, spec.K)
    return max(1, min(spec.M, by_work, by_mem))


class LayerDigest:
    """Running digests of one layer in one protocol, fed row ranges in order."""

    def __init__(self, spec, mode_name, kbits, f, parties, with_dealt, along_m):
        self.spec, self.mode_name, self.kbits, self.f, self.P = spec, mode_name, kbits, f, parties
        self.with_dealt, self.along_m = with_dealt, along_m
        self.h = {}
        self.cs = [[0] * parties for _ in range(3)]
        self.first = True
        self.mask = O.MASK128 if kbits == 64 else O.MASK64

    def _upd(self, name, arr):
        h = self.h.get(name)
        if h is None:
            h = self.h[name] = hashlib.sha256()
        h.update(canon(arr, self.kbits))

    def feed(self, L: "O.OracleLayer"):
        P, first = self.P, self.first
        compact = self.mode_name == "compact"
        # row-indexed arrays of every range; K-indexed ones from the first range
        if self.with_dealt:
            for n in DEALT_MK + DEALT_MN + (TRUNC_DEALT if self.f else ()):
                for p in range(P):
                    self._upd(f"{n}/{p}", L[n][p])
            if first:
                for n in DEALT_KN:
                    for p in range(P):
                        self._upd(f"{n}/{p}", L[n][p])
        self._upd("E", L["E"])
        self._upd("D", L["D"])
        for n in ("Z", "tZ") + (TRUNC_OUT if self.f else ()):
            for p in range(P):
                self._upd(f"{n}/{p}", L[n][p])
        if first:
            self._upd("U", L["U"])
        if compact:
            if self.along_m:      # vectors of length K and N: one range holds the whole layer
                self._upd("cvec/Ec", L["Ec"])
                for p in range(P):
                    self._upd(f"cvec/tAc/{p}", L["tAc"][p])
            elif first:
                self._upd("cvec/Uc", L["Uc"])
                for p in range(P):
                    self._upd(f"cvec/tBc/{p}", L["tBc"][p])
            self._upd("cvec/Dc", L["Dc"])
            self._upd("cvec/EUc", L["EUc"])
            for n in ("tCc", "tRc", "tZc", "tDc"):
                for p in range(P):
                    self._upd(f"cvec/{n}/{p}", L[n][p])
        # check values: E and D add over row ranges (their combiners are indexed
        # by the global element), U is complete in every range
        for w in range(3):
            for p in range(P):
                v = O.u128(L.cs[w, p])
                if w == 1:
                    if first:
                        self.cs[w][p] = v
                    elif self.cs[w][p] != v:
                        raise AssertionError("check of U differs between row ranges")
                else:
                    self.cs[w][p] = (self.cs[w][p] + v) & self.mask
        self.first = False

    def result(self):
        sums = [sum(self.cs[w]) & self.mask for w in range(3)]
        if any(sums):
            raise AssertionError(f"{self.spec.name}: the honest run does not pass its checks")
        digests = {k: v.hexdigest()[:DIGEST_HEX] for k, v in sorted(self.h.items())}
        cs = [[format(v, "x") for v in row] for row in self.cs]
        return digests, cs


def run_case(case: str, threads: int, only=None) -> dict:
    """Digests of every layer of a case (only: the layer indices to run)."""
    config, kbits, f, parties, implicit, cmp, modes = CASES[case]
    specs = W.CONFIGS[config]()
    key = W.KEY_SEED
    pick = [li for li in range(len(specs)) if only is None or li in only]
    tasks = []  # (mode name, layer index, r0, r1)
    for mname in modes:
        for li in pick:
            s = specs[li]
            c = compress_of(s, cmp) if mname == "compact" else 0
            rows = chunk_rows(s, c == 1)
            for r0 in range(0, s.M, rows):
                tasks.append((mname, li, r0, min(s.M, r0 + rows)))
    mode_ids = dict(MODES)

    def work(t):
        mname, li, r0, r1 = t
        s = specs[li]
        c = compress_of(s, cmp) if mname == "compact" else 0
        conv = s.conv if (implicit and s.conv is not None) else None
        L = O.OracleLayer(s.M, s.K, s.N, s.seed, s.layer_id, key, r0, r1, f, 0, kbits, c, conv, parties)
        return L.deal().online(mode_ids[mname]).check(mode_ids[mname])

    layers = {}
    cur = {}
    window = threads + 4
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        futs = {}
        nxt = 0
        for i, t in enumerate(tasks):
            while nxt < len(tasks) and nxt < i + window:
                futs[nxt] = ex.submit(work, tasks[nxt])
                nxt += 1
            L = futs.pop(i).result()
            mname, li, r0, r1 = t
            s = specs[li]
            k = (mname, li)
            if k not in cur:
                c = compress_of(s, cmp) if mname == "compact" else 0
                cur[k] = LayerDigest(s, mname, kbits, f, parties, with_dealt=(mname == modes[0]), along_m=(c == 1))
            cur[k].feed(L)
            del L
            if r1 == s.M:
                dg, cs = cur.pop(k).result()
                rec = layers.setdefault(s.name, {"M": s.M, "K": s.K, "N": s.N, "seed": s.seed,
                                                 "layer_id": s.layer_id, "conv": list(s.conv) if
                                                 (implicit and s.conv is not None) else None,
                                                 "compress": {}, "dealt": {}, "online": {}, "cs": {}})
                if mname == modes[0]:
                    rec["dealt"] = {n: v for n, v in dg.items() if n.split("/")[0] in
                                    DEALT_MK + DEALT_KN + DEALT_MN + TRUNC_DEALT}
                rec["online"][mname] = {n: v for n, v in dg.items() if n not in rec["dealt"]}
                rec["cs"][mname] = cs
                rec["compress"][mname] = compress_of(s, cmp) if mname == "compact" else 0
    return {
        "case": case, "config": config, "kbits": kbits, "f": f, "parties": parties,
        "implicit_conv": implicit, "compress_setting": cmp, "modes": list(modes), "key_seed": key,
        "oracle_source_sha256": hashlib.sha256(open(O.SRC, "rb").read()).hexdigest()[:DIGEST_HEX],
        "layers": [dict(name=specs[li].name, **layers[specs[li].name]) for li in pick],
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("cases", nargs="*", help="cases to write (default: all)")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    O.build()
    os.makedirs(OUT_DIR, exist_ok=True)
    for case in args.cases or list(CASES):
        t0 = time.time()
        rec = run_case(case, args.threads)
        rec["oracle_seconds"] = round(time.time() - t0, 1)
        rec["threads"] = args.threads
        with open(os.path.join(OUT_DIR, case + ".json"), "w") as fh:
            json.dump(rec, fh, indent=0, sort_keys=False)
            fh.write("\n")
        print(f"{case}: {len(rec['layers'])} layers, {rec['oracle_seconds']} s", flush=True)


if __name__ == "__main__":
    main()
