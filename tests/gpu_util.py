"""Helpers of the GPU parity tests: run layers through the C ABI and compare
them element by element with the oracle (both sides start from the same
seeds; no value crosses from the GPU path into the oracle)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle as O

DEALT = ["X", "tX", "A", "tA", "Y", "tY", "B", "tB", "C", "tC", "R", "tR"]
MK = {"X", "tX", "A", "tA", "E"}
KN = {"Y", "tY", "B", "tB", "U"}
MN = {"C", "tC", "R", "tR", "Z", "tZ", "D", "Rf", "tRf", "Zf", "tZf"}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_np(t: torch.Tensor) -> np.ndarray:
    return t.detach().contiguous().cpu().numpy().view(np.uint64)


def gpu_layers(ctx, specs, device="cuda:0"):
    from paper_2311_04406_amd import Layer
    return [Layer(s.M, s.K, s.N, s.seed, s.layer_id, device=device, f=getattr(s, "f", 0),
                  in_bits=getattr(s, "in_bits", 0), limbs=getattr(ctx, "limbs", 2),
                  compress=getattr(s, "compress", 0), conv=getattr(s, "conv", None),
                  parties=getattr(ctx, "parties", 2)) for s in specs]


def oracle_compress(spec):
    """The oracle's compressed dimension for a spec's compress setting (0 N, 1 M, 2 the cheaper)."""
    c = getattr(spec, "compress", 0)
    return O.cheaper_compress(spec.M, spec.K, spec.N) if c == 2 else c


def oracle_run(mode, spec, key_seed, r0=0, r1=None, kbits=64, parties=2):
    return O.run_layer(mode, spec.M, spec.K, spec.N, spec.seed, spec.layer_id, key_seed, r0, r1,
                       getattr(spec, "f", 0), getattr(spec, "in_bits", 0), kbits,
                       oracle_compress(spec) if mode == O.MODE_COMPACT else 0, getattr(spec, "conv", None),
                       parties)


def oracle_view(o, limbs):
    """The oracle's (lo, hi) limbs cut to the GPU tensors' limb count (with one
    limb the oracle's high limb must be zero)."""
    if limbs == 2:
        return o
    assert not o[..., 1].any()
    return o[..., :1]


def _rows(name, arr, r0, r1):
    if name in MK or name in MN:
        return arr[r0:r1]
    return arr


def compare_layer(gl, ol, mode, r0=0, r1=None, dealt=True, what=""):
    """Bit-exact comparison of every array of one layer (rows [r0, r1) of the
    M-indexed ones)."""
    if r1 is None:
        r1 = gl.M
    lw = gl.limbs if hasattr(gl, "limbs") else 2
    np_ = getattr(gl, "parties", 2)
    assert np_ == ol.parties, (what, "parties")
    names = (DEALT if dealt else []) + ["Z", "tZ"]
    if getattr(gl, "f", 0) > 0:
        names += (["Rf", "tRf"] if dealt else []) + ["Zf", "tZf"]
    for n in names:
        for p in range(np_):
            g = to_np(_rows(n, gl[n][p], r0, r1))
            o = oracle_view(ol[n][p], lw)
            assert g.shape == o.shape, (what, n, g.shape, o.shape)
            if not np.array_equal(g, o):
                bad = np.argwhere((g != o).any(axis=-1))
                raise AssertionError(f"{what}: {n}[{p}] differs at {len(bad)} places, first {bad[:3].tolist()}")
    for n in ("E", "U", "D"):
        g = to_np(_rows(n, gl[n], r0, r1))
        on = oracle_view(ol[n], lw)
        if not np.array_equal(g, on):
            bad = np.argwhere((g != on).any(axis=-1))
            raise AssertionError(f"{what}: {n} differs at {len(bad)} places, first {bad[:3].tolist()}")
    if mode == O.MODE_COMPACT:
        parts = {k: to_np(v) for k, v in gl.cvec_parts().items()}
        along_m = getattr(gl, "along_m", False)
        assert along_m == (ol.compress == 1), (what, "compressed dimension")
        if along_m:  # vectors of length K and N: the whole layer
            assert (r0, r1) == (0, gl.M)
            pairs = [("Ec", ol["Ec"]), ("tAc0", ol["tAc"][0]), ("tAc1", ol["tAc"][1])]
        else:
            pairs = [("Uc", ol["Uc"])] + [(f"tBc{p}", ol["tBc"][p]) for p in range(np_)]
        for n, on in [("Dc", "Dc"), ("EUc", "EUc")]:
            pairs.append((n, ol[on]))
        for base in ("tCc", "tRc", "tZc", "tDc"):
            for p in range(np_):
                pairs.append((f"{base}{p}", ol[base][p]))
        for n, o in pairs:
            g = parts[n]
            if not along_m and not (n == "Uc" or n.startswith("tBc")):
                g = g[r0:r1]  # the length-M vectors of the sampled rows
            o = oracle_view(o, lw)
            assert g.shape == o.shape, (what, n, g.shape, o.shape)
            assert np.array_equal(g, o), (what, n)


def compare_cs(gres, ol, which=(0, 1, 2), what=""):
    for w in which:
        assert len(gres.cs[w]) == ol.parties, (what, "parties")
        for p in range(ol.parties):
            assert gres.cs[w][p] == O.u128(ol.cs[w, p]), (what, w, p)


def cs_sums(res, kbits: int = 64):
    """Sum over the parties of each check value (E, U, D) of a check record,
    mod 2^{k+s}: 2^128 for k = s = 64, 2^64 for k = s = 32."""
    mod = 1 << (2 * kbits)
    return [sum(res.cs[w]) % mod for w in range(3)]


def free():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
