"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle,
bit-exact (everything is integer arithmetic mod 2^128)."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import compare_cs, compare_layer, cs_sums, free, gpu_layers, oracle_run, say, to_np
from paper_2311_04406_amd.binding import RESULT_WORDS

pytestmark = pytest.mark.gpu

KEY = 7
MODES = [O.MODE_SPDZ2K, O.MODE_COMPACT]


class Spec:
    def __init__(self, M, K, N, seed=1, layer_id=1, name="", f=0, in_bits=0):
        self.M, self.K, self.N, self.seed, self.layer_id, self.name = M, K, N, seed, layer_id, name or f"{M}x{K}x{N}"
        self.f, self.in_bits = f, in_bits


@pytest.fixture(scope="module")
def ctx():
    O.build()
    from paper_2311_04406_amd import Context
    c = Context(device=0, key_seed=KEY)
    yield c
    c.close()


def run_all(ctx, mode, specs):
    layers = gpu_layers(ctx, specs)
    ctx.gen_triple_tags(layers)
    ctx.tag_linear(mode, layers)
    status, res = ctx.mac_check(mode, layers)
    torch.cuda.synchronize()
    return layers, status, res


# shapes that span several tiles, ragged edges in every dimension, the
# skinny path (N <= 8), K not a multiple of 32 and K long enough to be split
SMALL = [Spec(1, 1, 1), Spec(3, 5, 7, 2, 2), Spec(64, 128, 32, 1000, 1, "fc64x128x32"), Spec(70, 100, 130, 3, 3),
         Spec(130, 33, 65, 4, 4), Spec(5, 300, 9, 5, 5), Spec(17, 40, 8, 6, 6), Spec(33, 70, 1, 7, 7),
         Spec(96, 600, 200, 8, 8), Spec(40, 2100, 70, 9, 9), Spec(65, 4500, 66, 10, 10)]


def test_key_shares(ctx):
    assert ctx.key_shares() == [int(x) for x in O.key_shares(KEY)]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("spec", SMALL, ids=lambda s: s.name)
def test_small_layers_bit_exact(ctx, mode, spec):
    say(f"[parity] mode={mode} shape={spec.name}")
    layers, status, res = run_all(ctx, mode, [spec])
    ol = oracle_run(mode, spec, KEY)
    compare_layer(layers[0], ol, mode, what=spec.name)
    compare_cs(res[0], ol, what=spec.name)
    assert status == 0 and res[0].accept and ol.accept()
    free()


@pytest.mark.parametrize("mode", MODES)
def test_several_layers_in_one_call(ctx, mode):
    specs = [SMALL[3], SMALL[5], SMALL[7], Spec(64, 128, 32, 11, 12)]
    say(f"[parity] multi-layer mode={mode}")
    layers, status, res = run_all(ctx, mode, specs)
    for s, gl, r in zip(specs, layers, res):
        ol = oracle_run(mode, s, KEY)
        compare_layer(gl, ol, mode, what=s.name)
        compare_cs(r, ol, what=s.name)
    assert status == 0
    free()


@pytest.mark.parametrize("mode", MODES)
def test_repeat_runs_identical(ctx, mode):
    """Determinism across launches (cross-workgroup sums are exact)."""
    s = Spec(96, 600, 200, 8, 8)
    layers, _, r1 = run_all(ctx, mode, [s])
    z1 = [to_np(layers[0]["Z"][p]) for p in range(2)] + [to_np(layers[0]["tZ"][p]) for p in range(2)]
    ctx.tag_linear(mode, layers)
    _, r2 = ctx.mac_check(mode, layers)
    z2 = [to_np(layers[0]["Z"][p]) for p in range(2)] + [to_np(layers[0]["tZ"][p]) for p in range(2)]
    assert all(np.array_equal(a, b) for a, b in zip(z1, z2))
    assert r1[0].cs == r2[0].cs
    free()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("spec", SMALL, ids=lambda s: s.name)
def test_fused_verification_matches(ctx, mode, spec):
    """ct_tag_linear_check gives the same outputs and check records as
    ct_tag_linear followed by ct_mac_check, and as the oracle."""
    from paper_2311_04406_amd import Context
    say(f"[fused] mode={mode} shape={spec.name}")
    layers = gpu_layers(ctx, [spec])
    ctx.gen_triple_tags(layers)
    out = torch.zeros(RESULT_WORDS, dtype=torch.int64, device="cuda:0")
    ctx.tag_linear_check(mode, layers, out)
    torch.cuda.synchronize()
    fused = Context.decode_results(out, 1)[0]
    ol = oracle_run(mode, spec, KEY)
    compare_layer(layers[0], ol, mode, what=spec.name)
    compare_cs(fused, ol, what=spec.name)
    assert fused.accept
    status, sep = ctx.mac_check(mode, layers)
    assert status == 0 and sep[0].cs == fused.cs
    free()


@pytest.mark.parametrize("mode", MODES)
def test_launch_configurations_give_identical_results(ctx, mode):
    """The tile order, XCD remap and K-split length change only the schedule:
    outputs and check records are bit-identical, and equal the oracle's."""
    from paper_2311_04406_amd import Context
    specs = [Spec(200, 700, 300, 31, 5), Spec(70, 100, 130, 3, 3), Spec(33, 70, 1, 7, 7)]
    layers = gpu_layers(ctx, specs)
    ctx.gen_triple_tags(layers)
    out = torch.zeros(RESULT_WORDS * len(specs), dtype=torch.int64, device="cuda:0")
    ref = None
    for g, x, sp in [(1, 0, 0), (4, 1, 8), (16, 0, 32), (2, 1, 128), (8, 1, 0), (64, 1, 16), (2, 4, 16), (1, 16, 0),
                     (8, 8, 32), (4, 3, 8)]:
        say(f"[tuning] mode={mode} group_m={g} xcd={x} split={sp}")
        ctx.set_tuning(g, x, sp)
        ctx.tag_linear_check(mode, layers, out)
        res = [r.cs for r in Context.decode_results(out, len(specs))]
        got = [to_np(l[n][p]) for l in layers for n in ("Z", "tZ") for p in range(2)]
        if ref is None:
            ref = (res, got)
            for s, gl, r in zip(specs, layers, Context.decode_results(out, len(specs))):
                ol = oracle_run(mode, s, KEY)
                compare_layer(gl, ol, mode, what=s.name)
                compare_cs(r, ol, what=s.name)
        else:
            assert res == ref[0]
            assert all(np.array_equal(a, b) for a, b in zip(got, ref[1]))
    best = ctx.autotune(mode, layers)
    assert best["group_m"] >= 1 and best["gemm_ms"] > 0
    ctx.set_tuning(1, 0, 0)
    free()


TAMPER = [("X", 1, 5, 0), ("tA", 0, 63, 0), ("B", 0, 31, 1), ("tY", 1, 0, 1), ("C", 1, 17, 2), ("tR", 0, 40, 2)]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("target", TAMPER, ids=lambda t: f"{t[0]}{t[1]}b{t[2]}")
def test_flipped_share_bit_aborts(ctx, mode, target):
    """One flipped bit in one party's share makes ct_mac_check return CT_ABORT,
    with the same check values as the oracle given the same flip."""
    from paper_2311_04406_amd import CT_ABORT
    name, party, bit, w = target
    s = Spec(40, 70, 50, 21, 3)
    say(f"[tamper] mode={mode} {name}[{party}] bit {bit}")
    layers = gpu_layers(ctx, [s])
    ctx.gen_triple_tags(layers)
    t = layers[0][name][party]
    flat = t.view(-1, 2)
    idx = 37 % flat.shape[0]
    limb = 0 if bit < 64 else 1
    flat[idx, limb] ^= (1 << (bit % 64)) if bit % 64 < 63 else -(1 << 63)
    out = torch.zeros(RESULT_WORDS, dtype=torch.int64, device="cuda:0")
    ctx.tag_linear_check(mode, layers, out)
    from paper_2311_04406_amd import Context
    fused = Context.decode_results(out, 1)[0]
    status, res = ctx.mac_check(mode, layers)
    assert status == CT_ABORT and not res[0].accept and not fused.accept
    assert cs_sums(res[0])[w] != 0
    assert fused.cs == res[0].cs
    ol = O.OracleLayer(s.M, s.K, s.N, s.seed, s.layer_id, KEY).deal()
    ol[name][party].reshape(-1, 2)[idx, limb] ^= np.uint64(1 << (bit % 64))
    ol.online(mode).check(mode)
    compare_layer(layers[0], ol, mode, what="tampered")
    compare_cs(res[0], ol, what="tampered")
    free()


# truncation by the opened D (f > 0): wide, skinny, ragged and split-K layers,
# uniform and signed 16-bit inputs
TRUNC = [Spec(70, 100, 130, 21, 21, f=13, in_bits=16), Spec(33, 70, 1, 22, 22, f=13, in_bits=16),
         Spec(5, 300, 9, 23, 23, f=40), Spec(40, 2100, 70, 24, 24, f=1, in_bits=20),
         Spec(17, 40, 8, 25, 25, f=63)]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("spec", TRUNC, ids=lambda s: f"{s.name}_f{s.f}_b{s.in_bits}")
def test_truncation_bit_exact(ctx, mode, spec):
    say(f"[parity] truncation mode={mode} shape={spec.name} f={spec.f} in_bits={spec.in_bits}")
    layers, status, res = run_all(ctx, mode, [spec])
    ol = oracle_run(mode, spec, KEY)
    compare_layer(layers[0], ol, mode, what=spec.name)
    compare_cs(res[0], ol, what=spec.name)
    assert status == 0 and res[0].accept and ol.accept()
    free()


@pytest.mark.parametrize("mode", MODES)
def test_truncation_fused_batch(ctx, mode):
    """A batch mixing f = 0 and f > 0 layers through the fused call equals the oracle."""
    from paper_2311_04406_amd import Context
    specs = [Spec(64, 128, 32, 31, 31), TRUNC[0], TRUNC[1], TRUNC[3]]
    say(f"[parity] truncation fused batch mode={mode}")
    layers = gpu_layers(ctx, specs)
    ctx.gen_triple_tags(layers)
    out = torch.zeros(RESULT_WORDS * len(specs), dtype=torch.int64, device="cuda:0")
    ctx.tag_linear_check(mode, layers, out)
    res = Context.decode_results(out, len(specs))
    for l, s, r in zip(layers, specs, res):
        ol = oracle_run(mode, s, KEY)
        compare_layer(l, ol, mode, what=s.name)
        compare_cs(r, ol, what=s.name)
        assert r.accept
    free()
