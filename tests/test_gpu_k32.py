"""GPU parity for the k = s = 32 parameter set (shares and tags in Z_{2^64},
32-bit key shares and combiners; Sec. 4.1): the HIP path through the C ABI
against the oracle run with kbits = 32, bit-exact."""
import pytest
import torch

import oracle as O
from gpu_util import compare_cs, compare_layer, free, gpu_layers, oracle_run, say, to_np
from paper_2311_04406_amd.binding import RESULT_WORDS

pytestmark = pytest.mark.gpu

KEY = 7
MODES = [O.MODE_SPDZ2K, O.MODE_COMPACT]


class Spec:
    def __init__(self, M, K, N, seed=1, layer_id=1, f=0, in_bits=0):
        self.M, self.K, self.N, self.seed, self.layer_id, self.f, self.in_bits = M, K, N, seed, layer_id, f, in_bits
        self.name = f"{M}x{K}x{N}" + (f"_f{f}" if f else "")


SMALL = [Spec(1, 1, 1), Spec(3, 5, 7, 2, 2), Spec(64, 128, 32, 1000, 1), Spec(70, 100, 130, 3, 3),
         Spec(130, 33, 65, 4, 4), Spec(33, 70, 1, 7, 7), Spec(17, 40, 8, 6, 6), Spec(96, 600, 200, 8, 8),
         Spec(65, 4500, 66, 10, 10), Spec(40, 2100, 70, 9, 9, f=11, in_bits=12), Spec(33, 70, 1, 11, 11, f=5)]


@pytest.fixture(scope="module")
def ctx():
    O.build()
    from paper_2311_04406_amd import Context
    c = Context(device=0, key_seed=KEY, kbits=32)
    yield c
    c.close()


def test_k32_key_shares(ctx):
    assert ctx.key_shares() == [int(x) for x in O.key_shares(KEY, 32)]
    assert all(v < 1 << 32 for v in ctx.key_shares())


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("spec", SMALL, ids=lambda s: s.name)
def test_k32_bit_exact(ctx, mode, spec):
    say(f"[k32] mode={mode} shape={spec.name}")
    layers = gpu_layers(ctx, [spec])
    assert layers[0].limbs == 1
    ctx.gen_triple_tags(layers)
    ctx.tag_linear(mode, layers)
    status, res = ctx.mac_check(mode, layers)
    torch.cuda.synchronize()
    ol = oracle_run(mode, spec, KEY, kbits=32)
    compare_layer(layers[0], ol, mode, what=spec.name)
    compare_cs(res[0], ol, what=spec.name)
    assert status == 0 and res[0].accept and ol.accept()
    free()


@pytest.mark.parametrize("mode", MODES)
def test_k32_fused_batch_and_graph(ctx, mode):
    """A mixed batch through the fused call and through a captured plan."""
    from paper_2311_04406_amd import Context
    specs = [SMALL[2], SMALL[3], SMALL[5], SMALL[9]]
    layers = gpu_layers(ctx, specs)
    ctx.gen_triple_tags(layers)
    out = torch.zeros(RESULT_WORDS * len(specs), dtype=torch.int64, device="cuda:0")
    ctx.tag_linear_check(mode, layers, out)
    res = Context.decode_results(out, len(specs))
    for l, s, r in zip(layers, specs, res):
        ol = oracle_run(mode, s, KEY, kbits=32)
        compare_layer(l, ol, mode, what=s.name)
        compare_cs(r, ol, what=s.name)
        assert r.accept
    ref = [to_np(l["Z"][0]).copy() for l in layers]
    plan = ctx.plan(mode, layers, out)
    for rep in range(3):
        for l in layers:
            l["Z"][0].zero_()
        out.zero_()
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for l, z in zip(layers, ref):
            assert (to_np(l["Z"][0]) == z).all(), rep
        assert all(r.accept for r in Context.decode_results(out, len(specs)))
    plan.close()
    free()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("target,bit", [("X", 3), ("tA", 31), ("tB", 7), ("C", 20)])
def test_k32_flipped_bit_aborts(ctx, mode, target, bit):
    spec = Spec(20, 50, 40, 21, 21)
    layers = gpu_layers(ctx, [spec])
    ctx.gen_triple_tags(layers)
    layers[0][target][1].view(-1)[17] ^= 1 << bit
    ctx.tag_linear(mode, layers)
    status, res = ctx.mac_check(mode, layers)
    from paper_2311_04406_amd import CT_ABORT
    assert status == CT_ABORT and not res[0].accept
    free()


@pytest.mark.parametrize("mode", MODES)
def test_k32_sampled_encoder_layer(ctx, mode):
    """An encoder FFN layer (128 x 3072 x 768) against the oracle on 24 rows."""
    spec = Spec(128, 3072, 768, 1100, 4)
    layers = gpu_layers(ctx, [spec])
    ctx.gen_triple_tags(layers)
    out = torch.zeros(RESULT_WORDS, dtype=torch.int64, device="cuda:0")
    ctx.tag_linear_check(mode, layers, out)
    torch.cuda.synchronize()
    ol = oracle_run(mode, spec, KEY, 40, 64, kbits=32)
    compare_layer(layers[0], ol, mode, r0=40, r1=64, what="ffn2 rows 40..64")
    from paper_2311_04406_amd import Context
    assert Context.decode_results(out, 1)[0].accept
    free()
