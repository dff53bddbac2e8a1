"""GPU parity of the compact tag compressed along M (W^c = chi^T W; Eq. (5)
multiplied by chi^T from the left) and of the per-layer choice of the
compressed dimension by the operation count of Sec. 3.4.3: the HIP path
through the C ABI against the oracle, bit for bit."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import compare_cs, compare_layer, cs_sums, free, gpu_layers, oracle_run, say, to_np
from paper_2311_04406_amd.binding import RESULT_WORDS

pytestmark = pytest.mark.gpu

KEY = 7
ALONG_M, AUTO = 1, 2


class Spec:
    def __init__(self, M, K, N, seed=1, layer_id=1, compress=ALONG_M, f=0, in_bits=0):
        self.M, self.K, self.N, self.seed, self.layer_id = M, K, N, seed, layer_id
        self.compress, self.f, self.in_bits = compress, f, in_bits
        self.name = f"{M}x{K}x{N}_c{compress}" + (f"_f{f}" if f else "")


# every row-pass variant (N = 1, 2, 3..4, 5..8, > 8), ragged strips (K not a
# multiple of the strip width) and row blocks (M not a multiple of 32), one
# strip and many, several column-sweep row blocks
SMALL = [Spec(1, 1, 1), Spec(5, 3, 2, 2, 2), Spec(70, 300, 1, 3, 3), Spec(33, 257, 2, 4, 4),
         Spec(64, 129, 3, 5, 5), Spec(45, 100, 8, 6, 6), Spec(130, 700, 20, 7, 7), Spec(96, 64, 70, 8, 8),
         Spec(40, 2100, 70, 9, 9), Spec(17, 40, 90, 10, 10), Spec(300, 1030, 1, 11, 11),
         Spec(65, 513, 5, 12, 12, f=9, in_bits=10)]


@pytest.fixture(scope="module")
def ctx():
    O.build()
    from paper_2311_04406_amd import Context
    c = Context(device=0, key_seed=KEY)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx32():
    from paper_2311_04406_amd import Context
    c = Context(device=0, key_seed=KEY, kbits=32)
    yield c
    c.close()


def run_one(c, spec, kbits, fused):
    say(f"[compress] kbits={kbits} fused={fused} shape={spec.name}")
    layers = gpu_layers(c, [spec])
    assert layers[0].along_m == (O.cheaper_compress(spec.M, spec.K, spec.N) == 1 if spec.compress == AUTO
                                 else spec.compress == ALONG_M)
    c.gen_triple_tags(layers)
    if fused:
        out = torch.zeros(RESULT_WORDS, dtype=torch.int64, device="cuda:0")
        c.tag_linear_check(O.MODE_COMPACT, layers, out)
        from paper_2311_04406_amd import Context
        res = Context.decode_results(out, 1)[0]
        status = 0 if res.accept else 4
    else:
        c.tag_linear(O.MODE_COMPACT, layers)
        status, rr = c.mac_check(O.MODE_COMPACT, layers)
        res = rr[0]
    torch.cuda.synchronize()
    ol = oracle_run(O.MODE_COMPACT, spec, KEY, kbits=kbits)
    assert ol.compress == (1 if layers[0].along_m else 0)
    compare_layer(layers[0], ol, O.MODE_COMPACT, what=spec.name)
    compare_cs(res, ol, what=spec.name)
    assert status == 0 and res.accept and ol.accept()
    free()


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("spec", SMALL, ids=lambda s: s.name)
def test_along_m_bit_exact(ctx, spec, fused):
    run_one(ctx, spec, 64, fused)


@pytest.mark.parametrize("spec", SMALL[::2], ids=lambda s: s.name)
def test_along_m_bit_exact_k32(ctx32, spec):
    run_one(ctx32, spec, 32, True)


def test_auto_mixed_batch_and_graph(ctx):
    """A batch mixing both compressed dimensions (AUTO picks per layer) through
    the fused call and a captured plan, replayed three times."""
    from paper_2311_04406_amd import Context
    specs = [Spec(70, 300, 1, 3, 3, AUTO), Spec(64, 200, 96, 21, 21, AUTO), Spec(96, 64, 70, 8, 8, AUTO),
             Spec(20, 90, 40, 22, 22, AUTO), Spec(33, 257, 2, 4, 4, 0), Spec(45, 100, 8, 6, 6, ALONG_M)]
    layers = gpu_layers(ctx, specs)
    assert [l.along_m for l in layers] == [True, False, True, False, False, True]
    ctx.gen_triple_tags(layers)
    out = torch.zeros(RESULT_WORDS * len(specs), dtype=torch.int64, device="cuda:0")
    ctx.tag_linear_check(O.MODE_COMPACT, layers, out)
    res = Context.decode_results(out, len(specs))
    refs = []
    for l, s, r in zip(layers, specs, res):
        ol = oracle_run(O.MODE_COMPACT, s, KEY)
        compare_layer(l, ol, O.MODE_COMPACT, what=s.name)
        compare_cs(r, ol, what=s.name)
        assert r.accept
        refs.append((to_np(l["Z"][0]).copy(), to_np(l["cvec"]).copy()))
    plan = ctx.plan(O.MODE_COMPACT, layers, out)
    for rep in range(3):
        for l in layers:
            l["Z"][0].zero_()
            l["cvec"].zero_()
        out.zero_()
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for l, (z, cv) in zip(layers, refs):
            assert (to_np(l["Z"][0]) == z).all() and (to_np(l["cvec"]) == cv).all(), rep
        assert all(r.accept for r in Context.decode_results(out, len(specs)))
    plan.close()
    free()


@pytest.mark.parametrize("target,bit,w", [("tC", 3, 2), ("tR", 40, 2), ("R", 0, 2), ("C", 63, 2),
                                          ("tA", 17, 0), ("tB", 9, 1), ("X", 5, 0)])
def test_along_m_flipped_bit_aborts(ctx, target, bit, w):
    from paper_2311_04406_amd import CT_ABORT
    spec = Spec(40, 300, 3, 31, 31)
    layers = gpu_layers(ctx, [spec])
    ctx.gen_triple_tags(layers)
    # a bit below 2^64 of the low limb of element 18 (values are authenticated mod 2^k)
    t = layers[0][target][1]
    t.view(-1, t.shape[-1])[18, 0] ^= 1 << bit
    ctx.tag_linear(O.MODE_COMPACT, layers)
    status, res = ctx.mac_check(O.MODE_COMPACT, layers)
    assert status == CT_ABORT and not res[0].accept
    sums = cs_sums(res[0])
    assert sums[w] != 0, sums
    free()


@pytest.mark.parametrize("shape", [(256, 2304, 196), (512, 4608, 49)])
def test_cnn_layers_compressed_along_m(ctx, shape):
    """The two convolutions of the CNN workload that AUTO compresses along M,
    at full size, against the whole-layer oracle."""
    M, K, N = shape
    spec = Spec(M, K, N, 1003 if M == 256 else 1004, 3 if M == 256 else 4, AUTO)
    run_one(ctx, spec, 64, True)


def test_classifier_compressed_along_m(ctx):
    """The 25088 -> 4096 classifier at batch 1 (4096 x 25088 x 1), compressed
    along M: output shares and tags against the oracle on sampled rows; the
    compact tags satisfy the MAC relation sum_p [tZ^c]_p = Delta~ chi^T Z~ and
    sum_p [tD^c]_p = Delta~ D~^c; the layer is accepted, and a flipped bit of a
    tag share of C (reached only through the compact tag) is caught."""
    from paper_2311_04406_amd import CT_ABORT
    spec = Spec(4096, 25088, 1, 1005, 5, AUTO)
    layers = gpu_layers(ctx, [spec])
    L = layers[0]
    assert L.along_m
    ctx.gen_triple_tags(layers)
    ctx.tag_linear(O.MODE_COMPACT, layers)
    status, res = ctx.mac_check(O.MODE_COMPACT, layers)
    torch.cuda.synchronize()
    assert status == 0 and res[0].accept
    for r0 in (0, 2051, 4090):
        # the shares, tags and opened values do not depend on the compressed dimension
        ol = oracle_run(O.MODE_COMPACT, Spec(4096, 25088, 1, 1005, 5, 0), KEY, r0, r0 + 6)
        for n in ("Z", "tZ"):
            for p in range(2):
                assert np.array_equal(to_np(L[n][p][r0:r0 + 6]), ol[n][p]), (n, p, r0)
        assert np.array_equal(to_np(L["D"][r0:r0 + 6]), ol["D"])
    delta = sum(int(v) for v in O.key_shares(KEY))
    chi = [int(v) for v in O.draw_many(1005, O.stream(5, 0x30), 0, 4096)]
    mask = (1 << 128) - 1
    z = O.to_ints(to_np(L["Z"][0]).reshape(4096, 2)) + O.to_ints(to_np(L["Z"][1]).reshape(4096, 2))
    cz = sum(c * int(v) for c, v in zip(chi, z)) & mask
    parts = {k: to_np(v) for k, v in L.cvec_parts().items()}
    tzc = (O.u128(parts["tZc0"][0]) + O.u128(parts["tZc1"][0])) & mask
    tdc = (O.u128(parts["tDc0"][0]) + O.u128(parts["tDc1"][0])) & mask
    assert tzc == delta * cz & mask
    assert tdc == delta * O.u128(parts["Dc"][0]) & mask
    L["tC"][0].view(-1)[2000] ^= 1 << 7
    ctx.tag_linear(O.MODE_COMPACT, layers)
    status, res = ctx.mac_check(O.MODE_COMPACT, layers)
    assert status == CT_ABORT and cs_sums(res[0])[2] != 0 and cs_sums(res[0])[0] == 0
    del layers, L
    free()
