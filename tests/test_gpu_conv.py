"""GPU parity of convolution layers with the im2col matrix left implicit
(Eq. (4)): the input, its mask and U live in the input's C x H x W shape, U
is opened and checked on those elements, the matrix-core operands and the
compression along N gather the im2col entries.  The HIP path through the C
ABI against the oracle, bit for bit."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import compare_cs, compare_layer, cs_sums, free, gpu_layers, oracle_run, say, to_np
from paper_2311_04406_amd.binding import RESULT_WORDS

pytestmark = pytest.mark.gpu

KEY = 7
MODES = [O.MODE_SPDZ2K, O.MODE_COMPACT]


class Conv:
    def __init__(self, cout, C, H, W, k, s, p, seed=1, layer_id=1, compress=0, f=0):
        Ho, Wo = (H + 2 * p - k) // s + 1, (W + 2 * p - k) // s + 1
        self.M, self.K, self.N = cout, C * k * k, Ho * Wo
        self.conv = (C, H, W, k, s, p)
        self.seed, self.layer_id, self.compress, self.f, self.in_bits = seed, layer_id, compress, f, 0
        self.name = f"conv{cout}x{C}x{H}x{W}k{k}s{s}p{p}_c{compress}" + (f"_f{f}" if f else "")


# strides 1 and 2, padding 0 and 1, kernels 1, 2, 3; ragged tiles; a split-K
# layer (K = 2700); M above and below N
SMALL = [Conv(5, 3, 7, 9, 3, 1, 1, 2, 2), Conv(16, 8, 12, 12, 3, 2, 1, 3, 3), Conv(70, 5, 10, 11, 1, 1, 0, 4, 4),
         Conv(64, 16, 14, 14, 3, 1, 1, 5, 5), Conv(33, 40, 9, 9, 2, 1, 0, 6, 6), Conv(130, 64, 8, 8, 3, 1, 1, 7, 7),
         Conv(20, 300, 6, 6, 3, 1, 1, 8, 8), Conv(9, 4, 11, 7, 3, 2, 0, 9, 9, f=11)]


@pytest.fixture(scope="module")
def ctx():
    O.build()
    from paper_2311_04406_amd import Context
    c = Context(device=0, key_seed=KEY)
    yield c
    c.close()


def run_one(c, spec, mode, fused, kbits=64):
    from paper_2311_04406_amd import Context
    say(f"[conv] kbits={kbits} mode={mode} fused={fused} {spec.name}")
    layers = gpu_layers(c, [spec])
    c.gen_triple_tags(layers)
    if fused:
        out = torch.zeros(RESULT_WORDS, dtype=torch.int64, device="cuda:0")
        c.tag_linear_check(mode, layers, out)
        res = Context.decode_results(out, 1)[0]
        status = 0 if res.accept else 4
    else:
        c.tag_linear(mode, layers)
        status, rr = c.mac_check(mode, layers)
        res = rr[0]
    torch.cuda.synchronize()
    ol = oracle_run(mode, spec, KEY, kbits=kbits)
    compare_layer(layers[0], ol, mode, what=spec.name)
    compare_cs(res, ol, what=spec.name)
    assert status == 0 and res.accept and ol.accept()
    free()


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("spec", SMALL, ids=lambda s: s.name)
def test_conv_bit_exact(ctx, spec, mode, fused):
    run_one(ctx, spec, mode, fused)


@pytest.mark.parametrize("spec", [Conv(5, 3, 7, 9, 3, 1, 1, 2, 2, compress=2),
                                  Conv(130, 64, 8, 8, 3, 1, 1, 7, 7, compress=2),
                                  Conv(20, 300, 6, 6, 3, 1, 1, 8, 8, compress=1)], ids=lambda s: s.name)
def test_conv_compressed_along_m(ctx, spec):
    run_one(ctx, spec, O.MODE_COMPACT, True)


@pytest.mark.parametrize("mode", MODES)
def test_conv_k32(mode):
    from paper_2311_04406_amd import Context
    c = Context(device=0, key_seed=KEY, kbits=32)
    for spec in (SMALL[0], SMALL[3], SMALL[6]):
        run_one(c, spec, mode, True, kbits=32)
    c.close()


def test_conv_and_plain_layers_in_one_plan(ctx):
    """Convolutions (both compressed dimensions) and plain products in one
    fused batch and one captured plan, replayed three times."""
    from paper_2311_04406_amd import Context

    class Plain:
        def __init__(self, M, K, N, seed, lid):
            self.M, self.K, self.N, self.seed, self.layer_id, self.compress = M, K, N, seed, lid, 0
            self.name = f"{M}x{K}x{N}"
    specs = [SMALL[0], Plain(70, 100, 130, 21, 21), SMALL[5], Conv(130, 64, 8, 8, 3, 1, 1, 22, 22, compress=2),
             Plain(33, 70, 1, 23, 23)]
    mode = O.MODE_COMPACT
    layers = gpu_layers(ctx, specs)
    ctx.gen_triple_tags(layers)
    out = torch.zeros(RESULT_WORDS * len(specs), dtype=torch.int64, device="cuda:0")
    ctx.tag_linear_check(mode, layers, out)
    res = Context.decode_results(out, len(specs))
    refs = []
    for l, s, r in zip(layers, specs, res):
        ol = oracle_run(mode, s, KEY)
        compare_layer(l, ol, mode, what=s.name)
        compare_cs(r, ol, what=s.name)
        refs.append((to_np(l["Z"][1]).copy(), to_np(l["U"]).copy(), to_np(l["cvec"]).copy()))
    plan = ctx.plan(mode, layers, out)
    for rep in range(3):
        for l in layers:
            l["Z"][1].zero_()
            l["U"].zero_()
            l["cvec"].zero_()
        out.zero_()
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for l, (z, u, cv) in zip(layers, refs):
            assert (to_np(l["Z"][1]) == z).all() and (to_np(l["U"]) == u).all() and (to_np(l["cvec"]) == cv).all()
        assert all(r.accept for r in Context.decode_results(out, len(specs)))
    plan.close()
    free()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("target", ["Y", "tY", "B", "tB"])
def test_conv_flipped_input_bit_aborts(ctx, mode, target):
    from paper_2311_04406_amd import CT_ABORT
    spec = SMALL[1]
    layers = gpu_layers(ctx, [spec])
    ctx.gen_triple_tags(layers)
    t = layers[0][target][0]
    t.view(-1, t.shape[-1])[11, 0] ^= 1 << 33
    ctx.tag_linear(mode, layers)
    status, res = ctx.mac_check(mode, layers)
    assert status == CT_ABORT and cs_sums(res[0])[1] != 0
    free()


def test_conv_geometry_is_validated(ctx):
    from paper_2311_04406_amd import CtError, Layer
    bad = [Layer(4, 18, 24, 1, 1, conv=(2, 5, 5, 3, 1, 1)),      # N should be 25
           Layer(4, 18, 4, 1, 1, conv=(2, 4, 4, 3, 2, 1)),       # N = 4 <= 8
           Layer(4, 18, 25, 1, 1, conv=(2, 5, 5, 3, 1, 3))]      # pad >= kernel
    for l in bad:
        with pytest.raises(CtError):
            ctx.gen_triple_tags([l])
    free()


@pytest.mark.parametrize("mode", MODES)
def test_cnn_convolutions_implicit_full_size(ctx, mode):
    """The four convolutions of the CNN workload with the implicit im2col,
    against the oracle on sampled rows (the input side, U and its check,
    complete)."""
    from paper_2311_04406_amd import workloads as W
    specs = [s for s in W.cnn() if s.conv is not None]
    assert len(specs) == 4
    for s in specs:
        spec = Conv(s.M, *s.conv, s.seed, s.layer_id)
        assert (spec.K, spec.N) == (s.K, s.N)
        say(f"[conv] full size {s.name} mode={mode}")
        layers = gpu_layers(ctx, [spec])
        ctx.gen_triple_tags(layers)
        ctx.tag_linear(mode, layers)
        status, res = ctx.mac_check(mode, layers)
        torch.cuda.synchronize()
        assert status == 0 and res[0].accept
        for r0 in (0, s.M - 5):
            ol = oracle_run(mode, spec, KEY, r0, r0 + 5)
            compare_layer(layers[0], ol, mode, r0, r0 + 5, what=f"{s.name} rows {r0}")
            compare_cs(res[0], ol, which=(1,), what=s.name)
        free()
