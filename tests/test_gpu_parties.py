"""GPU parity with more than two parties (the appendix on scaling with
parties): 3 to 5 parties simulated in one process, every result -- every
party's shares and tags, the opened values, the compact vectors and each
party's check values -- bit-exact against the n-party oracle."""
import pytest
import torch

import oracle as O
from gpu_util import compare_cs, compare_layer, cs_sums, free, gpu_layers, oracle_run, say, to_np
from paper_2311_04406_amd.binding import RESULT_WORDS

pytestmark = pytest.mark.gpu

KEY = 7
MODES = [O.MODE_SPDZ2K, O.MODE_COMPACT]


class Spec:
    def __init__(self, M, K, N, seed=1, layer_id=1, f=0, in_bits=0):
        self.M, self.K, self.N, self.seed, self.layer_id, self.f, self.in_bits = M, K, N, seed, layer_id, f, in_bits
        self.name = f"{M}x{K}x{N}" + (f"_f{f}" if f else "")


# skinny (N = 1, 3, 8), matrix-core with ragged tiles, split K, truncation
SPECS = [Spec(1, 1, 1), Spec(33, 70, 1, 2, 2), Spec(17, 40, 3, 3, 3), Spec(45, 100, 8, 4, 4),
         Spec(70, 100, 130, 5, 5), Spec(64, 128, 32, 6, 6), Spec(40, 2100, 70, 7, 7), Spec(65, 300, 20, 8, 8, f=13)]


def ctx_for(parties, kbits=64):
    from paper_2311_04406_amd import Context
    return Context(device=0, key_seed=KEY, parties=parties, kbits=kbits)


@pytest.fixture(scope="module")
def contexts():
    O.build()
    cs = {p: ctx_for(p) for p in (3, 4, 5)}
    yield cs
    for c in cs.values():
        c.close()


def run_one(c, spec, mode, fused, kbits=64):
    from paper_2311_04406_amd import Context
    say(f"[parties] n={c.parties} kbits={kbits} mode={mode} fused={fused} {spec.name}")
    assert c.key_shares() == [int(x) for x in O.key_shares(KEY, kbits, c.parties)]
    layers = gpu_layers(c, [spec])
    c.gen_triple_tags(layers)
    if fused:
        out = torch.zeros(RESULT_WORDS, dtype=torch.int64, device="cuda:0")
        c.tag_linear_check(mode, layers, out)
        res = Context.decode_results(out, 1, c.parties)[0]
        status = 0 if res.accept else 4
    else:
        c.tag_linear(mode, layers)
        status, rr = c.mac_check(mode, layers)
        res = rr[0]
    torch.cuda.synchronize()
    ol = oracle_run(mode, spec, KEY, kbits=kbits, parties=c.parties)
    compare_layer(layers[0], ol, mode, what=spec.name)
    compare_cs(res, ol, what=spec.name)
    assert status == 0 and res.accept and ol.accept()
    free()


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("parties", [3, 5])
@pytest.mark.parametrize("spec", SPECS, ids=lambda s: s.name)
def test_parties_bit_exact(contexts, spec, parties, mode, fused):
    run_one(contexts[parties], spec, mode, fused)


@pytest.mark.parametrize("mode", MODES)
def test_four_parties_and_k32(contexts, mode):
    for spec in (SPECS[1], SPECS[4], SPECS[6]):
        run_one(contexts[4], spec, mode, True)
    c = ctx_for(3, kbits=32)
    for spec in (SPECS[2], SPECS[5], SPECS[7]):
        run_one(c, spec, mode, True, kbits=32)
    c.close()


@pytest.mark.parametrize("mode", MODES)
def test_parties_batch_and_plan(contexts, mode):
    """A mixed batch through the fused call and a captured plan (3 replays)."""
    from paper_2311_04406_amd import Context
    c = contexts[3]
    specs = [SPECS[1], SPECS[4], SPECS[3], SPECS[6]]
    layers = gpu_layers(c, specs)
    c.gen_triple_tags(layers)
    out = torch.zeros(RESULT_WORDS * len(specs), dtype=torch.int64, device="cuda:0")
    c.tag_linear_check(mode, layers, out)
    res = Context.decode_results(out, len(specs), 3)
    refs = []
    for l, s, r in zip(layers, specs, res):
        ol = oracle_run(mode, s, KEY, parties=3)
        compare_layer(l, ol, mode, what=s.name)
        compare_cs(r, ol, what=s.name)
        refs.append([to_np(l["Z"][p]).copy() for p in range(3)])
    plan = c.plan(mode, layers, out)
    for rep in range(3):
        for l in layers:
            for p in range(3):
                l["Z"][p].zero_()
        out.zero_()
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for l, z in zip(layers, refs):
            assert all((to_np(l["Z"][p]) == z[p]).all() for p in range(3)), rep
        assert all(r.accept for r in Context.decode_results(out, len(specs), 3))
    plan.close()
    free()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("target,w", [("X", 0), ("tA", 0), ("Y", 1), ("tB", 1), ("C", 2), ("tR", 2)])
def test_parties_flipped_bit_aborts(contexts, mode, target, w):
    from paper_2311_04406_amd import CT_ABORT
    c = contexts[4]
    for party in (0, 2, 3):
        layers = gpu_layers(c, [Spec(20, 50, 40, 21, 21)])
        c.gen_triple_tags(layers)
        t = layers[0][target][party]
        t.view(-1, t.shape[-1])[17, 0] ^= 1 << 29
        c.tag_linear(mode, layers)
        status, res = c.mac_check(mode, layers)
        assert status == CT_ABORT and cs_sums(res[0])[w] != 0, (target, party)
        free()


def test_parties_restrictions(contexts):
    """More than two parties: plain products compressed along N, no server;
    parties outside 2..5 are rejected."""
    from paper_2311_04406_amd import CtError, Layer, Server
    c = contexts[3]
    with pytest.raises(CtError):
        c.gen_triple_tags([Layer(4, 18, 25, 1, 1, conv=(2, 5, 5, 3, 1, 1), parties=3)])
    with pytest.raises(CtError):
        c.tag_linear(O.MODE_COMPACT, [Layer(40, 18, 5, 1, 1, compress=1, parties=3)])
    with pytest.raises(CtError):
        Server(c, 1 << 20)
    for bad in (1, 6):
        with pytest.raises(CtError):
            ctx_for(bad)
    free()
