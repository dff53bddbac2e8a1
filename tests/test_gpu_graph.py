"""Captured plans (ct_plan_*): the online phase recorded once into a HIP graph
and replayed.  Every replay must reproduce the eager call bit for bit, with
eager work and synchronizations between replays, and must recompute from the
current contents of the bound input buffers."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import compare_cs, compare_layer, free, gpu_layers, oracle_run, say, to_np
from paper_2311_04406_amd.binding import RESULT_WORDS

pytestmark = pytest.mark.gpu

KEY = 7
MODES = [O.MODE_SPDZ2K, O.MODE_COMPACT]
OUTS = ["Z", "tZ"]
PUB = ["E", "U", "D", "cvec"]


class Spec:
    def __init__(self, M, K, N, seed, layer_id):
        self.M, self.K, self.N, self.seed, self.layer_id = M, K, N, seed, layer_id
        self.name = f"{M}x{K}x{N}"


# wide, ragged, skinny (N <= 8) and K-split layers in one batch
BATCH = [Spec(70, 100, 130, 31, 1), Spec(5, 300, 9, 32, 2), Spec(33, 70, 1, 33, 3), Spec(40, 2100, 70, 34, 4),
         Spec(64, 128, 32, 35, 5)]


@pytest.fixture(scope="module")
def ctx():
    O.build()
    from paper_2311_04406_amd import Context
    c = Context(device=0, key_seed=KEY)
    yield c
    c.close()


def snapshot(layers, out):
    snap = []
    for l in layers:
        d = {}
        for n in OUTS:
            d[n] = [to_np(l[n][p]).copy() for p in range(2)]
        for n in PUB:
            d[n] = to_np(l[n]).copy()
        snap.append(d)
    return snap, to_np(out).copy()


def clear(layers, out):
    for l in layers:
        for n in OUTS:
            for p in range(2):
                l[n][p].zero_()
        for n in PUB:
            l[n].zero_()
    out.zero_()


def same(layers, out, ref, what):
    snap, res = snapshot(layers, out)
    for i, (a, b) in enumerate(zip(snap, ref[0])):
        for n in a:
            if isinstance(a[n], list):
                for p in range(2):
                    assert np.array_equal(a[n][p], b[n][p]), (what, i, n, p)
            else:
                assert np.array_equal(a[n], b[n]), (what, i, n)
    assert np.array_equal(res, ref[1]), (what, "results")


@pytest.mark.parametrize("mode", MODES)
def test_plan_replays_match_eager(ctx, mode):
    from paper_2311_04406_amd import Context
    say(f"[graph] mode={mode} batch of {len(BATCH)}")
    layers = gpu_layers(ctx, BATCH)
    out = torch.zeros(RESULT_WORDS * len(BATCH), dtype=torch.int64, device="cuda:0")
    ctx.gen_triple_tags(layers)
    ctx.tag_linear_check(mode, layers, out)
    torch.cuda.synchronize()
    ref = snapshot(layers, out)
    assert all(r.accept for r in Context.decode_results(out, len(BATCH)))
    plan = ctx.plan(mode, layers, out)
    other = gpu_layers(ctx, [Spec(50, 60, 70, 99, 9)])
    ctx.gen_triple_tags(other)
    for rep in range(4):
        clear(layers, out)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        same(layers, out, ref, f"replay {rep}")
        # eager work between replays, on the same stream
        ctx.tag_linear(mode, other)
        torch.cuda.synchronize()
    # one layer of the batch against the oracle as well
    ol = oracle_run(mode, BATCH[0], KEY)
    compare_layer(layers[0], ol, mode, what="replayed")
    compare_cs(Context.decode_results(out, len(BATCH))[0], ol, what="replayed")
    plan.close()
    free()


@pytest.mark.parametrize("mode", MODES)
def test_plan_recomputes_from_current_inputs(ctx, mode):
    from paper_2311_04406_amd import Context
    say(f"[graph] new inputs mode={mode}")
    specs = BATCH[:3]
    layers = gpu_layers(ctx, specs)
    out = torch.zeros(RESULT_WORDS * len(specs), dtype=torch.int64, device="cuda:0")
    ctx.gen_triple_tags(layers)
    plan = ctx.plan(mode, layers, None)
    plan_chk = ctx.plan(mode, layers, out)
    # fresh inputs and triples dealt into the same buffers (other seeds)
    for l in layers:
        l.seed += 1000
    ctx.gen_triple_tags(layers)
    for l, s in zip(layers, specs):
        l.seed = s.seed
    ctx.tag_linear_check(mode, layers, out)
    torch.cuda.synchronize()
    ref = snapshot(layers, out)
    clear(layers, out)
    plan.launch()           # online phase only
    plan_chk.launch()       # online phase + fused verification
    torch.cuda.synchronize()
    same(layers, out, ref, "new inputs")
    res = Context.decode_results(out, len(specs))
    assert all(r.accept for r in res)
    # a flipped tag bit of an input share is caught by the replayed check
    layers[0]["tX"][1][0, 0, 0] ^= 1 << 5
    plan_chk.launch()
    torch.cuda.synchronize()
    res = Context.decode_results(out, len(specs))
    assert not res[0].accept and res[1].accept and res[2].accept
    plan.close()
    plan_chk.close()
    free()


@pytest.mark.parametrize("mode", MODES)
def test_one_stream_matches_two(ctx, mode):
    """A mixed batch (skinny layer amid matrix-core ones) run with its two
    layer groups on two streams (the default) and all on the context stream
    (ct_set_overlap(0)), eagerly and as a plan: the same outputs and the same
    check records at the same positions."""
    say(f"[graph] overlap on/off mode={mode}")
    layers = gpu_layers(ctx, BATCH)
    out = torch.zeros(RESULT_WORDS * len(BATCH), dtype=torch.int64, device="cuda:0")
    ctx.gen_triple_tags(layers)
    ctx.tag_linear_check(mode, layers, out)
    torch.cuda.synchronize()
    ref = snapshot(layers, out)
    try:
        ctx.set_overlap(False)
        clear(layers, out)
        ctx.tag_linear_check(mode, layers, out)
        torch.cuda.synchronize()
        same(layers, out, ref, "one stream, eager")
        plan = ctx.plan(mode, layers, out)
        for rep in range(2):
            clear(layers, out)
            torch.cuda.synchronize()
            plan.launch()
            torch.cuda.synchronize()
            same(layers, out, ref, f"one stream, replay {rep}")
        plan.close()
    finally:
        ctx.set_overlap(True)
    free()


def test_plan_rejects_invalid(ctx):
    from paper_2311_04406_amd import CtError, Layer
    l = Layer(4, 4, 4, 1, 1)
    l.f = 1
    with pytest.raises(CtError):
        ctx.plan(O.MODE_COMPACT, [l])
