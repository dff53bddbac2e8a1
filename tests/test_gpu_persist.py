"""The persistent launch of the online phase (ct_set_launch(CT_LAUNCH_PERSISTENT)):
one launch walks every stage over all layers of a batch, meeting at grid
barriers (Sec. 3.3: a batch of layers tagged and verified together).  Its
outputs and check records must equal the staged kernels' bit for bit, eagerly
and replayed from a captured plan; one layer is also compared with the
oracle.  Batches outside its scope (a skinny layer) take the staged kernels."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import compare_cs, compare_layer, free, gpu_layers, oracle_run, say, to_np
from paper_2311_04406_amd.binding import (LAUNCH_PERSISTENT, LAUNCH_STAGED, RESULT_WORDS, TILE_REGS_128x64,
                                          TILE_REGS_64x64)

pytestmark = pytest.mark.gpu

KEY = 7
MODES = [O.MODE_SPDZ2K, O.MODE_COMPACT]
OUTS = ["Z", "tZ"]
PUB = ["E", "U", "D", "cvec"]


class Spec:
    def __init__(self, M, K, N, seed, layer_id, f=0, in_bits=0):
        self.M, self.K, self.N, self.seed, self.layer_id, self.f, self.in_bits = M, K, N, seed, layer_id, f, in_bits
        self.name = f"{M}x{K}x{N}"


# matrix-core layers only: ragged in every dimension, N just above the skinny
# bound, a long K, a truncated output, several tiles of each kind
BATCH = [Spec(70, 100, 130, 31, 1), Spec(5, 300, 9, 32, 2), Spec(40, 2100, 70, 34, 4), Spec(64, 128, 32, 35, 5),
         Spec(200, 96, 150, 36, 6), Spec(33, 40, 257, 37, 7, f=9, in_bits=10), Spec(130, 700, 65, 38, 8)]
# with a skinny layer (N <= 8): outside the persistent launch's scope
MIXED = BATCH[:2] + [Spec(33, 70, 1, 33, 3)]


def make_ctx(kbits):
    O.build()
    from paper_2311_04406_amd import Context
    return Context(device=0, key_seed=KEY, kbits=kbits)


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx(64)
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


def staged_then_persistent(ctx, mode, specs, what):
    """The staged result of a batch, then the persistent one into cleared
    outputs; returns the layers, the check records and the stages timed."""
    from paper_2311_04406_amd import Context
    layers = gpu_layers(ctx, specs)
    out = torch.zeros(RESULT_WORDS * len(specs), dtype=torch.int64, device="cuda:0")
    ctx.gen_triple_tags(layers)
    ctx.set_launch(LAUNCH_STAGED)
    ctx.tag_linear_check(mode, layers, out)
    torch.cuda.synchronize()
    ref = snapshot(layers, out)
    assert all(r.accept for r in Context.decode_results(out, len(specs))), what
    clear(layers, out)
    torch.cuda.synchronize()
    try:
        ctx.set_launch(LAUNCH_PERSISTENT)
        ctx.set_timing(True)
        ctx.stage_times()
        ctx.tag_linear_check(mode, layers, out)
        torch.cuda.synchronize()
        stages = ctx.stage_times()
    finally:
        ctx.set_timing(False)
        ctx.set_launch(LAUNCH_STAGED)
    same(layers, out, ref, what)
    return layers, out, ref, stages


@pytest.mark.parametrize("mode", MODES)
def test_persistent_matches_staged(ctx, mode):
    from paper_2311_04406_amd import Context
    say(f"[persist] mode={mode} batch of {len(BATCH)}")
    layers, out, _, stages = staged_then_persistent(ctx, mode, BATCH, "persistent")
    assert "persistent" in stages and "ring_gemm" not in stages and "row_pass" not in stages, stages
    res = Context.decode_results(out, len(BATCH))
    assert all(r.accept and r.reserved == 0 for r in res)
    for i in (0, 5):
        ol = oracle_run(mode, BATCH[i], KEY)
        compare_layer(layers[i], ol, mode, what=f"persistent {BATCH[i].name}")
        compare_cs(res[i], ol, what=f"persistent {BATCH[i].name}")
    free()


@pytest.mark.parametrize("mode", MODES)
def test_persistent_split_products(ctx, mode):
    """K-split products (their constant terms copied first, partial products
    added atomically) inside the persistent launch."""
    say(f"[persist] split products mode={mode}")
    specs = [Spec(40, 2100, 70, 34, 4), Spec(64, 1500, 96, 41, 9)]
    try:
        ctx.set_tuning(1, 0, 16, TILE_REGS_64x64)
        staged_then_persistent(ctx, mode, specs, "split")
    finally:
        ctx.set_tuning()
    free()


@pytest.mark.parametrize("mode", MODES)
def test_persistent_plan_replays(ctx, mode):
    """Captured with the persistent launch (the barrier counter is cleared by a
    kernel inside the graph): every replay, with eager work between them,
    reproduces the staged result; a flipped input tag bit is rejected."""
    from paper_2311_04406_amd import Context
    say(f"[persist] plan mode={mode}")
    specs = BATCH[:4]
    layers, out, ref, _ = staged_then_persistent(ctx, mode, specs, "eager")
    try:
        ctx.set_launch(LAUNCH_PERSISTENT)
        plan = ctx.plan(mode, layers, out)
    finally:
        ctx.set_launch(LAUNCH_STAGED)
    other = gpu_layers(ctx, [Spec(50, 60, 70, 99, 19)])
    ctx.gen_triple_tags(other)
    for rep in range(3):
        clear(layers, out)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        same(layers, out, ref, f"replay {rep}")
        ctx.tag_linear(mode, other)
        torch.cuda.synchronize()
    layers[1]["tX"][1][0, 0, 0] ^= 1 << 7
    plan.launch()
    torch.cuda.synchronize()
    res = Context.decode_results(out, len(specs))
    assert not res[1].accept and res[0].accept and res[2].accept and res[3].accept
    assert all(r.reserved == 0 for r in res)
    plan.close()
    free()


@pytest.mark.parametrize("mode", MODES)
def test_persistent_static_workspace(ctx, mode):
    """The entry point with the static per-GPU workspace, as one persistent
    launch: the staged result."""
    say(f"[persist] static workspace mode={mode}")
    layers, out, ref, _ = staged_then_persistent(ctx, mode, BATCH[:3], "static, eager")
    clear(layers, out)
    torch.cuda.synchronize()
    try:
        ctx.set_launch(LAUNCH_PERSISTENT)
        ctx.tag_linear_check_static(mode, layers, out)
        torch.cuda.synchronize()
    finally:
        ctx.set_launch(LAUNCH_STAGED)
    same(layers, out, ref, "static workspace")
    free()


@pytest.mark.parametrize("mode", MODES)
def test_mixed_batch_takes_staged_kernels(ctx, mode):
    say(f"[persist] mixed batch mode={mode}")
    _, _, _, stages = staged_then_persistent(ctx, mode, MIXED, "mixed")
    assert "persistent" not in stages and "row_pass" in stages, stages
    free()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("tile", [TILE_REGS_64x64, TILE_REGS_128x64], ids=["mt1", "mt2"])
def test_persistent_k32(mode, tile):
    """k = s = 32: one output tile per wavefront, and two (128 x 64 workgroup
    tiles) as the launch picks for large batches."""
    say(f"[persist] k32 mode={mode} tile={tile}")
    c = make_ctx(32)
    try:
        c.set_tuning(4, 0, 0, tile)
        layers, out, _, stages = staged_then_persistent(c, mode, BATCH, f"k32 tile {tile}")
        assert "persistent" in stages, stages
        ol = oracle_run(mode, BATCH[4], KEY, kbits=32)
        from paper_2311_04406_amd import Context
        compare_layer(layers[4], ol, mode, what="k32 persistent")
        compare_cs(Context.decode_results(out, len(BATCH))[4], ol, what="k32 persistent")
    finally:
        c.close()
    free()


def test_run_out_barrier_is_reported(ctx):
    """A barrier bound of zero ticks, set from the host: the first waits run
    out at once, every later one ends at once, every kernel finishes, and
    every layer's check record reports the run-out (accept 0, reserved 1).
    With the default bound the same context runs the batch correctly again."""
    from paper_2311_04406_amd import Context
    mode = O.MODE_COMPACT
    say("[persist] run-out barrier")
    specs = BATCH[:3]
    layers = gpu_layers(ctx, specs)
    out = torch.zeros(RESULT_WORDS * len(specs), dtype=torch.int64, device="cuda:0")
    ctx.gen_triple_tags(layers)
    try:
        ctx.set_launch(LAUNCH_PERSISTENT)
        ctx.set_launch_wait(0)
        ctx.tag_linear_check(mode, layers, out)
        torch.cuda.synchronize()
        res = Context.decode_results(out, len(specs))
        assert all(not r.accept and r.reserved == 1 for r in res), [(r.accept, r.reserved) for r in res]
        ctx.set_launch_wait()
        clear(layers, out)
        ctx.tag_linear_check(mode, layers, out)
        torch.cuda.synchronize()
        res = Context.decode_results(out, len(specs))
        assert all(r.accept and r.reserved == 0 for r in res)
    finally:
        ctx.set_launch(LAUNCH_STAGED)
        ctx.set_launch_wait()
    ol = oracle_run(mode, specs[0], KEY)
    compare_layer(layers[0], ol, mode, what="after a run-out launch")
    compare_cs(res[0], ol, what="after a run-out launch")
    free()


def test_set_launch_rejects_unknown_mode(ctx):
    from paper_2311_04406_amd import CtError
    with pytest.raises(CtError):
        ctx.set_launch(7)
