"""Every product kernel and workgroup tile shape (ct_tuning.tile) against the
oracle, bit-exact, in both protocols and both parameter sets, on shapes that
reach the tile edge cases: M with a ragged last 64- or 128-row tile and with
a lone 64-row tail (the 128 x 64 shapes then have no second left tile), N
with a ragged last column tile, K with a ragged last slice, and K ranges
split into partial products that are added atomically (forced through a
small split target).  One fused call per shape, as the benchmark runs."""
import pytest
import torch

import oracle as O
from gpu_util import compare_cs, compare_layer, free, gpu_layers, oracle_run, say
from paper_2311_04406_amd.binding import (RESULT_WORDS, TILE_LDS_128x64, TILE_LDS_64x64, TILE_REGS_128x64,
                                          TILE_REGS_64x64, TILE_REGS_FIT)

pytestmark = pytest.mark.gpu
KEY = 7
MODES = [O.MODE_SPDZ2K, O.MODE_COMPACT]


class Spec:
    def __init__(self, M, K, N, seed, layer_id):
        self.M, self.K, self.N, self.seed, self.layer_id = M, K, N, seed, layer_id
        self.name = f"{M}x{K}x{N}"


# (spec, split_target): 0 = no forced split; 8 slices of 32 force K splits.
# The fitted workgroup tile (TILE_REGS_FIT) of each shape is noted.
SHAPES = [(Spec(200, 300, 150, 31, 1), 0),     # ragged M (128-row: 128 + 72), N and K; fit 128 x 32
          (Spec(192, 96, 70, 32, 2), 0),       # 128-row tiles: one full, one lone 64-row tail; fit 64 x 64
          (Spec(130, 1000, 65, 33, 3), 8),     # 2 rows past a 128 tile; K = 1000 in 4 splits; fit 32 x 128
          (Spec(64, 2048, 128, 34, 4), 8),     # one 64-row tile; 8 splits; fit 64 x 64
          (Spec(33, 257, 9, 35, 5), 0),        # smallest matrix-core N; fit 64 x 64
          (Spec(90, 200, 250, 38, 8), 0),      # fit 32 x 128: ragged 32-row and 128-column tiles
          (Spec(250, 70, 90, 39, 9), 8)]       # fit 128 x 32, K in 3 slices (no split)
ALL = [TILE_LDS_64x64, TILE_REGS_64x64, TILE_REGS_FIT, TILE_LDS_128x64, TILE_REGS_128x64]
TILES = {64: ALL, 32: ALL}


@pytest.fixture(scope="module", params=[64, 32])
def ctx(request):
    from paper_2311_04406_amd import Context
    c = Context(device=0, key_seed=KEY, kbits=request.param)
    yield c
    c.close()


@pytest.mark.parametrize("mode", MODES)
def test_tile_shapes_bit_exact(ctx, mode):
    from paper_2311_04406_amd import Context
    for spec, split in SHAPES:
        ol = oracle_run(mode, spec, KEY, kbits=ctx.kbits)
        for tile in TILES[ctx.kbits]:
            say(f"[tiles] k={ctx.kbits} mode={mode} {spec.name} tile={tile} split={split}")
            ctx.set_tuning(1, 0, split, tile)
            layers = gpu_layers(ctx, [spec])
            ctx.gen_triple_tags(layers)
            out = torch.zeros(RESULT_WORDS, dtype=torch.int64, device="cuda:0")
            ctx.tag_linear_check(mode, layers, out)
            torch.cuda.synchronize()
            res = Context.decode_results(out, 1)[0]
            compare_layer(layers[0], ol, mode, dealt=False, what=f"{spec.name} tile {tile}")
            compare_cs(res, ol, what=f"{spec.name} tile {tile}")
            assert res.accept
            del layers
    ctx.set_tuning(1, 0, 0, 0)
    free()


def test_autotune_names_a_tile_shape(ctx):
    spec = Spec(256, 512, 256, 36, 6)
    layers = gpu_layers(ctx, [spec])
    ctx.gen_triple_tags(layers)
    t = ctx.autotune(O.MODE_COMPACT, layers, reps=1)
    assert t["tile"] in ("lds_64x64", "regs_64x64", "regs_fit", "lds_128x64", "regs_128x64"), t
    assert t["gemm_ms"] > 0
    assert ctx.get_tuning(O.MODE_COMPACT, layers)["tile"] == t["tile"]
    ol = oracle_run(O.MODE_COMPACT, spec, KEY, kbits=ctx.kbits)
    ctx.tag_linear(O.MODE_COMPACT, layers)   # under the tuned configuration
    torch.cuda.synchronize()
    compare_layer(layers[0], ol, O.MODE_COMPACT, dealt=False, what="tuned")
    del layers
    free()
