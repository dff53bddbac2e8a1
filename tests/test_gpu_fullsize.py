"""GPU parity at the benchmark configurations' full sizes, in the launch
configuration bench.py times (all layers of a configuration in one call):
full element-by-element comparison where the oracle finishes in seconds,
sampled rows of the rest (the oracle computes any row range on its own), the
check values of U in full, honest acceptance of every layer, and identical
results for a layer alone and inside the batch."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import compare_cs, compare_layer, free, gpu_layers, oracle_run, say, to_np
from paper_2311_04406_amd import workloads as W
from paper_2311_04406_amd.binding import RESULT_WORDS

pytestmark = pytest.mark.gpu
KEY = W.KEY_SEED


@pytest.fixture(scope="module")
def ctx():
    O.build()
    from paper_2311_04406_amd import Context
    c = Context(device=0, key_seed=KEY)
    yield c
    c.close()


def run_config(ctx, mode, specs):
    """All layers in one fused call (the benchmark's launch configuration),
    then the standalone verification, which must agree record by record."""
    from paper_2311_04406_amd import Context
    layers = gpu_layers(ctx, specs)
    ctx.gen_triple_tags(layers)
    out = torch.zeros(RESULT_WORDS * len(specs), dtype=torch.int64, device="cuda:0")
    ctx.tag_linear_check(mode, layers, out)
    fused = Context.decode_results(out, len(specs))
    status, res = ctx.mac_check(mode, layers)
    torch.cuda.synchronize()
    assert [f.cs for f in fused] == [r.cs for r in res]
    return layers, status, res


def sample_rows(gl, spec, mode, rows):
    for (r0, r1) in rows:
        ol = oracle_run(mode, spec, KEY, r0, r1)
        compare_layer(gl, ol, mode, r0, r1, what=f"{spec.name} rows [{r0},{r1})")
        # the U check is complete in every row-range run
        return ol


@pytest.mark.parametrize("mode", [O.MODE_SPDZ2K, O.MODE_COMPACT])
def test_cnn_config(ctx, mode):
    specs = W.cnn()
    say(f"[fullsize] cnn mode={mode}")
    layers, status, res = run_config(ctx, mode, specs)
    assert status == 0 and all(r.accept for r in res)
    for s, gl, r in zip(specs, layers, res):
        if s.N > 8:
            say(f"  full oracle {s.name}")
            ol = oracle_run(mode, s, KEY)
            compare_layer(gl, ol, mode, what=s.name)
            compare_cs(r, ol, what=s.name)
        else:
            say(f"  sampled rows {s.name}")
            for rr in [(0, 3), (s.M // 2 + 7, s.M // 2 + 9), (s.M - 2, s.M)]:
                ol = oracle_run(mode, s, KEY, *rr)
                compare_layer(gl, ol, mode, *rr, what=f"{s.name} rows {rr}")
            compare_cs(r, ol, which=(1,), what=s.name)
    free()


@pytest.mark.parametrize("mode", [O.MODE_SPDZ2K, O.MODE_COMPACT])
def test_transformer_config(ctx, mode):
    specs = W.transformer()
    say(f"[fullsize] transformer mode={mode} ({len(specs)} layers)")
    layers, status, res = run_config(ctx, mode, specs)
    assert status == 0 and all(r.accept for r in res)
    # encoder 0 in full in the CompactTag protocol; sampled rows elsewhere
    for i, (s, gl, r) in enumerate(zip(specs, layers, res)):
        if i < 4 and mode == O.MODE_COMPACT:
            say(f"  full oracle {s.name}")
            ol = oracle_run(mode, s, KEY)
            compare_layer(gl, ol, mode, what=s.name)
            compare_cs(r, ol, what=s.name)
        elif i % 7 == 3:
            say(f"  sampled rows {s.name}")
            ol = oracle_run(mode, s, KEY, s.M - 2, s.M)
            compare_layer(gl, ol, mode, s.M - 2, s.M, what=s.name)
            compare_cs(r, ol, which=(1,), what=s.name)
    free()


@pytest.mark.parametrize("mode", [O.MODE_SPDZ2K, O.MODE_COMPACT])
def test_training_products(ctx, mode):
    """One encoder's forward and backward products (dX = dZ W^T, dW = X^T dZ
    shapes) in one call: sampled rows of every layer against the oracle."""
    specs = W.training(1)
    say(f"[fullsize] training products mode={mode} ({len(specs)} layers)")
    layers, status, res = run_config(ctx, mode, specs)
    assert status == 0 and all(r.accept for r in res)
    for s, gl, r in zip(specs, layers, res):
        rr = (s.M // 3, s.M // 3 + 2)
        ol = oracle_run(mode, s, KEY, *rr)
        compare_layer(gl, ol, mode, *rr, what=f"{s.name} rows {rr}")
        compare_cs(r, ol, which=(1,), what=s.name)
    free()


def test_batched_config_and_alone_vs_mix(ctx):
    """64 layers of uneven shapes in one call; a layer's outputs and check
    values are the same alone as in the mix (tolerance 0: integer results)."""
    mode = O.MODE_COMPACT
    specs = W.batched()
    say(f"[fullsize] batched {len(specs)} layers")
    layers, status, res = run_config(ctx, mode, specs)
    assert status == 0 and all(r.accept for r in res)
    for i in (0, 5, 17, 33, 63):
        s = specs[i]
        say(f"  sampled rows {s.name} {s.M}x{s.K}x{s.N}")
        ol = oracle_run(mode, s, KEY, 0, min(2, s.M))
        compare_layer(layers[i], ol, mode, 0, min(2, s.M), what=s.name)
        compare_cs(res[i], ol, which=(1,), what=s.name)
    for i in (3, 40):
        say(f"  alone vs mix {specs[i].name}")
        alone = gpu_layers(ctx, [specs[i]])
        ctx.gen_triple_tags(alone)
        ctx.tag_linear(mode, alone)
        st, r1 = ctx.mac_check(mode, alone)
        assert st == 0
        assert r1[0].cs == res[i].cs
        for n in ("Z", "tZ"):
            for p in range(2):
                assert torch.equal(alone[0][n][p], layers[i][n][p]), (n, p)
        assert torch.equal(alone[0]["cvec"], layers[i]["cvec"])
        assert torch.equal(alone[0]["D"], layers[i]["D"])
        del alone
    free()
