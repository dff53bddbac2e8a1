"""ct_tag_linear_check_static (the online phase with the fused verification,
workspace in the library's static per-GPU array) against ct_tag_linear_check
(workspace from the caller): identical outputs and check records, bit for
bit, in both protocols, on two calls in a row -- a mixed batch first, then a
smaller one, which finds the array holding the first call's contents.  A
batch whose workspaces exceed the array is refused before anything runs."""
import pytest
import torch

import oracle as O
from gpu_util import free, gpu_layers, say

pytestmark = pytest.mark.gpu
KEY = 7


class Spec:
    def __init__(self, M, K, N, seed, lid, conv=None):
        self.M, self.K, self.N, self.seed, self.layer_id, self.conv = M, K, N, seed, lid, conv


FIRST = [Spec(200, 300, 150, 51, 1), Spec(64, 576, 100, 52, 2, (64, 10, 10, 3, 1, 1)), Spec(100, 700, 5, 53, 3),
         Spec(130, 65, 520, 54, 4)]
SECOND = [Spec(70, 130, 90, 61, 11)]


def outputs(gl):
    t = {n: gl[n] for n in ("E", "U", "D", "cvec")}
    for n in ("Z", "tZ"):
        for p in range(gl.parties):
            t[f"{n}{p}"] = gl[n][p]
    return t


@pytest.fixture(scope="module")
def ctx():
    from paper_2311_04406_amd import Context
    c = Context(device=0, key_seed=KEY)
    yield c
    c.close()


@pytest.mark.parametrize("mode", [O.MODE_SPDZ2K, O.MODE_COMPACT])
def test_static_workspace_matches_caller_workspace(ctx, mode):
    from paper_2311_04406_amd import Context
    from paper_2311_04406_amd.binding import RESULT_WORDS
    for call, specs in enumerate((FIRST, SECOND)):
        say(f"[no-alloc] mode={mode} call {call}: {[(s.M, s.K, s.N) for s in specs]}")
        ref = gpu_layers(ctx, specs)
        got = gpu_layers(ctx, specs)
        ctx.gen_triple_tags(ref)
        ctx.gen_triple_tags(got)
        out_ref = torch.zeros(RESULT_WORDS * len(specs), dtype=torch.int64, device="cuda:0")
        out_got = torch.full_like(out_ref, -1)
        ctx.tag_linear_check(mode, ref, out_ref)
        for g in got:   # the static call must not touch the caller's workspace
            g["work"].fill_(-1)
        ctx.tag_linear_check_static(mode, got, out_got)
        torch.cuda.synchronize()
        for s, r, g in zip(specs, ref, got):
            a, b = outputs(r), outputs(g)
            for n in a:
                assert torch.equal(a[n], b[n]), (call, s.M, s.K, s.N, n)
            assert bool((g["work"] == -1).all()), (call, "caller workspace written")
        rr = Context.decode_results(out_ref, len(specs))
        rg = Context.decode_results(out_got, len(specs))
        assert [x.cs for x in rr] == [x.cs for x in rg]
        assert all(x.accept for x in rg)
        del ref, got
        free()


def test_static_workspace_too_small_is_refused(ctx):
    from paper_2311_04406_amd import CtError
    from paper_2311_04406_amd.binding import RESULT_WORDS, STATIC_WORK_BYTES, work_len
    big = Spec(2048, 2048, 2048, 71, 21)   # about 3 x 64 MiB of folded operands plus 5 x 2 x 64 MiB of tiles
    assert work_len(big.M, big.K, big.N) * 16 > STATIC_WORK_BYTES
    layers = gpu_layers(ctx, [big])
    out = torch.zeros(RESULT_WORDS, dtype=torch.int64, device="cuda:0")
    with pytest.raises(CtError) as e:
        ctx.tag_linear_check_static(O.MODE_COMPACT, layers, out)
    assert "static workspace" in str(e.value)
    torch.cuda.synchronize()
    assert not bool(out.any())   # nothing ran
    del layers
    free()
