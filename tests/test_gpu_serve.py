"""The request server on the GPU: requests of mixed layer shapes that arrive
while others run are batched and overlap on the device, and every result is
the same, bit for bit, as the same layer computed alone through the plain
calls (and, for one layer, as the oracle)."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import compare_cs, compare_layer, cs_sums, free, oracle_run, say, to_np
from paper_2311_04406_amd.workloads import poisson_arrivals, request_choices

pytestmark = pytest.mark.gpu

KEY = 7
# wide (matrix-core), ragged, skinny (N <= 8), long-K (split) shapes
SHAPES = [(64, 576, 300), (128, 1152, 78), (70, 100, 130), (33, 70, 1), (256, 230, 19), (40, 2100, 70),
          (17, 40, 8)]
ARRAYS = ["X", "tX", "A", "tA", "Y", "tY", "B", "tB", "C", "tC", "R", "tR", "Z", "tZ"]


class Spec:
    def __init__(self, M, K, N, seed, layer_id):
        self.M, self.K, self.N, self.seed, self.layer_id = M, K, N, seed, layer_id


def requests(count, rate, seed, shapes, t0_us, id0=0):
    """(id, kind, (M, K, N, seed, layer_id), arrival_us) of a seeded Poisson stream."""
    arr = poisson_arrivals(rate, count, seed)
    ch = request_choices(count, len(shapes), seed)
    out = []
    for i in range(count):
        M, K, N = shapes[ch[i][1]]
        rid = id0 + i
        out.append((rid, ch[i][0], (M, K, N, 9000 + rid, 500 + rid), t0_us + arr[i] * 1e6))
    return out


@pytest.fixture(scope="module")
def alone_ctx():
    O.build()
    from paper_2311_04406_amd import Context
    c = Context(device=0, key_seed=KEY)
    yield c
    c.close()


def alone(ctx, mode, M, K, N, seed, lid):
    from paper_2311_04406_amd import Layer
    l = Layer(M, K, N, seed, lid)
    ctx.gen_triple_tags([l])
    ctx.tag_linear(mode, [l])
    st, res = ctx.mac_check(mode, [l])
    torch.cuda.synchronize()
    return l, st, res[0]


def same_layer(a, b, what, mode=O.MODE_COMPACT):
    for n in ARRAYS:
        for p in range(2):
            assert torch.equal(a[n][p], b[n][p]), (what, n, p)
    # the compressed vectors are outputs of the CompactTag protocol only
    for n in ("E", "U", "D") + (("cvec",) if mode == O.MODE_COMPACT else ()):
        assert torch.equal(a[n], b[n]), (what, n)


def overlapping(comps):
    """Two batches on different slots whose device intervals overlap."""
    batches = {}
    for c in comps:
        batches.setdefault((c["slot"], c["admit_us"]), c["done_us"])
    iv = sorted((a, d, s) for (s, a), d in batches.items())
    for i in range(len(iv)):
        for j in range(i + 1, len(iv)):
            if iv[j][0] >= iv[i][1]:
                break
            if iv[j][2] != iv[i][2]:
                return True
    return False


@pytest.mark.parametrize("mode", [O.MODE_COMPACT, O.MODE_SPDZ2K])
def test_mix_equals_alone(alone_ctx, mode):
    from paper_2311_04406_amd import REQ_CHECK, REQ_TAG, Context, Server
    say(f"[serve] mix vs alone mode={mode}")
    ctx = Context(device=0, key_seed=KEY)
    srv = Server(ctx, 4 << 30, slots=3, max_batch=8, mode=mode)
    reqs = requests(48, 20000.0, 5000 + mode, SHAPES, srv.now_us() + 3000.0)
    srv.submit(reqs)
    srv.drain(120)
    comps = srv.poll()
    st = srv.stats()
    say(f"[serve] stats {st}")
    assert len(comps) == len(reqs) and st["completed"] == len(reqs)
    assert all(c["status"] == 0 for c in comps), [c for c in comps if c["status"]]
    assert max(c["batch_size"] for c in comps) > 1          # continuous batching happened
    assert overlapping(comps)                                # and batches overlapped on the device
    by_id = {r[0]: r for r in reqs}
    for c in comps:
        assert c["admit_us"] >= c["arrival_us"] - 1.0 and c["done_us"] > c["admit_us"]
        if c["kind"] == REQ_TAG:
            assert c["layer"] == c["id"]
        else:
            assert by_id[c["id"]][1] == REQ_CHECK and c["layer"] != c["id"]
            assert by_id[c["layer"]][2][:3] == by_id[c["id"]][2][:3]     # a layer of the requested shape
    tags = [c for c in comps if c["kind"] == REQ_TAG]
    checks = {}
    for c in comps:
        if c["kind"] == REQ_CHECK:
            checks.setdefault(c["layer"], []).append(c)
    for c in tags:
        M, K, N, seed, lid = by_id[c["id"]][2]
        ref, ref_st, ref_res = alone(alone_ctx, mode, M, K, N, seed, lid)
        assert ref_st == 0 and ref_res.accept
        mine = srv.layer(c["id"])
        same_layer(mine, ref, f"request {c['id']} {M}x{K}x{N}", mode)
        for chk in checks.get(c["id"], []):
            assert chk["result"].accept and chk["result"].cs == ref_res.cs
        del ref, mine
    # one layer of the mix against the oracle as well
    c = next(c for c in tags if by_id[c["id"]][2][0] * by_id[c["id"]][2][1] * by_id[c["id"]][2][2] < 3e6)
    M, K, N, seed, lid = by_id[c["id"]][2]
    ol = oracle_run(mode, Spec(M, K, N, seed, lid), KEY)
    compare_layer(srv.layer(c["id"]), ol, mode, what="served")
    srv.close()
    ctx.close()
    free()


def test_eviction_rejection_and_tamper(alone_ctx):
    from paper_2311_04406_amd import REQ_CHECK, REQ_TAG, Context, Server
    from paper_2311_04406_amd.binding import CT_ABORT, CT_ENOMEM
    mode = O.MODE_COMPACT
    say("[serve] tight arena")
    ctx = Context(device=0, key_seed=KEY)
    srv = Server(ctx, 300 << 20, slots=2, max_batch=4, mode=mode)
    t0 = srv.now_us() + 3000.0
    reqs = requests(40, 5000.0, 5100, SHAPES, t0)
    # one layer larger than the whole arena
    reqs.append((1000, REQ_TAG, (4096, 25088, 1, 1, 1), t0 + 100.0))
    srv.submit(reqs)
    srv.drain(120)
    comps = {c["id"]: c for c in srv.poll()}
    st = srv.stats()
    say(f"[serve] stats {st}")
    assert len(comps) == len(reqs)
    assert comps[1000]["status"] == CT_ENOMEM
    assert all(c["status"] == 0 for i, c in comps.items() if i != 1000)
    assert st["evictions"] > 0 and st["rejected"] == 1 and st["arena_peak"] <= 300 << 20
    # layers still resident equal the same layers computed alone
    by_id = {r[0]: r for r in reqs}
    resident = [i for i, c in comps.items() if c["kind"] == REQ_TAG and c["status"] == 0]
    seen = 0
    for i in resident:
        try:
            mine = srv.layer(i)
        except Exception:
            continue  # evicted
        M, K, N, seed, lid = by_id[i][2]
        ref, _, _ = alone(alone_ctx, mode, M, K, N, seed, lid)
        same_layer(mine, ref, f"request {i}")
        seen += 1
    assert seen > 0
    # a flipped bit of a resident input tag share is caught by a later CHECK of its shape
    shape = (21, 45, 37)
    srv.submit([(2000, REQ_TAG, shape + (77, 4000), srv.now_us())])
    srv.drain(60)
    assert srv.poll()[0]["status"] == 0
    lay = srv.layer(2000)
    lay["tX"][0][3, 4, 0] ^= 1 << 40
    torch.cuda.synchronize()
    srv.submit([(2001, REQ_CHECK, shape + (0, 0), srv.now_us())])
    srv.drain(60)
    c = srv.poll()[0]
    assert c["kind"] == REQ_CHECK and c["layer"] == 2000 and c["status"] == CT_ABORT
    assert not c["result"].accept
    sums = cs_sums(c["result"])
    assert sums[0] != 0 and sums[1] == 0 and sums[2] == 0   # only the check of E fails
    srv.close()
    ctx.close()
    free()


@pytest.mark.parametrize("mode", [O.MODE_COMPACT, O.MODE_SPDZ2K])
def test_prepared_layers_equal_alone(alone_ctx, mode):
    """PREP requests deal layers ahead of their TAG requests (the offline
    phase); those TAGs run the online phase only, and every served layer --
    prepared or not -- equals the same layer computed alone, bit for bit.
    A repeated id of a resident layer is refused without running."""
    from paper_2311_04406_amd import REQ_PREP, REQ_TAG, Context, Server
    from paper_2311_04406_amd.binding import CT_EINVAL
    say(f"[serve] prepared layers mode={mode}")
    ctx = Context(device=0, key_seed=KEY)
    srv = Server(ctx, 4 << 30, slots=3, max_batch=8, mode=mode)
    t0 = srv.now_us() + 3000.0
    tags = requests(24, 20000.0, 5200 + mode, SHAPES, t0 + 2000.0)
    tags = [(i, REQ_TAG, lay, t) for i, _, lay, t in tags]
    preps = [(1000 + i, REQ_PREP, lay, t0 + 50.0 * i) for i, _, lay, t in tags if i % 3 != 2]
    srv.submit(preps + tags)
    srv.drain(120)
    comps = srv.poll()
    st = srv.stats()
    say(f"[serve] stats {st}")
    assert len(comps) == len(preps) + len(tags) and all(c["status"] == 0 for c in comps)
    assert st["prepared"] == len(preps) and 0 < st["online_only"] <= len(preps)
    by_id = {r[0]: r for r in tags}
    for c in comps:
        if c["kind"] != REQ_TAG:
            continue
        assert c["layer"] == c["id"]
        M, K, N, seed, lid = by_id[c["id"]][2]
        ref, ref_st, ref_res = alone(alone_ctx, mode, M, K, N, seed, lid)
        same_layer(srv.layer(c["id"]), ref, f"request {c['id']} {M}x{K}x{N}", mode)
        del ref
    srv.submit([(0, REQ_TAG, by_id[0][2], srv.now_us())])   # id 0 is resident
    srv.drain(60)
    c = srv.poll()[0]
    assert c["id"] == 0 and c["status"] == CT_EINVAL and srv.stats()["duplicates"] == 1
    srv.close()
    ctx.close()
    free()


def test_server_rejects_invalid_parameters():
    from paper_2311_04406_amd import Context, CtError, Server
    ctx = Context(device=0, key_seed=KEY)
    with pytest.raises(CtError):
        Server(ctx, 1 << 20, slots=0)
    with pytest.raises(CtError):
        Server(ctx, 1 << 20, max_batch=1000)
    srv = Server(ctx, 1 << 20, slots=1, max_batch=1)
    with pytest.raises(CtError):
        srv.submit([(1, 5, (4, 4, 4, 1, 1), 0.0)])
    with pytest.raises(CtError):
        srv.submit([(1, 0, (0, 4, 4, 1, 1), 0.0)])
    srv.close()
    ctx.close()
