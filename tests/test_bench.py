"""Host logic of bench.py: the algorithmic byte and operation counts the
roofline divides by, the digest that keys the committed counter figures, and
the refusal of more than one GPU.  No GPU needed."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2311_04406_amd.workloads import LayerSpec  # noqa: E402

WIDE = LayerSpec("wide", 70, 100, 130, 1, 1)      # matrix-core layer (N > 8)
SKINNY = LayerSpec("skinny", 33, 70, 1, 2, 2)     # products in the row pass
CONV = LayerSpec("conv", 64, 27, 64, 3, 3, (3, 8, 8, 3, 1, 1))  # 3 x 8 x 8 input, 3x3 kernel


def work(stage, specs, mode="compact", **kw):
    return bench.stage_work(stage, specs, mode, **kw)


def test_two_party_row_and_open_counts():
    mk, kn = SKINNY.M * SKINNY.K, SKINNY.K * SKINNY.N
    # 8 share arrays read and the opened value written, 16 B each
    assert work("row_pass", [SKINNY]) == ("hbm", 144 * mk)
    assert work("open_u", [SKINNY]) == ("hbm", 144 * kn)
    # a matrix-core layer also writes A_0 + E (and in SPDZ2k the two folded tag operands)
    wmk = WIDE.M * WIDE.K
    assert work("row_pass", [WIDE]) == ("hbm", (144 + 16) * wmk)
    assert work("row_pass", [WIDE], "spdz2k") == ("hbm", (144 + 48) * wmk)


def test_fused_opening_moves_the_right_operands_out_of_pack():
    kn, mk = WIDE.K * WIDE.N, WIDE.M * WIDE.K
    # two-party matrix-core layer: U is opened with the digit tiles of [B]_0, [B]_1, U
    assert work("open_u", [WIDE]) == ("hbm", 0)
    assert work("open_pack", [WIDE]) == ("hbm", (144 + 48) * kn)
    assert work("pack", [WIDE]) == ("hbm", 96 * mk)                   # left operands only
    assert work("pack", [WIDE], "spdz2k") == ("hbm", 160 * mk + 64 * kn)  # + the two tag operands
    # beyond two parties nothing is fused
    assert work("open_pack", [WIDE], parties=3) == ("hbm", 0)
    assert work("open_u", [WIDE], parties=3) == ("hbm", (64 * 3 + 16) * kn)


def test_n_party_counts():
    for n in (3, 4, 5):
        mk, mn = SKINNY.M * SKINNY.K, SKINNY.M * SKINNY.N
        assert work("row_pass", [SKINNY], parties=n) == ("hbm", (64 * n + 16) * mk)
        # the n-party post pass compresses [tC]_p in a pass of its own
        assert work("post", [SKINNY], parties=n) == ("hbm", (64 * n + 16) * mn)
    assert work("post", [SKINNY]) == ("hbm", 176 * SKINNY.M * SKINNY.N)


def test_products_and_ring_size():
    ops = work("ring_gemm", [WIDE, SKINNY])
    assert ops == ("mfma", 2 * bench.DIGIT_PAIRS * 2 * 2 * WIDE.M * WIDE.K * WIDE.N)
    # k = s = 32: 36 digit products per ring MAC, every byte figure halves
    assert work("ring_gemm", [WIDE], kbits=32) == ("mfma", 2 * 36 * 2 * 2 * WIDE.M * WIDE.K * WIDE.N)
    assert work("row_pass", [SKINNY], kbits=32) == ("hbm", 72 * SKINNY.M * SKINNY.K)
    assert work("copy_base", [WIDE]) is None
    assert work("no_such_stage", [WIDE]) is None


def test_implicit_convolution_counts():
    c, h, w = CONV.conv[:3]
    nr, kn = c * h * w, CONV.K * CONV.N
    assert work("open_u", [CONV], implicit=True) == ("hbm", 144 * nr)
    assert work("open_pack", [CONV], implicit=True) == ("hbm", 0)
    assert work("conv_compress", [CONV], implicit=True) == ("hbm", 48 * nr)
    assert work("pack", [CONV], implicit=True) == ("hbm", 96 * CONV.M * CONV.K + 3 * (16 * nr + 32 * kn))


def test_digest_ignores_comments_only():
    src = "int a; // note\n/* block\n comment */ int b;  \n\n"
    assert bench.strip_comments(src) == "int a;\n int b;"
    assert bench.strip_comments(src) != bench.strip_comments(src.replace("int b", "int c"))
    d = bench.source_digest()
    assert len(d) == 16 and d == bench.source_digest()


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_persistent_launch_scope():
    """The bench's rule for when the persistent launch applies follows the
    library's: two parties, matrix-core layers only, no implicit convolution,
    nothing compressed along M."""
    from paper_2311_04406_amd import workloads as W
    assert bench.persistent_applies(W.batched(), "n", 2, True)
    assert not bench.persistent_applies(W.batched(), "n", 3, True)
    assert not bench.persistent_applies(W.cnn(), "n", 2, True)     # classifier N = 1, convolutions
    assert bench.persistent_applies(W.transformer(1), "n", 2, True)
    assert not bench.persistent_applies(W.transformer(1), "m", 2, True)
