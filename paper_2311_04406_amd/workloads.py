"""Synthetic workloads: layer shapes and seeds of the benchmark configurations.

Holds shapes, seeds and the seeded shape/arrival generators only -- none of
the protocol's arithmetic.  Every layer's data is produced on demand by the
dealer (``ct_gen_triple_tags``) from its (seed, layer_id); values are uniform
ring elements.

The paper names no dataset.  The shapes stand in for the linear layers of its
models: VGG-style 3x3 convolutions at batch 1 written as im2col products
(M = C_out, K = 9 C_in, N = H W, Eq. (4) with the usual +1 output size), a
VGG classifier layer at batch 1, and BERT-base-width encoder products at
sequence length 128.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

MASK64 = (1 << 64) - 1
KEY_SEED = 7  # key shares of every benchmark context


@dataclass(frozen=True)
class LayerSpec:
    name: str
    M: int
    K: int
    N: int
    seed: int
    layer_id: int
    conv: tuple | None = None   # (C, H, W, k, stride, pad) of a convolution, whose Y is the im2col of its input

    @property
    def mkn(self) -> int:
        return self.M * self.K * self.N


def _sm_mix(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def _sm_draw(seed: int, stream: int, i: int) -> int:
    """SplitMix64 counter draw (Steele, Lea, Flood 2014), for shapes and arrivals."""
    key = _sm_mix(seed ^ _sm_mix(stream))
    return _sm_mix(key + (i + 1) * 0x9E3779B97F4A7C15)


def fc_small():
    """One fully connected layer, W 64 x 128 times X 128 x 32."""
    return [LayerSpec("fc64x128x32", 64, 128, 32, 1000, 1)]


def cnn():
    """VGG-style 3x3 convolutions (pad 1, stride 1) at batch 1 as im2col
    products, and the 25088 -> 4096 classifier layer at batch 1."""
    shapes = [("conv64@56x56", 64, 576, 3136, (64, 56, 56, 3, 1, 1)),
              ("conv128@28x28", 128, 1152, 784, (128, 28, 28, 3, 1, 1)),
              ("conv256@14x14", 256, 2304, 196, (256, 14, 14, 3, 1, 1)),
              ("conv512@7x7", 512, 4608, 49, (512, 7, 7, 3, 1, 1)),
              ("fc25088x4096", 4096, 25088, 1, None)]
    return [LayerSpec(n, M, K, N, 1001 + i, i + 1, g) for i, (n, M, K, N, g) in enumerate(shapes)]


def transformer(encoders: int = 12):
    """Encoder products at sequence 128, hidden 768: QKV, attention output,
    FFN up and down, for `encoders` layers (one shared key)."""
    per = [("qkv", 128, 768, 2304), ("attn_out", 128, 768, 768), ("ffn1", 128, 768, 3072),
           ("ffn2", 128, 3072, 768)]
    out = []
    for e in range(encoders):
        for j, (n, M, K, N) in enumerate(per):
            lid = 4 * e + j + 1
            out.append(LayerSpec(f"enc{e}.{n}", M, K, N, 1100, lid))
    return out


def batched(count: int = 64, seed: int = 4000):
    """`count` layers with M, K, N log-uniform in [32, 4096]:
    dim = clamp(floor(32 * 2^(7u)), 32, 4096), u = (draw >> 11) 2^-53."""
    stream = (0xFFFF << 16) | 0x50
    out = []
    for l in range(count):
        dims = []
        for j in range(3):
            u = (_sm_draw(seed, stream, 3 * l + j) >> 11) * 2.0 ** -53
            dims.append(min(4096, max(32, int(math.floor(32 * 2.0 ** (7 * u))))))
        out.append(LayerSpec(f"batched{l}", dims[0], dims[1], dims[2], seed + 1 + l, 2000 + l))
    return out


def training(encoders: int = 12):
    """The products of one encoder training step at sequence 128, hidden 768:
    for each forward product Z = X W (M x K x N) its backward products
    dX = dZ W^T (M x N x K) and dW = X^T dZ (K x M x N) -- the same path with
    the operands' roles exchanged."""
    per = [("qkv", 128, 768, 2304), ("attn_out", 128, 768, 768), ("ffn1", 128, 768, 3072),
           ("ffn2", 128, 3072, 768)]
    out = []
    lid = 1
    for e in range(encoders):
        for n, M, K, N in per:
            for tag, shape in (("fwd", (M, K, N)), ("dX", (M, N, K)), ("dW", (K, M, N))):
                out.append(LayerSpec(f"enc{e}.{n}.{tag}", *shape, 1200, lid))
                lid += 1
    return out


def serving_shapes():
    """The request shape set: the CNN and the encoder products."""
    return cnn() + transformer(1)


def poisson_arrivals(rate: float, count: int, seed: int = 5000):
    """Arrival times (s) of a Poisson stream: gaps -ln(1 - u) / rate."""
    stream = (0xFFFF << 16) | 0x51
    t, out = 0.0, []
    for i in range(count):
        u = (_sm_draw(seed, stream, i) >> 11) * 2.0 ** -53
        t += -math.log(1.0 - u) / rate
        out.append(t)
    return out


def request_choices(count: int, nshapes: int, seed: int = 5000):
    """(kind, shape index) per request: kind 0 = tag generation, 1 = check."""
    ks, ss = (0xFFFF << 16) | 0x52, (0xFFFF << 16) | 0x53
    return [(_sm_draw(seed, ks, i) & 1, _sm_draw(seed, ss, i) % nshapes) for i in range(count)]


CONFIGS = {"fc_small": fc_small, "cnn": cnn, "transformer": transformer, "batched": batched,
           "training": training}
