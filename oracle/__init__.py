"""CPU oracle for the CompactTag linear-layer hot path (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It drives the plain C oracle in
``ct_oracle.c`` through ctypes; it shares no code with the GPU library, and the
GPU library never falls back to it.

Ring elements of Z_{2^{k+s}} are numpy ``uint64`` arrays whose last axis holds
the (lo, hi) limbs (k = s = 64 or 32; with 32 the high limb is zero).
``run_layer`` executes the whole procedure (two parties by default) of one
linear layer -- the dealer (preprocessing of Fig. 7), the online phase and
the verification -- optionally restricted to a range of rows of the M
dimension, which is how full-size layers are sampled.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ct_oracle.c")
# CT_ORACLE_LIB names a library built from ct_oracle.c elsewhere (e.g. with
# sanitizers); it is then used as it is and never rebuilt here.
_LIB_OVERRIDE = os.environ.get("CT_ORACLE_LIB") or None
LIB_PATH = _LIB_OVERRIDE or os.path.join(HERE, "libct_oracle.so")

MODE_SPDZ2K = 0
MODE_COMPACT = 1
MAX_PARTIES = 5
MODES = {"spdz2k": MODE_SPDZ2K, "compact": MODE_COMPACT}
MASK64 = (1 << 64) - 1
MASK128 = (1 << 128) - 1


def _gpu_initialised() -> bool:
    """Whether this process has initialised the GPU through torch."""
    t = sys.modules.get("torch")
    try:
        return bool(t is not None and t.cuda.is_initialized())
    except Exception:
        return False


def stale() -> bool:
    """Whether libct_oracle.so is missing or older than its source."""
    return not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no intrinsics; each call runs on its
    calling thread).  A process that has initialised the GPU never compiles
    (that would fork a compiler from it): there a missing or stale library
    raises, so build it before the first GPU call."""
    if _LIB_OVERRIDE:
        return LIB_PATH
    if force or stale():
        if _gpu_initialised():
            raise RuntimeError(f"{LIB_PATH} is missing or older than {SRC}, and this process has initialised "
                               "the GPU: build the oracle before any GPU call (python3 -c 'import oracle; "
                               "oracle.build()')")
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-o", tmp, SRC])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Desc(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("K", ctypes.c_int64), ("N", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("layer_id", ctypes.c_uint64),
                ("r0", ctypes.c_int64), ("r1", ctypes.c_int64), ("f", ctypes.c_int64), ("in_bits", ctypes.c_int64),
                ("kbits", ctypes.c_int64), ("compress", ctypes.c_int64),
                ("conv_c", ctypes.c_int64), ("conv_h", ctypes.c_int64), ("conv_w", ctypes.c_int64),
                ("conv_k", ctypes.c_int64), ("conv_stride", ctypes.c_int64), ("conv_pad", ctypes.c_int64),
                ("parties", ctypes.c_int64)]


_P2 = ctypes.c_void_p * MAX_PARTIES   # one pointer per party slot
_BUF_FIELDS = [
    ("X", 2), ("tX", 2), ("A", 2), ("tA", 2), ("E", 1),
    ("Y", 2), ("tY", 2), ("B", 2), ("tB", 2), ("U", 1),
    ("C", 2), ("tC", 2), ("R", 2), ("tR", 2), ("Z", 2), ("tZ", 2), ("D", 1),
    ("Uc", 1), ("tBc", 2),
    ("Dc", 1), ("EUc", 1), ("tCc", 2), ("tRc", 2), ("tZc", 2), ("tDc", 2),
    ("Ec", 1), ("tAc", 2),
    ("Rf", 2), ("tRf", 2), ("Zf", 2), ("tZf", 2),
]


class _Bufs(ctypes.Structure):
    _fields_ = [(n, _P2 if c == 2 else ctypes.c_void_p) for n, c in _BUF_FIELDS] + [
        ("cs", ctypes.c_uint64 * (3 * MAX_PARTIES * 2)), ("tag_mults", ctypes.c_uint64 * MAX_PARTIES)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        u64, i64, vp = ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p
        L.or_mix64.restype = u64
        L.or_mix64.argtypes = [u64]
        L.or_stream_key.restype = u64
        L.or_stream_key.argtypes = [u64, u64]
        L.or_draw.restype = u64
        L.or_draw.argtypes = [u64, u64, u64]
        L.or_draw_many.argtypes = [u64, u64, u64, i64, vp]
        L.or_key_shares.argtypes = [u64, vp]
        L.or_key_shares_k.argtypes = [u64, i64, vp]
        L.or_key_shares_n.argtypes = [u64, i64, i64, vp]
        L.or_set_kbits.argtypes = [i64]
        L.or_deal.argtypes = [ctypes.POINTER(_Desc), vp, ctypes.c_int, ctypes.POINTER(_Bufs)]
        L.or_online.argtypes = [ctypes.c_int, ctypes.POINTER(_Desc), vp, ctypes.POINTER(_Bufs)]
        L.or_check.argtypes = [ctypes.c_int, ctypes.POINTER(_Desc), vp, ctypes.POINTER(_Bufs)]
        L.or_matmul.argtypes = [i64, i64, i64, vp, vp, vp]
        L.or_compress.argtypes = [i64, i64, vp, vp, vp]
        L.or_compress_rows.argtypes = [i64, i64, vp, vp, vp]
        L.or_im2col.argtypes = [ctypes.POINTER(_Desc), vp, vp]
        L.or_right_len.restype = i64
        L.or_right_len.argtypes = [ctypes.POINTER(_Desc)]
        L.or_batchrec_cs.argtypes = [i64, vp, vp, vp, u64, vp]
        L.or_compact_cs.argtypes = [i64, vp, vp, vp, u64, vp]
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# conversions

def to_ints(a: np.ndarray):
    """(..., 2) uint64 limbs -> nested Python ints (object ndarray)."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    lo = a[..., 0].astype(object)
    hi = a[..., 1].astype(object)
    return lo + (hi << 64)


def from_ints(x) -> np.ndarray:
    x = np.asarray(x, dtype=object)
    out = np.empty(x.shape + (2,), dtype=np.uint64)
    flat = x.reshape(-1)
    o = out.reshape(-1, 2)
    for i, v in enumerate(flat):
        v = int(v) & MASK128
        o[i, 0] = v & MASK64
        o[i, 1] = v >> 64
    return out


def u128(limbs) -> int:
    limbs = np.asarray(limbs, dtype=np.uint64)
    return int(limbs[0]) | (int(limbs[1]) << 64)


def _ptr(a: np.ndarray) -> int:
    assert a.flags.c_contiguous
    return a.ctypes.data


# ---------------------------------------------------------------------------
# PRNG and keys

def mix64(z: int) -> int:
    return int(lib().or_mix64(z & MASK64))


def draw(seed: int, stream: int, i: int) -> int:
    return int(lib().or_draw(seed & MASK64, stream & MASK64, i))


def draw_many(seed: int, stream: int, first: int, n: int) -> np.ndarray:
    out = np.empty(max(n, 1), dtype=np.uint64)
    lib().or_draw_many(seed & MASK64, stream & MASK64, first, n, _ptr(out))
    return out[:n]


def stream(layer_id: int, purpose: int) -> int:
    return ((layer_id << 16) | purpose) & MASK64


def key_shares(key_seed: int, kbits: int = 64, parties: int = 2) -> np.ndarray:
    out = np.zeros(parties, dtype=np.uint64)
    lib().or_key_shares_n(key_seed & MASK64, kbits, parties, _ptr(out))
    return out


def set_kbits(kbits: int):
    """Ring width (k = s) of the building blocks matmul, compress, batchrec_cs, compact_cs."""
    lib().or_set_kbits(kbits)


# ---------------------------------------------------------------------------
# one layer

@dataclass
class OracleLayer:
    M: int
    K: int
    N: int
    seed: int
    layer_id: int
    key_seed: int
    r0: int = 0
    r1: int | None = None
    f: int = 0
    in_bits: int = 0
    kbits: int = 64
    compress: int = 0                   # 0: along N (columns), 1: along M (rows; all rows)
    conv: tuple | None = None           # (C, H, W, k, stride, pad): Y is the im2col of a C x H x W input
    parties: int = 2                    # 2..MAX_PARTIES
    arrays: dict = field(default_factory=dict)
    cs: np.ndarray | None = None        # [3 (E,U,D)][2 parties][2 limbs]
    tag_mults: np.ndarray | None = None
    delta: np.ndarray | None = None

    def __post_init__(self):
        if self.r1 is None:
            self.r1 = self.M
        rows, K, N = self.r1 - self.r0, self.K, self.N
        if self.conv is not None:
            C, H, W, k, st, pd = self.conv
            Ho, Wo = (H + 2 * pd - k) // st + 1, (W + 2 * pd - k) // st + 1
            if min(C, H, W, k, st) < 1 or pd < 0 or Ho < 1 or Wo < 1 or K != C * k * k or N != Ho * Wo:
                raise ValueError("convolution geometry does not give this K and N")
        if not 2 <= self.parties <= MAX_PARTIES:
            raise ValueError(f"parties must be in [2, {MAX_PARTIES}]")
        kn = (self.conv[0], self.conv[1] * self.conv[2]) if self.conv is not None else (K, N)
        P = self.parties
        shapes = {}
        for n in ("X", "tX", "A", "tA"):
            shapes[n] = (P, rows, K)
        for n in ("Y", "tY", "B", "tB"):
            shapes[n] = (P,) + kn
        for n in ("C", "tC", "R", "tR", "Z", "tZ", "Rf", "tRf", "Zf", "tZf"):
            shapes[n] = (P, rows, N)
        if self.compress not in (0, 1) or (self.compress == 1 and (self.r0, self.r1) != (0, self.M)):
            raise ValueError("compress is 0 (along N) or 1 (along M, over all rows)")
        L = N if self.compress == 1 else rows     # length of the compressed M x N quantities
        shapes.update(E=(rows, K), U=kn, D=(rows, N), Uc=(K,), tBc=(P, K), Dc=(L,), EUc=(L,),
                      tCc=(P, L), tRc=(P, L), tZc=(P, L), tDc=(P, L), Ec=(K,), tAc=(P, K))
        for n, s in shapes.items():
            self.arrays[n] = np.zeros(s + (2,), dtype=np.uint64)
        self.delta = key_shares(self.key_seed, self.kbits, self.parties)

    def _desc(self):
        return _Desc(self.M, self.K, self.N, self.seed & MASK64, self.layer_id & MASK64, self.r0, self.r1,
                     self.f, self.in_bits, self.kbits, self.compress, *(self.conv or (0, 0, 0, 0, 0, 0)),
                     self.parties)

    def _bufs(self):
        b = _Bufs()
        for n, c in _BUF_FIELDS:
            a = self.arrays[n]
            if c == 2:
                setattr(b, n, _P2(*[_ptr(a[p]) for p in range(self.parties)]))
            else:
                setattr(b, n, _ptr(a))
        return b

    def deal(self, with_inputs: bool = True):
        b = self._bufs()
        lib().or_deal(ctypes.byref(self._desc()), _ptr(self.delta), int(with_inputs), ctypes.byref(b))
        return self

    def online(self, mode: int):
        b = self._bufs()
        lib().or_online(mode, ctypes.byref(self._desc()), _ptr(self.delta), ctypes.byref(b))
        self.tag_mults = np.array(b.tag_mults, dtype=np.uint64)[:self.parties]
        return self

    def check(self, mode: int):
        b = self._bufs()
        lib().or_check(mode, ctypes.byref(self._desc()), _ptr(self.delta), ctypes.byref(b))
        self.cs = np.array(b.cs, dtype=np.uint64).reshape(3, MAX_PARTIES, 2)[:, :self.parties].copy()
        return self

    def cs_sums(self):
        """sum over parties of each check value, mod 2^{k+s}: [E, U, D]."""
        mask = MASK128 if self.kbits == 64 else MASK64
        return [sum(u128(self.cs[w, p]) for p in range(self.parties)) & mask for w in range(3)]

    def accept(self) -> bool:
        return all(s == 0 for s in self.cs_sums())

    def __getitem__(self, name):
        return self.arrays[name]


def run_layer(mode: int, M: int, K: int, N: int, seed: int, layer_id: int, key_seed: int,
              r0: int = 0, r1: int | None = None, f: int = 0, in_bits: int = 0, kbits: int = 64,
              compress: int = 0, conv: tuple | None = None, parties: int = 2) -> OracleLayer:
    """Dealer, online phase and verification of one layer on rows [r0, r1)
    (with f > 0 the product is truncated by f fractional bits; kbits = k = s;
    compress = 1 compresses along M, over all rows; conv = (C, H, W, k,
    stride, pad) makes the layer a convolution of a C x H x W input)."""
    L = OracleLayer(M, K, N, seed, layer_id, key_seed, r0, r1, f, in_bits, kbits, compress, conv, parties)
    return L.deal().online(mode).check(mode)


# ---------------------------------------------------------------------------
# building blocks with chosen combiners

def matmul(P: np.ndarray, Q: np.ndarray) -> np.ndarray:
    M, K = P.shape[:2]
    N = Q.shape[1]
    out = np.zeros((M, N, 2), dtype=np.uint64)
    lib().or_matmul(M, K, N, _ptr(np.ascontiguousarray(P)), _ptr(np.ascontiguousarray(Q)), _ptr(out))
    return out


def compress(Mx: np.ndarray, chi: np.ndarray) -> np.ndarray:
    rows, N = Mx.shape[:2]
    out = np.zeros((rows, 2), dtype=np.uint64)
    lib().or_compress(rows, N, _ptr(np.ascontiguousarray(Mx)), _ptr(np.ascontiguousarray(chi, dtype=np.uint64)),
                      _ptr(out))
    return out


def im2col(L: OracleLayer, a: np.ndarray) -> np.ndarray:
    """The K x N im2col matrix (Eq. (4)) of a C x (H W) array of a convolution layer."""
    out = np.zeros((L.K, L.N, 2), dtype=np.uint64)
    lib().or_im2col(ctypes.byref(L._desc()), _ptr(np.ascontiguousarray(a)), _ptr(out))
    return out


def compress_rows(Mx: np.ndarray, chi: np.ndarray) -> np.ndarray:
    """chi^T Mx: one entry per column of Mx."""
    rows, N = Mx.shape[:2]
    out = np.zeros((N, 2), dtype=np.uint64)
    lib().or_compress_rows(rows, N, _ptr(np.ascontiguousarray(Mx)),
                           _ptr(np.ascontiguousarray(chi, dtype=np.uint64)), _ptr(out))
    return out


def batchrec_cs(W: np.ndarray, tW: np.ndarray, chi: np.ndarray, delta_p: int) -> int:
    out = np.zeros(2, dtype=np.uint64)
    n = W.size // 2
    lib().or_batchrec_cs(n, _ptr(np.ascontiguousarray(W)), _ptr(np.ascontiguousarray(tW)),
                         _ptr(np.ascontiguousarray(chi, dtype=np.uint64)), delta_p & MASK64, _ptr(out))
    return u128(out)


def compact_cs(Dc: np.ndarray, tDc: np.ndarray, chihat: np.ndarray, delta_p: int) -> int:
    out = np.zeros(2, dtype=np.uint64)
    lib().or_compact_cs(Dc.shape[0], _ptr(np.ascontiguousarray(Dc)), _ptr(np.ascontiguousarray(tDc)),
                        _ptr(np.ascontiguousarray(chihat, dtype=np.uint64)), delta_p & MASK64, _ptr(out))
    return u128(out)


# ---------------------------------------------------------------------------
# closed-form operation counts of Sec. 3.4.3 (per party)

def spdz2k_tag_mults(M: int, K: int, N: int) -> int:
    return 3 * M * K * N + M * N


def compact_tag_mults(M: int, K: int, N: int, compress: int = 0) -> int:
    """compress = 1 (along M) exchanges the roles of M and N."""
    if compress == 1:
        return 4 * M * N + 2 * K * M + 3 * N * K + N
    return 4 * M * N + 2 * K * N + 3 * M * K + M


def cheaper_compress(M: int, K: int, N: int) -> int:
    """The compressed dimension with the smaller count: 1 (M) exactly when M > N."""
    return 1 if compact_tag_mults(M, K, N, 1) < compact_tag_mults(M, K, N, 0) else 0
