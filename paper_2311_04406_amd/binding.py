"""ctypes binding of libcompacttag (argument marshalling only).

Every step of the hot path runs in the HIP library; this module only builds
the C structures of ``include/compacttag.h`` from torch tensors and forwards
the calls.  Device memory and the stream come from PyTorch (ROCm build): each
ring matrix is a ``torch.int64`` tensor of shape ``[rows, cols, limbs]``
holding the little-endian 64-bit limbs of its elements -- two for Z_{2^128}
(k = s = 64), one for Z_{2^64} (k = s = 32).

There is no CPU fallback: if the library is not built or no GPU is visible,
``load()`` raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcompacttag.so")

MODE_SPDZ2K = 0
MODE_COMPACT = 1
CT_OK, CT_EINVAL, CT_ENOMEM, CT_EDEVICE, CT_ABORT = 0, 1, 2, 3, 4
STATUS = {0: "CT_OK", 1: "CT_EINVAL", 2: "CT_ENOMEM", 3: "CT_EDEVICE", 4: "CT_ABORT"}
STATIC_WORK_BYTES = 256 << 20   # CT_STATIC_WORK_BYTES
MASK64 = (1 << 64) - 1
SKINNY_N = 8


def work_len(M: int, K: int, N: int, parties: int = 2) -> int:
    """CT_WORK_LEN_NP of compacttag.h: workspace elements of one layer."""
    if N <= SKINNY_N:
        return 0
    tiles = lambda d: ((d + 63) // 64) * ((K + 31) // 32)
    return (parties + 1) * M * K + (2 * parties + 1) * 2048 * (tiles(M) + tiles(N))


MAX_PARTIES = 5   # CT_MAX_PARTIES


class CtParams(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("key_seed", ctypes.c_uint64), ("k_bits", ctypes.c_int),
                ("s_bits", ctypes.c_int), ("hip_stream", ctypes.c_void_p), ("max_layers", ctypes.c_int),
                ("parties", ctypes.c_int)]


class CtLayerDesc(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("K", ctypes.c_int64), ("N", ctypes.c_int64), ("f", ctypes.c_int32),
                ("in_bits", ctypes.c_int32), ("seed", ctypes.c_uint64), ("layer_id", ctypes.c_uint64),
                ("compress", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("conv_c", ctypes.c_int32), ("conv_h", ctypes.c_int32), ("conv_w", ctypes.c_int32),
                ("conv_k", ctypes.c_int32), ("conv_stride", ctypes.c_int32), ("conv_pad", ctypes.c_int32)]


# compressed dimension of the compact tag (CT_COMPRESS_*)
COMPRESS_N, COMPRESS_M, COMPRESS_AUTO = 0, 1, 2


def compress_along_m(M: int, N: int, compress: int) -> bool:
    """CT_COMPRESS_ALONG_M: AUTO takes M exactly when M > N."""
    return compress == COMPRESS_M or (compress == COMPRESS_AUTO and M > N)


def cvec_len(M: int, K: int, N: int, compress: int = COMPRESS_N) -> int:
    """CT_CVEC_LEN_FOR: 3 K + 10 L, L = N when compressing along M, else M."""
    return 3 * K + 10 * (N if compress_along_m(M, N, compress) else M)


_P2 = ctypes.c_void_p * MAX_PARTIES   # one pointer per party slot
BUF_PAIRS = ["X", "tX", "A", "tA", "Y", "tY", "B", "tB", "C", "tC", "R", "tR", "Z", "tZ"]
BUF_SINGLE = ["E", "U", "D", "cvec", "work"]
BUF_TRUNC = ["Rf", "tRf", "Zf", "tZf"]  # f > 0 only


class CtLayerBufs(ctypes.Structure):
    _fields_ = [(n, _P2) for n in BUF_PAIRS] + [(n, ctypes.c_void_p) for n in BUF_SINGLE] + \
               [(n, _P2) for n in BUF_TRUNC]


class CtStageTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("total_ms", ctypes.c_double), ("launches", ctypes.c_int64)]


class CtTuning(ctypes.Structure):
    _fields_ = [("group_m", ctypes.c_int32), ("xcd_remap", ctypes.c_int32), ("split_target", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("gemm_ms", ctypes.c_double)]


# product kernel and workgroup tile shape (CT_TILE_*)
TILE_AUTO, TILE_LDS_64x64, TILE_LDS_128x64, TILE_REGS_64x64, TILE_REGS_128x64, TILE_REGS_FIT = 0, 1, 2, 3, 4, 5
# launch of the online phase (CT_LAUNCH_*)
LAUNCH_STAGED, LAUNCH_PERSISTENT = 0, 1
LAUNCH_WAIT_DEFAULT = 200000000  # 2 s of the device's 100 MHz wall clock
TILE_NAMES = {0: "auto", 1: "lds_64x64", 2: "lds_128x64", 3: "regs_64x64", 4: "regs_128x64", 5: "regs_fit"}


class CtCheckResult(ctypes.Structure):
    _fields_ = [("cs", ctypes.c_uint64 * (3 * MAX_PARTIES * 2)), ("accept", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


# int64 words of one ct_check_result (the device result records of the fused calls)
RESULT_WORDS = ctypes.sizeof(CtCheckResult) // 8


REQ_TAG, REQ_CHECK, REQ_PREP = 0, 1, 2


class CtServerParams(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t), ("slots", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("mode", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class CtRequest(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("layer", CtLayerDesc), ("arrival_us", ctypes.c_double)]


class CtCompletion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("kind", ctypes.c_int32), ("status", ctypes.c_int32),
                ("layer", ctypes.c_int64), ("arrival_us", ctypes.c_double), ("admit_us", ctypes.c_double),
                ("done_us", ctypes.c_double), ("batch_size", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("result", CtCheckResult)]


class CtServerCounts(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "rejected", "converted", "evictions",
                                              "batches", "max_batch", "resident_layers")] + \
               [(n, ctypes.c_uint64) for n in ("arena_bytes", "arena_peak", "arena_used")] + \
               [("duplicates", ctypes.c_int64), ("prepared", ctypes.c_int64), ("online_only", ctypes.c_int64)]


_lib = None


def load() -> ctypes.CDLL:
    """Loads the built HIP library; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2311_04406_amd.build` "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i = ctypes.c_void_p, ctypes.c_int
    L.ct_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(CtParams)]
    L.ct_destroy.argtypes = [vp]
    L.ct_key_shares.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
    L.ct_gen_triple_tags.argtypes = [vp, ctypes.POINTER(CtLayerDesc), ctypes.POINTER(CtLayerBufs), i, i]
    L.ct_tag_linear.argtypes = [vp, i, ctypes.POINTER(CtLayerDesc), ctypes.POINTER(CtLayerBufs), i]
    L.ct_mac_check_device.argtypes = [vp, i, ctypes.POINTER(CtLayerDesc), ctypes.POINTER(CtLayerBufs), i, vp]
    L.ct_tag_linear_check.argtypes = [vp, i, ctypes.POINTER(CtLayerDesc), ctypes.POINTER(CtLayerBufs), i, vp]
    L.ct_tag_linear_check_static.argtypes = [vp, i, ctypes.POINTER(CtLayerDesc), ctypes.POINTER(CtLayerBufs), i,
                                             vp]
    L.ct_mac_check.argtypes = [vp, i, ctypes.POINTER(CtLayerDesc), ctypes.POINTER(CtLayerBufs), i,
                               ctypes.POINTER(CtCheckResult)]
    L.ct_set_timing.argtypes = [vp, i]
    L.ct_set_overlap.argtypes = [vp, i]
    L.ct_set_launch.argtypes = [vp, i]
    L.ct_set_launch_wait.argtypes = [vp, ctypes.c_uint64]
    L.ct_stage_times.argtypes = [vp, ctypes.POINTER(CtStageTime), i, ctypes.POINTER(ctypes.c_int)]
    L.ct_autotune.argtypes = [vp, i, ctypes.POINTER(CtLayerDesc), ctypes.POINTER(CtLayerBufs), i, i,
                              ctypes.POINTER(CtTuning)]
    L.ct_get_tuning.argtypes = [vp, i, ctypes.POINTER(CtLayerDesc), i, ctypes.POINTER(CtTuning)]
    L.ct_set_tuning.argtypes = [vp, ctypes.POINTER(CtTuning)]
    L.ct_plan_create.argtypes = [vp, i, ctypes.POINTER(CtLayerDesc), ctypes.POINTER(CtLayerBufs), i, vp,
                                 ctypes.POINTER(vp)]
    L.ct_plan_launch.argtypes = [vp]
    L.ct_plan_destroy.argtypes = [vp]
    L.ct_server_create.argtypes = [vp, ctypes.POINTER(CtServerParams), ctypes.POINTER(vp)]
    L.ct_server_now_us.argtypes = [vp]
    L.ct_server_now_us.restype = ctypes.c_double
    L.ct_server_submit.argtypes = [vp, ctypes.POINTER(CtRequest), i]
    L.ct_server_poll.argtypes = [vp, ctypes.POINTER(CtCompletion), i, ctypes.POINTER(ctypes.c_int)]
    L.ct_server_drain.argtypes = [vp, ctypes.c_double]
    L.ct_server_layer.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(CtLayerDesc), ctypes.POINTER(CtLayerBufs)]
    L.ct_server_stats.argtypes = [vp, ctypes.POINTER(CtServerCounts)]
    L.ct_server_destroy.argtypes = [vp]
    L.ct_server_last_error.argtypes = [vp]
    L.ct_server_last_error.restype = ctypes.c_char_p
    L.ct_last_error.argtypes = [vp]
    L.ct_last_error.restype = ctypes.c_char_p
    for f in ("ct_create", "ct_destroy", "ct_key_shares", "ct_gen_triple_tags", "ct_tag_linear",
              "ct_mac_check_device", "ct_mac_check", "ct_tag_linear_check_static", "ct_set_timing", "ct_set_overlap", "ct_set_launch", "ct_set_launch_wait", "ct_stage_times", "ct_tag_linear_check",
              "ct_autotune", "ct_get_tuning", "ct_set_tuning", "ct_plan_create", "ct_plan_launch",
              "ct_plan_destroy", "ct_server_create", "ct_server_submit", "ct_server_poll", "ct_server_drain",
              "ct_server_layer", "ct_server_stats", "ct_server_destroy"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


class CtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


@dataclass
class CheckResult:
    cs: list            # cs[W][p] as Python ints, W in (E, U, D), p over the parties
    accept: bool
    reserved: int = 0   # 1: a persistent launch's barrier wait ran out


def _result(r: CtCheckResult, parties: int = 2) -> CheckResult:
    v = list(r.cs)
    m = 2 * MAX_PARTIES
    cs = [[v[m * w + 2 * p] | (v[m * w + 2 * p + 1] << 64) for p in range(parties)] for w in range(3)]
    return CheckResult(cs=cs, accept=bool(r.accept), reserved=int(r.reserved))


class Layer:
    """Device buffers of one linear layer (every party), as torch tensors of
    `limbs` 64-bit words per element (2: k = s = 64; 1: k = s = 32)."""

    def __init__(self, M: int, K: int, N: int, seed: int, layer_id: int, device="cuda:0", f: int = 0,
                 in_bits: int = 0, limbs: int = 2, compress: int = COMPRESS_N, conv=None, parties: int = 2):
        """conv = (C, H, W, k, stride, pad): a convolution whose right operand
        is the implicit im2col matrix of a C x H x W input; Y, tY, B, tB and U
        then have the input's shape, stored as C x (H W).  parties: the share
        arrays hold one tensor per party."""
        self.M, self.K, self.N, self.seed, self.layer_id, self.f = M, K, N, seed, layer_id, f
        self.in_bits, self.limbs, self.compress, self.parties = in_bits, limbs, compress, parties
        self.conv = tuple(conv) if conv is not None else None
        self.t = {}
        kn = (self.conv[0], self.conv[1] * self.conv[2]) if self.conv else (K, N)
        dims = {"MK": (M, K), "KN": kn, "MN": (M, N)}
        groups = {"MK": ["X", "tX", "A", "tA"], "KN": ["Y", "tY", "B", "tB"],
                  "MN": ["C", "tC", "R", "tR", "Z", "tZ"] + (BUF_TRUNC if f > 0 else [])}
        w = limbs
        for g, names in groups.items():
            for n in names:
                self.t[n] = [torch.zeros(dims[g] + (w,), dtype=torch.int64, device=device) for _ in range(parties)]
        self.t["E"] = torch.zeros((M, K, w), dtype=torch.int64, device=device)
        self.t["U"] = torch.zeros(kn + (w,), dtype=torch.int64, device=device)
        self.t["D"] = torch.zeros((M, N, w), dtype=torch.int64, device=device)
        nc = cvec_len(M, K, N, compress) if parties == 2 else (1 + parties) * K + (2 + 4 * parties) * M
        self.t["cvec"] = torch.zeros((nc, w), dtype=torch.int64, device=device)
        self.t["work"] = torch.zeros((max(1, work_len(M, K, N, parties)), w), dtype=torch.int64, device=device)

    @classmethod
    def wrap(cls, M: int, K: int, N: int, seed: int, layer_id: int, tensors: dict,
             compress: int = COMPRESS_N) -> "Layer":
        """A Layer over existing device tensors (no allocation)."""
        obj = cls.__new__(cls)
        obj.M, obj.K, obj.N, obj.seed, obj.layer_id, obj.f = M, K, N, seed, layer_id, 0
        obj.in_bits, obj.limbs, obj.compress, obj.conv, obj.parties = 0, 2, compress, None, 2
        obj.t = dict(tensors)
        return obj

    @staticmethod
    def footprint_bytes(M: int, K: int, N: int) -> int:
        return 16 * (9 * M * K + 9 * K * N + 13 * M * N + 3 * K + 10 * M + work_len(M, K, N))

    def __getitem__(self, name):
        return self.t[name]

    def desc(self) -> CtLayerDesc:
        return CtLayerDesc(self.M, self.K, self.N, self.f, self.in_bits, self.seed & MASK64, self.layer_id & MASK64,
                           self.compress, 0, *(self.conv or (0, 0, 0, 0, 0, 0)))

    @property
    def along_m(self) -> bool:
        return compress_along_m(self.M, self.N, self.compress)

    def bufs(self) -> CtLayerBufs:
        b = CtLayerBufs()
        for n in BUF_PAIRS:
            setattr(b, n, _P2(*[t.data_ptr() for t in self.t[n]]))
        for n in BUF_SINGLE:
            setattr(b, n, self.t[n].data_ptr())
        for n in BUF_TRUNC:
            if n in self.t:
                setattr(b, n, _P2(*[t.data_ptr() for t in self.t[n]]))
        return b

    # cvec views (element offsets of compacttag.h); compressed along M, the
    # K-long parts hold E^c, [tA^c]_p (named Ec, tAc0, tAc1) and the others have N entries
    def cvec_parts(self):
        K, c = self.K, self.t["cvec"]
        if getattr(self, "parties", 2) > 2:  # CT_CVEC_LEN_NP layout
            P, M = self.parties, self.M
            o = {"Uc": (0, K)}
            for p in range(P):
                o[f"tBc{p}"] = ((1 + p) * K, K)
            dc = (1 + P) * K
            o["Dc"], o["EUc"] = (dc, M), (dc + M, M)
            for g, name in enumerate(("tCc", "tRc", "tZc", "tDc")):
                for p in range(P):
                    o[f"{name}{p}"] = (dc + (2 + g * P + p) * M, M)
            return {n: c[a:a + l] for n, (a, l) in o.items()}
        M = self.N if self.along_m else self.M
        k3 = ("Ec", "tAc0", "tAc1") if self.along_m else ("Uc", "tBc0", "tBc1")
        o = {k3[0]: (0, K), k3[1]: (K, K), k3[2]: (2 * K, K), "Dc": (3 * K, M), "EUc": (3 * K + M, M)}
        base = 3 * K + 2 * M
        for i, n in enumerate(["tCc0", "tCc1", "tRc0", "tRc1", "tZc0", "tZc1", "tDc0", "tDc1"]):
            o[n] = (base + i * M, M)
        return {n: c[a:a + l] for n, (a, l) in o.items()}


def _arrays(layers):
    n = len(layers)
    D = (CtLayerDesc * n)(*[l.desc() for l in layers])
    B = (CtLayerBufs * n)(*[l.bufs() for l in layers])
    return n, D, B


class Context:
    """A libcompacttag context bound to one device and one HIP stream."""

    def __init__(self, device: int = 0, key_seed: int = 0, stream=None, max_layers: int = 256, kbits: int = 64,
                 parties: int = 2):
        """kbits = k = s: 64 (shares and tags in Z_{2^128}) or 32 (in Z_{2^64})."""
        self.lib = load()
        self.kbits = kbits
        self.parties = parties
        self.limbs = 2 if kbits == 64 else 1
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: libcompacttag needs an MI355X (there is no CPU fallback)")
        self.device = device
        self.torch_device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.torch_device)
        self.stream = stream
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        p = CtParams(device, key_seed & MASK64, kbits, kbits, handle, max_layers, parties)
        h = ctypes.c_void_p()
        s = self.lib.ct_create(ctypes.byref(h), ctypes.byref(p))
        if s != CT_OK:
            raise CtError(s, "ct_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.ct_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s: int, allow_abort: bool = False):
        if s == CT_OK or (allow_abort and s == CT_ABORT):
            return s
        raise CtError(s, self.lib.ct_last_error(self.h).decode())

    def key_shares(self):
        out = (ctypes.c_uint64 * MAX_PARTIES)()
        self._check(self.lib.ct_key_shares(self.h, out))
        return [int(out[p]) for p in range(self.parties)]

    def gen_triple_tags(self, layers, with_inputs: bool = True):
        n, D, B = _arrays(layers)
        self._check(self.lib.ct_gen_triple_tags(self.h, D, B, n, int(with_inputs)))

    def tag_linear(self, mode: int, layers):
        n, D, B = _arrays(layers)
        self._check(self.lib.ct_tag_linear(self.h, mode, D, B, n))

    def mac_check_device(self, mode: int, layers, out: torch.Tensor):
        """out: int64 device tensor of n * RESULT_WORDS entries (n ct_check_result records)."""
        n, D, B = _arrays(layers)
        assert out.numel() * 8 >= n * ctypes.sizeof(CtCheckResult)
        self._check(self.lib.ct_mac_check_device(self.h, mode, D, B, n, ctypes.c_void_p(out.data_ptr())))

    def tag_linear_check(self, mode: int, layers, out: torch.Tensor):
        """Online phase with the verification fused in; n check records to `out` (device)."""
        n, D, B = _arrays(layers)
        assert out.numel() * 8 >= n * ctypes.sizeof(CtCheckResult)
        self._check(self.lib.ct_tag_linear_check(self.h, mode, D, B, n, ctypes.c_void_p(out.data_ptr())))

    def tag_linear_check_static(self, mode: int, layers, out: torch.Tensor):
        """As tag_linear_check, with the workspace taken from the library's
        static per-GPU array (the layers' own work tensors are not used)."""
        n, D, B = _arrays(layers)
        assert out.numel() * 8 >= n * ctypes.sizeof(CtCheckResult)
        self._check(self.lib.ct_tag_linear_check_static(self.h, mode, D, B, n, ctypes.c_void_p(out.data_ptr())))

    def mac_check(self, mode: int, layers):
        n, D, B = _arrays(layers)
        res = (CtCheckResult * n)()
        s = self._check(self.lib.ct_mac_check(self.h, mode, D, B, n, res), allow_abort=True)
        out = [_result(r, self.parties) for r in res]
        return s, out

    def autotune(self, mode: int, layers, reps: int = 2) -> dict:
        """Chooses the matrix-core launch configuration for this layer batch's
        shape class (runs the online phase once per candidate)."""
        n, D, B = _arrays(layers)
        t = CtTuning()
        self._check(self.lib.ct_autotune(self.h, mode, D, B, n, reps, ctypes.byref(t)))
        return {"group_m": t.group_m, "xcd_remap": t.xcd_remap, "split_target": t.split_target,
                "tile": TILE_NAMES.get(t.tile, t.tile), "gemm_ms": t.gemm_ms}

    def get_tuning(self, mode: int, layers) -> dict:
        n, D, B = _arrays(layers)
        t = CtTuning()
        self._check(self.lib.ct_get_tuning(self.h, mode, D, n, ctypes.byref(t)))
        return {"group_m": t.group_m, "xcd_remap": t.xcd_remap, "split_target": t.split_target,
                "tile": TILE_NAMES.get(t.tile, t.tile)}

    def set_tuning(self, group_m: int = 1, xcd_remap: int = 0, split_target: int = 0, tile: int = TILE_AUTO):
        """Launch configuration of shape classes never tuned (tile: TILE_*)."""
        t = CtTuning(group_m, xcd_remap, split_target, tile, 0.0)
        self._check(self.lib.ct_set_tuning(self.h, ctypes.byref(t)))

    def set_timing(self, enable: bool):
        self._check(self.lib.ct_set_timing(self.h, int(enable)))

    def set_overlap(self, enable: bool):
        """Mixed batches on two streams (default) or all on the context stream."""
        self._check(self.lib.ct_set_overlap(self.h, int(enable)))

    def set_launch(self, mode: int):
        """LAUNCH_STAGED (one kernel per stage) or LAUNCH_PERSISTENT (one launch)."""
        self._check(self.lib.ct_set_launch(self.h, int(mode)))

    def set_launch_wait(self, ticks: int = LAUNCH_WAIT_DEFAULT):
        """Bound of the persistent launch's barrier waits (100 MHz ticks)."""
        self._check(self.lib.ct_set_launch_wait(self.h, int(ticks)))

    def stage_times(self):
        """{stage: (total_ms, launches)} since the previous call (synchronizes)."""
        buf = (CtStageTime * 32)()
        cnt = ctypes.c_int()
        self._check(self.lib.ct_stage_times(self.h, buf, 32, ctypes.byref(cnt)))
        return {buf[i].name.decode(): (buf[i].total_ms, int(buf[i].launches)) for i in range(min(cnt.value, 32))}

    def layer(self, M: int, K: int, N: int, seed: int, layer_id: int, f: int = 0, in_bits: int = 0,
              compress: int = COMPRESS_N, conv=None) -> Layer:
        """Buffers of one layer for this context's parameter set."""
        return Layer(M, K, N, seed, layer_id, device=self.torch_device, f=f, in_bits=in_bits, limbs=self.limbs,
                     compress=compress, conv=conv, parties=self.parties)

    def plan(self, mode: int, layers, out: torch.Tensor | None = None) -> "Plan":
        """Captures the online phase of this layer batch (with the fused
        verification if `out` is given) into a HIP graph; see Plan."""
        n, D, B = _arrays(layers)
        if out is not None:
            assert out.numel() * 8 >= n * ctypes.sizeof(CtCheckResult)
        h = ctypes.c_void_p()
        self._check(self.lib.ct_plan_create(self.h, mode, D, B, n,
                                            ctypes.c_void_p(out.data_ptr()) if out is not None else None,
                                            ctypes.byref(h)))
        return Plan(self, h, layers, out)

    @staticmethod
    def decode_results(t: torch.Tensor, n: int, parties: int = 2):
        """Decodes ct_check_result records copied back from mac_check_device."""
        raw = t.detach().cpu().contiguous().numpy().tobytes()
        arr = (CtCheckResult * n).from_buffer_copy(raw[: n * ctypes.sizeof(CtCheckResult)])
        return [_result(r, parties) for r in arr]


class Plan:
    """A captured online phase (ct_plan): launch() replays its HIP graph on
    the context stream; the layers and result tensor stay bound to it."""

    def __init__(self, ctx: Context, handle, layers, out):
        self.ctx, self.h, self.layers, self.out = ctx, handle, list(layers), out

    def launch(self):
        self.ctx._check(self.ctx.lib.ct_plan_launch(self.h))

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.ct_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _status_name(s: int) -> str:
    return STATUS.get(s, str(s))


class Server:
    """The request server (ct_server_*): continuous batching of tag-generation
    and check requests over one device arena, allocated here with PyTorch.
    The server's worker thread owns `ctx` until close()."""

    def __init__(self, ctx: Context, arena_bytes: int, slots: int = 2, max_batch: int = 32,
                 mode: int = MODE_COMPACT):
        self.ctx, self.lib = ctx, ctx.lib
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=ctx.torch_device)
        torch.cuda.synchronize(ctx.torch_device)
        p = CtServerParams(self.arena.data_ptr(), arena_bytes, slots, max_batch, mode, 0)
        h = ctypes.c_void_p()
        s = self.lib.ct_server_create(ctx.h, ctypes.byref(p), ctypes.byref(h))
        if s != CT_OK:
            raise CtError(s, self.lib.ct_last_error(ctx.h).decode())
        self.h = h

    def _check(self, s: int):
        if s != CT_OK:
            raise CtError(s, self.lib.ct_server_last_error(self.h).decode())

    def now_us(self) -> float:
        return float(self.lib.ct_server_now_us(self.h))

    def submit(self, reqs):
        """reqs: iterable of (id, kind, (M, K, N, seed, layer_id[, compress]), arrival_us)."""
        reqs = list(reqs)
        arr = (CtRequest * max(1, len(reqs)))()
        for i, (rid, kind, lay, t) in enumerate(reqs):
            M, K, N, seed, lid = lay[:5]
            cmp = lay[5] if len(lay) > 5 else COMPRESS_N
            arr[i] = CtRequest(rid, kind, 0, CtLayerDesc(M, K, N, 0, 0, seed & MASK64, lid & MASK64, cmp, 0), t)
        self._check(self.lib.ct_server_submit(self.h, arr, len(reqs)))

    def poll(self, max_items: int = 4096):
        buf = (CtCompletion * max_items)()
        cnt = ctypes.c_int()
        self._check(self.lib.ct_server_poll(self.h, buf, max_items, ctypes.byref(cnt)))
        out = []
        for i in range(cnt.value):
            c = buf[i]
            out.append({"id": c.id, "kind": c.kind, "status": c.status, "status_name": _status_name(c.status),
                        "layer": c.layer, "arrival_us": c.arrival_us, "admit_us": c.admit_us,
                        "done_us": c.done_us, "batch_size": c.batch_size, "slot": c.slot,
                        "result": _result(c.result)})
        return out

    def drain(self, timeout_s: float = 120.0):
        self._check(self.lib.ct_server_drain(self.h, timeout_s))

    def layer(self, rid: int) -> Layer:
        """The resident layer written by TAG request rid, as torch views into the arena."""
        d, b = CtLayerDesc(), CtLayerBufs()
        self._check(self.lib.ct_server_layer(self.h, rid, ctypes.byref(d), ctypes.byref(b)))
        M, K, N = d.M, d.K, d.N
        base = self.arena.data_ptr()

        def view(ptr, rows, cols):
            off = ptr - base
            return self.arena[off: off + rows * cols * 16].view(torch.int64).view(rows, cols, 2)
        dims = {"MK": (M, K), "KN": (K, N), "MN": (M, N)}
        groups = {"MK": ["X", "tX", "A", "tA"], "KN": ["Y", "tY", "B", "tB"],
                  "MN": ["C", "tC", "R", "tR", "Z", "tZ"]}
        t = {}
        for g, names in groups.items():
            for n in names:
                pair = getattr(b, n)
                t[n] = [view(pair[q], *dims[g]) for q in range(2)]
        t["E"] = view(b.E, M, K)
        t["U"] = view(b.U, K, N)
        t["D"] = view(b.D, M, N)
        off = b.cvec - base
        n = cvec_len(M, K, N, d.compress)
        t["cvec"] = self.arena[off: off + n * 16].view(torch.int64).view(n, 2)
        return Layer.wrap(M, K, N, d.seed, d.layer_id, t, d.compress)

    def stats(self) -> dict:
        c = CtServerCounts()
        self._check(self.lib.ct_server_stats(self.h, ctypes.byref(c)))
        return {n: int(getattr(c, n)) for n, _ in CtServerCounts._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.ct_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
