#!/usr/bin/env python3
"""Benchmark of the linear-layer hot path on one MI355X.

A step is one pass of the whole hot path over one batch of layers: the online
phase (open E and U, output-share products, tags) with the verification
fused in (batch tag checks of E and U, check of D), for every layer of the
workload, launched as one captured HIP graph (ct_plan_launch; a batch that
mixes matrix-core layers with row-pass-only layers runs the two groups on two
streams forked and joined inside the graph).  The per-kernel breakdown comes
from a second, untimed pass with per-launch timing, which runs every stage
once over the whole batch on one stream.  The dealer
runs once before the timed region and is not timed.  Inputs are synthetic
(uniform ring elements from the dealer's seeded generator) and resident in
HBM.

Prints one JSON line.  Default workload: the batched layer set (64 linear
layers with M, K, N log-uniform in [32, 4096], seeded; the largest
configuration by sum M K N), CompactTag protocol, with beside it: the same
step as eager calls, the SPDZ2k protocol, one plain launch per layer, the
check as a separate call, the step as one persistent launch, a per-kernel breakdown with the dominant kernel's
roofline, the captured steps of the CNN and encoder layer sets (--extra), a
serving leg (open-loop Poisson arrivals of single-layer requests, p50/p99
latency) and the oracle on the host (all host threads up to 16, and one).
--config serving runs the full serving sweep.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tagged ring-MACs/sec (Z_2^64 GEMM Gops) + p50/p99 tag latency, 1 MI355X"
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
INT8_PEAK_TOPS = 5000.0      # MI355X dense int8 MFMA, 5.0 POP/s
DIGIT_PAIRS = 136            # int8 digit products per 128-bit ring multiply-accumulate


def along_m(s, compress: str) -> bool:
    """Whether the compact tag of layer s is compressed along M (AUTO: exactly when M > N)."""
    return compress == "m" or (compress == "auto" and s.M > s.N)


def persistent_applies(specs, compress: str, parties: int, implicit: bool) -> bool:
    """Whether ct_set_launch(CT_LAUNCH_PERSISTENT) runs a batch as the one
    persistent launch (two parties; every layer a matrix-core layer that is
    not an implicit-im2col convolution and not compressed along M) or as the
    staged kernels."""
    return parties == 2 and all(s.N > 8 and not (implicit and s.conv is not None) and not along_m(s, compress)
                                for s in specs)


def stage_work(stage: str, specs, mode: str, f: int = 0, kbits: int = 64, compress: str = "n",
               implicit: bool = False, parties: int = 2):
    """Algorithmic work of one launch of a kernel stage over the layer batch:
    ("hbm", bytes) or ("mfma", int8 ops), for the fused step
    (online phase + verification).  16 B per Z_2^128 element; per element,
    with n parties (two: the figures in brackets):
      open_u     K x N: reads Y_p, B_p, tY_p, tB_p (4 n), writes U:
                 64 n + 16 B [144]; two-party matrix-core layers that are
                 not convolutions take open_pack instead
      open_pack  those layers, K x N: the same, and writes the digit tiles
                 of [B]_0, [B]_1, U (16 B each per element): 192 B
      row_pass   M x K: reads X_p, A_p, tX_p, tA_p (4 n), writes E:
                 64 n + 16 B [144], plus the folded operands written for
                 matrix-core layers (A_0 + E; SPDZ2k also tA_p + Delta_p E):
                 16 [16] / 16 + 16 n [48] B
      pack       matrix-core layers: reads each operand once and writes its
                 digit tiles, 32 B per element: M x K: E, A_0 + E, [A]_p
                 (p > 0; SPDZ2k also the n folded tag operands):
                 32 (n + 1) [96] / 32 (2 n + 1) [160] B; K x N: [B]_p, U
                 (SPDZ2k also [tB]_p): the same counts, less the three
                 operands open_pack writes
      copy_base  M x N base copies of the products whose K range is split
                 (32 B per element); which products split depends on the
                 tile plan, so no byte figure is given
      ring_gemm  2 * 136 int8 ops per ring MAC; 2 n M K N ring MACs per
                 layer (4 n in SPDZ2k), layers with N > 8
      post       M x N: CompactTag reads R_p, Z_p, tR_p, tC_p (4 n), writes
                 D, tZ_p (n + 1): 80 n + 16 B [176] (beyond two parties tC_p
                 is compressed in a pass of its own: 64 n + 16 B); SPDZ2k reads R_p, Z_p,
                 tR_p, tZ_p (4 n), writes D: 64 n + 16 B [144]; with f > 0
                 also reads R^f_p, tR^f_p and writes Z^f_p, tZ^f_p: + 64 n B.
      col_tag    layers compressed along M, K x N: reads U, tB_p: 16 n + 16 B.
    With implicit convolutions (im2col left implicit) the right operand's
    arrays have the input's C H W elements: open_u moves its bytes per input
    element, the packing of each right operand reads 16 B per input element
    and writes 32 B per K x N entry, and conv_compress reads U, tB_p:
    16 n + 16 B per input element.
    With k = s = 32 elements are 8 B (every byte figure halves) and a ring
    MAC is 36 digit products."""
    scale = 1 if kbits == 64 else 0.5
    pairs = DIGIT_PAIRS if kbits == 64 else 36
    spdz = mode == "spdz2k"
    tot = 0
    for s in specs:
        M, K, N = s.M, s.K, s.N
        mk, kn, mn = M * K, K * N, M * N
        wide = N > 8
        conv = implicit and s.conv is not None
        nr = s.conv[0] * s.conv[1] * s.conv[2] if conv else kn
        n = parties
        elem = 64 * n + 16                  # 4 n share arrays read, one opened value written
        nops = (2 * n + 1) if spdz else (n + 1)  # packed operands per side
        fused = n == 2 and wide and not conv     # U opened and right operands packed in one pass
        if stage == "open_u":
            tot += 0 if fused else elem * nr
        elif stage == "open_pack":
            tot += (elem + 48) * kn if fused else 0
        elif stage == "row_pass":
            tot += elem * mk + ((16 + 16 * n if spdz else 16) * mk if wide else 0)
        elif stage == "pack":
            right = nops * (16 * nr + 32 * kn) if conv else 32 * (nops - (3 if fused else 0)) * kn
            tot += (32 * nops * mk + right) if wide else 0
        elif stage == "conv_compress":
            tot += (16 * n + 16) * nr if conv and not spdz and not along_m(s, compress) else 0
        elif stage == "copy_base":
            return None
        elif stage == "ring_gemm":
            tot += 2 * pairs * (4 if spdz else 2) * parties * M * K * N if wide else 0
        elif stage == "post":
            tot += ((64 * n + 16 if spdz or n > 2 else 80 * n + 16) + (64 * n if f > 0 else 0)) * mn
        elif stage == "col_tag":
            tot += (16 * n + 16) * kn if not spdz and along_m(s, compress) else 0
        else:
            return None
    if stage == "ring_gemm":
        return ("mfma", tot)
    return ("hbm", int(tot * scale))


# Sources that determine what the device kernels do; the hardware counters in
# profiles/traffic.json are valid only for the digest they were taken on.
KERNEL_SOURCES = ("ct_device.h", "ct_internal.h", "ct_sweep.h", "ct_passes.h", "ct_kernels.hip", "ct_gemm.hip",
                  "ct_parties.hip")


def strip_comments(src: str) -> str:
    """C/C++ source without its comments and trailing blanks: what the counters
    depend on (string literals in these files hold no comment markers)."""
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(line.rstrip() for line in src.splitlines() if line.strip())


def source_digest() -> str:
    """Digest of the kernel sources' code (comments ignored)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(strip_comments(open(os.path.join(ROOT, "paper_2311_04406_amd", "csrc", f)).read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get(workload, {}).get(kernel)
        if e and e.get("source_digest") == source_digest():
            return e["bytes_per_launch"]
    except Exception:
        return None
    return None


def measured_counters(kernel: str, workload: str):
    """MFMA busy fraction and clock of a product kernel from the committed
    rocprofv3 counter summary (profiles/counters.json), if it was taken on
    the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    try:
        e = json.load(open(path)).get(workload, {}).get(kernel)
        if e and e.get("source_digest") == source_digest():
            return {"mfma_busy": e["mfma_busy"], "clock_ghz": e.get("clock_ghz")}
    except Exception:
        return None
    return None


def pct(v, q):
    v = sorted(v)
    if not v:
        return None
    i = min(len(v) - 1, max(0, int(round(q / 100.0 * (len(v) - 1)))))
    return v[i]


def run_steps(ctx, mode_id, layer_groups, out_dev, steps, warmup, torch, timing=False, fused=True, plan=None):
    """Runs warmup + steps; each step launches the captured plan (one HIP
    graph launch) if given, else enqueues every group (one call per group):
    ct_tag_linear_check (fused) or ct_tag_linear + ct_mac_check_device.
    Returns (total seconds, per-step ms list, stage times)."""
    def step():
        if plan is not None:
            plan.launch()
            return
        for g in layer_groups:
            if fused:
                ctx.tag_linear_check(mode_id, g, out_dev)
            else:
                ctx.tag_linear(mode_id, g)
                ctx.mac_check_device(mode_id, g, out_dev)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if timing:
        ctx.set_timing(True)
        ctx.stage_times()  # reset
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        evs[i][0].record()
        step()
        evs[i][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = [a.elapsed_time(b) for a, b in evs]
    stages = None
    if timing:
        stages = ctx.stage_times()
        ctx.set_timing(False)
    return t1 - t0, per, stages


def cpu_threads() -> int:
    """Host threads for the oracle: the cores this process may run on, at most
    16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_sample(specs, budget_mkn: int = 1 << 30):
    """A bounded sample of the workload for the oracle: up to 16 layers spread
    over the batch, each on its first rows, at most budget / (number of
    layers) M K N per layer.  Returns [(spec, rows)]."""
    step = max(1, len(specs) // 16)
    pick = specs[::step][:16]
    per = budget_mkn // len(pick)
    out = []
    for s in pick:
        rows = max(1, min(s.M, per // max(1, s.K * s.N)))
        out.append((s, rows))
    return out


def cpu_baseline(specs, min_seconds: float = 10.0, kbits: int = 64, implicit: bool = False, parties: int = 2,
                 threads: int = 1, mode: int = 1):
    """The oracle (plain C, -O2) on a bounded sample of the workload (see
    cpu_sample): online phase + verification of the timed step's protocol,
    convolutions as the timed step runs them; the dealer is untimed.  With
    threads > 1 every sampled layer's rows are cut into ranges (about four
    per layer on large layers) that run concurrently on a thread pool (the
    oracle releases the interpreter lock; each range opens U and compresses
    the K x N operands itself, as a separate party computation would).  The
    sample is repeated until at least min_seconds of wall time have
    accumulated."""
    import concurrent.futures as cf

    import oracle as O
    from paper_2311_04406_amd.workloads import KEY_SEED
    parts = cpu_sample(specs)
    tasks = []
    for s, rows in parts:
        pieces = 1 if threads == 1 else max(1, min(4, rows // 8, (rows * s.K * s.N) // (1 << 24)))
        step = -(-rows // pieces)
        for r0 in range(0, rows, step):
            tasks.append((s, r0, min(rows, r0 + step)))
    tasks.sort(key=lambda t: -(t[2] - t[1]) * t[0].K * t[0].N)

    def deal(t):
        s, r0, r1 = t
        return O.OracleLayer(s.M, s.K, s.N, s.seed, s.layer_id, KEY_SEED, r0, r1, kbits=kbits,
                             conv=s.conv if implicit else None, parties=parties).deal()

    def run(L):
        L.online(mode).check(mode)
        return L
    t_tot, macs, passes = 0.0, 0, 0
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        dealt = list(ex.map(deal, tasks))   # untimed
        while passes == 0 or t_tot < min_seconds:
            t0 = time.perf_counter()
            if threads == 1:
                for L in dealt:
                    run(L)
            else:
                list(ex.map(run, dealt))
            t_tot += time.perf_counter() - t0
            macs += sum((r1 - r0) * s.K * s.N for s, r0, r1 in tasks)
            passes += 1
    full = [L for L, (s, r0, r1) in zip(dealt, tasks) if (r0, r1) == (0, s.M)]
    assert all(L.accept() for L in full)
    desc = ", ".join(f"{s.name} rows [0,{rows})" for s, rows in parts)
    return {"value": macs / t_tot / 1e9, "unit": "G ring-MAC/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(parts)} layers: {desc}; {len(tasks)} row ranges, {passes} passes; "
                      f"{'CompactTag' if mode == 1 else 'SPDZ2k'} online phase + verification, plain C oracle on "
                      f"{threads} host thread{'s' if threads > 1 else ''}; {t_tot:.1f} s",
            "seconds": t_tot, "ring_macs": macs}


def extra_run(torch, ctx, name: str, mode_id: int, args, implicit: bool, cmp: int) -> dict:
    """The captured step of another workload (same protocol and parameters):
    dealer untimed, the launch configuration autotuned unless disabled,
    warm-up, then the timed graph launches; honest acceptance checked."""
    from paper_2311_04406_amd import RESULT_WORDS, Context, workloads
    specs = workloads.CONFIGS[name]()
    layers = [ctx.layer(s.M, s.K, s.N, s.seed, s.layer_id, f=args.f, in_bits=args.in_bits, compress=cmp,
                        conv=s.conv if implicit else None) for s in specs]
    ctx.gen_triple_tags(layers)
    out_dev = torch.zeros(len(layers) * RESULT_WORDS, dtype=torch.int64, device="cuda:0")
    if not args.no_autotune and not args.tuning:
        ctx.autotune(mode_id, layers)
    plan = ctx.plan(mode_id, layers, out_dev)
    T, per, _ = run_steps(ctx, mode_id, [layers], out_dev, args.steps, args.warmup, torch, plan=plan)
    plan.close()
    res = Context.decode_results(out_dev, len(layers), args.parties)
    mkn = sum(s.mkn for s in specs)
    del layers
    return {"value": round(mkn * args.steps / T / 1e9, 3), "ms_per_step": round(T / args.steps * 1e3, 4),
            "p50_ms": round(pct(per, 50), 4), "p99_ms": round(pct(per, 99), 4), "layers": len(specs),
            "sum_MKN": mkn, "accept": all(r.accept for r in res)}


def serving_run(torch, ctx, mode_id, rate: float, count: int, arena_bytes: int, slots: int, max_batch: int,
                seed: int = 5000, warm: float = 0.1, prep_lead_ms: float | None = None):
    """One open-loop serving run: `count` requests of a seeded Poisson stream
    at `rate` req/s, each one layer of the CNN or encoder shape set, tag
    generation or check with probability 1/2, submitted with their scheduled
    arrival times to a fresh server.  With prep_lead_ms, every tag-generation
    request is preceded, prep_lead_ms earlier, by a preprocessing request for
    its layer (the offline phase: the dealer), so that the request itself
    runs the online phase only.  The first `warm` fraction is excluded from
    the statistics.  Latency = completion - scheduled arrival."""
    from paper_2311_04406_amd import REQ_PREP, REQ_TAG, Server, workloads
    shapes = workloads.serving_shapes()
    arr = workloads.poisson_arrivals(rate, count, seed)
    ch = workloads.request_choices(count, len(shapes), seed)
    srv = Server(ctx, arena_bytes, slots=slots, max_batch=max_batch, mode=mode_id)
    t0 = srv.now_us() + 5000.0 + (prep_lead_ms or 0.0) * 1e3
    reqs, preps = [], []
    for i in range(count):
        s = shapes[ch[i][1]]
        lay = (s.M, s.K, s.N, 50000 + i, 10000 + i)
        reqs.append((i, ch[i][0], lay, t0 + arr[i] * 1e6))
        if prep_lead_ms is not None and ch[i][0] == REQ_TAG:
            preps.append((count + i, REQ_PREP, lay, t0 + arr[i] * 1e6 - prep_lead_ms * 1e3))
    srv.submit(preps + reqs)
    srv.drain(600)
    comps = [c for c in srv.poll(count + len(preps) + 16) if c["kind"] != REQ_PREP]
    st = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    by_id = {r[0]: r for r in reqs}
    nwarm = int(count * warm)
    live = [c for c in comps if nwarm <= c["id"] < count]
    bad = [c for c in comps if c["status"] != 0]
    lat = sorted((c["done_us"] - c["arrival_us"]) / 1e3 for c in live)
    lat_tag = sorted((c["done_us"] - c["arrival_us"]) / 1e3 for c in live if c["kind"] == REQ_TAG)
    lat_chk = sorted((c["done_us"] - c["arrival_us"]) / 1e3 for c in live if c["kind"] != REQ_TAG)
    t_first = min(c["arrival_us"] for c in live)
    t_last = max(c["done_us"] for c in live)
    span = (t_last - t_first) * 1e-6
    macs = sum(by_id[c["id"]][2][0] * by_id[c["id"]][2][1] * by_id[c["id"]][2][2]
               for c in live if c["kind"] == REQ_TAG)
    return {"rate_rps": rate, "requests": count, "measured": len(live), "errors": len(bad),
            "achieved_rps": round(len(live) / span, 1), "tag_gops": round(macs / span / 1e9, 3),
            "p50_ms": round(pct(lat, 50), 3), "p99_ms": round(pct(lat, 99), 3),
            "tag_p50_ms": round(pct(lat_tag, 50), 3) if lat_tag else None,
            "tag_p99_ms": round(pct(lat_tag, 99), 3) if lat_tag else None,
            "check_p50_ms": round(pct(lat_chk, 50), 3) if lat_chk else None,
            "check_p99_ms": round(pct(lat_chk, 99), 3) if lat_chk else None,
            "batches": st["batches"], "mean_batch": round(st["completed"] / max(st["batches"], 1), 2),
            "max_batch": st["max_batch"], "converted_checks": st["converted"], "evictions": st["evictions"],
            "arena_peak_GB": round(st["arena_peak"] / 1e9, 2),
            "prep_lead_ms": prep_lead_ms, "prepared": st["prepared"], "online_only": st["online_only"]}


SERVE_RATES = (100, 200, 500, 1000, 2000, 5000)
SERVE_ARENA = 192 << 30  # of the 288 GB: the request stream's layers (the classifier's are 14.8 GB)
SERVE_SLOTS = 3
SERVE_BATCH = 32


def serve_count(rate: float) -> int:
    """At least 10 s of arrivals or at least 2000 requests."""
    return int(min(2000, math.ceil(10 * rate)))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="batched",
                    choices=["cnn", "transformer", "batched", "training", "fc_small", "serving"])
    ap.add_argument("--serve-rate", type=float, default=1000.0,
                    help="offered rate (req/s) of the serving leg of a layer-batch run")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-prep-ms", type=float, default=20.0,
                    help="lead (ms) of the preprocessing requests in the online-phase serving runs")
    ap.add_argument("--f", type=int, default=0, help="truncate every product by f fractional bits (0..k-1)")
    ap.add_argument("--kbits", type=int, default=64, choices=[64, 32],
                    help="parameter set k = s: 64 (shares in Z_2^128) or 32 (shares in Z_2^64)")
    ap.add_argument("--in-bits", type=int, default=0, help="dealer inputs as signed in-bits-bit integers (0: uniform)")
    ap.add_argument("--mode", default="compact", choices=["compact", "spdz2k"])
    ap.add_argument("--compress", default="n", choices=["n", "m", "auto"],
                    help="dimension the compact tag compresses: N, M, or per layer the cheaper (M iff M > N)")
    ap.add_argument("--parties", type=int, default=2,
                    help="parties simulated in one process (2 to 5; more than 2: explicit convolutions, no server)")
    ap.add_argument("--conv", default="implicit", choices=["explicit", "implicit"],
                    help="convolutions as products with an explicit K x N im2col operand, or with the im2col "
                         "left implicit (input, mask and U of the input's C x H x W shape)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the SPDZ2k and per-layer comparison runs")
    ap.add_argument("--no-autotune", action="store_true", help="use the default matrix-core launch configuration")
    ap.add_argument("--tuning", default=None,
                    help="fixed launch configuration group_m,xcd_remap,split_target[,tile] (tile: CT_TILE_* number)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="copy this many MiB once with a plain device copy before the steps (calibrates "
                         "hardware byte counters against a kernel of known traffic)")
    ap.add_argument("--extra", default="cnn,transformer",
                    help="further workloads whose captured step is timed beside the main one (comma list; "
                         "'' for none)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run mixed batches on one stream (every kernel alone, as a per-kernel profile needs)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the layers shard across GPUs by layer or by output columns, which is not built here",
              file=sys.stderr)
        sys.exit(2)

    if not args.no_cpu_baseline and args.config != "serving":
        # compiled before any GPU call: a process that has initialised the GPU
        # must not fork a compiler
        import oracle
        oracle.build()

    import torch
    from paper_2311_04406_amd import MODE_COMPACT, MODE_SPDZ2K, RESULT_WORDS, Context, Layer, workloads
    from paper_2311_04406_amd.binding import LAUNCH_PERSISTENT, LAUNCH_STAGED

    if args.config == "serving":
        return serving_main(args, torch)
    specs = workloads.CONFIGS[args.config]()
    mode_id = MODE_COMPACT if args.mode == "compact" else MODE_SPDZ2K
    ctx = Context(device=0, key_seed=workloads.KEY_SEED, max_layers=max(256, len(specs)), kbits=args.kbits,
                  parties=args.parties)
    if args.no_overlap:
        ctx.set_overlap(False)
    cmp = {"n": 0, "m": 1, "auto": 2}[args.compress]
    implicit = args.conv == "implicit" and args.parties == 2
    layers = [ctx.layer(s.M, s.K, s.N, s.seed, s.layer_id, f=args.f, in_bits=args.in_bits, compress=cmp,
                        conv=s.conv if implicit else None) for s in specs]
    print(f"[bench] config {args.config}: {len(specs)} layers, dealer ...", file=sys.stderr, flush=True)
    ctx.gen_triple_tags(layers)
    torch.cuda.synchronize()
    out_dev = torch.zeros(len(layers) * RESULT_WORDS, dtype=torch.int64, device="cuda:0")
    mkn = sum(s.mkn for s in specs)

    if args.copy_probe > 0:
        n = args.copy_probe * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.int64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tuning = None
    if args.tuning:
        v = [int(x) for x in args.tuning.split(",")]
        ctx.set_tuning(*v)
        tuning = ctx.get_tuning(mode_id, layers)
    elif not args.no_autotune:
        print("[bench] autotuning the matrix-core launch configuration ...", file=sys.stderr, flush=True)
        tuning = ctx.autotune(mode_id, layers)
    print(f"[bench] timed {args.mode}: {args.warmup} warmup + {args.steps} steps", file=sys.stderr, flush=True)
    # the timed step: one graph launch of the captured online phase + verification
    plan = ctx.plan(mode_id, layers, out_dev)
    T, per, _ = run_steps(ctx, mode_id, [layers], out_dev, args.steps, args.warmup, torch, plan=plan)
    Te, pere, _ = run_steps(ctx, mode_id, [layers], out_dev, args.steps, args.warmup, torch)
    # per-kernel durations: a second pass with an event pair around every launch
    _, _, stages = run_steps(ctx, mode_id, [layers], out_dev, args.steps, 0, torch, timing=True)
    res = Context.decode_results(out_dev, len(layers), args.parties)
    if not all(r.accept for r in res):
        print("[bench] ERROR: an honest run was rejected", file=sys.stderr)
        sys.exit(1)
    ms = T / args.steps * 1e3
    value = mkn * args.steps / T / 1e9

    # per-stage figures and the dominant kernel's roofline
    stage_rows = {}
    for name, (tot_ms, n) in stages.items():
        avg = tot_ms / max(n, 1)
        w = stage_work(name, specs, args.mode, args.f, args.kbits, args.compress, implicit, args.parties)
        row = {"ms_per_launch": round(avg, 5), "launches": n, "share_of_step": round(tot_ms / args.steps / ms, 4)}
        if w is not None and w[1] > 0:
            bound, units = w
            if bound == "hbm":
                row.update(bound="hbm", achieved_GBps=round(units / (avg * 1e-3) / 1e9, 1),
                           frac=round(units / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), algorithmic_bytes=units)
            else:
                row.update(bound="mfma", achieved_TOPS=round(units / (avg * 1e-3) / 1e12, 1),
                           frac=round(units / (avg * 1e-3) / 1e12 / INT8_PEAK_TOPS, 4), int8_ops=units)
        stage_rows[name] = row
    ranked = sorted(((k, v) for k, v in stage_rows.items() if "bound" in v),
                    key=lambda kv: -kv[1]["ms_per_launch"] * kv[1]["launches"])
    roofline = None
    if ranked:
        k, v = ranked[0]
        if v["bound"] == "hbm":
            roofline = {"kernel": k, "bound": "hbm", "achieved": v["achieved_GBps"], "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": v["frac"]}
        else:
            roofline = {"kernel": k, "bound": "mfma", "achieved": v["achieved_TOPS"], "peak": INT8_PEAK_TOPS,
                        "unit": "TOPS (int8)", "frac": v["frac"]}
        wl_key = (f"{args.config}/{args.mode}" + (f"/f{args.f}" if args.f else "") + ("/k32" if args.kbits == 32 else "")
                  + (f"/c{args.compress}" if args.compress != "n" else "") + ("/implicit" if implicit else "")
                  + (f"/p{args.parties}" if args.parties != 2 else ""))
        roofline["traffic"] = measured_traffic(k, wl_key)
        if v["bound"] == "mfma":
            roofline["counters"] = measured_counters(k, wl_key)
        roofline["share_of_step"] = v["share_of_step"]

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "G ring-MAC/s (Z_2^64 GEMM Gops, 1 op = 1 MAC)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "p50_ms": round(pct(per, 50), 4), "p99_ms": round(pct(per, 99), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u128" if args.kbits == 64 else "u64", "data": "synthetic",
        "config": {"workload": f"{args.config}: " + ", ".join(f"{s.name} ({s.M}x{s.K}x{s.N})" for s in specs)
                   if len(specs) <= 8 else f"{args.config}: {len(specs)} layers, sum MKN {mkn}",
                   "protocol": args.mode, "parties": args.parties,
                   "ring": ("values Z_2^64, shares and tags Z_2^128" if args.kbits == 64 else
                            "values Z_2^32, shares and tags Z_2^64"),
                   "layers_per_call": len(specs), "sum_MKN": mkn, "f": args.f, "in_bits": args.in_bits,
                   "compress": args.compress, "conv": "implicit" if implicit else "explicit",
                   "compressed_along_m": [s.name for s in specs if along_m(s, args.compress)]
                   if len(specs) <= 8 else sum(along_m(s, args.compress) for s in specs)},
        "roofline": roofline,
        "eager": {"value": round(mkn * args.steps / Te / 1e9, 3), "ms_per_step": round(Te / args.steps * 1e3, 4),
                  "p50_ms": round(pct(pere, 50), 4), "p99_ms": round(pct(pere, 99), 4)},
        "stages": stage_rows,
        "tuning": tuning,
    }

    if not args.no_compare:
        other = MODE_SPDZ2K if mode_id == MODE_COMPACT else MODE_COMPACT
        oname = "spdz2k" if other == MODE_SPDZ2K else "compact"
        if not args.no_autotune:
            ctx.autotune(other, layers)
            for l in layers:
                ctx.autotune(mode_id, [l])
        plan2 = ctx.plan(other, layers, out_dev)
        T2, per2, _ = run_steps(ctx, other, [layers], out_dev, args.steps, args.warmup, torch, plan=plan2)
        plan2.close()
        out[oname] = {"value": round(mkn * args.steps / T2 / 1e9, 3), "ms_per_step": round(T2 / args.steps * 1e3, 4),
                      "p50_ms": round(pct(per2, 50), 4), "p99_ms": round(pct(per2, 99), 4)}
        T3, per3, _ = run_steps(ctx, mode_id, [[l] for l in layers], out_dev, args.steps, args.warmup, torch)
        out["per_layer_launch"] = {"value": round(mkn * args.steps / T3 / 1e9, 3),
                                   "ms_per_step": round(T3 / args.steps * 1e3, 4),
                                   "p50_ms": round(pct(per3, 50), 4), "p99_ms": round(pct(per3, 99), 4)}
        T4, per4, _ = run_steps(ctx, mode_id, [layers], out_dev, args.steps, args.warmup, torch, fused=False)
        out["separate_check"] = {"value": round(mkn * args.steps / T4 / 1e9, 3),
                                 "ms_per_step": round(T4 / args.steps * 1e3, 4),
                                 "p50_ms": round(pct(per4, 50), 4), "p99_ms": round(pct(per4, 99), 4)}
        if persistent_applies(specs, args.compress, args.parties, implicit):
            # the same captured step as one persistent launch (every stage at
            # the products' occupancy, grid barriers between stages)
            ctx.set_launch(LAUNCH_PERSISTENT)
            plan5 = ctx.plan(mode_id, layers, out_dev)
            ctx.set_launch(LAUNCH_STAGED)
            T5, per5, _ = run_steps(ctx, mode_id, [layers], out_dev, args.steps, args.warmup, torch, plan=plan5)
            plan5.close()
            ok5 = all(r.accept and r.reserved == 0 for r in Context.decode_results(out_dev, len(layers), args.parties))
            out["persistent_launch"] = {"value": round(mkn * args.steps / T5 / 1e9, 3),
                                        "ms_per_step": round(T5 / args.steps * 1e3, 4),
                                        "p50_ms": round(pct(per5, 50), 4), "p99_ms": round(pct(per5, 99), 4),
                                        "accept": ok5}
    plan.close()
    del plan
    if not args.no_serve and args.kbits == 64 and args.parties == 2:  # the server runs two parties, k = s = 64
        print(f"[bench] serving leg at {args.serve_rate:g} req/s ...", file=sys.stderr, flush=True)
        layers = None
        torch.cuda.empty_cache()
        out["serving"] = serving_run(torch, ctx, mode_id, args.serve_rate, serve_count(args.serve_rate),
                                     SERVE_ARENA, SERVE_SLOTS, SERVE_BATCH)
        out["serving_online"] = serving_run(torch, ctx, mode_id, args.serve_rate, serve_count(args.serve_rate),
                                            SERVE_ARENA, SERVE_SLOTS, SERVE_BATCH, prep_lead_ms=args.serve_prep_ms)
    if args.extra:
        del layers
        torch.cuda.empty_cache()
        out["extra"] = {}
        for name in [x for x in args.extra.split(",") if x and x != args.config]:
            print(f"[bench] extra workload {name} ...", file=sys.stderr, flush=True)
            out["extra"][name] = extra_run(torch, ctx, name, mode_id, args, implicit, cmp)
            torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        nt = cpu_threads()
        print(f"[bench] cpu baseline (oracle, {nt} threads and 1) ...", file=sys.stderr, flush=True)
        cb = cpu_baseline(specs, kbits=args.kbits, implicit=implicit, parties=args.parties, threads=nt,
                          mode=mode_id)
        c1 = cpu_baseline(specs, kbits=args.kbits, implicit=implicit, parties=args.parties, threads=1,
                          mode=mode_id)
        out["cpu_baseline"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in cb.items()}
        out["cpu_baseline"]["single_core"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in c1.items()
                                              if k in ("value", "seconds", "ring_macs", "cores")}
    ctx.close()
    print(json.dumps(out), flush=True)


def serving_main(args, torch):
    """The serving configuration: an open-loop Poisson sweep over the offered
    rates; `value` is the tagged ring-MAC throughput at the highest rate."""
    from paper_2311_04406_amd import MODE_COMPACT, MODE_SPDZ2K, Context, workloads
    mode_id = MODE_COMPACT if args.mode == "compact" else MODE_SPDZ2K
    ctx = Context(device=0, key_seed=workloads.KEY_SEED)
    rows = []
    online = []
    for rate in SERVE_RATES:
        print(f"[bench] serving {rate} req/s ...", file=sys.stderr, flush=True)
        rows.append(serving_run(torch, ctx, mode_id, rate, serve_count(rate), SERVE_ARENA, SERVE_SLOTS,
                                SERVE_BATCH))
        print(f"[bench]   {rows[-1]}", file=sys.stderr, flush=True)
        online.append(serving_run(torch, ctx, mode_id, rate, serve_count(rate), SERVE_ARENA, SERVE_SLOTS,
                                  SERVE_BATCH, prep_lead_ms=args.serve_prep_ms))
        print(f"[bench]   online phase only: {online[-1]}", file=sys.stderr, flush=True)
    ctx.close()
    top = rows[-1]
    ref = next((r for r in rows if r["rate_rps"] == args.serve_rate), rows[0])
    shapes = workloads.serving_shapes()
    out = {
        "metric": METRIC, "value": top["tag_gops"], "unit": "G ring-MAC/s (Z_2^64 GEMM Gops, 1 op = 1 MAC)",
        "n_gpus": 1, "steps": sum(r["requests"] for r in rows), "warmup": 0, "ms_per_step": None,
        "p50_ms": ref["p50_ms"], "p99_ms": ref["p99_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u128", "data": "synthetic",
        "config": {"workload": "serving: open-loop Poisson arrivals at " + ", ".join(str(r) for r in SERVE_RATES)
                   + " req/s; each request one layer of " + ", ".join(f"{s.name} ({s.M}x{s.K}x{s.N})"
                                                                       for s in shapes)
                   + "; tag generation (dealer + online phase) or check, 1/2 each",
                   "protocol": args.mode, "parties": 2, "ring": "values Z_2^64, shares and tags Z_2^128",
                   "arena_GB": SERVE_ARENA / 2**30, "slots": SERVE_SLOTS, "max_batch": SERVE_BATCH,
                   "latency_rate_rps": ref["rate_rps"]},
        "serving": rows,
        "serving_online": online,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
