"""Benchmark: all-pairs Levenshtein on 4096 DNA sequences (lengths 1000-1600).

One step = one lev_allpairs call over the whole set (8,386,560 pairs): length
binning, staging and the persistent bit-parallel kernel.  Inputs are
resident on the GPU before the timed region starts; the launch variant is
autotuned before it.  Further legs, reported in the same JSON line: pair
lists through lev_batch ("pairs": the 2 M training labels of the learned
workload and 8.4 M random pairs of the all-pairs set), the 512-pair NW fill
+ traceback ("nw"), the same pairs under an affine-gap score matrix
("gotoh") and by the exact banded distance ("band"), the exact tree build of
20,000 protein sequences ("tree": autotuned, graph-replayed levels), the
online insertion of 1,000 sequences into the exact tree of 99,000
("insert"), the learned pruning of the tree build on 100,000 sequences
("pruned": embedder training, exact vs pruned build time, teacher-forced
agreement, control rankers, alignment quality of the pruned trees'
alignments) and the alignment-quality metrics ("quality") and machine rates
("machine").

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--quick]
                    [--no-tune] [--legs a,b,...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("GCUPS & pairs/s (batched Levenshtein+NW, bit-exact); "
          "surrogate vs exact tree-build speedup")
# Roofline peak of the bit-parallel Levenshtein kernel.  Integer VALU: 256 CUs
# x 4 SIMDs x 16 lanes x 2 instructions issued per cycle (gfx950 dual-issues
# VALU; the same rate gives the 157.3 TFLOP/s fp32 vector figure) x 2.4 GHz
# = 78.6 T 32-bit lane-ops/s.  The reference cost of the recurrence is 32
# lane-ops per 64-cell word step (16 64-bit logical ops, two 32-bit halves
# each), so the peak is 78.6e12 * 64 / 32 = 157.3 T cells/s.
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2 * 2.4e9
K_REF = 32
LEV_PEAK_TCUPS = VALU_PEAK_LANE_OPS * 64 / K_REF / 1e12
HBM_PEAK_GBS = 8000.0
# HBM traffic of a kernel comes from rocprofv3 counter runs recorded in
# profiles/counters.json (FETCH_SIZE x its copy-calibration factor +
# WRITE_SIZE, per launch), each entry stamped with a hash of the kernel's
# source files; it is reported only while those files are unchanged.
COUNTERS = os.path.join(ROOT, "profiles", "counters.json")


def source_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counted(kernel, variant=None):
    """The recorded counter entry of a kernel (and launch variant) if its
    sources are unchanged since the counters were taken, else None."""
    try:
        with open(COUNTERS) as fh:
            c = json.load(fh)
    except OSError:
        return None
    e = c.get(kernel)
    if e is None or source_hash(e["sources"]) != e["source_hash"]:
        return None
    if variant is not None:
        return e.get("variants", {}).get(str(variant))
    return e


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--legs", default="pairs,nw,gotoh,band,tree,insert,pruned,quality,machine",
                    help="legs after the all-pairs one: any of pairs, nw, gotoh, band, tree, "
                         "insert, cnn, pruned, quality, machine (comma list; cnn is not in "
                         "the default set, the pruned leg trains and embeds too)")
    ap.add_argument("--quick", action="store_true", help="only the all-pairs leg")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch variants (no autotuning before timing)")
    ap.add_argument("--epochs", type=int, default=2, help="embedder epochs over 2M pairs")
    ap.add_argument("--topk", type=int, default=16)
    ap.add_argument("--exact-below", type=int, default=256,
                    help="hybrid point: clusters of at most this many members keep the full median")
    ap.add_argument("--points", default="",
                    help="pruned builds to run instead of the default set, as ranker:topk:"
                         "exact_below items (rankers cnn, cnn_raw, shortest, random, "
                         "sampled4, sampled8, sampled16)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    return ap.parse_args()


def copy_probe():
    """A plain device-to-device copy of exactly 1 GiB, for scaling the HBM
    byte counters (FETCH_SIZE / WRITE_SIZE) of the other kernels."""
    import torch
    n = 1 << 30
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n}), flush=True)


def cpu_baseline(d, seconds, device_out):
    """The oracle (plain Wagner-Fischer, OpenMP over pairs) on a seeded
    sample of the same pairs, for about `seconds` of wall time; its
    distances are also compared with the device's condensed output
    (returned as the second value: True when every sampled pair agrees)."""
    from oracle import pyoracle as orc
    n = d["n"]
    L = np.diff(d["offsets"])
    rng = np.random.default_rng(2024)
    done_cells = 0
    done_pairs = 0
    agree = True
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        ia = rng.integers(0, n, size=512)
        ib = rng.integers(0, n, size=512)
        keep = ia != ib
        ia, ib = ia[keep], ib[keep]
        want = orc.lev_pairs(d["codes"], d["offsets"], d["codes"], d["offsets"], ia, ib)
        i, j = np.minimum(ia, ib), np.maximum(ia, ib)
        agree &= bool((device_out[i * n - i * (i + 1) // 2 + (j - i - 1)] == want).all())
        done_cells += int((L[ia] * L[ib]).sum())
        done_pairs += len(ia)
    dt = time.perf_counter() - t0
    return ({"value": round(done_cells / dt / 1e9, 3), "unit": "GCUPS",
             "cores": orc.num_threads(), "kind": "oracle",
             "sample": f"{done_pairs} seeded random pairs of the same 4096-sequence set "
                       f"({done_cells:.3e} cells, {dt:.1f} s); pairs/s = "
                       f"{done_pairs / dt:.1f}"}, agree)


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding "
              "of the pair triangle is designed but not built", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2601_15458_amd import msadp, synth

    d = synth.allpairs()
    n = d["n"]
    L = np.diff(d["offsets"]).astype(np.int64)
    tot = int(L.sum())
    cells = (tot * tot - int((L * L).sum())) // 2
    pairs = n * (n - 1) // 2
    A = msadp.to_device(d["codes"], d["offsets"], d["sigma"])
    ap = msadp.AllPairs(A)
    stream = torch.cuda.current_stream()
    tuning = None if args.no_tune else tune_lev(msadp, torch, A, ap, stream)
    for _ in range(args.warmup):
        ap(stream)
    torch.cuda.synchronize()
    ap.st.check("lev_allpairs")

    # the device distances, for the CPU-baseline leg's check of its sample
    out = ap.out[:pairs].cpu().numpy().astype(np.int64)

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        ap(stream)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    call_ms = [a.elapsed_time(b) for a, b in ev]
    ms = float(np.mean(call_ms))
    ap.st.check("lev_allpairs")
    tcups = cells / (ms * 1e-3) / 1e12
    chosen = tuning["chosen"] if tuning else 32
    ce = counted("k_lev_allpairs", chosen)
    traffic = ce["hbm_bytes"] if ce else None
    res = {
        "metric": METRIC,
        "value": round(cells / (wall / args.steps) / 1e9, 1),
        "unit": "GCUPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "lev_allpairs: 4096 DNA seqs, lengths U{1000..1600}, "
                               "seed 2, uint16 condensed output",
                   "pairs": pairs, "cells": cells},
        "pairs_per_s": round(pairs / (wall / args.steps), 1),
        "tuning": tuning,
        "roofline": {"bound": "alu", "achieved": round(tcups, 2),
                     "peak": round(LEV_PEAK_TCUPS, 1), "unit": "Tcell/s",
                     "frac": round(tcups / LEV_PEAK_TCUPS, 4),
                     "traffic": traffic,
                     "kernel": "k_lev_allpairs", "call_ms_mean": round(ms, 3),
                     "peak_basis": "32 VALU lane-ops per 64-cell word step at 78.6 T "
                                   "lane-ops/s (dual issue)"},
    }
    if ce and ce.get("valu_insts"):
        # the chip's own count: VALU instructions x 64 lanes over the call
        lane_ops = ce["valu_insts"] * 64 / (ms * 1e-3) / 1e12
        res["roofline"]["counted_valu"] = {
            "lane_ops_per_s": round(lane_ops, 2), "unit": "T/s",
            "frac_of_78.6": round(lane_ops / (VALU_PEAK_LANE_OPS / 1e12), 4),
            "valu_per_word_step": ce.get("valu_per_word_step"),
            "dual_issue_share": ce.get("valu2_share")}
    legs = [] if args.quick else [x for x in args.legs.split(",") if x]
    for name, fn in (("pairs", bench_pairs), ("nw", bench_nw), ("gotoh", bench_gotoh),
                     ("band", bench_band), ("tree", bench_tree), ("insert", bench_insert),
                     ("cnn", bench_cnn), ("pruned", bench_pruned),
                     ("quality", bench_quality), ("machine", bench_machine)):
        if name in legs:
            try:
                res[name] = fn(msadp, synth, torch, args)
            except Exception as e:   # report, keep the headline line
                res[name] = {"error": f"{type(e).__name__}: {e}"}
                _log(f"{name} leg failed: {e}")
    if not args.no_cpu:
        res["cpu_baseline"], res["parity_sample_ok"] = cpu_baseline(d, args.cpu_seconds, out)
    print(json.dumps(res), flush=True)


def oracle_beside(args, fn, cells, sample):
    """The oracle on a bounded sample of a leg's work, on the host's cores,
    timed beside the device (skipped with --no-cpu)."""
    if args.no_cpu:
        return None
    from oracle import pyoracle as orc
    t0 = time.perf_counter()
    fn()
    dt = time.perf_counter() - t0
    return {"kind": "oracle", "sample": sample, "cells": int(cells), "seconds": round(dt, 3),
            "gcups": round(cells / dt / 1e9, 3) if cells else None, "cores": orc.num_threads()}


def alu_roofline(entry, ms, kernel):
    """A kernel's VALU issue against the chip's VALU figure: the counted
    SQ_INSTS_VALU of one dispatch (profiles/counters.json) x 64 lanes over
    the timed call; None without a current counter entry."""
    if not entry or not entry.get("valu_insts"):
        return None
    peak = VALU_PEAK_LANE_OPS / 1e12
    a = entry["valu_insts"] * 64 / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(a, 2), "peak": round(peak, 1),
            "unit": "T lane-ops/s", "frac": round(a / peak, 4), "kernel": kernel,
            "valu_insts": entry["valu_insts"], "dual_issue_share": entry.get("valu2_share")}


def _time_calls(torch, fn, stream, reps):
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_quality(msadp, synth, torch, args):
    """Alignment quality (Sec. 2.3 and the Table 2 columns) of the
    4096-sequence set's own alignment: guide tree and merge on the device,
    then the pair counts over all 8,386,560 pairs and the metrics, the
    distortion against the all-pairs Levenshtein distances."""
    d = synth.allpairs()
    n = d["n"]
    A = msadp.to_device(d["codes"], d["offsets"], d["sigma"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tree, msa = msadp.align(A, use_graph=True)
    t_align = time.perf_counter() - t0
    lev = msadp.lev_allpairs(A)
    gap = d["sigma"]
    Q = msadp.Quality(msa, gap)
    max_len = int(np.diff(d["offsets"]).max())
    stream = torch.cuda.current_stream()
    counts = Q.pair_counts(stream=stream)
    q = Q.metrics(counts, max_len, lev=lev, stream=stream)
    reps = max(args.steps, 3)
    ms_counts = _time_calls(torch, lambda: Q.pair_counts(stream=stream), stream, reps)
    ms_metrics = _time_calls(torch, lambda: Q.metrics(counts, max_len, lev=lev, stream=stream),
                             stream, reps)
    Q.st.check("msa_pair_counts")
    # every row pair of an alignment costs at least the two sequences'
    # Levenshtein distance (the counts' parity with the oracle is in tests/)
    bound = bool((counts[0].cpu().numpy() >= lev.cpu().numpy()).all())
    pairs = n * (n - 1) // 2
    rows, width = msa.shape
    words = -(-width // 32)
    nb = max(1, int(gap).bit_length())
    ops = pairs * words * (2 * nb + 4)           # VALU lane-ops of the pair-count kernel
    achieved = ops / (ms_counts * 1e-3) / 1e12
    peak = VALU_PEAK_LANE_OPS / 1e12
    return {"workload": "alignment quality: the 4096-sequence DNA set (lengths U{1000..1600}, "
                        "seed 2) aligned on the device, all 8,386,560 row pairs",
            "align_s": round(t_align, 3), "width": int(width),
            "metrics": {k: (round(v, 6) if isinstance(v, float) else v) for k, v in q.items()},
            "pair_counts_ms": round(ms_counts, 3), "metrics_ms": round(ms_metrics, 3),
            "pairs_per_s": round(pairs / (ms_counts * 1e-3), 1),
            "hamming_ge_lev_all_pairs": bound,
            "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": round(peak, 1),
                         "unit": "T lane-ops/s", "frac": round(achieved / peak, 4),
                         "traffic": None, "kernel": "k_qual_planes + k_qual_tri (one call)",
                         "ops_per_pair_word": 2 * nb + 4}}


def bench_machine(msadp, synth, torch, args):
    """Measured machine rates beside the vendor figures the roofline
    fractions use: VALU 32-bit lane-instructions/s (independent xor/add
    chains), MFMA operations/s for the shapes the kernels use, and HBM
    bytes/s of a streaming copy (read + write bytes over kernel time)."""
    stream = torch.cuda.current_stream()
    blocks = 256 * 8                       # eight wavefronts per SIMD
    sink = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    out = {}
    ops = msadp.probe_valu(blocks, 4096, sink, stream)
    ms = _time_calls(torch, lambda: msadp.probe_valu(blocks, 4096, sink, stream), stream, 3)
    out["valu_lane_ops"] = {"measured": round(ops / (ms * 1e-3) / 1e12, 2), "unit": "T/s",
                            "vendor_single_issue": round(VALU_PEAK_LANE_OPS / 2e12, 1),
                            "vendor_dual_issue": round(VALU_PEAK_LANE_OPS / 1e12, 1)}
    vendor = {"bf16": 2500.0, "i8": 5000.0}
    for kind in msadp.PROBE_MFMA:
        per_trip = msadp.probe_mfma(kind, blocks, 1, sink, stream)
        iters = max(1, (1 << 45) // per_trip)      # 7-14 ms at the vendor rates
        ops = msadp.probe_mfma(kind, blocks, iters, sink, stream)
        ms = _time_calls(torch, lambda: msadp.probe_mfma(kind, blocks, iters, sink, stream),
                         stream, 3)
        out["mfma_" + kind] = {"measured": round(ops / (ms * 1e-3) / 1e12, 1),
                               "unit": "TFLOP/s" if kind.startswith("bf16") else "TOP/s",
                               "vendor": vendor[kind.split("_")[0]]}
    n = 1 << 30
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    rates = {}
    for b in (256, 512, 1024):            # the best of a few grid sizes
        nb = msadp.probe_copy(src, dst, b, stream)
        ms = _time_calls(torch, lambda: msadp.probe_copy(src, dst, b, stream), stream, 5)
        rates[b] = nb / (ms * 1e-3) / 1e9
    best = max(rates, key=rates.get)
    out["hbm_copy"] = {"measured": round(rates[best], 1), "unit": "GB/s",
                       "vendor": HBM_PEAK_GBS, "bytes": nb, "workgroups": best}
    torch.cuda.synchronize()
    del src, dst
    return out


def tune_lev(msadp, torch, A, ap, stream, reps=2):
    """Autotuning before the timed region: every word class that needs no
    more passes than the default, fastest kept in the tuning table."""
    words = msadp.lev_words_bin(A)
    dflt = next(c for c in (4, 8, 16, 24, 32) if c >= min(words, 32))
    max_passes = max(2, -(-words // dflt))
    ms = {}
    for c in msadp.tune_candidates(msadp.MSA_TUNE_LEV):
        if -(-words // c) > max_passes:
            continue
        msadp.tune_set(msadp.MSA_TUNE_LEV, A.sigma, words, c)
        ms[c] = round(_time_calls(torch, lambda: ap(stream), stream, reps), 3)
    best = min(ms, key=ms.get)
    msadp.tune_set(msadp.MSA_TUNE_LEV, A.sigma, words, best)
    _log(f"lev word classes (ms per call): {ms}; using {best}")
    return {"kind": "lev words per pass", "default": dflt, "chosen": best, "ms": ms}


def bench_nw(msadp, synth, torch, args):
    """512 long DNA pairs: NW fill (traceback codes to HBM) then traceback."""
    d = synth.nw_long()
    P = d["n_pairs"]
    A = msadp.to_device(d["a_codes"], d["a_offsets"], 4)
    B = msadp.to_device(d["b_codes"], d["b_offsets"], 4)
    ia = np.arange(P)
    nb = msadp.NwBatch(A, B, ia, ia)
    stream = torch.cuda.current_stream()
    tuning = None
    if not args.no_tune:
        waves = -(-(-(-A.max_len // 32)) // 64)
        ms = {}
        for R in msadp.tune_candidates(msadp.MSA_TUNE_NW):
            msadp.tune_set(msadp.MSA_TUNE_NW, A.sigma, waves, R)
            ms[R] = round(_time_calls(torch, lambda: nb.fill(stream), stream, 2), 3)
        best = min(ms, key=ms.get)
        msadp.tune_set(msadp.MSA_TUNE_NW, A.sigma, waves, best)
        _log(f"nw barrier intervals (fill ms): {ms}; using {best}")
        tuning = {"kind": "nw steps between barriers", "default": 32, "chosen": best, "ms": ms}
    nb.fill(stream)
    nb.traceback(stream)
    torch.cuda.synchronize()
    nb.st.check("nw")
    la = np.diff(d["a_offsets"])
    lb = np.diff(d["b_offsets"])
    cells = int((la * lb).sum())
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fill, tb = [], []
    for _ in range(max(args.steps, 3)):
        e[0].record(stream)
        nb.fill(stream)
        e[1].record(stream)
        nb.traceback(stream)
        e[2].record(stream)
        torch.cuda.synchronize()
        fill.append(e[0].elapsed_time(e[1]))
        tb.append(e[1].elapsed_time(e[2]))
    f = float(np.median(fill))
    t = float(np.median(tb))
    tb_bytes = int(sum(msadp.lib().nw_tb_bytes(int(a), int(b)) for a, b in zip(la, lb)))
    from oracle import pyoracle as orc
    sel = np.arange(4)
    cpu = oracle_beside(args, lambda: orc.nw_pairs(d["a_codes"], d["a_offsets"], d["b_codes"],
                                                   d["b_offsets"], sel, sel),
                        (la[sel] * lb[sel]).sum(),
                        "full-matrix NW with traceback on pairs 0-3 of the 512")
    return {"workload": "nw_batch+nw_traceback: 512 DNA pairs, lengths U{5000..10000}, 10% "
                        "divergence, unit costs, seed 4", "tuning": tuning, "cpu_oracle": cpu,
            "cells": cells, "fill_ms": round(f, 3), "traceback_ms": round(t, 3),
            "fill_gcups": round(cells / f / 1e6, 1),
            "gcups_fill_plus_traceback": round(cells / (f + t) / 1e6, 1),
            "pairs_per_s": round(P / ((f + t) * 1e-3), 1),
            "tb_bytes": tb_bytes,
            "fill_hbm_gbs": round(tb_bytes / f / 1e6, 1),
            "fill_hbm_frac": round(tb_bytes / f / 1e6 / HBM_PEAK_GBS, 4),
            "roofline": {"bound": "hbm", "achieved": round(tb_bytes / f / 1e6, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(tb_bytes / f / 1e6 / HBM_PEAK_GBS, 4),
                         "traffic": (counted("k_nw_fill", tuning["chosen"] if tuning else 32)
                                     or {}).get("hbm_bytes"),
                         "kernel": "k_nw_fill"},
            # the same fill against the VALU figure (it is latency-bound: see
            # the kernel's discussion)
            "roofline_alu": alu_roofline(counted("k_nw_fill", tuning["chosen"] if tuning else 32),
                                         f, "k_nw_fill")}


def bench_pairs(msadp, synth, torch, args):
    """Pair lists through lev_batch, layout autotuned: the 2,000,000 training
    pairs of the learned workload (100,000 DNA sequences of 100-500, about 20
    pairs per sequence: one pattern per lane) and 8,386,560 random pairs of
    the all-pairs set (about 2,000 per sequence: shared patterns)."""
    from paper_2601_15458_amd import learned
    stream = torch.cuda.current_stream()
    out = {}
    work = []
    d = synth.learned()
    S = msadp.to_device(d["codes"], d["offsets"], d["sigma"])
    ia, ib = learned.sample_pairs(d["family"], 2_000_000, seed=11)
    work.append(("labels", "2,000,000 training pairs (50 % within-family) of 100,000 DNA "
                 "seqs, lengths 100-500, seed 5/11", S, ia, ib, np.diff(d["offsets"])))
    a = synth.allpairs()
    n = a["n"]
    A = msadp.to_device(a["codes"], a["offsets"], a["sigma"])
    rng = np.random.default_rng(8)
    np_ = n * (n - 1) // 2
    work.append(("random_allpairs_set", "8,386,560 uniform random pairs of the 4096 DNA seqs "
                 "(lengths 1000-1600), seed 2/8", A, rng.integers(0, n, np_).astype(np.int32),
                 rng.integers(0, n, np_).astype(np.int32), np.diff(a["offsets"])))
    for name, desc, X, xa, xb, L in work:
        lb = msadp.LevBatch(X, X, xa, xb)
        best, _ = msadp.autotune_pairs(lb, reps=2, stream=stream)
        ms = _time_calls(torch, lambda: lb(stream), stream, max(args.steps, 3))
        lb.st.check("lev_batch")
        cells = float((L[xa].astype(np.float64) * L[xb]).sum())
        tc = cells / (ms * 1e-3) / 1e12
        out[name] = {"workload": desc, "pairs": int(len(xa)), "cells": cells,
                     "layout": {1: "one pattern per lane", 2: "a pattern across lanes",
                                64: "shared patterns"}[best],
                     "ms": round(ms, 3), "t_cells_per_s": round(tc, 1),
                     "pairs_per_s": round(len(xa) / (ms * 1e-3), 1),
                     "frac_of_157.3": round(tc / LEV_PEAK_TCUPS, 4)}
        _log(f"pairs {name}: {ms:.2f} ms, {tc:.1f} T cells/s ({out[name]['layout']})")
        del lb
    return out


def _dna_scores():
    """Stand-in nucleotide matrix (+5 match, -4 mismatch): the paper's
    extended-IUPAC table is not available here."""
    return np.where(np.eye(4, dtype=bool), 5, -4).astype(np.int32)


def bench_gotoh(msadp, synth, torch, args):
    """The 512 long DNA pairs under the cost model of Sec. 2.4: a substitution
    matrix (stand-in) and affine gaps with opening ten times the extension
    (open 10, extension 1): fill (one code byte per cell) and traceback."""
    d = synth.nw_long()
    P = d["n_pairs"]
    A = msadp.to_device(d["a_codes"], d["a_offsets"], 4)
    B = msadp.to_device(d["b_codes"], d["b_offsets"], 4)
    g = msadp.GotohBatch(A, B, np.arange(P), np.arange(P), _dna_scores(), 10, 1)
    stream = torch.cuda.current_stream()
    g.fill(stream)
    g.traceback(stream)
    torch.cuda.synchronize()
    g.st.check("gotoh")
    la = np.diff(d["a_offsets"])
    lb = np.diff(d["b_offsets"])
    cells = int((la * lb).sum())
    reps = max(args.steps, 3)
    f = _time_calls(torch, lambda: g.fill(stream), stream, reps)
    t = _time_calls(torch, lambda: g.traceback(stream), stream, reps)
    tb = int(sum(msadp.lib().gotoh_tb_bytes(int(a), int(b)) for a, b in zip(la, lb)))
    from oracle import pyoracle as orc
    sel = np.argsort(la * lb, kind="stable")[:4].astype(np.int32)
    cpu = oracle_beside(args, lambda: orc.gotoh_pairs(d["a_codes"], d["a_offsets"], d["b_codes"],
                                                      d["b_offsets"], sel, sel, _dna_scores(),
                                                      10, 1),
                        (la[sel] * lb[sel]).sum(),
                        "Gotoh's three full matrices and the walk on the 4 smallest pairs")
    return {"workload": "gotoh_batch+gotoh_traceback: 512 DNA pairs, lengths U{5000..10000}, "
                        "10% divergence, +5/-4 matrix, open 10, extension 1, seed 4",
            "cpu_oracle": cpu,
            "cells": cells, "fill_ms": round(f, 3), "traceback_ms": round(t, 3),
            "fill_gcups": round(cells / f / 1e6, 1),
            "gcups_fill_plus_traceback": round(cells / (f + t) / 1e6, 1),
            "tb_bytes": tb, "fill_hbm_gbs": round(tb / f / 1e6, 1),
            # one code byte per cell written: the fill's design bound is HBM
            # writes
            "roofline": {"bound": "hbm", "achieved": round(tb / f / 1e6, 1), "peak": 8000.0,
                         "unit": "GB/s", "frac": round(tb / f / 1e6 / 8000.0, 4),
                         "traffic": (counted("k_gotoh_fill") or {}).get("hbm_bytes"),
                         "kernel": "k_gotoh_fill"},
            # what does bound it: VALU issue, counted
            "roofline_alu": alu_roofline(counted("k_gotoh_fill"), f, "k_gotoh_fill")}


def bench_band(msadp, synth, torch, args):
    """Exact banded Levenshtein (lev_band) on the 512 long DNA pairs, against
    the full-matrix fill of the same pairs: effective GCUPS = all m x n cells
    over the banded time."""
    d = synth.nw_long()
    P = d["n_pairs"]
    A = msadp.to_device(d["a_codes"], d["a_offsets"], 4)
    B = msadp.to_device(d["b_codes"], d["b_offsets"], 4)
    la = np.diff(d["a_offsets"])
    lb = np.diff(d["b_offsets"])
    cells = int((la * lb).sum())
    stream = torch.cuda.current_stream()
    reps = max(args.steps, 3)
    out = {"workload": "lev_band: 512 DNA pairs, lengths U{5000..10000}, 10% divergence, "
                       "seed 4", "cells": cells, "by_k0": {}}
    for k0 in (256, 2048):
        band = msadp.LevBand(A, B, np.arange(P), np.arange(P), k0, 4000)
        band(stream)
        ms = _time_calls(torch, lambda: band(stream), stream, reps)
        band.st.check("lev_band")
        ku = band.k_used[:P].cpu().numpy()
        out["by_k0"][k0] = {"ms": round(ms, 3), "effective_gcups": round(cells / ms / 1e6, 1),
                            "k_used_max": int(ku.max()), "verified": int((ku > 0).sum())}
    nb = msadp.NwBatch(A, B, np.arange(P), np.arange(P))
    full = _time_calls(torch, lambda: nb.fill(stream), stream, reps)
    out["full_matrix_fill_ms"] = round(full, 3)
    out["full_matrix_gcups"] = round(cells / full / 1e6, 1)
    # the full-matrix distance of the same pairs through lev_batch, whose
    # default layout for long patterns with one partner each is a pair per
    # group of 64 lanes (2-3 pattern words per lane, carries passed by DPP)
    xb = msadp.LevBatch(A, B, np.arange(P), np.arange(P))
    xb(stream)
    lev_ms = _time_calls(torch, lambda: xb(stream), stream, reps)
    xb.st.check("lev_batch")
    out["lev_batch_across_lanes"] = {"ms": round(lev_ms, 3),
                                     "gcups": round(cells / lev_ms / 1e6, 1)}
    from oracle import pyoracle as orc
    sel = np.arange(32)
    out["cpu_oracle"] = oracle_beside(
        args, lambda: orc.lev_pairs(d["a_codes"], d["a_offsets"], d["b_codes"], d["b_offsets"],
                                    sel, sel),
        (la[sel] * lb[sel]).sum(), "Wagner-Fischer (all cells) on pairs 0-31 of the 512")
    return out


def tree_cells(t, L):
    """Levenshtein cells of one exact build: per internal node the medoid
    triangle and three pole rows (c, l and r against every member)."""
    perm = t["perm"].astype(np.int64)
    Lp = L[perm]
    c1 = np.concatenate([[0], np.cumsum(Lp)])
    c2 = np.concatenate([[0], np.cumsum(Lp * Lp)])
    ms, mc = t["mstart"].astype(np.int64), t["mcount"].astype(np.int64)
    v = np.flatnonzero(t["left"] >= 0)
    s1 = c1[ms[v] + mc[v]] - c1[ms[v]]
    s2 = c2[ms[v] + mc[v]] - c2[ms[v]]
    poles = L[t["center"][v]] + L[t["lpole"][v]] + L[t["rpole"][v]]
    return int(((s1 * s1 - s2) // 2 + poles * s1).sum())


def bench_insert(msadp, synth, torch, args):
    """Online insertion: 1,000 sequences of the learned workload's families
    (seeded choice) inserted into the exact tree of the other 99,000, against
    rebuilding the tree of all 100,000; both trees' alignments get the
    Sec. 2.3 metrics on the same 10,000 rows (the 1,000 new and 9,000 old)."""
    from paper_2601_15458_amd import learned
    d = synth.learned()
    n = d["n"]
    rng = np.random.default_rng(42)
    new = np.sort(rng.choice(n, size=1000, replace=False))
    keep = np.setdiff1d(np.arange(n), new)
    order = np.concatenate([keep, new])
    allset = synth.subset(d, order)
    n_old = len(keep)
    o = allset["offsets"]
    S_old = msadp.to_device(allset["codes"][: o[n_old]], o[: n_old + 1], d["sigma"])
    S = msadp.to_device(allset["codes"], allset["offsets"], d["sigma"])
    stream = torch.cuda.current_stream()
    old_b = msadp.TreeBuilder(S_old)
    t0 = time.perf_counter()
    old = old_b(stream)
    torch.cuda.synchronize()
    t_old = time.perf_counter() - t0
    old_b.st.check("tree_build")
    _log(f"insert: old tree of {n_old} in {t_old:.2f} s")
    msadp.tree_insert(S, n_old, old)          # warm-up
    ts = []
    for _ in range(max(3, min(args.steps, 5))):
        t0 = time.perf_counter()
        grown = msadp.tree_insert(S, n_old, old)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    t_ins = float(np.median(ts))
    full_b = msadp.TreeBuilder(S)
    t0 = time.perf_counter()
    full = full_b(stream)
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t0
    full_b.st.check("tree_build")
    sub = np.sort(np.concatenate([np.arange(n_old, n),
                                  rng.choice(n_old, 9000, replace=False)]))
    sub_d = synth.subset(allset, sub)
    S_sub = msadp.to_device(sub_d["codes"], sub_d["offsets"], d["sigma"])
    lev_sub = msadp.lev_allpairs(S_sub)
    max_len_sub = int(np.diff(sub_d["offsets"]).max())

    def quality(tree):
        t0 = time.perf_counter()
        msa = msadp.msa_merge(S, tree)
        t_merge = time.perf_counter() - t0
        Q = msadp.Quality(msa[sub], d["sigma"])
        q = Q.metrics(Q.pair_counts(), max_len_sub, lev=lev_sub)
        q = {k: (round(v, 6) if isinstance(v, float) else v) for k, v in q.items()}
        q["width"] = int(msa.shape[1])
        q["merge_s"] = round(t_merge, 3)
        return q

    gh, fh = grown.host(), full.host()
    from oracle import pyoracle as orc
    cpu = None
    if not args.no_cpu:
        small = synth.subset(allset, np.concatenate([np.arange(150),
                                                     np.arange(n_old, n_old + 20)]))
        seqs_small = synth.from_csr(small["codes"], small["offsets"])
        old_small = orc.tree(*synth.to_csr(seqs_small[:150]))
        cpu = oracle_beside(args, lambda: orc.tree_insert(small["codes"], small["offsets"], 150,
                                                          old_small),
                            0, "20 sequences into the oracle's tree of 150 (routing, "
                               "re-partition, renumbering; cells not counted)")
    out = {"workload": "tree_insert: 1,000 of the 100,000 learned-workload DNA seqs (seed 42) "
                       "into the exact tree of the other 99,000",
           "old_build_s": round(t_old, 3), "insert_s": round(t_ins, 4),
           "rebuild_s": round(t_full, 3), "speedup_vs_rebuild": round(t_full / t_ins, 1),
           "nodes_old": int(old.n_nodes), "nodes_inserted": int(gh["n_nodes"]),
           "nodes_rebuilt": int(fh["n_nodes"]),
           "rebuilt_clusters_kept": round(learned.reproduced_clusters(fh, gh), 4),
           "cpu_oracle": cpu,
           "alignment_quality": {"rows": "the 1,000 new and 9,000 seeded old rows, all pairs",
                                 "inserted": quality(grown), "rebuilt": quality(full)}}
    _log(f"insert: {out}")
    return out


def bench_tree(msadp, synth, torch, args):
    """Exact Alg. 1 build of the 20,000-sequence protein set: kernel class
    autotuned, levels replayed from a HIP graph (and, for comparison,
    launched one by one)."""
    d = synth.protein_tree()
    S = msadp.to_device(d["codes"], d["offsets"], d["sigma"])
    stream = torch.cuda.Stream()
    tuning = None
    if not args.no_tune:
        best, ms = msadp.autotune_tree(S, reps=1, stream=stream)
        tuning = {"kind": "tree words per pass", "chosen": best, "ms": round(ms, 1)}
        _log(f"tree class: {best} ({ms:.1f} ms)")
    times = {}
    for graph in (True, False):
        tb = msadp.TreeBuilder(S, use_graph=graph)
        with torch.cuda.stream(stream):
            tb(stream)
            torch.cuda.synchronize()
            ts = []
            for _ in range(max(args.steps, 3)):
                t0 = time.perf_counter()
                tree = tb(stream)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
        tb.st.check("tree_build")
        times[graph] = float(np.median(ts))
        if graph:
            host = tree.host()
    L = np.diff(d["offsets"]).astype(np.int64)
    cells = tree_cells(host, L)
    tg = times[True]
    # the oracle's Alg. 1 and the device's on the same seeded 150-sequence
    # subset (the full set would take the oracle hours)
    from oracle import pyoracle as orc
    sub = synth.subset(d, np.random.default_rng(39).choice(d["n"], 150, replace=False))
    Ss = msadp.to_device(sub["codes"], sub["offsets"], d["sigma"])
    msadp.tree_build(Ss)
    t0 = time.perf_counter()
    small = msadp.tree_build(Ss)
    t_small = time.perf_counter() - t0
    ls = np.diff(sub["offsets"]).astype(np.int64)
    cpu = oracle_beside(args, lambda: orc.tree(sub["codes"], sub["offsets"]),
                        tree_cells(small, ls),
                        "Alg. 1 (full median) on a seeded 150-sequence subset")
    if cpu:
        cpu["device_seconds_same_subset"] = round(t_small, 4)
    return {"workload": "tree_build: 20,000 protein seqs (200 families, lognormal lengths "
                        "median 350 in [50, 2000], 30% divergence), seed 3", "tuning": tuning,
            "n_nodes": int(host["n_nodes"]), "depth": int(host["depth"].max()),
            "build_s_graph": round(tg, 4), "build_s_launches": round(times[False], 4),
            "cells": cells, "gcups": round(cells / tg / 1e9, 1), "cpu_oracle": cpu}


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cnn_rates(learned, d, losses, t_train, positions, t_embed):
    """Embedder throughput: a training step is a forward, an input-gradient
    and a weight-gradient pass (3x the forward multiply-adds); the roofline
    is the BF16 dense MFMA peak."""
    f = learned.flops_per_position()
    all_pos = int(np.diff(d["offsets"]).sum())
    embed_tf = all_pos * f / t_embed / 1e12
    train_tf = 3 * positions * f / t_train / 1e12
    return {"train_step_ms": round(t_train / len(losses) * 1e3, 2),
            "train_pairs_per_s": round(len(losses) * 4096 / t_train, 1),
            "train_tflops": round(train_tf, 1),
            "embed_seqs_per_s": round(d["n"] / t_embed, 1),
            "embed_tflops": round(embed_tf, 1),
            "flops_per_position": f,
            "roofline": {"bound": "mfma", "achieved": round(embed_tf, 1), "peak": 2500.0,
                         "unit": "TFLOP/s", "frac": round(embed_tf / 2500.0, 4),
                         "traffic": None, "kernel": "k_conv (embedding pass, all kernels)"}}


def bench_cnn(msadp, synth, torch, args):
    """The embedder alone on the learned workload: training on the 2M
    labelled pairs (args.epochs epochs of 4096-pair steps) and one embedding
    pass over the 100,000 sequences; then two fresh runs of the first 50
    steps from the same seed, whose weights must agree bit for bit."""
    from paper_2601_15458_amd import learned
    d = synth.learned()
    S = msadp.to_device(d["codes"], d["offsets"], d["sigma"])
    ia, ib = learned.sample_pairs(d["family"], 2_000_000, seed=11)
    dist = learned.lev_labels(S, ia, ib)
    E, losses, t_train, positions = learned.train(S, ia, ib, dist, epochs=args.epochs, seed=13)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E.embed(S)
    torch.cuda.synchronize()
    t_embed = time.perf_counter() - t0
    out = {"workload": "cnn_train_step + cnn_embed: 100,000 DNA seqs (lengths 100-500), "
                       "2M pairs, batches of 4096, seed 5/11/13",
           "epochs": args.epochs, "steps": len(losses),
           "loss_first_last": [round(float(losses[:50].mean()), 5),
                               round(float(losses[-50:].mean()), 5)],
           "rates": cnn_rates(learned, d, losses, t_train, positions, t_embed)}
    sel = 50 * 4096
    weights = []
    for _ in range(2):
        E2, _, _, _ = learned.train(S, ia[:sel], ib[:sel], dist[:sel], epochs=1, seed=13)
        weights.append(E2.get()[0])
    out["bit_identical_weights_two_runs_50_steps"] = all(
        np.array_equal(a, c) and np.array_equal(b, e)
        for (a, b), (c, e) in zip(weights[0], weights[1]))
    return out


def bench_pruned(msadp, synth, torch, args):
    """Learned pruning on 100,000 DNA sequences of 1,000 families: train the
    embedder on 2M exact pairs, then the exact and the pruned tree build,
    teacher-forced agreement of (c, l, r) and the control rankers."""
    from paper_2601_15458_amd import learned
    d = synth.learned()
    S = msadp.to_device(d["codes"], d["offsets"], d["sigma"])
    _log(f"learned workload: {d['n']} seqs")
    ia, ib = learned.sample_pairs(d["family"], 2_000_000, seed=11)
    ha, hb = learned.sample_pairs(d["family"], 20_000, seed=12)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dist = learned.lev_labels(S, ia, ib)
    torch.cuda.synchronize()
    t_label = time.perf_counter() - t0
    hdist = learned.lev_labels(S, ha, hb)
    _log(f"labels {t_label:.2f} s; training {args.epochs} epochs")
    E, losses, t_train, positions = learned.train(S, ia, ib, dist, epochs=args.epochs, seed=13,
                                                  log=_log)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    emb = E.embed(S)
    torch.cuda.synchronize()
    t_embed = time.perf_counter() - t0
    mae, rel = learned.pair_error(emb, S, ha, hb, hdist)
    _log(f"trained in {t_train:.1f} s, held-out MAE {mae:.2f} edits ({rel:.4f} rel); "
         "exact build")
    # both builds replay each level from a HIP graph on their own stream, and
    # both are timed the same way: one warm-up build, then the median of
    # timed builds (device tree; the host copy is outside the timing)
    stream = torch.cuda.Stream()
    exact_b = msadp.TreeBuilder(S, use_graph=True)
    times = []
    with torch.cuda.stream(stream):
        exact_dev = exact_b(stream)
        torch.cuda.synchronize()
        for _ in range(max(1, min(args.steps, 2))):
            t0 = time.perf_counter()
            exact_dev = exact_b(stream)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
    exact_b.st.check("tree_build")
    t_exact = float(np.median(times))
    exact = exact_dev.host()
    # alignment quality (Sec. 2.3 metrics) of the exact tree's alignment on a
    # seeded 10,000-row subsample, as the paper measures large alignments
    sub = np.sort(np.random.default_rng(15).choice(d["n"], 10_000, replace=False))
    sub_d = synth.subset(d, sub)
    S_sub = msadp.to_device(sub_d["codes"], sub_d["offsets"], sub_d["sigma"])
    lev_sub = msadp.lev_allpairs(S_sub)
    max_len_sub = int(np.diff(sub_d["offsets"]).max())

    def msa_quality_of(tree_dev):
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            msa = msadp.msa_merge(S, tree_dev, stream=stream)
        t_merge = time.perf_counter() - t0
        Q = msadp.Quality(msa[sub], d["sigma"])
        q = Q.metrics(Q.pair_counts(), max_len_sub, lev=lev_sub)
        q = {k: (round(v, 6) if isinstance(v, float) else v) for k, v in q.items()}
        q["width"] = int(msa.shape[1])
        q["merge_s"] = round(t_merge, 3)
        return q

    exact_quality = msa_quality_of(exact_dev)
    _log(f"exact tree alignment: {exact_quality}")
    _log(f"exact build {t_exact:.2f} s ({exact['n_nodes']} nodes); pruned builds")
    out = {"workload": "tree build: 100,000 DNA seqs (1,000 families x 100, mutate d=0.30, "
                       "lengths 100-500, seed 5)",
           "train_pairs": len(ia), "epochs": args.epochs,
           "label_s": round(t_label, 3), "train_s": round(t_train, 2),
           "train_loss_first_last": [round(float(losses[:50].mean()), 5),
                                     round(float(losses[-50:].mean()), 5)],
           "embed_s": round(t_embed, 3), "heldout_mae_edits": round(mae, 3),
           "cnn": cnn_rates(learned, d, losses, t_train, positions, t_embed),
           "heldout_rel_err": round(rel, 4), "exact_build_s": round(t_exact, 3),
           "exact_nodes": int(exact["n_nodes"]),
           "alignment_quality": {"rows": "seeded 10,000-row subsample (seed 15), all pairs",
                                 "exact_tree": exact_quality}}
    off, ca, cb, corr = learned.calibrate(emb, S, d["family"])
    _log(f"calibration on within-family pairs: y = {ca:.3f} + {cb:.4f} y_hat "
         f"(corr {corr:.3f}) -> offset {off:.3f}")
    out["calibration"] = {"offset": round(off, 4), "intercept": round(ca, 4),
                          "slope": round(cb, 5), "corr": round(corr, 4)}
    # which distance passes run with a pair per group of lanes (the set's
    # patterns: 8 words, one or two per lane): timed per variant on the
    # sampled build (16 pivots, top 32) and kept for every build below
    words = (S.max_len + 63) // 64
    if args.no_tune:
        xl = {"value": msadp.tune_get(msadp.MSA_TUNE_TREE_XL, d["sigma"], words) or None,
              "tuned": False}
    else:
        with torch.cuda.stream(stream):
            best, ms = msadp.autotune_tree_xl(S, pivots=16, topk=32, stream=stream)
        xl = {"value": best, "tuned": True, "ms": round(ms, 1)}
        _log(f"across-lanes passes: {msadp.xl_describe(best)} ({ms:.1f} ms per sampled build)")
    if xl["value"]:
        xl["variant"] = msadp.xl_describe(xl["value"])
    out["across_lanes"] = xl
    # ranker -> (embedding, offset): the calibrated network, the raw network,
    # the length prior (shortest first) and noise
    rankers = {"cnn": (emb, off), "cnn_raw": (emb, 0.0),
               "shortest": (learned.control_embeddings(S, "zero"), 1.0),
               "random": (learned.control_embeddings(S, "random", seed=14), 0.0)}
    # the median over a smaller subset (Sec. 2.1): candidates ranked by their
    # summed exact distance to P hashed members ("sampledP"); no embedding
    for p in (4, 8, 16):
        rankers[f"sampled{p}"] = (None, 0.0)
    # (ranker, topk, exact_below): pure top-k pruning of every cluster, and
    # the hybrid that keeps the full median for clusters it finds cheap
    # the four rankers at top-16; more candidates (64, 96) and the hybrid
    # that keeps the full median for clusters of at most 2048 members, the
    # ways to reach 99 % agreement
    points = [("cnn", args.topk, 0), ("cnn_raw", args.topk, 0), ("shortest", args.topk, 0),
              ("random", args.topk, 0),
              ("cnn", 64, 0), ("cnn", 96, 0), ("shortest", 96, 0),
              ("cnn", args.topk, args.exact_below), ("cnn", args.topk, 8 * args.exact_below),
              ("sampled8", args.topk, 0), ("sampled16", args.topk, 0), ("sampled8", 32, 0),
              ("sampled16", 32, 0)]
    if args.points:
        points = []
        for item in args.points.split(","):
            name, topk, eb = item.split(":")
            if name not in rankers:
                raise ValueError(f"unknown ranker {name!r} (one of {sorted(rankers)})")
            points.append((name, int(topk), int(eb)))
    out["points"] = []
    quality_points = {("cnn", args.topk, 0), ("cnn", 96, 0), ("shortest", 96, 0),
                      ("sampled16", 32, 0)}
    for name, topk, eb in points:
        e, eo = rankers[name]
        piv = int(name[len("sampled"):]) if name.startswith("sampled") else 0
        b = msadp.TreeBuilder(S, use_graph=True, emb=e, topk=topk, exact_below=eb,
                              emb_offset=eo, pivots=piv)
        times = []
        with torch.cuda.stream(stream):
            b(stream)
            torch.cuda.synchronize()
            for _ in range(max(1, min(args.steps, 3))):
                t0 = time.perf_counter()
                t = b(stream)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
        b.st.check("tree_build_pruned")
        quality = None
        if (name, topk, eb) in quality_points:
            quality = msa_quality_of(t)
        t = t.host()
        clr = msadp.tree_eval_centers(S, exact, emb=e, topk=topk, exact_below=eb, emb_offset=eo,
                                      pivots=piv)
        agree = learned.agreement(exact, clr, min_size=17, pruned_above=max(topk, eb))
        rep = learned.reproduced_clusters(exact, t)
        nd, ex_mean, ex_max = learned.rowsum_excess(S, exact, clr, max(topk, eb))
        tp = float(np.median(times))
        # the network's rankings need the embedding pass (once per set);
        # the other rankers need none
        t_emb = t_embed if name.startswith("cnn") else 0.0
        out["points"].append({"ranker": name, "offset": round(eo, 4), "pivots": piv,
                              "topk": topk,
                              "exact_below": eb,
                              "build_s": round(tp, 4), "speedup": round(t_exact / tp, 2),
                              "speedup_with_embedding": round(t_exact / (tp + t_emb), 2),
                              "agreement": agree, "reproduced_clusters": round(rep, 4),
                              "center_differs": nd, "rowsum_excess_mean": round(ex_mean, 6),
                              "rowsum_excess_max": round(ex_max, 6),
                              "nodes": int(t["n_nodes"]), "alignment_quality": quality})
        _log(f"{name} topk={topk} exact_below={eb}: build {tp:.3f} s, speedup "
             f"{t_exact / tp:.1f}x, agreement {agree}, reproduced {rep:.4f}, "
             f"excess over {nd} differing centers mean {ex_mean:.2e} max {ex_max:.2e}")
    return out


if __name__ == "__main__":
    main()
