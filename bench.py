#!/usr/bin/env python3
"""Benchmark of the Kruskal-Wallis SNP x trait scan on one MI355X.

A step is one pass of the whole path over one workload with the inputs
resident in HBM: per-trait ranking (krux_rank) and the test of every trait
against every SNP (krux_test / krux_permute / krux_test_batched): genotype
packing, the fused MFMA rank-sum GEMM with its statistic / threshold /
p-value / compaction epilogue, exact evaluation of screened pairs, hit
sorting and the per-trait minimum-p passes.

Workloads (--workload; seeded synthetic data shaped like the paper's
102-sample human blood data set):
  paper_scale_hits (default)  K=102, 20,000 log-normal traits with 5% forced
      ties, 500,000 Hardy-Weinberg SNPs (MAF U[0.05, 0.5]), 500 planted pairs;
      sorted hits at p < 1e-5 plus the per-trait minimum p; fp16 path, beside
      the int8 path and the fp64-GEMM comparator on the same inputs
  precision_K500   K=500, 20,000 traits, 100,000 SNPs; hits at p < 1e-5 through
      the fp16, int8 (byte-split ranks) and fp64-GEMM paths, plus group rank
      sums of a slice compared bit for bit across the three
  permutations     K=102, 20,000 traits, 100,000 SNPs, 200 permutations of the
      samples; per-permutation hit counts at p < {1e-4, 1e-5, 1e-6} and the
      per-(permutation, trait) minimum p; beside it the full empirical FDR
      curve at p < 1e-5 (real and permuted hit lists, FDR at every real hit)
  cohorts_missing  8 cohorts, K in {48, ..., 1000}, 5,000-20,000 traits each,
      one 200,000-SNP panel with 2% missing genotypes; hits at p < 1e-5 per
      cohort
  sample_missing   the paper-scale workload with sample-structured missing
      genotypes (samples 5 and 40 missing in 90% of the SNPs, sample 77 in
      30%); the pattern-grouped scan timed beside the per-pair path
  multi_allelic    K=102, 20,000 traits, 50,000 markers with 4 genotype classes
      (class frequencies Dirichlet(1) per marker); hits at p < 1e-5 plus the
      per-trait minimum p through the lane-per-pair multi-allelic kernel
  missing_expression  the paper-scale workload with NaN expression values in
      2% of the traits (1-5 each); hits at p < 1e-5 plus the per-trait minimum
      p, timed beside the same traits without NaN values

The default run (paper_scale_hits) also measures precision_K500, permutations
and cohorts_missing with fewer steps and reports them under "other_configs",
and checks the paper-scale results against the CPU oracle on a prefix of the
SNPs ("parity", "parity_checks").  Prints ONE JSON line on stdout; progress
goes to stderr.
"""
import argparse
import json
import os
import sys
import time

METRIC = "SNP-trait pairs/sec at N=102 (exact MFMA vs FP64 GEMM), % MFMA peak"
PEAK_FP16_TFLOPS = 2500.0      # MI355X dense fp16 MFMA
PEAK_INT8_TOPS = 5000.0        # MI355X dense int8 MFMA
PEAK_FP64_TFLOPS = 78.6        # MI355X fp64 MFMA
DATA = "synthetic (seeded generators shaped like the paper's 102-sample blood data)"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


ROOT = os.path.dirname(os.path.abspath(__file__))
PROFILE = os.path.join(ROOT, "profiles", "scan_f16_diag_screen_K102_T20000_M500000.txt")


DOMINANT_KERNEL = "_ZN2kx11scan_kernelILi0ELi7ELi0ELi0ELi4ELi3EEEvNS_8ScanArgsE"


def _elf_symbols(elf, names):
    """Bytes of the named symbols of an ELF64 image (code objects here)."""
    import struct
    shoff, = struct.unpack_from("<Q", elf, 0x28)
    shentsize, shnum = struct.unpack_from("<HH", elf, 0x3A)
    secs = [struct.unpack_from("<IIQQQQIIQQ", elf, shoff + k * shentsize) for k in range(shnum)]
    out = {}
    for sh in secs:
        if sh[1] != 2:                      # SHT_SYMTAB
            continue
        strtab = secs[sh[6]]
        for k in range(sh[5] // 24):
            st_name, st_info, st_other, st_shndx, st_value, st_size = struct.unpack_from(
                "<IBBHQQ", elf, sh[4] + 24 * k)
            o = strtab[4] + st_name
            name = elf[o:elf.index(b"\0", o)].decode()
            if name in names and 0 < st_shndx < len(secs):
                sec = secs[st_shndx]
                start = sec[4] + st_value - sec[3]
                out[name] = elf[start:start + st_size]
    return out


def kernel_digest(lib_path, symbol):
    """sha256 of a kernel's gfx950 machine code and kernel descriptor, read from
    the code objects embedded in the library, or None if not found."""
    import hashlib
    import struct
    data = open(lib_path, "rb").read()
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    pos = data.find(magic)
    while pos >= 0:
        n, = struct.unpack_from("<Q", data, pos + len(magic))
        off = pos + len(magic) + 8
        for _ in range(n):
            o, size, tl = struct.unpack_from("<QQQ", data, off)
            triple = data[off + 24:off + 24 + tl]
            off += 24 + tl
            if b"gfx950" in triple and size:
                found = _elf_symbols(data[pos + o:pos + o + size], (symbol, symbol + ".kd"))
                if symbol in found:
                    return hashlib.sha256(found[symbol] + found.get(symbol + ".kd", b"")).hexdigest()
        pos = data.find(magic, pos + 1)
    return None


def measured_traffic():
    """HBM bytes per main-pass launch of the dominant kernel from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE runs, scaled by a plain copy),
    or None when the kernel's machine code in the built library differs from
    the one the counters were taken on."""
    try:
        fields = {}
        for line in open(PROFILE):
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        from paper_1307_3519_amd import krux
        if kernel_digest(krux.LIB_PATH, fields["kernel_symbol"]) != fields["kernel_sha256"]:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


class Runner:
    """Warmup + timed steps with the fused-kernel timer."""

    def __init__(self, ctx, torch):
        self.ctx = ctx
        self.torch = torch

    def run(self, step, steps, warmup):
        torch = self.torch
        res = None
        for _ in range(warmup):
            res = step()
        torch.cuda.synchronize()
        self.ctx.timer_start()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kms, kn = self.ctx.timer_read()
        # per step: all timed scan launches (two per main pass)
        return (t1 - t0) * 1e3 / steps, res, kms / max(steps, 1), kn


def same_hits(a, b):
    import numpy as np
    return bool(a[0] == b[0] and np.array_equal(a[1]["trait"], b[1]["trait"])
                and np.array_equal(a[1]["snp"], b[1]["snp"]))


def base_line(args, metric, value, unit, ms, dtype, config):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": DATA, "config": config}


def roofline(kernel, pairs, flops_per_pair, kern_ms, peak, unit, traffic=None):
    achieved = pairs * flops_per_pair / (kern_ms / 1e3) / 1e12
    return {"bound": "mfma", "kernel": kernel, "achieved": achieved, "peak": peak,
            "unit": unit, "frac": achieved / peak, "traffic": traffic, "kernel_ms": kern_ms,
            "flops_per_pair": flops_per_pair}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def oracle_baseline(args, T, n_total, label, run_sample):
    """Times the oracle on a bounded prefix of the SNPs: run_sample(n) scans
    all traits against the first n SNPs and returns the oracle's result.
    Returns (cpu_baseline dict, that result for the timed sample, n); the
    timed sample runs on all the oracle's threads, a smaller one on one."""
    import oracle
    threads = oracle.num_threads()
    probe = max(1, min(n_total, 200))
    t0 = time.perf_counter()
    run_sample(probe)
    rate = T * probe / (time.perf_counter() - t0)
    n_snp = int(min(n_total, max(probe, args.cpu_seconds * rate / max(T, 1))))
    log("oracle baseline: %d traits x %d SNPs (probe %.3e pairs/s)" % (T, n_snp, rate))
    t0 = time.perf_counter()
    res = run_sample(n_snp)
    dt = time.perf_counter() - t0
    log("oracle: %.3e pairs/s on %d threads" % (T * n_snp / dt, threads))
    # one thread, on about a quarter of the time budget
    n1 = int(min(n_snp, max(1, args.cpu_seconds / 4.0 * (rate / threads) / max(T, 1))))
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        run_sample(n1)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(threads)
    log("oracle: %.3e pairs/s on 1 thread" % (T * n1 / dt1))
    base = {"value": T * n_snp / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "all %d traits x the first %d of %d SNPs (%s), %.1f s"
                      % (T, n_snp, n_total, label, dt),
            "one_thread": {"value": T * n1 / dt1, "unit": "pairs/s",
                           "sample": "all %d traits x the first %d SNPs, %.1f s" % (T, n1, dt1)}}
    return base, res, n_snp


def oracle_rate(*args):
    return oracle_baseline(*args)[0]


def hits_match(got, want, snp_offset=0):
    """Identical (trait, snp) lists, H within 1e-12 relative, p within 1e-10
    relative (absolute floor 1e-300)."""
    import numpy as np
    if len(got["trait"]) != len(want["trait"]):
        return False
    if not (np.array_equal(got["trait"], want["trait"])
            and np.array_equal(got["snp"] - snp_offset, want["snp"])):
        return False
    rel = np.abs(got["H"] - want["H"]) / np.maximum(np.abs(want["H"]), 1e-300)
    dp = np.abs(got["p"] - want["p"]) <= np.maximum(1e-10 * np.abs(want["p"]), 1e-300)
    return bool(rel.max(initial=0.0) <= 1e-12 and dp.all())


def min_p_match(got, want):
    import numpy as np
    return bool(np.all(np.abs(got - want) <= np.maximum(1e-10 * np.abs(want), 1e-300)))


def oracle_scan_hits(oracle, x, g, p_c, min_p=True):
    """The oracle's hits (+ minimum p) in one pass, with a hit buffer large
    enough for the null rate and the planted pairs."""
    cap = max(1 << 16, int(x.shape[0] * g.shape[0] * p_c * 20))
    return oracle.scan(x, g, p_cs=(p_c,), hits=True, min_p=min_p, hit_cap=cap)


# ---------------------------------------------------------------- workloads
def paper_scale_hits(args, ctx, torch, np, datagen, krux):
    wl = dict(datagen.WORKLOADS[2])
    T = args.T or wl["T"]
    M = args.M or wl["M"]
    K = wl["K"]
    p_c = 1e-5
    log("generating workload K=%d T=%d M=%d" % (K, T, M))
    t0 = time.time()
    w = datagen.make_workload(2, T=T, M=M)
    log("generated in %.1fs" % (time.time() - t0))
    x = torch.from_numpy(w["expr"]).cuda()
    g = torch.from_numpy(w["geno"]).cuda()
    cap = 1 << 17          # hit-list capacity (about 2.4e4 hits are expected)
    bufs = {}
    runner = Runner(ctx, torch)

    def step_for(prec):
        def step():
            r, ts, _ = ctx.rank(x)
            res = ctx.test(r, ts, g, p_c=p_c, mode="hits", precision=prec, hit_capacity=cap,
                           min_p=not args.no_minp, out=bufs.get(prec))
            bufs[prec] = res
            return res
        return step

    log("fp16 path: %d warmup + %d timed steps" % (args.warmup, args.steps))
    ms, res, kern_ms, kn = runner.run(step_for("fp16"), args.steps, args.warmup)
    pairs = float(T) * float(M)
    value = pairs / (ms / 1e3)
    hits16 = krux.unpack_hits(res)
    minp = {"fp16": None if args.no_minp else res["min_p"].cpu().numpy()}
    planted = set(map(tuple, w["planted"][:, :2].tolist()))
    found = set(zip(hits16[1]["trait"].tolist(), hits16[1]["snp"].tolist()))
    log("fp16: %.3f ms/step, %.3e pairs/s, hits %d, planted recovered %d/%d"
        % (ms, value, hits16[0], len(planted & found), len(planted)))
    flops_per_pair = 2 * K * 2          # two genotype classes of a K-long contraction
    out = base_line(args, METRIC, value, "pairs/s", ms, "f16", {
        "workload": "paper_scale_hits", "K": K, "T": T, "M": M,
        "planted": int(w["planted"].shape[0]), "p_c": p_c,
        "outputs": "sorted hit list (p < 1e-5)" + ("" if args.no_minp else " + per-trait min p")})
    if not args.no_graph:
        # the same step (ranks, scan, exact pass, minimum-p fix-ups, hit sort)
        # captured once as a HIP graph and replayed as one launch per step;
        # reported beside the eager rate, which stays the value
        r0, ts0, _ = ctx.rank(x)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            rr, tt, _ = ctx.rank(x, out=(r0, ts0))
            ctx.test(rr, tt, g, p_c=p_c, mode="hits", precision="fp16", hit_capacity=cap,
                     min_p=not args.no_minp, out=bufs["fp16"])
        graph.replay()
        torch.cuda.synchronize()
        same = same_hits(krux.unpack_hits(bufs["fp16"]), hits16) and (
            args.no_minp or bool(np.array_equal(bufs["fp16"]["min_p"].cpu().numpy(), minp["fp16"])))
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.replay()
        torch.cuda.synchronize()
        gms = (time.perf_counter() - t0) * 1e3 / args.steps
        log("fp16, one graph launch per step: %.3f ms/step, hits and minima identical %s"
            % (gms, same))
        out["graph_replay"] = {"ms_per_step": gms, "value": pairs / (gms / 1e3), "unit": "pairs/s",
                               "identical_hits_and_min_p": same}
    rl = roofline("scan_kernel<F16, KS=7, DIAG, SCREEN>", pairs, flops_per_pair, kern_ms,
                  PEAK_FP16_TFLOPS, "TFLOP/s", measured_traffic())
    rl["kernel_launches"] = kn
    rl["kernel_ms_note"] = ("main pass per step: the complete-SNP kernel plus the "
                            "missing-genotype kernel, which returns at once here")
    out["roofline"] = rl
    out["n_hits"] = hits16[0]
    out["planted_recovered"] = [len(planted & found), len(planted)]

    if not args.no_compare:
        log("fp64 GEMM comparator: 1 warmup + 2 timed steps")
        ms64, res64, _, _ = runner.run(step_for("fp64"), 2, 1)
        same = same_hits(krux.unpack_hits(res64), hits16)
        minp["fp64"] = None if args.no_minp else res64["min_p"].cpu().numpy()
        log("fp64: %.3f ms/step, %.3e pairs/s, identical hits %s" % (ms64, pairs / (ms64 / 1e3), same))
        out["fp64_gemm"] = {"value": pairs / (ms64 / 1e3), "unit": "pairs/s", "ms_per_step": ms64,
                            "identical_hits": same,
                            "speedup_of_fp16": (pairs / (ms / 1e3)) / (pairs / (ms64 / 1e3)),
                            "peak_fp64_tflops": PEAK_FP64_TFLOPS}
        n8 = max(3, args.steps // 2)
        log("int8 path: %d warmup + %d timed steps" % (max(1, args.warmup // 2), n8))
        ms8, res8, k8ms, _ = runner.run(step_for("int8"), n8, max(1, args.warmup // 2))
        same8 = same_hits(krux.unpack_hits(res8), hits16)
        minp["int8"] = None if args.no_minp else res8["min_p"].cpu().numpy()
        out["int8"] = {"value": pairs / (ms8 / 1e3), "unit": "pairs/s", "ms_per_step": ms8,
                       "kernel_ms": k8ms,
                       "kernel_tops": pairs * flops_per_pair / (k8ms / 1e3) / 1e12,
                       "frac_of_int8_peak": pairs * flops_per_pair / (k8ms / 1e3) / 1e12 / PEAK_INT8_TOPS,
                       "identical_hits": same8}
        log("int8: %.3f ms/step, identical hits %s" % (ms8, same8))

    if not args.no_minp:
        # per-trait minimum p of the three paths on the whole workload
        for prec in ("int8", "fp64"):
            if minp.get(prec) is not None:
                out["int8" if prec == "int8" else "fp64_gemm"]["identical_min_p"] = bool(
                    np.array_equal(minp[prec], minp["fp16"]))
    if not args.no_cpu:
        import oracle
        base, o, n = oracle_baseline(
            args, T, M, "hits at p<1e-5 + per-trait min p",
            lambda n: oracle_scan_hits(oracle, w["expr"], w["geno"][:n], p_c))
        out["cpu_baseline"] = base
        # parity with the oracle at this shape: (1) the hits of the whole
        # run that fall in the oracle's SNP prefix, (2) a GPU scan of that
        # prefix (hits and per-trait minimum p), (3) the minima of the
        # three GPU paths on the whole workload against each other
        h = hits16[1]
        sel = h["snp"] < n
        pre = {k: v[sel] for k, v in h.items()}
        r, ts, _ = ctx.rank(x)
        sub = ctx.test(r, ts, g[:n], p_c=p_c, mode="hits", precision="fp16",
                       hit_capacity=1 << 17, min_p=True)
        n_sub, h_sub = krux.unpack_hits(sub)
        checks = {"oracle_snps": n, "oracle_hits": int(o["n_hits"]),
                  "full_run_hits_in_prefix": hits_match(pre, o["hits"]),
                  "prefix_scan_hits": n_sub == o["n_hits"] and hits_match(h_sub, o["hits"]),
                  "prefix_scan_min_p": min_p_match(sub["min_p"].cpu().numpy(), o["min_p"])}
        if not args.no_minp and not args.no_compare:
            checks["min_p_fp16_eq_fp64_eq_int8"] = bool(
                np.array_equal(minp["fp16"], minp["fp64"])
                and np.array_equal(minp["fp16"], minp["int8"]))
        out["parity"] = all(v for k, v in checks.items() if isinstance(v, bool))
        out["parity_checks"] = checks
        log("parity with the oracle: %s %s" % (out["parity"], checks))
    out["paper_context"] = {"kruX_matlab_single_cpu_pairs_per_s": 4.2e6,
                            "note": "derived from the paper's ~2,500 s for 19,610 x 530,222 "
                                    "pairs on one CPU; another machine and method, context only"}
    return out


def precision_k500(args, ctx, torch, np, datagen, krux):
    wl = dict(datagen.WORKLOADS[3])
    T = args.T or wl["T"]
    M = args.M or wl["M"]
    K = wl["K"]
    p_c = 1e-5
    log("generating workload K=%d T=%d M=%d" % (K, T, M))
    w = datagen.make_workload(3, T=T, M=M)
    x = torch.from_numpy(w["expr"]).cuda()
    g = torch.from_numpy(w["geno"]).cuda()
    runner = Runner(ctx, torch)
    bufs = {}

    def step_for(prec):
        def step():
            r, ts, _ = ctx.rank(x)
            res = ctx.test(r, ts, g, p_c=p_c, mode="hits", precision=prec, hit_capacity=1 << 17,
                           min_p=True, out=bufs.get(prec))
            bufs[prec] = res
            return res
        return step

    pairs = float(T) * float(M)
    flops_per_pair = 4 * K
    res = {}
    for prec, steps, warm in (("fp16", args.steps, args.warmup), ("int8", args.steps, args.warmup),
                              ("fp64", 2, 1)):
        log("%s: %d warmup + %d timed steps" % (prec, warm, steps))
        ms, r, kms, _ = runner.run(step_for(prec), steps, warm)
        res[prec] = (ms, krux.unpack_hits(r), kms, r["min_p"].cpu().numpy())
        log("%s: %.3f ms/step, %.3e pairs/s, hits %d" % (prec, ms, pairs / (ms / 1e3), res[prec][1][0]))
    ms = res["fp16"][0]
    out = base_line(args, "SNP-trait pairs/sec at N=500, three precisions", pairs / (ms / 1e3),
                    "pairs/s", ms, "f16", {"workload": "precision_K500", "K": K, "T": T, "M": M,
                                           "p_c": p_c, "outputs": "hits + per-trait min p"})
    out["roofline"] = roofline("scan_tiled<F16, PLAIN, SCREEN>", pairs, flops_per_pair,
                               res["fp16"][2], PEAK_FP16_TFLOPS, "TFLOP/s")
    for prec, peak in (("int8", PEAK_INT8_TOPS), ("fp64", PEAK_FP64_TFLOPS)):
        ms_p, hits_p, kms_p, mp_p = res[prec]
        d = {"value": pairs / (ms_p / 1e3), "unit": "pairs/s", "ms_per_step": ms_p,
             "identical_hits": same_hits(hits_p, res["fp16"][1]),
             "identical_min_p": bool(np.array_equal(mp_p, res["fp16"][3]))}
        if prec == "int8":
            d["kernel_ms"] = kms_p
            d["frac_of_int8_peak"] = pairs * flops_per_pair / (kms_p / 1e3) / 1e12 / peak
        out[prec] = d
    # group rank sums of a slice, bit for bit across the three precisions
    ms_slice = min(M, 2000)
    r, ts, _ = ctx.rank(x)
    sums = {p: ctx.test(r, ts, g[:ms_slice], mode="sums", precision=p)["sums"].cpu().numpy()
            for p in ("fp16", "int8", "fp64")}
    out["sums_slice"] = {"traits": T, "snps": ms_slice,
                         "fp16_eq_fp64": bool(np.array_equal(sums["fp16"], sums["fp64"])),
                         "int8_eq_fp64": bool(np.array_equal(sums["int8"], sums["fp64"]))}
    log("sums slice identical: %s" % out["sums_slice"])
    if not args.no_cpu:
        import oracle
        out["cpu_baseline"] = oracle_rate(
            args, T, M, "hits at p<1e-5 + per-trait min p",
            lambda n: oracle.scan(w["expr"], w["geno"][:n], p_cs=(p_c,), hits=True, min_p=True))
    return out


def permutations(args, ctx, torch, np, datagen, krux):
    wl = dict(datagen.WORKLOADS[4])
    T = args.T or wl["T"]
    M = args.M or wl["M"]
    K = wl["K"]
    P = args.P or wl["P"]
    p_cs = (1e-4, 1e-5, 1e-6)
    log("generating workload K=%d T=%d M=%d P=%d" % (K, T, M, P))
    w = datagen.make_workload(4, T=T, M=M, P=P)
    x = torch.from_numpy(w["expr"]).cuda()
    g = torch.from_numpy(w["geno"]).cuda()
    perms = torch.from_numpy(w["perms"]).cuda()
    runner = Runner(ctx, torch)
    buf = {}

    def step():
        r, ts, _ = ctx.rank(x)
        res = ctx.permute(r, ts, g, perms, p_cs=p_cs, min_p=True, out=buf.get("o"))
        buf["o"] = res
        return res

    steps = max(1, min(args.steps, 3))
    log("permutations: 1 warmup + %d timed steps" % steps)
    ms, res, kms, _ = runner.run(step, steps, 1)
    pairs = float(P) * T * M
    counts = res["counts"].cpu().numpy()
    log("permute: %.1f ms/step, %.3e pairs/s, mean counts %s" % (ms, pairs / (ms / 1e3),
                                                                 counts.mean(axis=0)))
    out = base_line(args, "permuted SNP-trait pairs/sec at N=102", pairs / (ms / 1e3), "pairs/s",
                    ms, "f16", {"workload": "permutations", "K": K, "T": T, "M": M, "P": P,
                                "p_c": list(p_cs),
                                "outputs": "per-permutation counts + per-(permutation, trait) min p"})
    out["steps"] = steps
    out["warmup"] = 1
    out["roofline"] = roofline("scan_kernel<F16, KS=7, DIAG, SCREEN>", pairs, 4 * K, kms,
                               PEAK_FP16_TFLOPS, "TFLOP/s")
    out["mean_counts"] = counts.mean(axis=0).tolist()
    # the same step captured once into a HIP graph and replayed as one launch
    r, ts, _ = ctx.rank(x)
    o = buf["o"]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ctx.permute(r, ts, g, perms, p_cs=p_cs, min_p=True, out=o)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rr, tt, _ = ctx.rank(x, out=(r, ts))
        ctx.permute(rr, tt, g, perms, p_cs=p_cs, min_p=True, out=o)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    gms = (time.perf_counter() - t0) * 1e3 / steps
    same = bool(np.array_equal(o["counts"].cpu().numpy(), counts))
    log("graph replay: %.1f ms/step, counts identical %s" % (gms, same))
    out["graph_replay"] = {"ms_per_step": gms, "value": pairs / (gms / 1e3), "unit": "pairs/s",
                           "identical_counts": same}
    # the full empirical FDR curve at p < 1e-5: real hits, permuted hits (all
    # P permutations), FDR at every real hit's p
    p_f = p_cs[1]
    fcap = 1 << 23

    def fdr_step():
        r, ts, _ = ctx.rank(x)
        real = ctx.test(r, ts, g, p_c=p_f, mode="hits", precision="fp16", hit_capacity=1 << 17,
                        min_p=False)
        ph = ctx.permute_hits(r, ts, g, perms, p_c=p_f, hit_capacity=fcap)
        return real, ph, ctx.fdr_curve(real, ph, P)

    fdr_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        real, ph, fdr = fdr_step()
    torch.cuda.synchronize()
    fms = (time.perf_counter() - t0) * 1e3 / steps
    n_real, hr = krux.unpack_hits(real)
    n_perm = int(ph["n_hits_t"].item())
    f = fdr[:n_real].cpu().numpy()
    order = np.argsort(hr["p"], kind="stable")
    at = [float(f[order[min(len(order) - 1, int(q * len(order)))]]) for q in (0.1, 0.5, 0.9)] \
        if n_real else []
    log("FDR curve: %.1f ms/step, %d real hits, %d permuted hits (%.1f per permutation)"
        % (fms, n_real, n_perm, n_perm / P))
    out["fdr_curve"] = {"ms_per_step": fms, "p_c": p_f, "n_real_hits": n_real,
                        "n_permuted_hits": n_perm,
                        "fdr_at_real_p_quantiles_0.1_0.5_0.9": at,
                        "outputs": "real hit list, permuted hit lists, FDR at every real hit"}
    if not args.no_cpu:
        import oracle
        out["cpu_baseline"] = oracle_rate(
            args, T, M, "one permutation, counts + min p",
            lambda n: oracle.scan(w["expr"], w["geno"][:n], p_cs=p_cs, perm=w["perms"][0],
                                  min_p=True))
    return out


def cohorts_missing(args, ctx, torch, np, datagen, krux):
    M = args.M or datagen.WORKLOADS[5]["M"]
    p_c = 1e-5
    log("generating 8 cohorts, M=%d" % M)
    t0 = time.time()
    cs = datagen.make_cohorts(M=M, T_scale=(args.T / 12500.0) if args.T else 1.0)
    log("generated in %.1fs: K %s, T %s" % (time.time() - t0, [c["K"] for c in cs],
                                            [c["T"] for c in cs]))
    dev = [dict(x=torch.from_numpy(c["expr"]).cuda(), geno=torch.from_numpy(c["geno"]).cuda())
           for c in cs]
    runner = Runner(ctx, torch)
    # launch configuration per sample count, tuned on a slice of the panel
    tuned = []
    t0 = time.time()
    for d, c in zip(dev, cs):
        r, ts, _ = ctx.rank(d["x"])
        ms_t = ctx.autotune(r, ts, d["geno"][: min(M, 50000)], precision="fp16")
        tuned.append(dict(K=c["K"], ms_slice=ms_t, **ctx.tuning_of(c["K"], "fp16")))
    log("autotuned in %.1fs: %s" % (time.time() - t0, tuned))

    def step():
        batch = []
        for d in dev:
            r, ts, _ = ctx.rank(d["x"])
            batch.append(dict(ranks2=r, tiesum=ts, geno=d["geno"]))
        return ctx.test_batched(batch, M, p_c=p_c, precision="fp16", hit_capacity=1 << 16,
                                min_p=False)

    steps = max(1, min(args.steps, 5))
    log("cohorts: 1 warmup + %d timed steps (eager)" % steps)
    ms_eager, res, kms, _ = runner.run(step, steps, 1)
    pairs = float(sum(c["T"] for c in cs)) * M
    flops = float(sum(c["T"] * 4 * c["K"] for c in cs)) * M
    n_hits = [krux.unpack_hits(r)[0] for r in res]
    log("cohorts eager: %.1f ms/step, %.3e pairs/s, hits %s" % (ms_eager, pairs / (ms_eager / 1e3),
                                                              n_hits))
    # the whole step (ranks of every cohort, every cohort's scan) captured
    # once into a HIP graph and replayed as one launch per step
    ranks = [ctx.rank(d["x"]) for d in dev]
    gbufs = ctx.test_batched_buffers([dict(ranks2=r[0]) for r in ranks], hit_capacity=1 << 16)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch = []
        for d, (r, ts, _) in zip(dev, ranks):
            rr, tt, _ = ctx.rank(d["x"], out=(r, ts))
            batch.append(dict(ranks2=rr, tiesum=tt, geno=d["geno"]))
        ctx.test_batched(batch, M, p_c=p_c, precision="fp16", hit_capacity=1 << 16, min_p=False,
                         out=gbufs)
    graph.replay()
    torch.cuda.synchronize()
    same = all(same_hits(krux.unpack_hits(a), krux.unpack_hits(b)) for a, b in zip(gbufs, res))
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    same = same and all(same_hits(krux.unpack_hits(a), krux.unpack_hits(b))
                        for a, b in zip(gbufs, res))
    log("cohorts, one graph launch per step: %.1f ms/step, %.3e pairs/s, hits identical %s"
        % (ms, pairs / (ms / 1e3), same))
    out = base_line(args, "SNP-trait pairs/sec over uneven cohorts", pairs / (ms / 1e3), "pairs/s",
                    ms, "f16", {"workload": "cohorts_missing", "K": [c["K"] for c in cs],
                                "T": [c["T"] for c in cs], "M": M, "p_missing": 0.02, "p_c": p_c,
                                "outputs": "hits per cohort",
                                "timing": "the whole step captured as one HIP graph, replayed"})
    out["steps"] = steps
    out["warmup"] = 1
    out["eager"] = {"ms_per_step": ms_eager, "value": pairs / (ms_eager / 1e3), "unit": "pairs/s"}
    out["graph_identical_hits"] = same
    out["roofline"] = roofline("scan kernels of all cohorts", pairs, flops / pairs, kms,
                               PEAK_FP16_TFLOPS, "TFLOP/s")
    out["n_hits"] = n_hits
    out["autotuned"] = tuned
    if not args.no_cpu:
        import oracle
        c0 = cs[2]          # the K = 102 cohort
        out["cpu_baseline"] = oracle_rate(
            args, c0["T"], M, "cohort K=%d, hits" % c0["K"],
            lambda n: oracle.scan(c0["expr"], c0["geno"][:n], p_cs=(p_c,), hits=True))
    return out


def missing_expression(args, ctx, torch, np, datagen, krux):
    wl = dict(datagen.WORKLOADS[2])
    T = args.T or wl["T"]
    M = args.M or wl["M"]
    K = wl["K"]
    p_c = 1e-5
    log("generating workload K=%d T=%d M=%d with missing expression values" % (K, T, M))
    w = datagen.make_workload(2, T=T, M=M)
    x_nan = datagen.set_nan_expression(datagen.streams(2)["nan"], w["expr"], 0.02, 5)
    n_nan = int(np.isnan(x_nan).any(axis=1).sum())
    log("%d traits with NaN values (%d values)" % (n_nan, int(np.isnan(x_nan).sum())))
    g = torch.from_numpy(w["geno"]).cuda()
    runner = Runner(ctx, torch)
    cap = 1 << 17
    res_ms = {}
    for label, xs in (("complete", w["expr"]), ("nan", x_nan)):
        x = torch.from_numpy(xs).cuda()
        bufs = {}

        def step():
            r, ts, _ = ctx.rank(x)
            res = ctx.test(r, ts, g, p_c=p_c, mode="hits", precision="fp16",
                           hit_capacity=cap, min_p=not args.no_minp, out=bufs.get("o"))
            bufs["o"] = res
            return res

        log("%s: %d warmup + %d timed steps" % (label, args.warmup, args.steps))
        ms, res, kern_ms, _ = runner.run(step, args.steps, args.warmup)
        res_ms[label] = (ms, kern_ms, krux.unpack_hits(res)[0])
        log("%s: %.3f ms/step, main pass %.3f ms, hits %d" % ((label,) + res_ms[label]))
    ms, kern_ms, n_hits = res_ms["nan"]
    pairs = float(T) * float(M)
    out = base_line(args, METRIC, pairs / (ms / 1e3), "pairs/s", ms, "f16", {
        "workload": "missing_expression", "K": K, "T": T, "M": M, "p_c": p_c,
        "nan_traits": n_nan, "nan_recipe": "2% of traits, 1-5 NaN values each",
        "outputs": "sorted hit list (p < 1e-5)" + ("" if args.no_minp else " + per-trait min p")})
    out["roofline"] = roofline("scan_kernel<F16, KS=7, DIAG, SCREEN>", pairs - n_nan * float(M),
                               2 * K * 2, kern_ms, PEAK_FP16_TFLOPS, "TFLOP/s")
    out["n_hits"] = n_hits
    out["complete_expression"] = {"ms_per_step": res_ms["complete"][0],
                                  "kernel_ms": res_ms["complete"][1],
                                  "n_hits": res_ms["complete"][2]}
    if not args.no_cpu:
        import oracle
        rows = np.flatnonzero(np.isnan(x_nan).any(axis=1))
        xs = x_nan[rows]
        out["cpu_baseline"] = oracle_rate(
            args, len(rows), M, "the traits with NaN values, hits at p<1e-5 + per-trait min p",
            lambda n: oracle.scan(xs, w["geno"][:n], p_cs=(p_c,), hits=True, min_p=True))
    return out


def sample_missing(args, ctx, torch, np, datagen, krux):
    wl = dict(datagen.WORKLOADS[2])
    T = args.T or wl["T"]
    M = args.M or wl["M"]
    K = wl["K"]
    p_c = 1e-5
    sets, fracs = [[5, 40], [77]], [0.9, 0.3]
    log("generating workload K=%d T=%d M=%d, failed samples %s at %s" % (K, T, M, sets, fracs))
    w = datagen.make_workload(2, T=T, M=M)
    g_np = datagen.set_missing_samples(datagen.streams(2)["missing"], w["geno"], sets, fracs)
    x = torch.from_numpy(w["expr"]).cuda()
    g = torch.from_numpy(g_np).cuda()
    runner = Runner(ctx, torch)
    cap = 1 << 17
    minp = not args.no_minp
    steps = max(1, min(args.steps, 10))
    warm = max(1, min(args.warmup, 3))

    def per_pair():
        r, ts, _ = ctx.rank(x)
        return ctx.test(r, ts, g, p_c=p_c, mode="hits", precision="fp16", hit_capacity=cap,
                        min_p=minp)

    def grouped():
        r, ts, _ = ctx.rank(x)
        return ctx.test_grouped(r, ts, g, p_c=p_c, precision="fp16", min_group=256,
                                hit_capacity=cap, min_p=minp)

    log("per-pair path: %d warmup + %d timed steps" % (warm, steps))
    ms_pp, res_pp, _, _ = runner.run(per_pair, steps, warm)
    log("grouped path: %d warmup + %d timed steps" % (warm, steps))
    ms_g, res_g, _, _ = runner.run(grouped, steps, warm)
    a, b = krux.unpack_hits(res_pp), krux.unpack_hits(res_g)
    same = same_hits(a, b) and (not minp or bool(torch.equal(res_pp["min_p"], res_g["min_p"])))
    log("per-pair %.2f ms/step, grouped %.2f ms/step, hits %d / %d, identical %s"
        % (ms_pp, ms_g, a[0], b[0], same))
    pairs = float(T) * float(M)
    out = base_line(args, METRIC, pairs / (ms_g / 1e3), "pairs/s", ms_g, "f16", {
        "workload": "sample_missing", "K": K, "T": T, "M": M, "p_c": p_c,
        "failed_samples": sets, "fraction_of_snps": fracs, "min_group": 256,
        "outputs": "sorted hit list (p < 1e-5)" + (" + per-trait min p" if minp else "")})
    out["steps"], out["warmup"] = steps, warm
    out["per_pair_path"] = {"ms_per_step": ms_pp, "value": pairs / (ms_pp / 1e3),
                            "unit": "pairs/s"}
    out["identical_results"] = same
    out["n_hits"] = b[0]
    if not args.no_cpu:
        import oracle
        out["cpu_baseline"] = oracle_rate(
            args, T, M, "hits at p<1e-5" + (" + per-trait min p" if minp else ""),
            lambda n: oracle.scan(w["expr"], g_np[:n], p_cs=(p_c,), hits=True, min_p=minp))
    return out


def multi_allelic(args, ctx, torch, np, datagen, krux):
    K, G = 102, 4
    T = args.T or 20000
    M = args.M or 50000
    p_c = 1e-5
    log("generating workload K=%d T=%d M=%d, %d genotype classes" % (K, T, M, G))
    w = datagen.make_workload(2, T=T, M=1)
    rng = np.random.default_rng(7)
    q = rng.dirichlet(np.ones(G), size=M)
    u = rng.random((M, K))
    g_np = (u[:, :, None] > np.cumsum(q, axis=1)[:, None, :]).sum(axis=2).astype(np.int8)
    x = torch.from_numpy(w["expr"]).cuda()
    g = torch.from_numpy(g_np).cuda()
    runner = Runner(ctx, torch)
    steps = max(1, min(args.steps, 10))

    def step():
        r, ts, _ = ctx.rank(x)
        return ctx.test_multi(r, ts, g, G, p_c=p_c, mode="hits", hit_capacity=1 << 17,
                              min_p=not args.no_minp)

    log("multi-allelic: 3 warmup + %d timed steps" % steps)
    ms, res, kms, kn = runner.run(step, steps, 3)
    n_hits = krux.unpack_hits(res)[0]
    pairs = float(T) * float(M)
    log("multi-allelic: %.2f ms/step, %.3e pairs/s, hits %d, MFMA screen %.3f ms"
        % (ms, pairs / (ms / 1e3), n_hits, kms))
    out = base_line(args, "SNP-trait pairs/sec, multi-allelic markers", pairs / (ms / 1e3),
                    "pairs/s", ms, "f16", {
                        "workload": "multi_allelic", "K": K, "T": T, "M": M, "classes": G,
                        "p_c": p_c, "outputs": "sorted hit list" +
                        ("" if args.no_minp else " + per-trait min p")})
    out["steps"], out["warmup"] = steps, 3
    out["n_hits"] = n_hits
    # G - 1 indicator columns of a K-long contraction per pair
    out["roofline"] = roofline("scan_multi_mfma<KS=7, G=4>", pairs, 2 * K * (G - 1), kms,
                               PEAK_FP16_TFLOPS, "TFLOP/s")
    if not args.no_cpu:
        from oracle import multi
        t0 = time.perf_counter()
        n_snp, Tn = 0, min(T, 20)
        while time.perf_counter() - t0 < args.cpu_seconds and n_snp < M:
            multi.scan(w["expr"][:Tn], g_np[n_snp:n_snp + 5], G, p_c=p_c)
            n_snp += 5
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": Tn * n_snp / dt, "unit": "pairs/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "%d traits x the first %d SNPs (multi-allelic Python "
                                         "oracle, exact rationals), %.1f s" % (Tn, n_snp, dt)}
    return out


# keys of a workload's line that its sub-object in the default line leaves out
SUB_DROP = ("n_gpus", "higher_is_better", "scaling", "vs_baseline", "data")

WORKLOADS = {"paper_scale_hits": paper_scale_hits, "precision_K500": precision_k500,
             "permutations": permutations, "cohorts_missing": cohorts_missing,
             "missing_expression": missing_expression, "sample_missing": sample_missing,
             "multi_allelic": multi_allelic}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="paper_scale_hits")
    ap.add_argument("--T", type=int, default=None, help="override trait count")
    ap.add_argument("--M", type=int, default=None, help="override SNP count")
    ap.add_argument("--P", type=int, default=None, help="override permutation count")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-compare", action="store_true", help="skip the fp64 / int8 paths")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the graph-replay timing of the headline step")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-minp", action="store_true", help="hit list only (no per-trait min p)")
    ap.add_argument("--no-extra", action="store_true",
                    help="paper_scale_hits only: skip the other three configurations "
                         "(precision_K500, permutations, cohorts_missing) that the default "
                         "run adds as sub-objects of the JSON line")
    ap.add_argument("--kernel-digest", action="store_true",
                    help="print the sha256 of the dominant kernel's machine code in the built "
                         "library (recorded with its counter summary) and exit")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one plain 256 MiB device-to-device copy first (reference for "
                         "scaling the HBM byte counters of a profiler run)")
    args = ap.parse_args()

    if args.kernel_digest:
        from paper_1307_3519_amd import krux
        print(DOMINANT_KERNEL, kernel_digest(krux.LIB_PATH, DOMINANT_KERNEL))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the scan shards over SNP slices with no "
              "communication in the compute, and no multi-GPU run is part of this build "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1307_3519_amd import datagen, krux

    ctx = krux.Context(0)
    if args.copy_probe:
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    out = WORKLOADS[args.workload](args, ctx, torch, np, datagen, krux)
    if args.workload == "paper_scale_hits" and not args.no_extra:
        # the other configurations of the method, measured in the same run
        # (fewer steps, no CPU baseline) and reported beside the headline
        import copy
        out["other_configs"] = {}
        for name in ("precision_K500", "permutations", "cohorts_missing"):
            sub = copy.copy(args)
            sub.no_cpu = True
            sub.T = sub.M = sub.P = None
            sub.steps, sub.warmup = min(args.steps, 10), min(args.warmup, 3)
            log("configuration %s" % name)
            r = WORKLOADS[name](sub, ctx, torch, np, datagen, krux)
            out["other_configs"][name] = {k: v for k, v in r.items() if k not in SUB_DROP}
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
