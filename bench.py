"""Throughput of the FAMST hot path on one MI355X.

One step = one full pass of the pipeline over the resident input: kNN graph
(matrix-core screening + float32 re-rank) -> graph, components and
lambda-edges -> refinement rounds -> spanning tree and its weight -> weight
gradient.  The headline value is points/s of the bfloat16-screened path;
the float32-screened path is timed beside it.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1]
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

PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3, "fp8": 5000.0}
HBM_GBS = 8000.0
FP32_VALU_TFLOPS = 157.3   # vector float32, fused multiply-add counted as two flops

# HBM bytes per launch of the dominant kernel, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch) scaled by what the same
# counters read for a plain copy of known size (FETCH x 2.0, WRITE x 1.0).
# Valid only for the kernel sources they were taken on: the sha1 of those
# files is checked at run time and the figure is reported as null after any
# change.  The summaries and commands are in profiles/.
MEASURED_TRAFFIC = {
    ("dist_topk", "gamma-int-1m-d128"): {
        "sources": {"paper_2507_14261_amd/csrc/screen_v2.hpp": "8b27565b9dff0b55176140ed5ecb7a42c316bec8",
                    "paper_2507_14261_amd/csrc/screen_regs.hpp": "f04dfe1780054e95ee03ac2c0b662a6271ae75f2",
                    "paper_2507_14261_amd/csrc/famst_common.hpp": "38cc843bdab55bea9b6987a1878e69497774fc7e"},
        "fetch_GB": 964.664, "write_GB": 0.288,
        "profile": "profiles/dist_topk_gamma-int-1m-d128_bf16_hbm_counters.md"},
    ("rerank", "gamma-int-1m-d128"): {
        "sources": {"paper_2507_14261_amd/csrc/knn.hip": "8938109143edc6833afe2c1ff2ce25193d51c410",
                    "paper_2507_14261_amd/csrc/select.hpp": "a8e57a59a59aa64045df243bd780742f4798e2db",
                    "paper_2507_14261_amd/csrc/famst_common.hpp": "38cc843bdab55bea9b6987a1878e69497774fc7e"},
        "fetch_GB": 5.267, "write_GB": 0.256,
        "profile": "profiles/dist_topk_gamma-int-1m-d128_bf16_hbm_counters.md"},
    ("prep", "gamma-int-1m-d128"): {
        "sources": {"paper_2507_14261_amd/csrc/knn.hip": "8938109143edc6833afe2c1ff2ce25193d51c410",
                    "paper_2507_14261_amd/csrc/famst_common.hpp": "38cc843bdab55bea9b6987a1878e69497774fc7e"},
        "fetch_GB": 0.512, "write_GB": 0.272,
        "profile": "profiles/dist_topk_gamma-int-1m-d128_bf16_hbm_counters.md"},
    ("mst_backward", "gamma-int-1m-d128"): {
        "sources": {"paper_2507_14261_amd/csrc/backward.hip": "068237775349ccb723a3d343f9d1edc4135d1886",
                    "paper_2507_14261_amd/csrc/famst_common.hpp": "38cc843bdab55bea9b6987a1878e69497774fc7e"},
        "fetch_GB": 1.704, "write_GB": 0.512,
        "profile": "profiles/dist_topk_gamma-int-1m-d128_bf16_hbm_counters.md"},
    ("dist_topk", "lowrank-500k-d960"): {
        "sources": {"paper_2507_14261_amd/csrc/screen_hd.hpp": "393e7e925b916357258f66fec6deefacc2f2b964",
                    "paper_2507_14261_amd/csrc/screen_regs.hpp": "f04dfe1780054e95ee03ac2c0b662a6271ae75f2",
                    "paper_2507_14261_amd/csrc/famst_common.hpp": "38cc843bdab55bea9b6987a1878e69497774fc7e"},
        "fetch_GB": 2708.6, "write_GB": 0.130,
        "profile": "profiles/dist_topk_lowrank-500k-d960_kernel_stats_and_hbm.md"},
    ("dist_topk", "vmf-4m-d96"): {
        "sources": {"paper_2507_14261_amd/csrc/screen_v2.hpp": "8b27565b9dff0b55176140ed5ecb7a42c316bec8",
                    "paper_2507_14261_amd/csrc/screen_regs.hpp": "f04dfe1780054e95ee03ac2c0b662a6271ae75f2",
                    "paper_2507_14261_amd/csrc/famst_common.hpp": "38cc843bdab55bea9b6987a1878e69497774fc7e"},
        "fetch_GB": 5764.2, "write_GB": 1.152,
        "profile": "profiles/dist_topk_vmf-4m-d96_bf16_kernel_stats_and_hbm.md"},
    ("exact_tree", "clouds-256-d64"): {
        "sources": {"paper_2507_14261_amd/csrc/mst.hip": "2dde04c5ee757ec24b70d6ac123096784b61d10f",
                    "paper_2507_14261_amd/csrc/famst_common.hpp": "38cc843bdab55bea9b6987a1878e69497774fc7e"},
        "fetch_GB": 40.701, "write_GB": 28.549,
        "profile": "profiles/exact_tree_clouds-256-d64_kernel_stats_and_hbm.md"},
}


GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_weights.json")


def golden(name):
    """The oracle's stored FAMST result for a workload (written by
    tests/golden/make_oracle_weights.py), or None."""
    if not os.path.exists(GOLDEN):
        return None
    with open(GOLDEN) as f:
        return json.load(f).get(name)


def measured_traffic(kernel, workload):
    """HBM GB per launch measured by the counters, or None if the kernel's
    sources changed since (or no measurement exists)."""
    import hashlib
    m = MEASURED_TRAFFIC.get((kernel, workload))
    if m is None:
        return None
    for rel, sha in m["sources"].items():
        with open(os.path.join(ROOT, rel), "rb") as f:
            if hashlib.sha1(f.read()).hexdigest() != sha:
                return None
    return round(m["fetch_GB"] + (m["write_GB"] or 0.0), 3)

# workload name -> (generator kwargs, k, lambda)
WORKLOADS = {
    "gamma-int-1m-d128": ("gamma_int", dict(n=1_000_000, d=128), 20, 10),
    "blobs-10k-d32": ("blobs", dict(n=10_000, d=32), 10, 5),
    # many components (about 1175 at k = 1): 6.9e5 component pairs, 1.7e7 lambda-samples
    "blobs-10k-d32-k1": ("blobs", dict(n=10_000, d=32), 1, 5),
    "vmf-4m-d96": ("vmf", dict(n=4_000_000, d=96), 16, 8),
    "lowrank-500k-d960": ("lowrank", dict(n=500_000, d=960), 20, 10),
}


PHASES = ["prep", "sketch", "pivots", "gather_rows", "dist_topk", "rerank", "exact_row", "sort", "scan",
          "graph_keys", "graph_fill", "uf_hook", "lambda_edges", "refine", "mst_keys", "edge_compact",
          "boruvka_min", "boruvka_hook", "boruvka_block", "tree_weight", "mst_backward", "exact_items", "exact_tree",
          "dense_prim_fused"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_step(F, Xd, k, lam, seed, rounds, precision, exact, e_cap, gW):
    out = F.famst(Xd, k, lam, seed=seed, max_rounds=rounds, precision=precision, exact=exact,
                  e_cap=e_cap)
    grad = F.mst_backward(Xd, out.tu, out.tv, gW)
    return out, grad


def time_path(F, torch, Xd, k, lam, seed, rounds, precision, exact, steps, warmup, profile):
    gW = torch.ones(1, device=Xd.device)
    e_cap = None
    out = None
    for _ in range(warmup):
        out, _ = run_step(F, Xd, k, lam, seed, rounds, precision, exact, e_cap, gW)
        e_cap = max(1, len(out.E))
    torch.cuda.synchronize()
    if profile:
        F.profile_reset()
        F.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        out, grad = run_step(F, Xd, k, lam, seed, rounds, precision, exact, e_cap, gW)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = {}
    if profile:
        F.profile_enable(False)
        for name in PHASES:
            nl, ms = F.profile_read(name)
            if nl:
                phases[name] = {"launches": nl, "total_ms": round(ms, 3)}
    return (t1 - t0) * 1000.0 / steps, out, phases


def bench_clouds(args, F, torch):
    """Batched clouds: the exact tree weight + gradient of every cloud in one
    persistent launch, and the k = 16 FAMST path over the same batch."""
    import datagen
    X, offs = datagen.clouds(n_clouds=256, lo=512, hi=8192, d=64, seed=0)
    n, d = X.shape
    Xd = torch.from_numpy(X).to("cuda:0")
    gW = torch.ones(len(offs) - 1, device=Xd.device)

    def exact_step():
        return F.mst_dense_fused(Xd, offs=offs)

    e_cap = [None]

    def knn_step():
        out = F.famst(Xd, 16, 5, seed=args.seed, max_rounds=args.rounds, precision="bf16", exact=False,
                      offs=offs, e_cap=e_cap[0])
        e_cap[0] = max(1, len(out.E))
        g = F.mst_backward(Xd, out.tu, out.tv, gW, offs=offs)
        return out, g

    res = {}
    last = {}
    for name, fn, kern in [("exact", exact_step, "exact_tree"), ("k16", knn_step, "dist_topk")]:
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        F.profile_reset()
        F.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        F.profile_enable(False)
        last[name] = out
        nl, ms = F.profile_read(kern)
        res[name] = {"ms_per_step": (t1 - t0) * 1e3 / args.steps, "kernel": kern,
                     "kernel_avg_ms": ms / nl if nl else None, "phases": {}}
        for ph in PHASES:
            pl, pms = F.profile_read(ph)
            if pl:
                res[name]["phases"][ph] = round(pms / args.steps, 3)
    # exact path (d <= 64), one launch: the tiles evaluate each unordered pair
    # once (64 differences, 64 fused multiply-adds, 15 additions: 207 flops)
    # and store both orders (sum_i n_i^2 floats); each of the n_i - 1 Prim
    # steps of a cloud reads the n_i - 1 off-root entries of one matrix row
    sizes = np.diff(offs).astype(np.float64)
    pairs = float(np.sum(sizes * (sizes - 1) / 2))
    mat_bytes = float(np.sum(sizes ** 2)) * 4
    prim_bytes = float(np.sum((sizes - 1) ** 2)) * 4
    pair_flops = pairs * 207
    # the largest cloud's Prim steps follow one another: the critical path
    crit_steps = int(sizes.max()) - 1
    # weight error of the k = 16 FAMST trees against the exact trees, per cloud
    W_exact = last["exact"][3].double().cpu().numpy()
    W_k16 = last["k16"][0].W.double().cpu().numpy()
    rel = (W_k16 - W_exact) / W_exact
    weight = None
    g = golden("clouds-256-d64")
    if g is not None and g["n"] == n:
        # against the oracle: its float64 Prim per cloud (exact mode) and its
        # FAMST per cloud (k = 16 mode, bf16 screening here)
        ge, gf = np.array(g["W_exact"]), np.array(g["W"])
        weight = {"exact_rel_err_vs_oracle_prim_max": float(np.max(np.abs(W_exact - ge) / ge)),
                  "k16_bf16_rel_err_vs_oracle_famst_max": float(np.max(np.abs(W_k16 - gf) / gf)),
                  "oracle_famst_rel_err_vs_exact_mean": float(np.mean((gf - ge) / ge))}
    ex = res["exact"]
    val = n / (ex["ms_per_step"] * 1e-3)
    kms = ex["kernel_avg_ms"]
    byts = mat_bytes + prim_bytes
    gbs = byts / (kms * 1e-3) / 1e9 if kms else None
    return {
        "metric": "points/s to approx MST at stated weight error, BF16/FP8+rerank vs FP32",
        "value": round(val, 1), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ex["ms_per_step"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": "clouds-256-d64", "clouds": len(sizes), "n_total": int(n), "d": d,
                   "mode": "exact tree (k = n_i - 1) + gradient: pair matrices and Prim in one persistent launch"},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1) if gbs else None, "peak": HBM_GBS,
                     "unit": "GB/s", "frac": round(gbs / HBM_GBS, 4) if gbs else None,
                     "traffic": measured_traffic("exact_tree", "clouds-256-d64"),
                     "traffic_unit": "GB per launch", "kernel": "exact_tree",
                     "avg_ms": round(kms, 3) if kms else None,
                     "algorithmic_GB": round(byts / 1e9, 3),
                     "note": "matrix stores plus Prim row reads; the launch ends with the largest cloud's "
                             "sequential Prim steps (latency), not at the HBM rate"},
        "exact_tree_alu": {"bound": "alu", "achieved": round(pair_flops / (kms * 1e-3) / 1e12, 2) if kms else None,
                           "peak": FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                           "frac": round(pair_flops / (kms * 1e-3) / 1e12 / FP32_VALU_TFLOPS, 4) if kms else None,
                           "algorithmic_TFLOP": round(pair_flops / 1e12, 4)},
        "critical_path": {"prim_steps": crit_steps,
                          "us_per_step_if_all": round(kms * 1e3 / crit_steps, 3) if kms else None},
        "k16_path": {"ms_per_step": round(res["k16"]["ms_per_step"], 3),
                     "weight_rel_err_vs_exact_mst": {"max": float(rel.max()), "mean": float(rel.mean()),
                                                     "min": float(rel.min()), "clouds": int(len(rel))},
                     "points_per_s": round(n / (res["k16"]["ms_per_step"] * 1e-3), 1),
                     "phases_ms_per_step": res["k16"]["phases"]},
        "weight": weight,
        "cpu_baseline": None,
    }


def _subsample(name):
    import datagen
    if name == "vmf-4m-d96":
        return "vmf-4m-d96-sub100k", datagen.subsample(4_000_000, 100_000, seed=1)
    if name == "lowrank-500k-d960":
        return "lowrank-500k-d960-sub50k", datagen.subsample(500_000, 50_000, seed=1)
    return None, None


def bench_workload(args, F, torch, name, precs, pk):
    """One single-cloud workload at full size: time per step, points/s and the
    distance kernel's roofline per precision; the weight error of each
    precision against the oracle's FAMST on the stored subsample."""
    import datagen
    gen_name, kw, k, lam = WORKLOADS[name]
    t0 = time.perf_counter()
    X = getattr(datagen, gen_name)(seed=0, **kw)
    n, d = X.shape
    log(f"generated {name}: n={n} d={d} in {time.perf_counter() - t0:.1f}s")
    Xd = torch.from_numpy(X).to("cuda:0")
    flops = 2.0 * n * n * d
    block = {"n": n, "d": d, "k": k, "lambda": lam}
    for prec, steps, warmup in precs:
        exact = prec == "fp32"
        ms, out, ph = time_path(F, torch, Xd, k, lam, args.seed, args.rounds, prec, exact, steps, warmup, True)
        dt = ph.get("dist_topk", {})
        avg = dt["total_ms"] / dt["launches"] if dt.get("launches") else None
        tf = flops / (avg * 1e-3) / 1e12 if avg else None
        block[prec] = {"mode": "exact" if exact else "screening + fp32 re-rank", "steps": steps,
                       "ms_per_step": round(ms, 3), "points_per_s": round(n / (ms * 1e-3), 1),
                       "W": float(out.W[0].item()), "components": out.graph.n_comp[0],
                       "dist_topk_avg_ms": round(avg, 3) if avg else None,
                       "dist_topk_tflops": round(tf, 2) if tf else None,
                       "frac_of_peak": round(tf / PEAK_TFLOPS[prec], 4) if tf else None,
                       "frac_of_measured": round(tf / pk[f"mfma_{prec}_tflops"], 4) if tf and pk else None,
                       "traffic_GB_per_launch": measured_traffic("dist_topk", name) if prec == "bf16" else None}
        log(f"{name} {prec}: {ms:.1f} ms/step")
    del Xd
    sub, idx = _subsample(name)
    g = golden(sub) if sub else None
    if g is not None:
        Xs = torch.from_numpy(np.ascontiguousarray(X[idx])).to("cuda:0")
        err = {}
        for prec, _, _ in precs:
            out = F.famst(Xs, k, lam, seed=g["seed"], max_rounds=g["max_rounds"], precision=prec,
                          exact=prec == "fp32")
            err[f"rel_err_{prec}_vs_oracle"] = (float(out.W[0].item()) - g["W"]) / g["W"]
        block["weight_on_subsample"] = dict(subsample=sub, n=g["n"], W_oracle_famst=g["W"], **err)
        del Xs
    torch.cuda.empty_cache()
    return block


def bench_more_workloads(args, F, torch, pk):
    """The other measured workloads, timed with fewer steps (one JSON line
    holds them all): 500K x 960 in bf16, fp8 and fp32; 4M x 96 in bf16 and
    fp8 (the fp32 path takes about 24 s per step there and is left out);
    the 256 clouds in their exact and k = 16 modes."""
    out = {}
    out["lowrank-500k-d960"] = bench_workload(args, F, torch, "lowrank-500k-d960",
                                              [("bf16", 2, 1), ("fp8", 2, 1), ("fp32", 1, 0)], pk)
    out["vmf-4m-d96"] = bench_workload(args, F, torch, "vmf-4m-d96", [("bf16", 2, 1), ("fp8", 1, 1)], pk)
    c = bench_clouds(args, F, torch)
    out["clouds-256-d64"] = {k2: c[k2] for k2 in ("value", "unit", "ms_per_step", "config", "roofline",
                                                  "exact_tree_alu", "critical_path", "k16_path", "weight")}
    return out


def calib_copy(torch):
    """A plain device copy of 512,000,000 bytes (read and written once), the
    reference against which the HBM counters are scaled."""
    Y = torch.ones(128_000_000, dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    Z = Y.clone()
    torch.cuda.synchronize()
    log(f"calibration copy: {Z.numel() * 4} bytes read and written")


def cpu_baseline(X, k, rows):
    import oracle
    t0 = time.perf_counter()
    nbr, sq = oracle.knn_exact(X, k, rows=rows, block=64)
    t1 = time.perf_counter()
    return nbr, t1 - t0


def sweep_precision(d):
    """Screening precision of the n x d sweep: float32 up to 16 dimensions
    (bf16's 8-bit mantissa cannot separate neighbours of dense low-dimensional
    clouds), bf16 above; candidates re-ranked in float32 (approximate mode:
    in two dimensions the expansion's rounding exceeds the nearest-neighbour
    distances of a million points, so exact mode would recompute every row)."""
    return "fp32" if d <= 16 else "bf16"


def bench_sweep(args, F, torch):
    """Parameter sweeps on synthetic blobs (10 isotropic Gaussian clusters,
    sigma 1, centres in [-10, 10]^d), one JSON line.
    kl: k in {5, 10, 15, 20} x lambda in {1, 2, 3, 4, 5, 10} on 10,000 x 32
        points, data seeds 0, 1, 2: relative weight error against the exact
        tree (dense Prim on the complete graph), components t (mean t-bar),
        refinement rounds, time per step; the paper's error and time trends
        against k and lambda.
    nd: n in {32k, 64k, 128k, 256k, 512k, 1024k} x d in {2, 16, 32, 128,
        544, 784} at k = 10, lambda = 5 (float32 screening up to 16
        dimensions, bf16 above, float32 re-rank): time per step and per
        phase, points/s, components; the paper's runtime against n and d.
        Pairs whose screening exceeds --sweep-max-flops are skipped."""
    import datagen
    rows = []
    if args.sweep == "kl":
        for k in (5, 10, 15, 20):
            for lam in (1, 2, 3, 4, 5, 10):
                per = []
                for seed in (0, 1, 2):
                    X = torch.from_numpy(datagen.blobs(n=10_000, d=32, seed=seed)).to("cuda:0")
                    W_exact = float(F.mst(X, algo="prim")[3][0].item())
                    ms, out, _ = time_path(F, torch, X, k, lam, args.seed, args.rounds, "fp32", True, 3, 1, False)
                    W = float(out.W[0].item())
                    per.append((ms, (W - W_exact) / W_exact, out.graph.n_comp[0], out.rounds))
                rows.append({"k": k, "lambda": lam, "seeds": 3,
                             "rel_err_vs_exact_mean": float(np.mean([p[1] for p in per])),
                             "rel_err_vs_exact_max": float(np.max([p[1] for p in per])),
                             "t_bar": float(np.mean([p[2] for p in per])),
                             "rounds_mean": float(np.mean([p[3] for p in per])),
                             "ms_per_step": round(float(np.mean([p[0] for p in per])), 3)})
                log(f"k={k} lambda={lam}: {rows[-1]}")
        config = {"workload": "blobs-10k-d32 (data seeds 0-2)", "precision": "fp32 screening, exact"}
    else:
        for d in (2, 16, 32, 128, 544, 784):
            for n in (32_768, 65_536, 131_072, 262_144, 524_288, 1_048_576):
                if 2.0 * n * n * d > args.sweep_max_flops:
                    rows.append({"n": n, "d": d, "skipped": "screening above --sweep-max-flops"})
                    continue
                X = torch.from_numpy(datagen.blobs(n=n, d=d, seed=0)).to("cuda:0")
                prec = sweep_precision(d)
                ms, out, ph = time_path(F, torch, X, 10, 5, args.seed, args.rounds, prec, False, 2, 1, True)
                rows.append({"n": n, "d": d, "precision": prec, "ms_per_step": round(ms, 3),
                             "points_per_s": round(n / (ms * 1e-3), 1), "t": out.graph.n_comp[0],
                             "rounds": out.rounds,
                             "phases_ms_per_step": {kk: round(v["total_ms"] / 2, 3) for kk, v in ph.items()}})
                log(f"n={n} d={d} {prec}: {rows[-1]['ms_per_step']} ms")
                del X
                torch.cuda.empty_cache()
        config = {"workload": "blobs", "k": 10, "lambda": 5, "precision": "fp32 screening for d <= 16, bf16 above, "
                  "fp32 re-rank"}
    return {"metric": f"parameter sweep ({args.sweep})", "unit": "see rows", "n_gpus": 1,
            "data": "synthetic", "config": config, "rows": rows}


def measure_peaks():
    """Measured ceilings of this device (outside every timed region): dense
    MFMA throughput of the three forms the screening issues (every wave of a
    full-chip grid issuing independent MFMAs on register operands) and HBM
    copy / read bandwidth over 1 GiB."""
    from paper_2507_14261_amd import peaks as P
    out = {"mfma_fp32_tflops": round(P.mfma_tflops("fp32", 200000), 1),
           "mfma_bf16_tflops": round(P.mfma_tflops("bf16", 400000), 1),
           "mfma_fp8_tflops": round(P.mfma_tflops("fp8", 200000), 1)}
    c, r = P.hbm_gbps(1 << 30, 5)
    out["hbm_copy_GBps"] = round(c, 1)
    out["hbm_read_GBps"] = round(r, 1)
    log(f"measured peaks: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gamma-int-1m-d128", choices=sorted(WORKLOADS) + ["clouds-256-d64"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--rounds", type=int, default=10)
    ap.add_argument("--fp32-steps", type=int, default=1)
    ap.add_argument("--cpu-rows", type=int, default=3072)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-fp32", action="store_true", help="do not time the float32-screened path")
    ap.add_argument("--skip-fp8", action="store_true", help="do not time the float8-screened path")
    ap.add_argument("--no-peaks", action="store_true", help="skip the measured MFMA / HBM ceilings")
    ap.add_argument("--sweep", choices=["kl", "nd"], default=None,
                    help="parameter sweep on blobs instead of the timed workload (one JSON line)")
    ap.add_argument("--sweep-max-flops", type=float, default=2.0e15,
                    help="n x d sweep: skip pairs whose screening (2 n^2 d flops) exceeds this")
    ap.add_argument("--only-headline", action="store_true",
                    help="time only the default workload (not 500K x 960, 4M x 96 and the clouds)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="finish with a plain device copy of X (known bytes) for counter calibration")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is described in the design notes, not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    import datagen
    import paper_2507_14261_amd as F

    F.load()
    if args.sweep:
        print(json.dumps(bench_sweep(args, F, torch)), flush=True)
        return
    if args.workload == "clouds-256-d64":
        res = bench_clouds(args, F, torch)
        pk = None if args.no_peaks else measure_peaks()
        res["measured_peaks"] = pk
        rf = res["roofline"]
        if pk and rf.get("achieved"):
            rf["measured_peak"] = pk["hbm_read_GBps"]
            rf["frac_of_measured"] = round(rf["achieved"] / pk["hbm_read_GBps"], 4)
        if args.calib_copy:
            calib_copy(torch)
        print(json.dumps(res), flush=True)
        return
    gen_name, kw, k, lam = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    X = getattr(datagen, gen_name)(seed=0, **kw)
    n, d = X.shape
    log(f"generated {args.workload}: n={n} d={d} in {time.perf_counter() - t0:.1f}s")
    Xd = torch.from_numpy(X).to("cuda:0")
    torch.cuda.synchronize()
    # host -> device upload of X, outside every timed region (the library
    # takes device pointers; value is the rate on resident input): the best
    # of three uploads from pinned host memory
    Xh = torch.from_numpy(X).pin_memory()
    h2d = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Xd.copy_(Xh, non_blocking=True)
        torch.cuda.synchronize()
        h2d.append(time.perf_counter() - t0)
    h2d_s = min(h2d)
    del Xh

    ms_bf16, out_b, phases_b = time_path(F, torch, Xd, k, lam, args.seed, args.rounds, "bf16", False,
                                         args.steps, args.warmup, True)
    log(f"bf16 path: {ms_bf16:.1f} ms/step")
    if args.skip_fp32:
        ms_fp32, out_f, phases_f = float("nan"), out_b, {}
    else:
        ms_fp32, out_f, phases_f = time_path(F, torch, Xd, k, lam, args.seed, args.rounds, "fp32", True,
                                             args.fp32_steps, 1, True)
        log(f"fp32 path: {ms_fp32:.1f} ms/step")
    if args.skip_fp8:
        ms_fp8, out_8, phases_8 = float("nan"), None, {}
    else:
        ms_fp8, out_8, phases_8 = time_path(F, torch, Xd, k, lam, args.seed, args.rounds, "fp8", False,
                                            args.fp32_steps, 1, True)
        log(f"fp8 path: {ms_fp8:.1f} ms/step")
    pk = None if args.no_peaks else measure_peaks()
    Wb = float(out_b.W[0].item())
    Wf = float(out_f.W[0].item())
    W8 = float(out_8.W[0].item()) if out_8 is not None else float("nan")

    # roofline of the dominant kernel (distance tiles): 2 n^2 d flops per launch
    flops = 2.0 * n * n * d
    nl, tot = phases_b.get("dist_topk", {}).get("launches", 0), phases_b.get("dist_topk", {}).get("total_ms", 0.0)
    avg_ms = tot / nl if nl else float("nan")
    achieved = flops / (avg_ms * 1e-3) / 1e12 if nl else None
    nlf, totf = phases_f.get("dist_topk", {}).get("launches", 0), phases_f.get("dist_topk", {}).get("total_ms", 0.0)
    avg_f = totf / nlf if nlf else float("nan")
    nl8, tot8 = phases_8.get("dist_topk", {}).get("launches", 0), phases_8.get("dist_topk", {}).get("total_ms", 0.0)
    avg_8 = tot8 / nl8 if nl8 else float("nan")

    # achieved bandwidth of the gather / streaming kernels (algorithmic bytes)
    KC = 32 if k <= 24 else 64
    ncol = int(out_b.graph.col.numel())
    mdeg = ncol / n
    nE = len(out_b.E)
    gbytes = {
        "prep": n * d * 4 + n * d * 2 + 8 * n,
        "rerank": n * (KC + 1) * d * 4 + n * k * 8,
        "refine": out_b.rounds * nE * (2 * mdeg + 2) * d * 4,
        "mst_backward": (n + 2 * (n - 1)) * d * 4 + n * d * 4,
    }
    bw = {}
    for name, b in gbytes.items():
        ph = phases_b.get(name)
        if ph and ph["total_ms"] > 0:
            per_launch_ms = ph["total_ms"] / ph["launches"]
            gbs = b / (per_launch_ms * 1e-3) / 1e9
            # HBM figures only from counter bytes: gathered rows that hit in L2
            # are in the algorithmic bytes but never reach HBM
            hbm = measured_traffic(name, args.workload)
            bw[name] = {"algorithmic_GB": round(b / 1e9, 3), "ms_per_launch": round(per_launch_ms, 3),
                        "algorithmic_GB_per_s": round(gbs, 1),
                        "hbm_GB": hbm,
                        "hbm_GB_per_s": round(hbm / (per_launch_ms * 1e-3), 1) if hbm else None,
                        "frac_of_hbm": round(hbm / (per_launch_ms * 1e-3) / HBM_GBS, 4) if hbm else None}

    # sampled exact-kNN parity at full size + the CPU oracle baseline
    rng = np.random.default_rng(1)
    rows = np.sort(rng.choice(n, size=args.cpu_rows, replace=False))
    cpu = None
    parity = None
    oracle_w = None
    if not args.no_cpu_baseline:
        ref_nbr, t_cpu = cpu_baseline(X, k, rows)
        # the same oracle on one thread (BLAS limited to one), on the first
        # twelfth of the sampled rows
        from threadpoolctl import threadpool_limits
        rows1 = rows[:max(64, len(rows) // 12)]
        with threadpool_limits(limits=1):
            _, t_cpu1 = cpu_baseline(X, k, rows1)
        nb_b = out_b.nbr[torch.from_numpy(rows).to(Xd.device)].cpu().numpy()
        nb_f = out_f.nbr[torch.from_numpy(rows).to(Xd.device)].cpu().numpy()
        rec_b = float(np.mean([len(set(a) & set(b)) / k for a, b in zip(nb_b, ref_nbr)]))
        rec_f = float(np.mean([len(set(a) & set(b)) / k for a, b in zip(nb_f, ref_nbr)]))
        parity = {"sample_rows": int(len(rows)), "recall_bf16": rec_b, "recall_fp32": rec_f}
        if out_8 is not None:
            nb_8 = out_8.nbr[torch.from_numpy(rows).to(Xd.device)].cpu().numpy()
            parity["recall_fp8"] = float(np.mean([len(set(a) & set(b)) / k for a, b in zip(nb_8, ref_nbr)]))
        if args.workload == "blobs-10k-d32":
            # weight error against the oracle's FAMST and against the exact MST
            # (float64 Prim on the complete graph): seconds on the host here
            import oracle
            t0 = time.perf_counter()
            ref = oracle.famst(X, k, lam, seed=args.seed, max_rounds=args.rounds)
            exact_w = oracle.prim_exact(X)[3]
            log(f"oracle FAMST and exact MST: {time.perf_counter() - t0:.1f} s")
            oracle_w = {"W_oracle_famst": ref.W, "W_exact_mst": exact_w,
                        "rel_err_bf16_vs_oracle": abs(Wb - ref.W) / ref.W,
                        "rel_err_fp32_vs_oracle": abs(Wf - ref.W) / ref.W,
                        "famst_rel_err_vs_exact_mst": (Wf - exact_w) / exact_w}
            if out_8 is not None:
                oracle_w["rel_err_fp8_vs_oracle"] = abs(W8 - ref.W) / ref.W
        cores = len(os.sched_getaffinity(0))
        cpu = {"value": round(len(rows) / t_cpu, 3), "unit": "points/s", "cores": cores, "kind": "oracle",
               "sample": (f"exact float64 kNN (the oracle's Phase 1, the dominant phase) of {len(rows)} "
                          f"query rows against all {n} points; {t_cpu:.1f} s"),
               "single_thread": {"value": round(len(rows1) / t_cpu1, 3), "cores": 1,
                                 "sample": f"the first {len(rows1)} of those rows; {t_cpu1:.1f} s"}}

    g = golden(args.workload)
    if g is not None and (g["n"], g["d"], g["k"], g["lam"]) == (n, d, k, lam) and args.seed == g["seed"]:
        # Eq. (1)'s relative error against the oracle's FAMST on the same input
        oracle_w = dict(oracle_w or {}, W_oracle_famst=g["W"],
                        rel_err_bf16_vs_oracle=(Wb - g["W"]) / g["W"],
                        rel_err_fp32_vs_oracle=(Wf - g["W"]) / g["W"] if not args.skip_fp32 else None,
                        rel_err_fp8_vs_oracle=(W8 - g["W"]) / g["W"] if out_8 is not None else None,
                        oracle_t=g["t"], oracle_refine_deltas=g["deltas"])
    extra = None if args.only_headline else bench_more_workloads(args, F, torch, pk)
    res = {
        "metric": "points/s to approx MST at stated weight error, BF16/FP8+rerank vs FP32",
        "value": round(n / (ms_bf16 * 1e-3), 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_bf16, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "d": d, "k": k, "lambda": lam,
                   "max_rounds": args.rounds, "seed": args.seed,
                   "precision": "bf16 screening + fp32 re-rank", "components": out_b.graph.n_comp[0],
                   "inter_component_edges": len(out_b.E), "refine_rounds": out_b.rounds},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2) if achieved else None,
                     "peak": PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_TFLOPS["bf16"], 4) if achieved else None,
                     "traffic": measured_traffic("dist_topk", args.workload), "traffic_unit": "GB per launch",
                     "kernel": "dist_topk", "avg_ms": round(avg_ms, 3),
                     "algorithmic_flops": flops,
                     "measured_peak": pk["mfma_bf16_tflops"] if pk else None,
                     "frac_of_measured": round(achieved / pk["mfma_bf16_tflops"], 4) if pk and achieved else None},
        "measured_peaks": pk,
        "cpu_baseline": cpu,
        "h2d": {"bytes": int(X.nbytes), "ms": round(h2d_s * 1e3, 3), "GB_per_s": round(X.nbytes / h2d_s / 1e9, 1),
                "points_per_s_with_upload": round(n / (ms_bf16 * 1e-3 + h2d_s), 1)},
        "weight": {"W_bf16": Wb, "W_fp32": Wf, "gpu_rel_diff_bf16_vs_fp32": abs(Wb - Wf) / Wf,
                   "W_fp8": W8, "gpu_rel_diff_fp8_vs_fp32": abs(W8 - Wf) / Wf if out_8 is not None else None,
                   **(oracle_w or {})},
        "fp32_path": None if args.skip_fp32 else {
                      "ms_per_step": round(ms_fp32, 3), "points_per_s": round(n / (ms_fp32 * 1e-3), 1),
                      "dist_topk_avg_ms": round(avg_f, 3),
                      "dist_topk_tflops": round(flops / (avg_f * 1e-3) / 1e12, 2) if nlf else None,
                      "frac_of_fp32_peak": round(flops / (avg_f * 1e-3) / 1e12 / PEAK_TFLOPS["fp32"], 4) if nlf else None,
                      "frac_of_measured_fp32": round(flops / (avg_f * 1e-3) / 1e12 / pk["mfma_fp32_tflops"], 4)
                      if nlf and pk else None},
        "bandwidth_bf16_path": bw,
        "phases_ms_bf16": phases_b,
        "phases_ms_fp32": phases_f,
        "fp8_path": None if out_8 is None else {
                     "precision": "fp8 e4m3 screening (per-row scales) + fp32 re-rank, approximate mode",
                     "ms_per_step": round(ms_fp8, 3), "points_per_s": round(n / (ms_fp8 * 1e-3), 1),
                     "dist_topk_avg_ms": round(avg_8, 3),
                     "dist_topk_tflops": round(flops / (avg_8 * 1e-3) / 1e12, 2) if nl8 else None,
                     "frac_of_fp8_peak": round(flops / (avg_8 * 1e-3) / 1e12 / PEAK_TFLOPS["fp8"], 4) if nl8 else None,
                     "frac_of_measured_fp8": round(flops / (avg_8 * 1e-3) / 1e12 / pk["mfma_fp8_tflops"], 4)
                     if nl8 and pk else None},
        "parity": parity,
        "workloads": extra,
    }
    if args.calib_copy:
        calib_copy(torch)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
