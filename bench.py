#!/usr/bin/env python3
"""Benchmark of the approximate-product hot path on one MI355X.

Headline workload (one "step"): the 3D decay matrix n = 32768 (4096 atoms
on a 16^3 lattice, jitter 0.1, x 8 basis functions), a_ij = (2u - 1)
exp(-dist), leaf 64, tau = 1e-6, A = B.  A step builds the quadtree from the
dense FP64 matrix already in HBM (leaf norms, null map, pyramid, leaf
copies), then runs the combined scheme (Hybrid: leaf-level truncation of
both operands, pruning, the persistent leaf-GEMM launch, C's pyramid and the
FP64 accounting) with FP64 leaf products, the paper's arithmetic.  The
headline value is kept-leaf GFLOP/s (2 * 64^3 per formed leaf product, the
flop count of Sec. 5.3) over whole steps.

Beside it: the same step in FP32, BF16 and split BF16 (leaf-GEMM rate and
error against the FP64 product), multiplies/s at a fixed error
||A A - C||_F <= 1e-5 ||A||_F ||B||_F per precision (Sec. 5.3's
target-accuracy comparison), the 1D batch of 18 multiplies (n = 16384),
the purification chain, the served stream and the oracle timed on the host.

Prints one JSON line (see the repository's measurement notes for fields).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "kept-leaf GFLOP/s + multiplies/sec at fixed ‖E‖_F; p50/p99 latency, FP32 vs FP64"
N, LEAF = 16384, 64
ALPHAS = (0.2, 0.5)
TAUS = (1e-4, 1e-6, 1e-8)
MODE_NAMES = ("truncmul", "spamm", "hybrid")
SEED = 1
FP32_MFMA_PEAK_TFLOPS = 157.3
FP64_MFMA_PEAK_TFLOPS = 78.6
BF16_MFMA_PEAK_TFLOPS = 2500.0
# 3D decay workload: 4096 atoms (16^3 lattice, jitter 0.1) x 8 functions
N3D, LEAF3D, ALPHA3D, TAU3D = 32768, 64, 1.0, 1e-6
SIGMA_REL = 1e-5  # fixed error: ||A A - C||_F <= SIGMA_REL ||A||_F ||B||_F
TAU_GRID = tuple(10.0 ** -k for k in range(0, 9))  # 1 ... 1e-8, decades
GEMM_SOURCE = os.path.join(ROOT, "paper_1906_08148_amd", "csrc", "k_gemm.hip")
TRAFFIC_GLOB = os.path.join(ROOT, "profiles", "*_decay3d_n32768_hybrid_traffic.json")
PREC_NAMES = {0: "f64", 1: "f32", 2: "bf16", 3: "bf16x3"}
PEAKS = {0: FP64_MFMA_PEAK_TFLOPS, 1: FP32_MFMA_PEAK_TFLOPS, 2: BF16_MFMA_PEAK_TFLOPS, 3: BF16_MFMA_PEAK_TFLOPS}


CTX_OPTIONS = {}  # options every context of the run is given (--gemm-tile, --gemm-quad)


def new_context(arena_bytes):
    from paper_1906_08148_amd import spamm
    ctx = spamm.Context(arena_bytes=arena_bytes)
    for k, v in CTX_OPTIONS.items():
        ctx.set_option(k, v)
    return ctx


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_inputs():
    import numpy as np
    import synth
    out = {}
    for a in ALPHAS:
        coords, data = synth.DecaySpec("1d", N, a, seed=SEED).leaf_blocks(LEAF)
        out[a] = (coords.astype(np.int32), data)
    return out


def gpu_inputs(host):
    import torch
    return {a: (torch.from_numpy(c).cuda(), torch.from_numpy(d).cuda()) for a, (c, d) in host.items()}


def requests(mats, prec):
    from paper_1906_08148_amd import spamm
    reqs = []
    for a in ALPHAS:
        for t in TAUS:
            for mi, _ in enumerate(MODE_NAMES):
                reqs.append(dict(A=mats[a], B=mats[a], tau=t, mode=mi, prec=prec))
    return reqs


def run_step(ctx, dev, prec, keep=False):
    """One pass of the whole path; returns (stats list, products or None)."""
    from paper_1906_08148_amd import spamm
    store = spamm.STORE_F64 if prec == spamm.F64 else spamm.STORE_F32
    built = ctx.build_blocks_batch([(N, LEAF, c, d) for c, d in dev.values()], stores=store)
    mats = dict(zip(dev.keys(), built))
    prods = ctx.multiply_batch(requests(mats, prec), stats=True)
    stats = [p.stats for p in prods]
    if keep:
        return stats, prods, mats
    for p in prods:
        p.C.release()
    for m in mats.values():
        m.release()
    return stats, None, None


def timed_steps(ctx, dev, prec, steps, warmup):
    """Throughput and latency over `steps` steps with the library's event
    timing off, then the same number of steps with it on for the per-phase
    and per-launch kernel times (events add a little host work)."""
    import torch
    for _ in range(warmup):
        run_step(ctx, dev, prec)
    torch.cuda.synchronize()
    lat = []
    flops = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        stats, _, _ = run_step(ctx, dev, prec)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s0)
        flops += sum(s["flops"] for s in stats)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ctx.timing(enable=True, reset=True)
    for _ in range(steps):
        run_step(ctx, dev, prec)
    torch.cuda.synchronize()
    tm = ctx.timing(enable=False, reset=True)
    return total, lat, flops, tm, stats


def multiply_only(ctx, dev, prec, steps, warmup):
    """The same 18 multiplies with both matrices built once beforehand: the
    norms are precomputed, the paper's timing convention (Sec. 5)."""
    import torch
    from paper_1906_08148_amd import spamm
    store = spamm.STORE_F64 if prec == spamm.F64 else spamm.STORE_F32
    built = ctx.build_blocks_batch([(N, LEAF, c, d) for c, d in dev.values()], stores=store)
    mats = dict(zip(dev.keys(), built))
    reqs = requests(mats, prec)
    for _ in range(warmup):
        for p in ctx.multiply_batch(reqs):
            p.C.release()
    torch.cuda.synchronize()
    flops = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        prods = ctx.multiply_batch(reqs)
        flops += sum(p.stats["flops"] for p in prods)
        for p in prods:
            p.C.release()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    for m in mats.values():
        m.release()
    return {"ms_per_step": round(total / steps * 1e3, 4), "gflops": round(flops / total / 1e9, 3)}


def store_for(prec):
    from paper_1906_08148_amd import spamm
    return {spamm.F64: spamm.STORE_F64, spamm.F32: spamm.STORE_F32}.get(prec, spamm.STORE_BF16)


def config3_steps(ctx, dA, prec, steps, warmup, mode=None, keep_last=False):
    """`steps` whole steps of the 3D workload in precision `prec`: build from
    the dense matrix in HBM, then one multiply (Hybrid by default) with its
    statistics.  The library's HIP events (recorded on the stream the
    kernels run on) are on during the timed steps, so the per-kernel-class
    times come from the timed region itself."""
    import torch
    from paper_1906_08148_amd import spamm
    mode = spamm.HYBRID if mode is None else mode

    def one():
        M = ctx.build(dA, LEAF3D, stores=store_for(prec))
        p = ctx.multiply(M, M, TAU3D, mode=mode, prec=prec)
        return M, p

    for _ in range(warmup):
        M, p = one()
        p.C.release()
        M.release()
    torch.cuda.synchronize()
    ctx.timing(enable=True, reset=True)
    lat, flops, last = [], 0.0, None
    t0 = time.perf_counter()
    for k in range(steps):
        s0 = time.perf_counter()
        M, p = one()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s0)
        flops += p.stats["flops"]
        M.release()
        if keep_last and k + 1 == steps:
            last = p
        else:
            p.C.release()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    tm = ctx.timing(enable=False, reset=True)
    g_ms = tm["gemm_ms"] / max(tm["gemm_launches"], 1)
    g_fl = tm["gemm_flops"] / max(tm["gemm_launches"], 1)
    return dict(total=total, lat=lat, flops=flops, tm=tm, stats=p.stats, gemm_ms=g_ms, gemm_flops=g_fl,
                gemm_tflops=g_fl / (g_ms * 1e-3) / 1e12, last=last)


def multiply_only_3d(ctx, dA, prec, steps, mode=None):
    """The same multiply with the quadtree built once beforehand: norms
    precomputed, the paper's timing convention (Sec. 5.3)."""
    import torch
    from paper_1906_08148_amd import spamm
    mode = spamm.HYBRID if mode is None else mode
    M = ctx.build(dA, LEAF3D, stores=store_for(prec))
    ctx.multiply(M, M, TAU3D, mode=mode, prec=prec).C.release()
    torch.cuda.synchronize()
    flops = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        p = ctx.multiply(M, M, TAU3D, mode=mode, prec=prec, stats=False)
        p.C.release()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    p = ctx.multiply(M, M, TAU3D, mode=mode, prec=prec)
    flops = p.stats["flops"] * steps
    p.C.release()
    M.release()
    return {"ms_per_multiply": round(total / steps * 1e3, 3), "gflops": round(flops / total / 1e9, 1),
            "multiplies_per_s": round(steps / total, 3)}


def config3_precisions(ctx, dA, steps, C64):
    """FP32, BF16 and split BF16 on the same step: whole-step and leaf-GEMM
    rates, the GEMM's fraction of its precision's MFMA peak, and
    ||C - C_FP64||_F / ||C_FP64||_F against the FP64 product."""
    import torch
    from paper_1906_08148_amd import spamm
    out = {}
    nref = float(torch.linalg.norm(C64))
    for prec in (spamm.F32, spamm.BF16X3, spamm.BF16):
        log(f"bench: 3D hybrid {PREC_NAMES[prec]}")
        r = config3_steps(ctx, dA, prec, steps, 1, keep_last=True)
        C = ctx.to_dense(r["last"].C)
        rel = float(torch.linalg.norm(C - C64)) / nref
        del C
        r["last"].C.release()
        out[PREC_NAMES[prec]] = {
            "ms_per_step": round(r["total"] / steps * 1e3, 2),
            "gflops": round(r["flops"] / r["total"] / 1e9, 1),
            "gemm_ms": round(r["gemm_ms"], 3), "gemm_tflops": round(r["gemm_tflops"], 2),
            "gemm_frac_of_peak": round(r["gemm_tflops"] / PEAKS[prec], 4), "peak_tflops": PEAKS[prec],
            "rel_err_vs_f64": rel, "prec_bound": r["stats"]["prec_bound"],
            "phases_ms_per_step": {k: round(r["tm"][k + "_ms"] / steps, 3)
                                   for k in ("build", "trunc", "prune", "gemm", "pyramid")}}
        torch.cuda.empty_cache()
    return out


def quad_comparison(ctx, dA, reps=2):
    """The 3D multiply (norms precomputed) in every precision on the two leaf
    GEMMs: quads of sibling C leaves (the default) and one C leaf per work
    unit; leaf-GEMM time per launch from the library's HIP events."""
    import torch
    from paper_1906_08148_amd import spamm
    M = ctx.build(dA, LEAF3D, stores=spamm.STORE_F64 | spamm.STORE_F32 | spamm.STORE_BF16)
    default = ctx.get_option("gemm_quad")
    out = {}
    for prec in (spamm.F64, spamm.F32, spamm.BF16X3, spamm.BF16):
        row = {}
        for quad in (0, 1):
            ctx.set_option("gemm_quad", quad)
            ctx.multiply(M, M, TAU3D, mode=spamm.HYBRID, prec=prec, stats=False).C.release()
            torch.cuda.synchronize()
            ctx.timing(enable=True, reset=True)
            for _ in range(reps):
                ctx.multiply(M, M, TAU3D, mode=spamm.HYBRID, prec=prec, stats=False).C.release()
            torch.cuda.synchronize()
            tm = ctx.timing(enable=False, reset=True)
            g_ms = tm["gemm_ms"] / max(tm["gemm_launches"], 1)
            g_fl = tm["gemm_flops"] / max(tm["gemm_launches"], 1)
            row["quad" if quad else "one_leaf"] = {"gemm_ms": round(g_ms, 3),
                                                   "gemm_tflops": round(g_fl / (g_ms * 1e-3) / 1e12, 2),
                                                   "plan_ms": round(tm["prune_ms"] / reps, 3)}
        row["gemm_speedup"] = round(row["one_leaf"]["gemm_ms"] / row["quad"]["gemm_ms"], 3)
        out[PREC_NAMES[prec]] = row
    ctx.set_option("gemm_quad", default)
    M.release()
    torch.cuda.empty_cache()
    return out


def fixed_error_3d(ctx, dA, reps=3):
    """Sec. 5.3's comparison at a target accuracy: for each precision, the
    largest tau on the decade grid 1 ... 1e-8 whose Hybrid product has
    ||A A - C||_F <= sigma = 1e-5 ||A||_F ||B||_F (the exact product A A in
    FP64 by the vendor GEMM, an independent reference), then multiplies/s at
    that tau with the quadtree built once (norms precomputed).  BF16 alone
    stays above sigma at every tau: its rounding error exceeds the budget."""
    import torch
    from paper_1906_08148_amd import spamm
    exact = dA @ dA
    nA = float(torch.linalg.norm(dA))
    sigma = SIGMA_REL * nA * nA
    M = ctx.build(dA, LEAF3D, stores=spamm.STORE_F64 | spamm.STORE_F32 | spamm.STORE_BF16)
    out = {"sigma": sigma, "sigma_rel": SIGMA_REL, "mode": "hybrid", "tau_grid": list(TAU_GRID), "precisions": {}}
    for prec in (spamm.F64, spamm.F32, spamm.BF16X3, spamm.BF16):
        tried = []
        chosen = None
        for tau in TAU_GRID:
            p = ctx.multiply(M, M, tau, mode=spamm.HYBRID, prec=prec)
            err = float(torch.linalg.norm(ctx.to_dense(p.C) - exact))
            tried.append({"tau": tau, "err": err, "n_kept": int(p.stats["n_kept"]),
                          "bound": p.stats["err_bound"] + p.stats["prec_bound"]})
            p.C.release()
            if err <= sigma:
                chosen = tau
                break
            # the error has reached the precision's rounding floor: smaller
            # tau cannot help
            if len(tried) >= 3 and err > 0.5 * tried[-2]["err"] and tau <= 1e-4:
                break
        rec = {"tau": chosen, "tried": tried}
        if chosen is not None:
            ctx.multiply(M, M, chosen, mode=spamm.HYBRID, prec=prec, stats=False).C.release()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.multiply(M, M, chosen, mode=spamm.HYBRID, prec=prec, stats=False).C.release()
            torch.cuda.synchronize()
            rec["multiplies_per_s"] = round(reps / (time.perf_counter() - t0), 3)
        out["precisions"][PREC_NAMES[prec]] = rec
        log(f"bench: fixed error {PREC_NAMES[prec]}: tau {chosen}")
    M.release()
    del exact
    torch.cuda.empty_cache()
    P = out["precisions"]
    if P["f32"].get("multiplies_per_s") and P["f64"].get("multiplies_per_s"):
        out["f32_over_f64"] = round(P["f32"]["multiplies_per_s"] / P["f64"]["multiplies_per_s"], 3)
    return out


def symmetric_3d(ctx, dA, C64):
    """The square of the symmetric 3D matrix with only the C leaves on and
    above the diagonal formed (each leaf below is its mirror's transpose),
    against the full product: time and agreement."""
    import torch
    from paper_1906_08148_amd import spamm
    out = {}
    M = ctx.build(dA, LEAF3D, stores=spamm.STORE_F64 | spamm.STORE_F32)
    nref = float(torch.linalg.norm(C64))
    for name, mode in (("spamm_sym", spamm.SPAMM_SYM), ("hybrid_sym", getattr(spamm, "HYBRID_SYM", None))):
        if mode is None:
            continue
        for prec in (spamm.F64, spamm.F32):
            ctx.multiply(M, M, TAU3D, mode=mode, prec=prec).C.release()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p = ctx.multiply(M, M, TAU3D, mode=mode, prec=prec)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rec = {"ms": round(dt * 1e3, 2), "n_kept_formed": int(p.stats["n_kept"])}
            if mode != spamm.SPAMM_SYM:
                rec["rel_diff_vs_full_hybrid_f64"] = float(torch.linalg.norm(ctx.to_dense(p.C) - C64)) / nref
            p.C.release()
            out[f"{name}/{PREC_NAMES[prec]}"] = rec
    M.release()
    return out


def autotune_3d(ctx, dA):
    """Leaf size (32 ... 256), MFMA tile and C leaves per workgroup (one, or
    quads at leaf 64) picked by the autotuner for the 3D
    workload (Hybrid, tau 1e-6) per precision, among the candidates whose
    error meets sigma = 1e-5 ||A||_F^2: by the library's guaranteed bound,
    and by the error measured against the exact product."""
    import torch
    from paper_1906_08148_amd import autotune, spamm
    out = {}
    exact = dA @ dA
    budget = SIGMA_REL * float(torch.linalg.norm(dA)) ** 2
    tuner = autotune.Tuner(ctx, leaves=(32, 64, 128, 256), tiles=(0, 1), reps=1)
    measured = lambda c, p: float(torch.linalg.norm(c.to_dense(p.C) - exact))
    for prec in (spamm.F32, spamm.BF16X3, spamm.BF16):
        for how, fn in (("bound", None), ("measured", measured)):
            if how == "bound" and prec != spamm.F32:
                continue  # the BF16 rounding bounds are above sigma at every leaf size
            log(f"bench: 3D autotune {PREC_NAMES[prec]} ({how} error)")
            sig = autotune.signature("3d", N3D, ALPHA3D, TAU3D, spamm.HYBRID, prec) + (how,)
            best = tuner.tune(lambda leaf: ctx.build(dA, leaf, stores=store_for(prec)), sig,
                              TAU3D, spamm.HYBRID, prec, budget=budget, error_fn=fn)
            out[f"{PREC_NAMES[prec]}/{how}"] = {
                "leaf": best["leaf"], "tile": best["tile"], "quad": best["quad"], "budget": budget,
                "table": [{k: (round(v, 6) if isinstance(v, float) and k == "seconds" else v) for k, v in r.items()}
                          for r in best["table"]]}
            torch.cuda.empty_cache()
    del exact
    ctx.set_option("gemm_tile", 1)
    ctx.set_option("gemm_quad", -1)
    return out


def paper_workloads():
    """The paper's own synthetic workloads (Sec. 5), in FP64 as there.

    Model problem: 1D decay n = 4e4, alpha = 0.005, A = B.  For each leaf size
    and method, the largest tau on the grid 1e-4 ... 1e-12 whose product has
    ||A A - C||_F <= sigma = 1e-6; its kept products (the paper's gemm calls)
    and multiply time with the norms precomputed, as there.  Truncmul runs in
    both readings: the leaf-level budget and the element-wise truncation of
    Thm. 1 (the truncation is not timed, like the norms).

    Leaf-library sweep: 2048 x 2048 matrices of random uniform blocks at fill
    0.1 ... 1.0, every product formed (Truncmul at tau = 0); kept-product
    GFLOP/s of batches of 32 multiplies."""
    import numpy as np
    import torch
    import synth
    from paper_1906_08148_amd import spamm
    n, alpha, sigma = 40000, 0.005, 1e-6
    t0 = time.perf_counter()
    A = synth.DecaySpec("1d", n, alpha, seed=SEED).dense()
    gen_s = time.perf_counter() - t0
    dA = torch.from_numpy(A).cuda()
    del A
    exact = dA @ dA
    ctx = new_context(80 << 30)
    modes = {"truncmul": spamm.TRUNCMUL, "spamm": spamm.SPAMM, "hybrid": spamm.HYBRID}
    model = {"workload": f"1D decay n={n}, alpha {alpha}, A=B, FP64, sigma {sigma}",
             "generate_s": round(gen_s, 1), "rows": []}
    for leaf in (32, 64, 128, 256):
        M = ctx.build(dA, leaf, stores=spamm.STORE_F64)
        ctx.multiply(M, M, 1e-4, mode=spamm.SPAMM, prec=spamm.F64).C.release()  # prune views
        base = None
        for name in ("truncmul", "truncmul_elementwise", "spamm", "hybrid"):
            best = {"leaf": leaf, "method": name, "tau": None}
            for k in range(4, 13):
                tau = 10.0 ** -k
                log(f"bench: model problem leaf {leaf} {name} tau 1e-{k}")
                Mt = None
                if name == "truncmul_elementwise":
                    Mt, _ = ctx.truncate_elementwise(M, tau)
                torch.cuda.synchronize()
                s0 = time.perf_counter()
                if Mt is not None:
                    p = ctx.multiply(Mt, Mt, 0.0, mode=spamm.TRUNCMUL, prec=spamm.F64)
                else:
                    p = ctx.multiply(M, M, tau, mode=modes[name], prec=spamm.F64)
                torch.cuda.synchronize()
                dt = time.perf_counter() - s0
                err = float(torch.linalg.norm(ctx.to_dense(p.C) - exact))
                kept = int(p.stats["n_kept"])
                p.C.release()
                if Mt is not None:
                    Mt.release()
                if err <= sigma:
                    best = {"leaf": leaf, "method": name, "tau": tau, "n_kept": kept, "ms": round(dt * 1e3, 2),
                            "err": err, "gflops": round(2.0 * leaf ** 3 * kept / dt / 1e9, 1)}
                    break
            if name == "truncmul" and best["tau"] is not None:
                base = best
            if base is not None and best["tau"] is not None:
                best["kept_vs_truncmul"] = round(best["n_kept"] / base["n_kept"], 3)
                best["time_vs_truncmul"] = round(best["ms"] / base["ms"], 3)
            model["rows"].append(best)
            torch.cuda.empty_cache()
        M.release()
    del exact, dA
    torch.cuda.empty_cache()
    sweep = {"workload": "2048 x 2048 random uniform blocks, FP64, every product (Truncmul, tau 0), "
                         "batches of 32 multiplies", "rows": []}
    for leaf in (32, 64, 128, 256):
        for fill in (0.1, 0.3, 0.5, 0.7, 1.0):
            log(f"bench: leaf library leaf {leaf} fill {fill}")
            mats = []
            for seed in (SEED, SEED + 1):
                coords, data = synth.random_blocks(seed, 2048, leaf, fill)
                mats.append(ctx.build_blocks(2048, leaf, torch.from_numpy(coords.astype(np.int32)).cuda(),
                                             torch.from_numpy(np.ascontiguousarray(data)).cuda(),
                                             stores=spamm.STORE_F64))
            reqs = [dict(A=mats[0], B=mats[1], tau=0.0, mode=spamm.TRUNCMUL, prec=spamm.F64)] * 32
            for p in ctx.multiply_batch(reqs):
                p.C.release()
            ts, flops = [], 0.0
            for _ in range(5):
                torch.cuda.synchronize()
                s0 = time.perf_counter()
                prods = ctx.multiply_batch(reqs)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - s0)
                flops = sum(p.stats["flops"] for p in prods)
                for p in prods:
                    p.C.release()
            dt = sorted(ts)[len(ts) // 2]
            sweep["rows"].append({"leaf": leaf, "fill": fill, "gflops": round(flops / dt / 1e9, 1),
                                  "frac_of_fp64_peak": round(flops / dt / 1e12 / FP64_MFMA_PEAK_TFLOPS, 4)})
            for m in mats:
                m.release()
    ctx.close()
    return {"model_problem": model, "leaf_library": sweep}


def purification(steps, mode=None, tau_c=0.0):
    """20 trace-driven purification steps (X^2 or 2X - X^2, tau 1e-6, the
    symmetric square of Hybrid by default: the iterates are symmetric) on the
    3D decay matrix n = 32768 scaled into [0, 1], FP64 and FP32 chains side
    by side; per step the trace, products, time and ||X32 - X64||_F.  With
    tau_c > 0 every iterate is truncated after its product (mirror pairs,
    budget tau_c)."""
    import torch
    import synth
    from paper_1906_08148_amd import purify, spamm
    A = synth.DecaySpec("3d", N3D, ALPHA3D, seed=SEED).dense()
    ctx = new_context(96 << 30)
    dA = torch.from_numpy(A).cuda()
    del A
    X = ctx.build(dA, LEAF3D, stores=spamm.STORE_F64 | spamm.STORE_F32)
    torch.cuda.synchronize()
    del dA
    mode = spamm.HYBRID_SYM if mode is None else mode
    recs, diffs, (lo, hi) = purify.sp2(ctx, X, N3D / 2, TAU3D, steps, precs=(spamm.F64, spamm.F32), mode=mode,
                                       tau_c=tau_c)
    X.release()
    ctx.close()
    out = {"workload": f"SP2 purification of the 3D decay matrix n={N3D}, leaf {LEAF3D}, "
                       f"{'hybrid_sym' if mode == spamm.HYBRID_SYM else 'hybrid'}, tau {TAU3D}, n_occ = n/2, "
                       f"{steps} steps" + (f", iterates truncated with tau_c {tau_c}" if tau_c > 0 else ""),
           "gershgorin": [lo, hi], "steps": []}
    for k in range(steps):
        r64, r32 = recs[spamm.F64][k], recs[spamm.F32][k]
        out["steps"].append({"k": k, "trace64": round(r64.trace, 6), "trace32": round(r32.trace, 6),
                             "branch64": r64.branch, "branch32": r32.branch,
                             "kept64": r64.n_kept, "kept32": r32.n_kept,
                             "ms64": round(r64.seconds * 1e3, 1), "ms32": round(r32.seconds * 1e3, 1),
                             "gflops32": round(r32.flops / r32.seconds / 1e9, 1),
                             "idempotency64": r64.idempotency, "x32_minus_x64": diffs[spamm.F32][k]})
        if tau_c > 0:
            out["steps"][-1].update(leaves64=r64.nonnull, dropped_sq64=r64.dropped_sq)
    t64 = sum(r.seconds for r in recs[spamm.F64])
    t32 = sum(r.seconds for r in recs[spamm.F32])
    out["total_s"] = {"f64": round(t64, 3), "f32": round(t32, 3)}
    return out


def serving(n_requests, n_max, rates=(0.5, 1.0, 2.0, 4.0)):
    """Served stream: the first `n_requests` requests with n <= n_max of the
    seeded request pool (n in 2048..65536, 1D/3D decay, alpha, tau, scheme
    drawn per request, FP32, A = B).  Capacity mu is measured alone (one
    lane, one request per batch); then Poisson arrivals at rate x mu for
    each x, two lanes with continuous batching and memory admission, fresh
    lanes (cold quadtree caches) per run.  At 2 mu the same stream also runs
    with each batch's post-sizing kernels launched as one HIP graph."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from paper_1906_08148_amd import serve
    pool = [r for r in serve.request_pool(512) if r.mat.n <= n_max][:n_requests]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(4) as ex:
        mats = list({r.mat: None for r in pool})
        inputs = dict(zip(mats, ex.map(lambda m: serve.make_input(m, 64), mats)))
    gen_s = time.perf_counter() - t0
    lane_bytes = 60 << 30
    srv = serve.Server(lanes=1, arena_bytes_per_lane=lane_bytes, max_batch=1, inputs=inputs, options=CTX_OPTIONS)
    t0 = time.perf_counter()
    alone = serve.run_stream(srv.sched, pool, rate=0)
    t_alone = time.perf_counter() - t0
    srv.close()
    del srv
    torch.cuda.empty_cache()
    mu = len(pool) / t_alone
    out = {"workload": f"first {len(pool)} requests with n <= {n_max} of the seeded pool (n in 2048..65536 step "
                       f"2048, 1D/3D decay, alpha U[0.2,1], tau 10^U[-8,-4], truncmul/spamm/hybrid, FP32, A=B)",
           "generate_s": round(gen_s, 1), "alone": serve.summarize(alone, t_alone), "mu_per_s": mu,
           "n_max_served": max(r.mat.n for r in pool),
           "kinds": [f"{r.mat.kind}:{r.mat.n}" for r in pool], "runs": {}}
    for x, graph in [(x, False) for x in rates] + [(2.0, True)]:
        log(f"bench: serving at {x} mu{' (graph)' if graph else ''}")
        srv = serve.Server(lanes=2, arena_bytes_per_lane=lane_bytes, max_batch=16, inputs=inputs, graph=graph,
                           options=CTX_OPTIONS)
        res = serve.run_stream(srv.sched, pool, rate=x * mu, seed=11)
        srv.close()
        log_ = list(srv.sched.log)
        del srv
        torch.cuda.empty_cache()
        sm = serve.summarize(res)
        sm["gflops_frac_of_fp32_peak"] = sm.get("gflops", 0.0) / 1e3 / FP32_MFMA_PEAK_TFLOPS
        sm["batches"] = len(log_)
        sm["largest_batch"] = max((len(b[2]) for b in log_), default=0)
        sm["over_alone_capacity"] = round(sm.get("multiplies_per_s", 0.0) / mu, 3)
        out["runs"][f"{x}{'_graph' if graph else ''}"] = sm
    return out


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_baseline_3d(sample_n=8192, one_thread=True):
    """The oracle as it stands on a bounded sample of the 3D workload: the
    leading sample_n x sample_n principal sub-matrix of the same matrix (the
    first sample_n / 8 atoms of the Morton order, a box of the same
    lattice), leaf 64, tau 1e-6, Hybrid, the whole oracle multiply (tree and
    norms, truncation, kept list, every C leaf, accounting), NumPy FP64 with
    BLAS on every core the host gives it; then again with one BLAS thread."""
    import oracle as O
    import synth
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_info = threadpool_limits = None
    A = synth.DecaySpec("3d", N3D, ALPHA3D, seed=SEED).block(0, sample_n, 0, sample_n)

    def run():
        ph = {}
        t0 = time.perf_counter()
        T = O.build(A, LEAF3D)
        ph["tree_and_norms"] = time.perf_counter() - t0
        s0 = time.perf_counter()
        r = O.multiply(T, T, TAU3D, O.HYBRID)
        ph["multiply"] = time.perf_counter() - s0
        return time.perf_counter() - t0, r.stats["flops"], ph

    dt, flops, ph = run()
    blas = None
    if threadpool_info is not None:
        blas = sum(p.get("num_threads", 0) for p in threadpool_info() if p.get("user_api") == "blas") or None
    out = {"value": round(flops / dt / 1e9, 4), "unit": "GFLOP/s", "cores": blas or 1, "kind": "oracle",
           "sample": f"leading {sample_n} x {sample_n} principal block of the 3D decay matrix (first "
                     f"{sample_n // 8} atoms), leaf {LEAF3D}, tau {TAU3D}, Hybrid: the whole oracle multiply "
                     f"({dt:.1f} s, {flops:.3e} kept-leaf flops), NumPy FP64; cores = BLAS threads "
                     f"(Python-level work is one thread)",
           "host_cores": os.cpu_count(), "seconds": round(dt, 2),
           "phases_s": {k: round(v, 3) for k, v in ph.items()}}
    if one_thread and threadpool_limits is not None:
        with threadpool_limits(1):
            dt1, fl1, _ = run()
        out["one_thread"] = {"value": round(fl1 / dt1 / 1e9, 4), "seconds": round(dt1, 2)}
    return out


def traffic_for(kernel_name):
    """HBM bytes per GEMM launch from the committed rocprofv3 counter summary
    of this kernel, only when it was taken on the current kernel source."""
    import glob
    src = hashlib.sha256(open(GEMM_SOURCE, "rb").read()).hexdigest()
    for f in sorted(glob.glob(TRAFFIC_GLOB)):
        try:
            rec = json.load(open(f))
        except Exception:
            continue
        if rec.get("kernel") == kernel_name and rec.get("kernel_source_sha256") == src:
            return rec.get("bytes_per_launch")
    return None


def batch_1d(ctx, steps, warmup):
    """The 1D batch: 18 multiplies of n = 16384 (alpha x tau x scheme) built
    from leaf-block lists, FP32 and FP64, one batch per step."""
    from paper_1906_08148_amd import spamm
    host = make_inputs()
    dev = gpu_inputs(host)
    out = {"workload": "1D decay n=16384 leaf 64, alpha {0.2,0.5} x tau {1e-4,1e-6,1e-8} x "
                       "{truncmul,spamm,hybrid}, A=B, built from leaf-block lists; 18 multiplies per step, one batch"}
    for prec in (spamm.F32, spamm.F64):
        total, lat, flops, tm, stats = timed_steps(ctx, dev, prec, steps, warmup)
        g = tm["gemm_ms"] / max(tm["gemm_launches"], 1)
        fl = tm["gemm_flops"] / max(tm["gemm_launches"], 1)
        out[PREC_NAMES[prec]] = {
            "gflops": round(flops / total / 1e9, 1), "ms_per_step": round(total / steps * 1e3, 4),
            "multiplies_per_s": round(len(stats) * steps / total, 1),
            "latency_ms": {"p50": round(pct(lat, 0.5) * 1e3, 4), "p99": round(pct(lat, 0.99) * 1e3, 4)},
            "gemm_tflops": round(fl / (g * 1e-3) / 1e12, 2),
            "gemm_frac_of_peak": round(fl / (g * 1e-3) / 1e12 / PEAKS[prec], 4),
            "phases_ms_per_step": {k: round(tm[k + "_ms"] / steps, 4)
                                   for k in ("build", "trunc", "prune", "gemm", "pyramid")},
            "norms_precomputed": multiply_only(ctx, dev, prec, steps, warmup)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=8192, help="size of the oracle's sample (principal block)")
    ap.add_argument("--skip-extras", action="store_true", help="only the timed headline steps (profiling)")
    ap.add_argument("--prec", default="f64", choices=sorted(PREC_NAMES.values()),
                    help="precision of the timed steps (profiling the other GEMMs)")
    ap.add_argument("--graph", action="store_true", help="launch each batch's post-sizing kernels as one HIP graph")
    ap.add_argument("--gemm-tile", type=int, default=None, help="MFMA tile variant (0: 32x32, 1: 16x16)")
    ap.add_argument("--gemm-quad", type=int, default=None, choices=(0, 1),
                    help="leaf-64 products in quads of sibling C leaves (1, the library default) or one C leaf "
                         "per work unit (0)")
    ap.add_argument("--steps-1d", type=int, default=20)
    ap.add_argument("--no-1d", action="store_true", help="skip the 1D batch section")
    ap.add_argument("--no-purify", action="store_true", help="skip the purification section")
    ap.add_argument("--no-autotune", action="store_true", help="skip the autotuner section")
    ap.add_argument("--paper-workloads", action="store_true",
                    help="also run the paper's model problem and leaf-library sweep (FP64; a few minutes)")
    ap.add_argument("--purify-steps", type=int, default=20)
    ap.add_argument("--serve-requests", type=int, default=64, help="requests of the served stream (0: skip)")
    ap.add_argument("--serve-nmax", type=int, default=32768, help="largest n of the served sample (pool: 65536)")
    ap.add_argument("--serving-only", action="store_true", help="only the served stream (its own JSON line)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="before the steps, copy a buffer of this many MiB on the device (a plain copy "
                         "kernel of known traffic, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU (sharding across GPUs is designed, not "
                                   "implemented); --gpus must be 1", "n_gpus": args.gpus}))
        return 2
    import torch
    import synth
    from paper_1906_08148_amd import spamm

    if args.gemm_tile is not None:
        CTX_OPTIONS["gemm_tile"] = args.gemm_tile
    if args.gemm_quad is not None:
        CTX_OPTIONS["gemm_quad"] = args.gemm_quad
    if args.serving_only:
        print(json.dumps({"serving": serving(args.serve_requests, args.serve_nmax)}))
        return 0
    prec = spamm.PRECS[args.prec]
    log("bench: generating the 3D decay matrix n=32768")
    t0 = time.perf_counter()
    A = synth.DecaySpec("3d", N3D, ALPHA3D, seed=SEED).dense()
    gen_s = time.perf_counter() - t0
    dA = torch.from_numpy(A).cuda()
    del A
    ctx = new_context(64 << 30)
    if args.graph:
        ctx.set_option("graph", 1)
    if args.copy_calibration_mb:
        src = torch.ones(args.copy_calibration_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    log(f"bench: 3D hybrid {args.prec} steps")
    r = config3_steps(ctx, dA, prec, args.steps, args.warmup, keep_last=not args.skip_extras)
    tile = ctx.get_option("gemm_tile")
    quad = r["tm"]["gemm_quad_launches"] > 0  # the GEMM the library chose for this workload
    if quad:
        kname = f"void spamm::k_gemm_quad<{prec}, {0 if prec == spamm.F64 else 1}, {LEAF3D}>"
    else:
        kname = f"void spamm::k_gemm<{prec}, {LEAF3D}, {0 if prec == spamm.F64 else tile}, {LEAF3D}>"
    st = r["stats"]
    out = {
        "metric": METRIC,
        "value": round(r["flops"] / r["total"] / 1e9, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["total"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"3D decay n={N3D} (4096 atoms on a 16^3 lattice x 8 functions), a_ij = (2u-1) "
                               f"exp(-dist), leaf {LEAF3D}, tau {TAU3D}, A=B; one step = build from the dense "
                               f"FP64 matrix in HBM + one Hybrid multiply ({args.prec} leaf products)",
                   "n": N3D, "leaf": LEAF3D, "tau": TAU3D, "mode": "hybrid", "seed": SEED},
        "multiplies_per_s": round(args.steps / r["total"], 3),
        "latency_ms": {"p50": round(pct(r["lat"], 0.5) * 1e3, 3), "p99": round(pct(r["lat"], 0.99) * 1e3, 3)},
        "kept_products_per_step": int(st["n_kept"]),
        "stats": {k: st[k] for k in ("n_candidates", "c_nonnull", "err_bound", "prec_bound", "dA", "B2")},
        "phases_ms_per_step": {k: round(r["tm"][k + "_ms"] / args.steps, 3)
                               for k in ("build", "trunc", "prune", "gemm", "pyramid")},
        "generate_s": round(gen_s, 1),
        "roofline": {"kernel": (f"k_gemm_quad<{args.prec.upper()}> (quads of sibling 64-leaves, pipelined MFMA "
                               f"leaf GEMM)" if quad else
                               f"k_gemm<{args.prec.upper()},{LEAF3D}> (persistent MFMA leaf GEMM)"),
                     "bound": "mfma", "achieved": round(r["gemm_tflops"], 3), "peak": PEAKS[prec],
                     "unit": "TFLOP/s", "frac": round(r["gemm_tflops"] / PEAKS[prec], 4),
                     "traffic": traffic_for(kname), "flops_per_launch": r["gemm_flops"],
                     "ms_per_launch": round(r["gemm_ms"], 4)},
    }
    C64 = None
    if r["last"] is not None:
        C64 = ctx.to_dense(r["last"].C)
        r["last"].C.release()
    if not args.skip_extras:
        log("bench: 3D multiply with norms precomputed")
        out["norms_precomputed"] = multiply_only_3d(ctx, dA, prec, args.steps)
        if prec == spamm.F64:
            out["precisions"] = config3_precisions(ctx, dA, max(2, args.steps // 2), C64)
            log("bench: 3D symmetric square")
            out["symmetric"] = symmetric_3d(ctx, dA, C64)
        del C64
        torch.cuda.empty_cache()
        log("bench: 3D quads vs one leaf per work unit")
        out["quad_vs_one_leaf"] = quad_comparison(ctx, dA)
        log("bench: 3D fixed error")
        out["fixed_error"] = fixed_error_3d(ctx, dA)
        if not args.no_autotune:
            out["autotune"] = autotune_3d(ctx, dA)
        ctx.close()
        del dA
        torch.cuda.empty_cache()
        ctx = new_context(16 << 30)
        if not args.no_1d:
            log("bench: 1D batch")
            out["batch_1d"] = batch_1d(ctx, args.steps_1d, 5)
        ctx.close()
        ctx = None
        if not args.no_purify:
            log("bench: purification n=32768")
            out["purification"] = purification(args.purify_steps)
        if args.serve_requests > 0:
            log("bench: serving")
            out["serving"] = serving(args.serve_requests, args.serve_nmax)
        if args.paper_workloads:
            log("bench: the paper's model problem and leaf-library sweep")
            out["paper_workloads"] = paper_workloads()
    if ctx is not None:
        ctx.close()
    if not args.no_cpu_baseline:
        log("bench: oracle CPU baseline")
        out["cpu_baseline"] = cpu_baseline_3d(args.cpu_sample_n)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
