#!/usr/bin/env python3
"""Benchmark of the approximate-product hot path on one MI355X.

Workload (one "step"): the 1D-decay sweep n = 16384, leaf 64,
a_ij = (2u - 1) exp(-alpha |i - j|), alpha in {0.2, 0.5}, tau in {1e-4, 1e-6,
1e-8}, schemes Truncmul / SpAMM / Hybrid, A = B.  A step builds both matrices
from their device-resident leaf-block lists (norms, null map, pyramid), then
runs the 18 multiplies as one batch: truncation, pruning, one persistent
leaf-GEMM launch, C pyramids and the FP64 accounting.  The headline value is
kept-leaf GFLOP/s (2 * 64^3 per formed leaf product) in FP32-MFMA mode; the
same step in FP64 mode is reported beside it.

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
GEMM_SOURCE = os.path.join(ROOT, "paper_1906_08148_amd", "csrc", "k_gemm.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_gemm_f32_leaf64_decay1d_n16384_batch18_traffic.json")


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


def dense3d(steps):
    """3D decay, n = 32768, leaf 64, tau = 1e-6, A = B: one multiply per
    (scheme, precision), timed alone (warm), with the leaf-GEMM time from the
    library's events and the relative difference from the FP64 product."""
    import torch
    import synth
    from paper_1906_08148_amd import spamm
    t0 = time.perf_counter()
    A = synth.DecaySpec("3d", N3D, ALPHA3D, seed=SEED).dense()
    gen_s = time.perf_counter() - t0
    ctx = spamm.Context(arena_bytes=64 << 30)
    dA = torch.from_numpy(A).cuda()
    del A
    M = ctx.build(dA, LEAF3D, stores=spamm.STORE_F64 | spamm.STORE_F32 | spamm.STORE_BF16)
    torch.cuda.synchronize()
    out = {"workload": f"3D decay n={N3D} (4096 atoms x 8 functions), alpha {ALPHA3D}, leaf {LEAF3D}, "
                       f"tau {TAU3D}, A=B", "generate_s": round(gen_s, 1), "runs": {}}
    peaks = {spamm.F64: FP64_MFMA_PEAK_TFLOPS, spamm.F32: FP32_MFMA_PEAK_TFLOPS,
             spamm.BF16: BF16_MFMA_PEAK_TFLOPS, spamm.BF16X3: BF16_MFMA_PEAK_TFLOPS}
    names = {spamm.F64: "f64", spamm.F32: "f32", spamm.BF16: "bf16", spamm.BF16X3: "bf16x3"}
    for mode, mname in ((spamm.SPAMM, "spamm"), (spamm.HYBRID, "hybrid"), (spamm.SPAMM_SYM, "spamm_sym")):
        ref = None
        for prec in ((spamm.F64, spamm.F32) if mode == spamm.SPAMM_SYM else
                     (spamm.F64, spamm.F32, spamm.BF16, spamm.BF16X3)):
            log(f"bench: 3D {mname} {names[prec]}")
            p = ctx.multiply(M, M, TAU3D, mode=mode, prec=prec)  # warm
            p.C.release()
            torch.cuda.synchronize()
            ts = []
            for _ in range(steps):
                ctx.timing(enable=True, reset=True)
                s0 = time.perf_counter()
                p = ctx.multiply(M, M, TAU3D, mode=mode, prec=prec)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - s0)
                tm = ctx.timing(enable=False, reset=True)
                if _ + 1 < steps:
                    p.C.release()
            dt = sorted(ts)[len(ts) // 2]
            st = p.stats
            gemm_s = tm["gemm_ms"] / max(tm["gemm_launches"], 1) * 1e-3
            rec = {"ms": round(dt * 1e3, 2), "gflops": round(st["flops"] / dt / 1e9, 1),
                   "n_kept": int(st["n_kept"]), "gemm_ms": round(gemm_s * 1e3, 2),
                   "gemm_tflops": round(st["flops"] / gemm_s / 1e12, 2),
                   "gemm_frac": round(st["flops"] / gemm_s / 1e12 / peaks[prec], 4),
                   "phases_ms": {k: round(tm[k + "_ms"], 2) for k in ("trunc", "prune", "gemm", "pyramid")}}
            C = ctx.to_dense(p.C)
            if prec == spamm.F64:
                ref = C
                rec["rel_err_vs_f64"] = 0.0
            else:
                rec["rel_err_vs_f64"] = float(torch.linalg.norm(C - ref) / torch.linalg.norm(ref))
                del C
            p.C.release()
            out["runs"][f"{mname}/{names[prec]}"] = rec
        del ref
        torch.cuda.empty_cache()
    M.release()
    # leaf size and MFMA tile picked by the autotuner (hybrid, FP32)
    from paper_1906_08148_amd import autotune
    log("bench: 3D autotune")
    tuner = autotune.Tuner(ctx, leaves=(32, 64, 128), tiles=(0, 1), reps=2)
    sig = autotune.signature("3d", N3D, ALPHA3D, TAU3D, spamm.HYBRID, spamm.F32)
    best = tuner.tune(lambda leaf: ctx.build(dA, leaf, stores=spamm.STORE_F32), sig, TAU3D, spamm.HYBRID, spamm.F32)
    out["autotune"] = {"leaf": best["leaf"], "tile": best["tile"],
                       "table": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
                                 for r in best["table"]]}
    del dA
    ctx.close()
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
    ctx = spamm.Context(arena_bytes=80 << 30)
    modes = {"truncmul": spamm.TRUNCMUL, "spamm": spamm.SPAMM, "hybrid": spamm.HYBRID}
    model = {"workload": f"1D decay n={n}, alpha {alpha}, A=B, FP64, sigma {sigma}",
             "generate_s": round(gen_s, 1), "rows": []}
    for leaf in (32, 64, 128):
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
    for leaf in (32, 64, 128):
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


def purification(steps):
    """20 trace-driven purification steps (X^2 or 2X - X^2, Hybrid, tau 1e-6)
    on the 3D decay matrix n = 32768 scaled into [0, 1], FP64 and FP32 chains
    side by side; per step the trace, products, time and ||X32 - X64||_F."""
    import torch
    import synth
    from paper_1906_08148_amd import purify, spamm
    A = synth.DecaySpec("3d", N3D, ALPHA3D, seed=SEED).dense()
    ctx = spamm.Context(arena_bytes=96 << 30)
    dA = torch.from_numpy(A).cuda()
    del A
    X = ctx.build(dA, LEAF3D, stores=spamm.STORE_F64 | spamm.STORE_F32)
    torch.cuda.synchronize()
    del dA
    recs, diffs, (lo, hi) = purify.sp2(ctx, X, N3D / 2, TAU3D, steps, precs=(spamm.F64, spamm.F32))
    X.release()
    ctx.close()
    out = {"workload": f"SP2 purification of the 3D decay matrix n={N3D}, leaf {LEAF3D}, hybrid, tau {TAU3D}, "
                       f"n_occ = n/2, {steps} steps", "gershgorin": [lo, hi], "steps": []}
    for k in range(steps):
        r64, r32 = recs[spamm.F64][k], recs[spamm.F32][k]
        out["steps"].append({"k": k, "trace64": round(r64.trace, 6), "trace32": round(r32.trace, 6),
                             "branch64": r64.branch, "branch32": r32.branch,
                             "kept64": r64.n_kept, "kept32": r32.n_kept,
                             "ms64": round(r64.seconds * 1e3, 1), "ms32": round(r32.seconds * 1e3, 1),
                             "gflops32": round(r32.flops / r32.seconds / 1e9, 1),
                             "idempotency64": r64.idempotency, "x32_minus_x64": diffs[spamm.F32][k]})
    t64 = sum(r.seconds for r in recs[spamm.F64])
    t32 = sum(r.seconds for r in recs[spamm.F32])
    out["total_s"] = {"f64": round(t64, 3), "f32": round(t32, 3)}
    return out


def serving(n_requests, n_max, rates=(0.5, 0.8, 1.0, 1.2)):
    """Served stream: the first `n_requests` requests with n <= n_max of the
    seeded request pool (n in 2048..65536, 1D/3D decay, alpha, tau, scheme
    drawn per request, FP32, A = B).  Capacity mu is measured alone (one lane, one request per
    batch); then Poisson arrivals at rate x mu for each x, two lanes with
    continuous batching and memory admission, fresh lanes (cold quadtree
    caches) per run."""
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
    srv = serve.Server(lanes=1, arena_bytes_per_lane=lane_bytes, max_batch=1, inputs=inputs)
    t0 = time.perf_counter()
    alone = serve.run_stream(srv.sched, pool, rate=0)
    t_alone = time.perf_counter() - t0
    srv.close()
    torch.cuda.empty_cache()
    mu = len(pool) / t_alone
    out = {"workload": f"first {len(pool)} requests with n <= {n_max} of the seeded pool (n in 2048..65536 step "
                       f"2048, 1D/3D decay, alpha U[0.2,1], tau 10^U[-8,-4], truncmul/spamm/hybrid, FP32, A=B)",
           "generate_s": round(gen_s, 1), "alone": serve.summarize(alone, t_alone), "mu_per_s": mu,
           "kinds": [f"{r.mat.kind}:{r.mat.n}" for r in pool], "runs": {}}
    for x in rates:
        log(f"bench: serving at {x} mu")
        srv = serve.Server(lanes=2, arena_bytes_per_lane=lane_bytes, max_batch=16, inputs=inputs)
        res = serve.run_stream(srv.sched, pool, rate=x * mu, seed=11)
        srv.close()
        torch.cuda.empty_cache()
        sm = serve.summarize(res)
        sm["gflops_frac_of_fp32_peak"] = sm.get("gflops", 0.0) / 1e3 / FP32_MFMA_PEAK_TFLOPS
        sm["batches"] = len(srv.sched.log)
        out["runs"][str(x)] = sm
    return out


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def errors(ctx, dev, host, prec):
    """||C - A A||_F of every request against the FP64 dense product (torch
    FP64 GEMM as an independent reference), outside the timed region."""
    import numpy as np
    import torch
    import synth
    stats, prods, mats = run_step(ctx, dev, prec, keep=True)
    out = []
    i = 0
    for a in ALPHAS:
        coords, data = host[a]
        A = torch.from_numpy(synth.dense_from_blocks(N, LEAF, coords, data)).cuda()
        exact = A @ A
        nA = float(torch.linalg.norm(A))
        for t in TAUS:
            for m in MODE_NAMES:
                C = ctx.to_dense(prods[i].C)
                err = float(torch.linalg.norm(C - exact))
                out.append(dict(alpha=a, tau=t, mode=m, err=err, sigma=1e-5 * nA * nA,
                                n_kept=stats[i]["n_kept"], bound=stats[i]["err_bound"],
                                prec_bound=stats[i]["prec_bound"]))
                i += 1
                del C
        del A, exact
    for p in prods:
        p.C.release()
    for m in mats.values():
        m.release()
    torch.cuda.empty_cache()
    return out


def fixed_error_rate(ctx, dev, prec, errs, reps):
    """Multiplies/s for the largest tau meeting ||E||_F <= 1e-5 ||A||_F^2 per
    (alpha, scheme), matrices prebuilt (norms precomputed, as in Sec. 5.3)."""
    import torch
    from paper_1906_08148_amd import spamm
    store = spamm.STORE_F64 if prec == spamm.F64 else spamm.STORE_F32
    mats = {a: ctx.build_blocks(N, LEAF, c, d, stores=store) for a, (c, d) in dev.items()}
    chosen = []
    for a in ALPHAS:
        for mi, m in enumerate(MODE_NAMES):
            ok = [e for e in errs if e["alpha"] == a and e["mode"] == m and e["err"] <= e["sigma"]]
            if ok:
                best = max(ok, key=lambda e: e["tau"])
                chosen.append(dict(alpha=a, mode=m, tau=best["tau"], err=best["err"], mi=mi))
    reqs = [dict(A=mats[c["alpha"]], B=mats[c["alpha"]], tau=c["tau"], mode=c["mi"], prec=prec) for c in chosen]
    for _ in range(2):
        for p in ctx.multiply_batch(reqs, stats=False):
            p.C.release()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for p in ctx.multiply_batch(reqs, stats=False):
            p.C.release()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for m in mats.values():
        m.release()
    return dict(multiplies_per_s=len(reqs) * reps / dt,
                chosen=[{k: c[k] for k in ("alpha", "mode", "tau", "err")} for c in chosen])


def cpu_baseline(host, min_s=10.0):
    """The oracle as it stands, with one BLAS thread, on whole steps of the
    same workload (both builds and all 18 multiplies), repeated until at
    least ``min_s`` seconds of CPU work have run."""
    import oracle as O
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(1)
    except Exception:  # pragma: no cover
        limiter = None
    t0 = time.perf_counter()
    flops = 0.0
    steps = 0
    while True:
        for a in ALPHAS:
            coords, data = host[a]
            tree = O.build_from_blocks(N, LEAF, coords, data)
            for t in TAUS:
                for mi in (O.TRUNCMUL, O.SPAMM, O.HYBRID):
                    flops += O.multiply(tree, tree, t, mi).stats["flops"]
        steps += 1
        if time.perf_counter() - t0 >= min_s:
            break
    dt = time.perf_counter() - t0
    # one more step, timed phase by phase: the leaf trees with their norms,
    # the truncations, the kept lists, and the rest of each multiply (C
    # accumulation and accounting)
    ph = {"build_and_norms": 0.0, "truncation": 0.0, "kept_list": 0.0, "c_and_accounting": 0.0}
    for a in ALPHAS:
        coords, data = host[a]
        s0 = time.perf_counter()
        tree = O.build_from_blocks(N, LEAF, coords, data)
        ph["build_and_norms"] += time.perf_counter() - s0
        for t in TAUS:
            s0 = time.perf_counter()
            tr = O.truncate(tree, t).tree
            ph["truncation"] += 2 * (time.perf_counter() - s0)  # Truncmul and Hybrid each truncate
            s0 = time.perf_counter()
            for Tu, use in ((tr, False), (tree, True), (tr, True)):
                O.kept_flat(Tu, Tu, t, use)
            kept_s = time.perf_counter() - s0
            ph["kept_list"] += kept_s
            s0 = time.perf_counter()
            for mi in (O.TRUNCMUL, O.SPAMM, O.HYBRID):
                O.multiply(tree, tree, t, mi)
            ph["c_and_accounting"] += time.perf_counter() - s0 - kept_s
    ph["c_and_accounting"] -= ph["truncation"]
    if limiter is not None:
        limiter.unregister()
    return {"value": round(flops / dt / 1e9, 4), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} whole step(s): both builds and all 18 multiplies, {dt:.1f} s, "
                      f"NumPy FP64, one BLAS thread",
            "host_cores": os.cpu_count(),
            "phases_s_per_step": {k: round(v, 4) for k, v in ph.items()}}


def traffic_for(tile):
    """HBM bytes per GEMM launch from the committed rocprofv3 counter summary,
    only when it was taken on the current kernel source and tile variant."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except Exception:
        return None
    src = hashlib.sha256(open(GEMM_SOURCE, "rb").read()).hexdigest()
    if rec.get("kernel_source_sha256") != src or rec.get("kernel") != f"void spamm::k_gemm<1, 64, {tile}>":
        return None
    return rec.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--skip-extras", action="store_true", help="only the timed FP32 steps (profiling)")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D decay n=32768 section")
    ap.add_argument("--graph", action="store_true", help="launch each batch's post-sizing kernels as one HIP graph")
    ap.add_argument("--gemm-tile", type=int, default=None, help="MFMA tile variant (0: 32x32, 1: 16x16)")
    ap.add_argument("--steps-3d", type=int, default=3)
    ap.add_argument("--no-purify", action="store_true", help="skip the purification section")
    ap.add_argument("--paper-workloads", action="store_true",
                    help="also run the paper's model problem and leaf-library sweep (FP64; a few minutes)")
    ap.add_argument("--purify-steps", type=int, default=20)
    ap.add_argument("--serve-requests", type=int, default=16, help="requests of the served stream (0: skip)")
    ap.add_argument("--serve-nmax", type=int, default=32768, help="largest n of the served sample (pool: 65536)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="before the steps, copy a buffer of this many MiB on the device (a plain copy "
                         "kernel of known traffic, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU (sharding across GPUs is designed, not "
                                   "implemented); --gpus must be 1", "n_gpus": args.gpus}))
        return 2
    import torch
    from paper_1906_08148_amd import spamm

    log("bench: generating inputs")
    host = make_inputs()
    dev = gpu_inputs(host)
    ctx = spamm.Context(arena_bytes=16 << 30)
    if args.graph:
        ctx.set_option("graph", 1)
    if args.gemm_tile is not None:
        ctx.set_option("gemm_tile", args.gemm_tile)
    if args.copy_calibration_mb:
        src = torch.ones(args.copy_calibration_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    log("bench: FP32 steps")
    total32, lat32, flops32, tm32, stats32 = timed_steps(ctx, dev, spamm.F32, args.steps, args.warmup)
    value = flops32 / total32 / 1e9
    gemm_per_launch_ms = tm32["gemm_ms"] / max(tm32["gemm_launches"], 1)
    flops_per_launch = tm32["gemm_flops"] / max(tm32["gemm_launches"], 1)
    achieved = flops_per_launch / (gemm_per_launch_ms * 1e-3) / 1e12
    tile = ctx.get_option("gemm_tile")
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total32 / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1D decay n=16384 leaf 64, alpha {0.2,0.5} x tau {1e-4,1e-6,1e-8} x "
                               "{truncmul,spamm,hybrid}, A=B, built from leaf-block lists; 18 multiplies "
                               "per step, one batch",
                   "n": N, "leaf": LEAF, "multiplies_per_step": len(stats32), "seed": SEED},
        "multiplies_per_s": round(len(stats32) * args.steps / total32, 2),
        "latency_ms": {"p50": round(pct(lat32, 0.5) * 1e3, 4), "p99": round(pct(lat32, 0.99) * 1e3, 4)},
        "kept_products_per_step": int(sum(s["n_kept"] for s in stats32)),
        "phases_ms_per_step": {k: round(tm32[k + "_ms"] / args.steps, 4)
                               for k in ("build", "trunc", "prune", "gemm", "pyramid")},
        # the same multiplies with the matrices (and their norms) built once
        "norms_precomputed": multiply_only(ctx, dev, spamm.F32, args.steps, args.warmup),
        "roofline": {"kernel": f"k_gemm<SPAMM_F32,64,{tile}> (persistent MFMA leaf GEMM, "
                               f"{'16x16' if tile else '32x32'} MFMA tiles)", "bound": "mfma",
                     "achieved": round(achieved, 3), "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP32_MFMA_PEAK_TFLOPS, 4),
                     "traffic": traffic_for(tile),
                     "flops_per_launch": flops_per_launch, "ms_per_launch": round(gemm_per_launch_ms, 5)},
    }
    if not args.skip_extras:
        log("bench: FP64 steps")
        total64, lat64, flops64, tm64, _ = timed_steps(ctx, dev, spamm.F64, args.steps, args.warmup)
        g64 = tm64["gemm_ms"] / max(tm64["gemm_launches"], 1)
        f64l = tm64["gemm_flops"] / max(tm64["gemm_launches"], 1)
        out["f64"] = {"value": round(flops64 / total64 / 1e9, 3), "unit": "GFLOP/s",
                      "ms_per_step": round(total64 / args.steps * 1e3, 4),
                      "multiplies_per_s": round(18 * args.steps / total64, 2),
                      "latency_ms": {"p50": round(pct(lat64, 0.5) * 1e3, 4),
                                     "p99": round(pct(lat64, 0.99) * 1e3, 4)},
                      "gemm_tflops": round(f64l / (g64 * 1e-3) / 1e12, 3),
                      "gemm_frac_of_fp64_peak": round(f64l / (g64 * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS, 4)}
        log("bench: errors and fixed-error rates")
        e32 = errors(ctx, dev, host, spamm.F32)
        e64 = errors(ctx, dev, host, spamm.F64)
        out["fixed_error"] = {
            "sigma": "1e-5 * ||A||_F * ||B||_F",
            "f32": fixed_error_rate(ctx, dev, spamm.F32, e32, 20),
            "f64": fixed_error_rate(ctx, dev, spamm.F64, e64, 20),
            # err <= bound + prec_bound: the approximation and the FP32 rounding
            "errors_f32": [{k: e[k] for k in ("alpha", "tau", "mode", "err", "bound", "prec_bound")}
                           for e in e32],
        }
        out["fixed_error"]["f32_over_f64"] = round(out["fixed_error"]["f32"]["multiplies_per_s"] /
                                                   out["fixed_error"]["f64"]["multiplies_per_s"], 3)
        # every FP32 error within the approximation bound plus the rounding bound
        out["fixed_error"]["bounds_hold"] = all(e["err"] <= e["bound"] + e["prec_bound"] for e in e32)
    if not args.skip_extras and not args.no_3d:
        log("bench: 3D decay n=32768")
        out["dense3d"] = dense3d(args.steps_3d)
    if not args.skip_extras and not args.no_purify:
        log("bench: purification n=32768")
        out["purification"] = purification(args.purify_steps)
    if not args.skip_extras and args.serve_requests > 0:
        log("bench: serving")
        out["serving"] = serving(args.serve_requests, args.serve_nmax)
    if args.paper_workloads:
        log("bench: the paper's model problem and leaf-library sweep")
        out["paper_workloads"] = paper_workloads()
    if not args.no_cpu_baseline:
        log("bench: oracle CPU baseline")
        out["cpu_baseline"] = cpu_baseline(host, args.cpu_seconds)
    ctx.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
