"""Leaf size and GEMM tile autotuner.

The leaf size trades pruning resolution against per-product efficiency: a
smaller leaf skips more negligible work (finer norm tests) but each product
is a smaller matrix multiply.  The GEMM tile variant (32 x 32 or 16 x 16
MFMA tiles for FP32 / BF16) changes the register budget and the issue
pattern of the leaf GEMM.  The tuner times the full multiply (prune + GEMM +
epilogue) for every candidate on the device and keeps the fastest; choices
are cached per workload signature and can be saved as JSON.
"""
import json
import math
import time

from . import spamm as S


def signature(kind: str, n: int, alpha: float, tau: float, mode: int, prec: int):
    """Workloads that share a signature are expected to share a best config:
    n by powers of two, alpha by halvings, tau by decades."""
    return (kind, int(round(math.log2(max(n, 1)))), int(round(math.log2(max(alpha, 1e-9)))),
            int(round(math.log10(max(tau, 1e-300)))) if tau > 0 else -999, int(mode), int(prec))


def _time_multiply(ctx, M, tau, mode, prec, reps):
    import torch
    p = ctx.multiply(M, M, tau, mode=mode, prec=prec)  # warm (derives compute copies)
    p.C.release()
    torch.cuda.synchronize()
    ts = []
    stats = None
    for _ in range(reps):
        t0 = time.perf_counter()
        p = ctx.multiply(M, M, tau, mode=mode, prec=prec)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        stats = p.stats
        p.C.release()
    return sorted(ts)[len(ts) // 2], stats


def choose(candidates, measure):
    """Run `measure(leaf, tile) -> seconds` over the candidates and return
    (best (leaf, tile), table).  Pure selection logic (testable without a
    device)."""
    table = []
    for leaf, tile in candidates:
        t = measure(leaf, tile)
        table.append({"leaf": leaf, "tile": tile, "seconds": t})
    best = min(table, key=lambda r: (r["seconds"], r["leaf"], r["tile"]))
    return (best["leaf"], best["tile"]), table


class Tuner:
    def __init__(self, ctx: S.Context, leaves=(32, 64, 128), tiles=(0, 1), reps=3):
        self.ctx, self.leaves, self.tiles, self.reps = ctx, leaves, tiles, reps
        self.cache = {}

    def tune(self, make_matrix, sig, tau, mode, prec):
        """`make_matrix(leaf)` builds the workload's matrix in this context.
        Returns {"leaf", "tile", "table"}; sets the context's tile option."""
        if sig in self.cache:
            best = self.cache[sig]
            self.ctx.set_option("gemm_tile", best["tile"])
            return best
        tiles = self.tiles if prec != S.F64 else (0,)
        built = {}
        extra = {}

        def measure(leaf, tile):
            if leaf not in built:
                built[leaf] = make_matrix(leaf)
            self.ctx.set_option("gemm_tile", tile)
            t, st = _time_multiply(self.ctx, built[leaf], tau, mode, prec, self.reps)
            extra[(leaf, tile)] = {"n_kept": int(st["n_kept"]), "flops": float(st["flops"])}
            return t

        (leaf, tile), table = choose([(l, t) for l in self.leaves for t in tiles], measure)
        for r in table:
            r.update(extra[(r["leaf"], r["tile"])])
        for M in built.values():
            M.release()
        self.ctx.set_option("gemm_tile", tile)
        best = {"leaf": leaf, "tile": tile, "table": table}
        self.cache[sig] = best
        return best

    def save(self, path):
        json.dump({json.dumps(list(k)): v for k, v in self.cache.items()}, open(path, "w"), indent=1)

    def load(self, path):
        for k, v in json.load(open(path)).items():
            self.cache[tuple(json.loads(k))] = v
