"""Leaf size and GEMM tile autotuner.

The leaf size trades pruning resolution against per-product efficiency: a
smaller leaf skips more negligible work (finer norm tests) but each product
is a smaller matrix multiply.  A different leaf also changes which products
are kept, and so the error of the result at the same tau (the paper picks a
different tau per block size for the same accuracy, Sec. 5.3).  The GEMM
tile variant (32 x 32 or 16 x 16 MFMA tiles for FP32 / BF16) changes the
register budget and the issue pattern of the leaf GEMM.

For every candidate the tuner times the full multiply (prune + GEMM +
epilogue) on the device and takes its error: by default the library's
guaranteed bound on ||A B - C||_F (the approximation bound plus the
rounding bound of the compute precision), or a measured error when the
caller gives a function for it.  Candidates whose error exceeds the
request's budget are rejected; the fastest of the rest wins.  Choices are
cached per workload signature and can be saved as JSON.
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


def choose(candidates, measure, budget=None):
    """Run `measure(leaf, tile) -> (seconds, error)` over the candidates and
    return (best (leaf, tile) or None, table).  A candidate whose error is
    above `budget` (None: no budget) is rejected whatever its time; the
    fastest admissible one wins, ties going to the smaller leaf, then tile.
    None when no candidate meets the budget.  Pure selection logic
    (testable without a device)."""
    table = []
    for leaf, tile in candidates:
        t, err = measure(leaf, tile)
        ok = budget is None or (err is not None and err <= budget)
        table.append({"leaf": leaf, "tile": tile, "seconds": t, "error": err, "admissible": ok})
    admissible = [r for r in table if r["admissible"]]
    if not admissible:
        return None, table
    best = min(admissible, key=lambda r: (r["seconds"], r["leaf"], r["tile"]))
    return (best["leaf"], best["tile"]), table


class Tuner:
    def __init__(self, ctx: S.Context, leaves=(32, 64, 128, 256), tiles=(0, 1), reps=3):
        self.ctx, self.leaves, self.tiles, self.reps = ctx, leaves, tiles, reps
        self.cache = {}

    def tune(self, make_matrix, sig, tau, mode, prec, budget=None, error_fn=None):
        """`make_matrix(leaf)` builds the workload's matrix in this context.
        `budget` bounds ||A B - C||_F; each candidate's error is
        error_fn(ctx, product) when given, else the product's err_bound +
        prec_bound.  Returns {"leaf", "tile", "table"} (leaf and tile None
        when no candidate meets the budget); sets the context's tile option
        to the winner's."""
        key = (sig, budget)
        if key in self.cache:
            best = self.cache[key]
            if best["tile"] is not None:
                self.ctx.set_option("gemm_tile", best["tile"])
            return best
        tiles = self.tiles if prec != S.F64 else (0,)
        built = {}
        extra = {}

        def measure(leaf, tile):
            if leaf not in built:  # one leaf size resident at a time (candidates go leaf by leaf)
                for M in built.values():
                    M.release()
                built.clear()
                built[leaf] = make_matrix(leaf)
            self.ctx.set_option("gemm_tile", tile)
            t, st = _time_multiply(self.ctx, built[leaf], tau, mode, prec, self.reps)
            if error_fn is not None:
                p = self.ctx.multiply(built[leaf], built[leaf], tau, mode=mode, prec=prec)
                err = float(error_fn(self.ctx, p))
                p.C.release()
            else:
                err = float(st["err_bound"] + st["prec_bound"])
            extra[(leaf, tile)] = {"n_kept": int(st["n_kept"]), "flops": float(st["flops"])}
            return t, err

        pick, table = choose([(l, t) for l in self.leaves for t in tiles], measure, budget)
        for r in table:
            r.update(extra[(r["leaf"], r["tile"])])
        for M in built.values():
            M.release()
        leaf, tile = pick if pick is not None else (None, None)
        if tile is not None:
            self.ctx.set_option("gemm_tile", tile)
        best = {"leaf": leaf, "tile": tile, "table": table, "budget": budget}
        self.cache[key] = best
        return best

    def save(self, path):
        json.dump({json.dumps(list(k)): v for k, v in self.cache.items()}, open(path, "w"), indent=1)

    def load(self, path):
        for k, v in json.load(open(path)).items():
            self.cache[tuple(json.loads(k))] = v
