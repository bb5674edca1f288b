"""Leaf size, GEMM tile and C blocks per workgroup autotuner.

The leaf size trades pruning resolution against per-product efficiency: a
smaller leaf skips more negligible work (finer norm tests) but each product
is a smaller matrix multiply.  A different leaf also changes which products
are kept, and so the error of the result at the same tau (the paper picks a
different tau per block size for the same accuracy, Sec. 5.3).  The GEMM
tile variant (32 x 32 or 16 x 16 MFMA tiles for FP32 / BF16) changes the
register budget and the issue pattern of the leaf GEMM.  At leaf 64 the
GEMM can also run the four sibling C leaves of a quadtree node in one
workgroup (quads, option gemm_quad), which halves the operand loads where
siblings share their k and costs time where they do not; at leaves 128 and
256 the same kernel runs a C leaf's 128 x 128 tile as a quad of its 64 x 64
blocks.

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


def candidates(leaves, tiles, quads=True):
    """(leaf, tile, quad) to try: every leaf with every tile on one C leaf
    (or 128-tile) per workgroup, and at leaves 64 to 256 quads once each
    (they take 16 x 16 tiles whatever the tile option says)."""
    out = [(l, t, 0) for l in leaves for t in tiles]
    if quads:
        out += [(l, 1, 1) for l in leaves if l >= 64]
    return out


def choose(cands, measure, budget=None):
    """Run `measure(leaf, tile, quad) -> (seconds, error)` over the
    candidates and return (best (leaf, tile, quad) or None, table).  A
    candidate whose error is above `budget` (None: no budget) is rejected
    whatever its time; the fastest admissible one wins, ties going to the
    smaller leaf, then tile, then one C leaf per workgroup.  None when no
    candidate meets the budget.  Pure selection logic (testable without a
    device)."""
    table = []
    for leaf, tile, quad in cands:
        t, err = measure(leaf, tile, quad)
        ok = budget is None or (err is not None and err <= budget)
        table.append({"leaf": leaf, "tile": tile, "quad": quad, "seconds": t, "error": err, "admissible": ok})
    admissible = [r for r in table if r["admissible"]]
    if not admissible:
        return None, table
    best = min(admissible, key=lambda r: (r["seconds"], r["leaf"], r["tile"], r["quad"]))
    return (best["leaf"], best["tile"], best["quad"]), table


class Tuner:
    def __init__(self, ctx: S.Context, leaves=(32, 64, 128, 256), tiles=(0, 1), reps=3, quads=True):
        self.ctx, self.leaves, self.tiles, self.reps, self.quads = ctx, leaves, tiles, reps, quads
        self.cache = {}

    def _apply(self, best):
        if best["tile"] is not None:
            self.ctx.set_option("gemm_tile", best["tile"])
            self.ctx.set_option("gemm_quad", best.get("quad", 0))

    def tune(self, make_matrix, sig, tau, mode, prec, budget=None, error_fn=None):
        """`make_matrix(leaf)` builds the workload's matrix in this context.
        `budget` bounds ||A B - C||_F; each candidate's error is
        error_fn(ctx, product) when given, else the product's err_bound +
        prec_bound.  Returns {"leaf", "tile", "quad", "table"} (None when
        no candidate meets the budget); sets the context's tile and quad
        options to the winner's."""
        key = (sig, budget)
        if key in self.cache:
            best = self.cache[key]
            self._apply(best)
            return best
        tiles = self.tiles if prec != S.F64 else (0,)
        built = {}
        extra = {}

        def measure(leaf, tile, quad):
            if leaf not in built:  # one leaf size resident at a time (candidates go leaf by leaf)
                for M in built.values():
                    M.release()
                built.clear()
                built[leaf] = make_matrix(leaf)
            self.ctx.set_option("gemm_tile", tile)
            self.ctx.set_option("gemm_quad", quad)
            t, st = _time_multiply(self.ctx, built[leaf], tau, mode, prec, self.reps)
            if error_fn is not None:
                p = self.ctx.multiply(built[leaf], built[leaf], tau, mode=mode, prec=prec)
                err = float(error_fn(self.ctx, p))
                p.C.release()
            else:
                err = float(st["err_bound"] + st["prec_bound"])
            extra[(leaf, tile, quad)] = {"n_kept": int(st["n_kept"]), "flops": float(st["flops"])}
            return t, err

        pick, table = choose(candidates(self.leaves, tiles, self.quads), measure, budget)
        for r in table:
            r.update(extra[(r["leaf"], r["tile"], r["quad"])])
        for M in built.values():
            M.release()
        leaf, tile, quad = pick if pick is not None else (None, None, None)
        best = {"leaf": leaf, "tile": tile, "quad": quad, "table": table, "budget": budget}
        self._apply(best)
        self.cache[key] = best
        return best

    def save(self, path):
        json.dump({json.dumps(list(k)): v for k, v in self.cache.items()}, open(path, "w"), indent=1)

    def load(self, path):
        for k, v in json.load(open(path)).items():
            self.cache[tuple(json.loads(k))] = v
