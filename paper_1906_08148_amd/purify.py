"""Density-matrix purification driven by the library's products.

The paper motivates SpAMM by purification (Introduction): X <- X^2 or
2X - X^2 until X is a projector.  This driver runs the second-order
trace-driven scheme (SP2) with every matrix operation done by the library:

* spectrum bounds: spamm_gershgorin on the quadtree;
* X_0 = (hi I - X) / (hi - lo): one FP64 product X * I with the epilogue
  alpha = -1 / (hi - lo), beta = hi / (hi - lo), D = I (X * I is exact);
* X_{k+1} = X_k^2 (trace above the target) or 2 X_k - X_k^2 (epilogue
  alpha = -1, beta = 2, D = X_k), each an approximate product with the chosen
  scheme, tau and precision; the trace comes from the product's statistics;
* differences ||A - B||_F: the FP64 product A * I with alpha = 1, beta = -1,
  D = B, whose C norm the library reports.  Since both branches give
  X_{k+1} - X_k = +-(X_k^2 - X_k), the step difference is the idempotency
  error of X_k;
* optionally (tau_c > 0) each new iterate is truncated after its product,
  the removal of small leaves from the product that the paper's
  Introduction names as common practice: the leaf-block truncation of
  Sec. 3 with budget tau_c, in mirror pairs (spamm_truncate_symmetric; the
  iterates are symmetric, and a pair is never split by rounding), so the
  lightest pairs go while their squared norms sum to at most tau_c^2.  The
  trace is the product's unless a diagonal leaf was removed, then that of
  the truncated iterate.
"""
import numpy as np
from dataclasses import dataclass, field

from . import spamm as S


@dataclass
class Step:
    k: int
    trace: float          # trace of X_k (decides the branch)
    branch: int           # 0: X^2, 1: 2X - X^2
    n_kept: int
    flops: float
    seconds: float
    idempotency: float    # ||C - X_k||_F = ||X_k^2 - X_k||_F (C: the product, before any truncation)
    stats: dict = field(default_factory=dict)
    dropped_sq: float = 0.0   # squared norm removed by the truncation after the product
    nonnull: int = 0          # non-null leaves of X_{k+1}


class Chain:
    """One SP2 chain in one precision; keeps only the current iterate."""

    def __init__(self, ctx: S.Context, X0: S.Matrix, trace0: float, n_occ: float, tau: float, prec: int,
                 mode: int = S.HYBRID, tau_c: float = 0.0):
        self.ctx, self.X, self.trace = ctx, X0, trace0
        self.n_occ, self.tau, self.prec, self.mode = n_occ, tau, prec, mode
        self.tau_c = tau_c
        self.k = 0

    def step(self, ident: S.Matrix) -> Step:
        import time
        import torch
        ctx, X = self.ctx, self.X
        branch = 0 if self.trace > self.n_occ else 1
        t0 = time.perf_counter()
        if branch == 0:
            p = ctx.multiply(X, X, self.tau, mode=self.mode, prec=self.prec)
        else:
            p = ctx.multiply(X, X, self.tau, mode=self.mode, prec=self.prec, alpha=-1.0, beta=2.0, D=X)
        C, trace, dropped = p.C, float(p.stats["trace"]), 0.0
        if self.tau_c > 0.0:
            Ct, dropped = ctx.truncate(C, self.tau_c, symmetric=True)
            if not np.array_equal(diag_leaves(ctx, Ct), diag_leaves(ctx, C)):
                trace = trace_of(ctx, Ct, ident)
        else:
            Ct = C
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        idem = diff_norm(ctx, C, X, ident)
        rec = Step(self.k, self.trace, branch, int(p.stats["n_kept"]), float(p.stats["flops"]), dt, idem,
                   dict(p.stats), dropped, int(Ct.info.nonnull))
        if Ct is not C:
            C.release()  # the truncated handle keeps the leaves it shares
        X.release()
        self.X, self.trace = Ct, trace
        self.k += 1
        return rec


def diag_leaves(ctx: S.Context, M: S.Matrix) -> np.ndarray:
    """Which diagonal leaves of M have a non-zero norm."""
    L = M.info.L
    return np.diag(S.morton_order_to_grid(ctx.norms(M, L), L)) > 0


def trace_of(ctx: S.Context, M: S.Matrix, ident: S.Matrix) -> float:
    """trace(M) in FP64 via M * I (exact)."""
    p = ctx.multiply(M, ident, 0.0, mode=S.SPAMM, prec=S.F64)
    v = float(p.stats["trace"])
    p.C.release()
    return v


def diff_norm(ctx: S.Context, A: S.Matrix, B: S.Matrix, ident: S.Matrix) -> float:
    """||A - B||_F in FP64 via C = 1 * (A I) - 1 * B."""
    p = ctx.multiply(A, ident, 0.0, mode=S.SPAMM, prec=S.F64, alpha=1.0, beta=-1.0, D=B)
    v = float(p.stats["normC"])
    p.C.release()
    return v


def scale_unit(ctx: S.Context, X: S.Matrix, ident: S.Matrix):
    """X_0 = (hi I - X) / (hi - lo) with Gershgorin bounds; returns (X_0,
    trace of X_0, lo, hi)."""
    lo, hi = ctx.gershgorin(X)
    d = hi - lo
    p = ctx.multiply(X, ident, 0.0, mode=S.SPAMM, prec=S.F64, alpha=-1.0 / d, beta=hi / d, D=ident)
    return p.C, float(p.stats["trace"]), lo, hi


def sp2(ctx: S.Context, X: S.Matrix, n_occ: float, tau: float, steps: int, precs=(S.F64, S.F32),
        mode: int = S.HYBRID, tau_c: float = 0.0):
    """Run one chain per precision side by side for `steps` steps (each
    iterate truncated with budget tau_c when tau_c > 0); every step also
    records ||X_k^(p) - X_k^(first precision)||_F.  Returns {prec: [Step]},
    {prec: [difference per step]}, (lo, hi)."""
    n, leaf = X.info.n, X.info.leaf
    ident = ctx.identity(n, leaf, stores=S.STORE_F64 | S.STORE_F32)
    X0, tr0, lo, hi = scale_unit(ctx, X, ident)
    chains = {}
    for i, pr in enumerate(precs):
        if i == 0:
            Xi = X0
        else:  # an independent copy of X_0 (X_0 * I, exact)
            p = ctx.multiply(X0, ident, 0.0, mode=S.SPAMM, prec=S.F64)
            Xi = p.C
        chains[pr] = Chain(ctx, Xi, tr0, n_occ, tau, pr, mode, tau_c)
    recs = {pr: [] for pr in precs}
    diffs = {pr: [] for pr in precs[1:]}
    for _ in range(steps):
        for pr in precs:
            recs[pr].append(chains[pr].step(ident))
        for pr in precs[1:]:
            diffs[pr].append(diff_norm(ctx, chains[pr].X, chains[precs[0]].X, ident))
    for c in chains.values():
        c.X.release()
    ident.release()
    return recs, diffs, (lo, hi)
