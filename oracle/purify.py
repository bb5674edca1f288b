"""Oracle for the purification chain that drives repeated SpAMM products.

Test infrastructure only: tests, the smoke check and the benchmark's CPU
baseline may import it; the library never does.

The paper motivates SpAMM by density-matrix purification (Introduction):
X_{k+1} = X_k^2 or 2 X_k - X_k^2, a map that sends every eigenvalue in
[0, 1] towards 0 or 1.  The choice between the two follows the trace (the
second-order spectral projection scheme, SP2): squaring lowers the trace,
2X - X^2 raises it, and the target trace is the number of occupied states.
Before the chain, the spectrum is mapped into [0, 1] with Gershgorin bounds,
X_0 = (hi I - A) / (hi - lo), so the smallest eigenvalues of A land near 1.
Every product is the oracle's multiply (a chosen scheme and tau), in FP64.
Optionally each new iterate is truncated after the product (the removal of
small leaves from the product matrix that the paper's Introduction reports
as common practice besides truncation before the multiply): the leaf-block
truncation of Sec. 3 with its own budget tau_c, in mirror pairs since the
iterates are symmetric (``truncate_pairs``), so ||X - X~||_F <= tau_c.
"""
import numpy as np

from . import spamm_oracle as O


def gershgorin(A: np.ndarray):
    """(lo, hi): every eigenvalue of A lies in [lo, hi] (Gershgorin discs)."""
    A = np.asarray(A, dtype=np.float64)
    d = np.diag(A)
    r = np.abs(A).sum(axis=1) - np.abs(d)
    return float(np.min(d - r)), float(np.max(d + r))


def scale_unit(A: np.ndarray):
    """X_0 = (hi I - A) / (hi - lo) with Gershgorin bounds; returns (X_0, lo, hi)."""
    lo, hi = gershgorin(A)
    n = A.shape[0]
    X0 = (hi * np.eye(n) - A) / (hi - lo)
    return X0, lo, hi


def sp2_chain(A: np.ndarray, bs: int, n_occ: float, tau: float, steps: int, mode: int = O.HYBRID,
              sym: bool = False, tau_c: float = 0.0):
    """Run `steps` SP2 steps on A scaled into [0, 1].  Each record holds the
    trace the decision used, the branch (0: X^2, 1: 2X - X^2), the number of
    leaf products formed and the new iterate (dense FP64).  With `sym` every
    square is the symmetric square (``multiply_symmetric``): the iterates
    stay exactly symmetric.  With tau_c > 0 every new iterate is truncated
    in mirror pairs (``truncate_pairs``, budget tau_c) before it is used; the
    record then also holds the squared norm dropped, the leaves left and
    whether the truncation boundary was a tie."""
    X, lo, hi = scale_unit(A)
    out = []
    for _ in range(steps):
        T = O.build(X, bs)
        tr = float(np.trace(X))
        r = O.multiply_symmetric(T, tau, mode) if sym else O.multiply(T, T, tau, mode)
        X2 = r.C.to_dense()
        if tr > n_occ:
            Xn, branch = X2, 0
        else:
            Xn, branch = 2.0 * X - X2, 1
        rec = dict(trace=tr, branch=branch, n_kept=int(r.stats["n_kept"]))
        if tau_c > 0.0:
            t = O.truncate_pairs(O.build(Xn, bs), tau_c)
            Xn = t.tree.to_dense()
            rec.update(dropped_sq=t.dropped_sq, nonnull=t.tree.nonnull_count(), trunc_tie=t.tie)
        rec["X"] = Xn
        out.append(rec)
        X = Xn
    return out, (lo, hi)
