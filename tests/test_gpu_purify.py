"""Purification chain on the device against the oracle's chain: 3D decay
n = 2048 (256 atoms x 8 functions), leaf 64, Hybrid, tau = 1e-6, 20 SP2
steps, n_occ = n / 2.  The FP64 chain follows the oracle step by step
(trace, branch, products formed, iterate); the FP32 chain stays close to
the FP64 one."""
import numpy as np
import pytest

import oracle as O
import synth
from oracle import purify as PU
from paper_1906_08148_amd import purify, spamm

from parity import rel_fro

pytestmark = pytest.mark.gpu

N, LEAF, TAU, STEPS = 2048, 64, 1e-6, 20


def test_sp2_chain_matches_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    print("case: purification n=2048", flush=True)
    A = synth.DecaySpec("3d", N, 1.0, seed=1).dense()
    ref, (lo_r, hi_r) = PU.sp2_chain(A, LEAF, N / 2, TAU, STEPS, O.HYBRID)
    ctx = spamm.Context(arena_bytes=4 << 30)
    X = ctx.build(torch.from_numpy(A).cuda(), LEAF)
    ident = ctx.identity(N, LEAF)
    X0, tr0, lo, hi = purify.scale_unit(ctx, X, ident)
    assert abs(lo - lo_r) <= 1e-12 * abs(lo_r) and abs(hi - hi_r) <= 1e-12 * abs(hi_r)
    X064 = ctx.multiply(X0, ident, 0.0, mode=spamm.SPAMM, prec=spamm.F64).C
    c64 = purify.Chain(ctx, X0, tr0, N / 2, TAU, spamm.F64)
    c32 = purify.Chain(ctx, X064, tr0, N / 2, TAU, spamm.F32)
    for k in range(STEPS):
        s64 = c64.step(ident)
        s32 = c32.step(ident)
        r = ref[k]
        assert s64.branch == r["branch"], k
        assert abs(s64.trace - r["trace"]) <= 1e-10 * abs(r["trace"]), k
        assert s64.n_kept == r["n_kept"], k
        X64 = ctx.to_dense(c64.X).cpu().numpy()
        e = rel_fro(X64, r["X"])
        assert e <= 1e-10, (k, e)
        d = purify.diff_norm(ctx, c32.X, c64.X, ident) / np.linalg.norm(r["X"])
        print(f"  step {k}: branch {s64.branch} trace {s64.trace:.6f} kept {s64.n_kept} "
              f"fp64 rel {e:.2e} fp32-fp64 rel {d:.2e} idem {s64.idempotency:.3e}", flush=True)
        assert d <= 1e-3, (k, d)
    for m in (c64.X, c32.X, ident, X):
        m.release()
    ctx.close()
