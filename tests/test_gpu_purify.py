"""Purification chain on the device against the oracle's chain: 3D decay,
leaf 64, Hybrid, tau = 1e-6, 20 SP2 steps, n_occ = n / 2.

* n = 2048 (256 atoms) and n = 4096 (512 atoms, an 8^3 cube): the FP64
  chain follows the oracle step by step (trace, branch, products formed,
  iterate); the FP32 chain stays close to the FP64 one.  Both with the
  plain Hybrid square and with the symmetric square (upper C leaves formed,
  the rest mirrored, pair truncation).
* n = 32768 (the 16^3 cube): the first step, against the oracle's first
  step -- scaling bounds, branch, kept list triple for triple, the step's
  accounting and sampled leaves of X_1."""
import numpy as np
import pytest

import oracle as O
import synth
from oracle import purify as PU
from paper_1906_08148_amd import purify, spamm

from parity import TIE_BAND, _leaf_k_sets, compare_kept, rel_fro

pytestmark = pytest.mark.gpu

LEAF, TAU, STEPS = 64, 1e-6, 20


@pytest.mark.parametrize("n,sym", [(2048, False), (4096, False), (2048, True), (4096, True)])
def test_sp2_chain_matches_oracle(n, sym):
    """sym: every square is the symmetric square (HYBRID_SYM, pair
    truncation), against the oracle's chain of the same reading."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    print(f"case: purification n={n} sym={sym} oracle chain", flush=True)
    A = synth.DecaySpec("3d", n, 1.0, seed=1).dense()
    ref, (lo_r, hi_r) = PU.sp2_chain(A, LEAF, n / 2, TAU, STEPS, O.HYBRID, sym=sym)
    mode = spamm.HYBRID_SYM if sym else spamm.HYBRID
    print(f"case: purification n={n} device chains", flush=True)
    ctx = spamm.Context(arena_bytes=8 << 30)
    X = ctx.build(torch.from_numpy(A).cuda(), LEAF)
    ident = ctx.identity(n, LEAF)
    X0, tr0, lo, hi = purify.scale_unit(ctx, X, ident)
    assert abs(lo - lo_r) <= 1e-12 * abs(lo_r) and abs(hi - hi_r) <= 1e-12 * abs(hi_r)
    X064 = ctx.multiply(X0, ident, 0.0, mode=spamm.SPAMM, prec=spamm.F64).C
    c64 = purify.Chain(ctx, X0, tr0, n / 2, TAU, spamm.F64, mode)
    c32 = purify.Chain(ctx, X064, tr0, n / 2, TAU, spamm.F32, mode)
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


def test_sp2_first_step_full_size():
    """n = 32768: the oracle runs the scaling and step 1 with its kept list
    and accounting in full and the iterate on sampled leaves."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    n = 32768
    print("case: purification n=32768 step 1 oracle", flush=True)
    A = synth.DecaySpec("3d", n, 1.0, seed=1).dense()
    X0r, lo_r, hi_r = PU.scale_unit(A)
    T0 = O.build(X0r, LEAF)
    G = T0.G
    rng = np.random.default_rng(17)
    sample = sorted({(i, i) for i in range(0, G, 16)} |
                    {tuple(int(v) for v in x) for x in rng.integers(0, G, size=(64, 2))})
    ref = O.multiply(T0, T0, TAU, O.HYBRID, c_blocks=sample)
    ties = O.tie_triples(ref.A_used, ref.B_used, TAU, TIE_BAND)
    tr0 = float(np.trace(X0r))
    branch_r = 0 if tr0 > n / 2 else 1
    print("case: purification n=32768 step 1 device", flush=True)
    ctx = spamm.Context(arena_bytes=64 << 30)
    dA = torch.from_numpy(A).cuda()
    X = ctx.build(dA, LEAF, stores=spamm.STORE_F64)
    del dA
    ident = ctx.identity(n, LEAF, stores=spamm.STORE_F64)
    X0, tr0g, lo, hi = purify.scale_unit(ctx, X, ident)
    assert abs(lo - lo_r) <= 1e-12 * abs(lo_r) and abs(hi - hi_r) <= 1e-12 * abs(hi_r)
    assert abs(tr0g - tr0) <= 1e-10 * abs(tr0)
    X0_of = dict(zip(sample, ctx.leaves(X0, sample)))
    c64 = purify.Chain(ctx, X0, tr0g, n / 2, TAU, spamm.F64)
    s = c64.step(ident)
    assert s.branch == branch_r
    # X_0 is formed in a different order on the two sides, so its leaf
    # norms may differ in the last bits, and X_0 is symmetric, so mirror
    # leaves of equal norm can straddle the truncation boundary (a tie):
    # with no tie the kept lists and the accounting match exactly; with a
    # truncation tie the products of the leaves dropped on one side only may
    # differ, and the sampled leaves are compared where the kept sets agree
    gk = ctx.kept(c64.X)
    if not ref.stats["trunc_tie"]:
        ndiff = compare_kept(gk, ref.kept, ties, G)
        if ndiff == 0:
            assert s.n_kept == ref.stats["n_kept"]
            assert s.stats["c_nonnull"] == ref.stats["c_nonnull"]
        assert s.stats["n_candidates"] == ref.stats["n_candidates"]
        assert abs(s.stats["err_bound"] - ref.stats["err_bound"]) <= 1e-10 * ref.stats["err_bound"]
    else:
        ndiff = -1
        # the drop sets differ by at most the straddling run
        assert abs(s.n_kept - ref.stats["n_kept"]) <= 4 * G
        assert s.stats["dA"] <= TAU and ref.stats["dA"] <= TAU
    ks_g, ks_r = _leaf_k_sets(gk), _leaf_k_sets(ref.kept)
    sample = [ij for ij in sample if ks_g.get(ij) == ks_r.get(ij)]
    assert len(sample) >= 64
    want = np.stack([ref.C.leaf(I, J) if ref.C.index[I, J] >= 0 else np.zeros((LEAF, LEAF))
                     for I, J in sample])
    if branch_r == 1:
        want = 2.0 * np.stack([X0_of[ij] for ij in sample]) - want
    got = ctx.leaves(c64.X, sample)
    r = rel_fro(got, want)
    print(f"  step 1: branch {s.branch} kept {s.n_kept} ties {len(ties)} differing {ndiff} "
          f"sampled rel {r:.3e}", flush=True)
    assert r <= 1e-12
    for m in (c64.X, ident, X):
        m.release()
    ctx.close()
