"""Truncation of a product after the multiply (the removal of small leaves
from the product matrix, which the paper's Introduction names as common
practice besides truncation before it): spamm_truncate and its mirror-pair
form spamm_truncate_symmetric applied to C, against the oracle's truncation
of the oracle's C, and the SP2 purification chain with every iterate
truncated, against the oracle's chain of the same reading.

The budgets sit halfway between two consecutive prefix sums of the
oracle's ordered weights, and the two weights at the boundary differ by far
more than the rounding between the two C's (the oracle reports no tie), so
the drop set is the same on both sides."""
import numpy as np
import pytest

import oracle as O
import synth
from oracle import purify as PU
from paper_1906_08148_amd import purify, spamm

from parity import TOL, check_norms, check_product, rel_fro

pytestmark = pytest.mark.gpu
NRM_TOL = {spamm.F64: 1e-12, spamm.F32: 1e-5}


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    c = spamm.Context(arena_bytes=8 << 30)
    yield c
    c.close()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def unit_weights(T, pairs):
    """The oracle's truncation units of tree T in drop order: weights."""
    pres, sq = T.leaf_present, T.leaf_sq
    if pairs:
        I, K = np.nonzero(np.triu(pres | pres.T))
        w = np.where(I == K, sq[I, K], sq[I, K] + sq[K, I])
    else:
        I, K = np.nonzero(pres)
        w = sq[I, K]
    return np.sort(w)


def budgets(T, pairs, rel_gap):
    """tau values dropping about 10%, 50% and 90% of the units, each halfway
    between two prefix sums, at a boundary whose two weights differ by more
    than rel_gap."""
    w = unit_weights(T, pairs)
    cum = np.cumsum(w)
    out = []
    for f in (0.1, 0.5, 0.9):
        r = int(f * len(w))
        while r < len(w) - 1 and (w[r] - w[r - 1]) <= rel_gap * w[r]:
            r += 1
        out.append(float(np.sqrt(0.5 * (cum[r - 1] + cum[r]))))
    return out


def leaf_map(ctx, M):
    L = M.info.L
    return spamm.morton_order_to_grid(ctx.norms(M, L), L) > 0


@pytest.mark.parametrize("prec", [spamm.F64, spamm.F32])
@pytest.mark.parametrize("symmetric", [False, True])
def test_truncating_a_product(ctx, prec, symmetric):
    """C = A B (non-symmetric, the plain form) or A A (symmetric A, the pair
    form), then C truncated: drop set, dropped squared norm, leaves and norm
    pyramid against the oracle; the kept leaves are C's own, bit for bit."""
    print(f"case: post-multiplication truncation prec={prec} symmetric={symmetric}", flush=True)
    A = synth.DecaySpec("3d", 2048, 1.0, seed=21).dense()
    B = A if symmetric else synth.DecaySpec("1d", 2048, 0.05, seed=22).dense()
    TA = O.build(A, 64)
    TB = TA if symmetric else O.build(B, 64)
    MA = ctx.build(dev(A), 64, stores=spamm.STORE_F64 | spamm.STORE_F32)
    MB = MA if symmetric else ctx.build(dev(B), 64, stores=spamm.STORE_F64 | spamm.STORE_F32)
    p, ref, branch = check_product(ctx, MA, MB, TA, TB, 3e-3, spamm.HYBRID, prec, alias=symmetric)
    assert branch == "full"
    Cd = ctx.to_dense(p.C).cpu().numpy()
    rg = 1e-9 if prec == spamm.F64 else 1e-4
    for tau_c in budgets(ref.C, symmetric, rg):
        tr = (O.truncate_pairs if symmetric else O.truncate)(ref.C, tau_c)
        assert not tr.tie
        Ct, dropped = ctx.truncate(p.C, tau_c, symmetric=symmetric)
        keep = tr.tree.leaf_present
        assert Ct.info.nonnull == tr.tree.nonnull_count()
        assert np.array_equal(leaf_map(ctx, Ct), keep)
        assert abs(dropped - tr.dropped_sq) <= NRM_TOL[prec] * tr.dropped_sq
        assert dropped <= tau_c * tau_c
        check_norms(ctx, Ct, tr.tree, rtol=NRM_TOL[prec])
        got = ctx.to_dense(Ct).cpu().numpy()
        mask = np.kron(keep, np.ones((64, 64), dtype=bool))[:2048, :2048]
        assert np.array_equal(got, np.where(mask, Cd, 0.0))
        assert rel_fro(got, tr.tree.to_dense()) <= TOL[prec]
        if symmetric:
            assert np.array_equal(keep, keep.T)
        Ct.release()
    p.C.release()
    if MB is not MA:
        MB.release()
    MA.release()


def test_sp2_with_truncated_iterates_matches_oracle(ctx):
    """n = 2048 (256 atoms), leaf 64, the symmetric Hybrid square at
    tau = 1e-6, every iterate truncated in mirror pairs with tau_c = 1e-3
    (up to 48 leaves of 1024 go per step): the FP64 chain follows the
    oracle's step by step (trace, branch, products formed, leaves left,
    dropped norm, iterate); the FP32 chain stays close."""
    import torch
    n, steps, tau, tau_c = 2048, 12, 1e-6, 1e-3
    print("case: purification with truncated iterates, oracle chain", flush=True)
    A = synth.DecaySpec("3d", n, 1.0, seed=1).dense()
    ref, _ = PU.sp2_chain(A, 64, n / 2, tau, steps, O.HYBRID, sym=True, tau_c=tau_c)
    assert sum(r["dropped_sq"] > 0 for r in ref) >= 6
    print("case: purification with truncated iterates, device chains", flush=True)
    X = ctx.build(dev(A), 64)
    ident = ctx.identity(n, 64)
    X0, tr0, _, _ = purify.scale_unit(ctx, X, ident)
    X064 = ctx.multiply(X0, ident, 0.0, mode=spamm.SPAMM, prec=spamm.F64).C
    c64 = purify.Chain(ctx, X0, tr0, n / 2, tau, spamm.F64, spamm.HYBRID_SYM, tau_c)
    c32 = purify.Chain(ctx, X064, tr0, n / 2, tau, spamm.F32, spamm.HYBRID_SYM, tau_c)
    for k in range(steps):
        s64, s32 = c64.step(ident), c32.step(ident)
        r = ref[k]
        assert not r["trunc_tie"], k
        assert s64.branch == r["branch"], k
        assert abs(s64.trace - r["trace"]) <= 1e-10 * abs(r["trace"]), k
        assert s64.n_kept == r["n_kept"], k
        assert s64.nonnull == r["nonnull"], k
        assert abs(s64.dropped_sq - r["dropped_sq"]) <= 1e-9 * max(r["dropped_sq"], 1e-300), k
        assert s64.dropped_sq <= tau_c * tau_c
        e = rel_fro(ctx.to_dense(c64.X).cpu().numpy(), r["X"])
        d = purify.diff_norm(ctx, c32.X, c64.X, ident) / np.linalg.norm(r["X"])
        print(f"  step {k}: branch {s64.branch} kept {s64.n_kept} leaves {s64.nonnull} "
              f"dropped {s64.dropped_sq:.3e} fp64 rel {e:.2e} fp32-fp64 rel {d:.2e}", flush=True)
        assert e <= 1e-10, (k, e)
        assert d <= 1e-3, (k, d)
    for m in (c64.X, c32.X, ident, X):
        m.release()
    torch.cuda.synchronize()


def test_symmetric_truncation_edge_cases(ctx):
    """The mirror-pair form on its own: tau = 0 drops nothing, a budget
    above ||A||_F drops every leaf, and on random blocks (a null map that is
    not symmetric, ragged n) a leaf whose mirror is null is a unit alone of
    its own weight; against the oracle's pair truncation of the same input."""
    print("case: symmetric truncation edge cases", flush=True)
    A = synth.DecaySpec("3d", 1000, 1.0, seed=23).dense()  # G = 16, ragged
    T = O.build(A, 64)
    M = ctx.build(dev(A), 64)
    Mt, dropped = ctx.truncate(M, 0.0, symmetric=True)
    assert dropped == 0.0 and Mt.info.nonnull == M.info.nonnull
    Mt.release()
    Mt, dropped = ctx.truncate(M, 2.0 * T.fro(), symmetric=True)
    assert Mt.info.nonnull == 0
    assert not np.any(leaf_map(ctx, Mt))
    assert abs(dropped - T.fro() ** 2) <= 1e-12 * T.fro() ** 2
    Mt.release()
    M.release()
    c, d = synth.random_blocks(31, 1000, 64, 0.4)
    keep = ~((c[:, 0] > c[:, 1]) & ((c[:, 0] + c[:, 1]) % 3 == 0))  # some lower leaves lose their mirror
    c, d = c[keep], d[keep]
    T = O.build_from_blocks(1000, 64, c, d)
    assert not np.array_equal(T.leaf_present, T.leaf_present.T)
    M = ctx.build_blocks(1000, 64, dev(c.astype(np.int32)), dev(d))
    for tau in budgets(T, True, 1e-9):
        tr = O.truncate_pairs(T, tau)
        assert not tr.tie
        Mt, dropped = ctx.truncate(M, tau, symmetric=True)
        assert Mt.info.nonnull == tr.tree.nonnull_count()
        assert np.array_equal(leaf_map(ctx, Mt), tr.tree.leaf_present)
        assert abs(dropped - tr.dropped_sq) <= 1e-12 * tr.dropped_sq
        assert np.array_equal(ctx.to_dense(Mt).cpu().numpy(), tr.tree.to_dense())
        Mt.release()
    M.release()
