"""Quads of sibling C leaves (leaf 64, option gemm_quad, on by default):
the leaf GEMM that runs the up to four children of a quadtree node of C in
one workgroup over the merged k order of their products; at leaves 128 and
256 the same kernel runs a C leaf's 128 x 128 tile as a quad of its four
64 x 64 blocks.  Checked against the CPU oracle in
every scheme and precision (ragged tails, banded matrices whose quads have
one to four children, 3D decay with partial pruning), against the one-leaf
path, for repeatability, batches, C leaves from D alone, the symmetric
square and the captured graph."""
import numpy as np
import pytest

import oracle as O
import synth
from paper_1906_08148_amd import spamm

from parity import TOL, check_product, rel_fro

pytestmark = pytest.mark.gpu
MODES = (spamm.TRUNCMUL, spamm.SPAMM, spamm.HYBRID)
PRECS = (spamm.F64, spamm.F32, spamm.BF16, spamm.BF16X3)
ALL = spamm.STORE_F64 | spamm.STORE_F32 | spamm.STORE_BF16


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    c = spamm.Context(arena_bytes=8 << 30)
    c.set_option("gemm_quad", 1)
    yield c
    c.close()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


# (n, kind, alpha, tau, modes): no tie triple and no truncation tie in any
# listed scheme (checked on the oracle)
CASES = [
    (1500, "1d", 0.05, 1e-6, MODES),        # G = 32, ragged last leaf row, band: quads of 1-4 children
    (700, "1d", 0.3, 1e-4, MODES),          # narrow band, G = 16
    (2048, "3d", 1.0, 3e-3, MODES),         # 3D decay, some products pruned
    (3000, "3d", 1.0, 3e-3, (spamm.SPAMM,)),  # G = 64, ragged, a third of the products kept
    (50, "1d", 0.3, 1e-6, MODES),           # a single C leaf (one quad of one child)
    (100, "1d", 0.3, 1e-6, MODES),          # G = 2: one full quad
    (200, "1d", 0.05, 1e-5, MODES),         # G = 4, ragged
]


@pytest.mark.parametrize("quad", [1, 0])
@pytest.mark.parametrize("n,kind,alpha,tau,modes", CASES)
def test_quad_matches_the_oracle(ctx, n, kind, alpha, tau, modes, quad):
    """Quads (the default) and the one-leaf GEMM, against the oracle."""
    print(f"case: quad={quad} n={n} {kind} alpha={alpha} tau={tau}", flush=True)
    ctx.set_option("gemm_quad", quad)
    A = synth.DecaySpec(kind, n, alpha, seed=3).dense()
    B = A if kind == "3d" else synth.DecaySpec(kind, n, alpha * 1.5, seed=4).dense()
    TA = O.build(A, 64)
    TB = TA if B is A else O.build(B, 64)
    MA = ctx.build(dev(A), 64, stores=ALL)
    MB = MA if B is A else ctx.build(dev(B), 64, stores=ALL)
    for mode in modes:
        for prec in PRECS:
            p, _, _ = check_product(ctx, MA, MB, TA, TB, tau, mode, prec, alias=B is A)
            p.C.release()
    ctx.set_option("gemm_quad", 1)
    if MB is not MA:
        MB.release()
    MA.release()


def test_quad_equals_one_leaf_path(ctx):
    """Same kept products, accounting and C leaves as the one-leaf GEMM,
    within each precision's tolerance, and bitwise repeatable."""
    import torch
    print("case: quad vs one-leaf path", flush=True)
    A = synth.DecaySpec("3d", 4096, 1.0, seed=5).dense()
    M = ctx.build(dev(A), 64, stores=ALL)
    for prec in PRECS:
        ctx.set_option("gemm_quad", 0)
        ref = ctx.multiply(M, M, 1e-3, mode=spamm.HYBRID, prec=prec)
        ctx.set_option("gemm_quad", 1)
        q1 = ctx.multiply(M, M, 1e-3, mode=spamm.HYBRID, prec=prec)
        q2 = ctx.multiply(M, M, 1e-3, mode=spamm.HYBRID, prec=prec)
        for k in ("n_kept", "n_candidates", "c_nonnull", "B1", "B2", "err_bound", "prec_bound"):
            assert q1.stats[k] == ref.stats[k], k
        assert np.array_equal(ctx.kept(q1.C), ctx.kept(ref.C))
        assert np.array_equal(ctx.skipped_bound(q1.C), ctx.skipped_bound(ref.C))
        Cq, Cr = ctx.to_dense(q1.C), ctx.to_dense(q2.C)
        assert torch.equal(Cq, Cr), f"prec {prec}: not repeatable"
        assert np.array_equal(ctx.norms(q1.C, -1), ctx.norms(q2.C, -1))
        r = rel_fro(Cq.cpu().numpy(), ctx.to_dense(ref.C).cpu().numpy())
        assert r <= TOL[prec], (prec, r)
        nq, nr = ctx.norms(q1.C), ctx.norms(ref.C)
        assert np.allclose(nq, nr, rtol=4 * TOL[prec], atol=0), prec
        if prec == spamm.F64:
            assert abs(q1.stats["trace"] - ref.stats["trace"]) <= 1e-12 * abs(ref.stats["trace"])
        for p in (ref, q1, q2):
            p.C.release()
    M.release()


def test_quad_batch_equals_alone(ctx):
    """Quads never span requests: each request of a mixed batch (quads of
    sibling leaves, quads of 128- and 256-leaf blocks, and leaf 32 on the
    one-leaf kernel) gives the C it gives alone, bit for bit."""
    import torch
    print("case: quad batch vs alone", flush=True)
    A = synth.DecaySpec("3d", 2048, 0.8, seed=10).dense()
    B = synth.DecaySpec("1d", 2048, 0.05, seed=11).dense()
    MA, MB, M32 = ctx.build(dev(A), 64, stores=ALL), ctx.build(dev(B), 64, stores=ALL), ctx.build(dev(A), 32)
    M128, M256 = ctx.build(dev(B), 128), ctx.build(dev(A), 256)
    reqs = [dict(A=MA, B=MA, tau=1e-4, mode=spamm.HYBRID, prec=spamm.F32),
            dict(A=M128, B=M128, tau=1e-6, mode=spamm.SPAMM, prec=spamm.F64),
            dict(A=M256, B=M256, tau=1e-3, mode=spamm.HYBRID, prec=spamm.F64),
            dict(A=MB, B=MB, tau=1e-6, mode=spamm.SPAMM, prec=spamm.F32),
            dict(A=M32, B=M32, tau=1e-5, mode=spamm.SPAMM, prec=spamm.F32),
            dict(A=MA, B=MB, tau=1e-6, mode=spamm.TRUNCMUL, prec=spamm.BF16X3),
            dict(A=MB, B=MA, tau=1e-5, mode=spamm.SPAMM, prec=spamm.F64)]
    alone = [ctx.multiply_batch([q])[0] for q in reqs]
    batch = ctx.multiply_batch(reqs)
    for a, b in zip(alone, batch):
        assert torch.equal(ctx.to_dense(a.C), ctx.to_dense(b.C))
        a.C.release()
        b.C.release()
    for m in (MA, MB, M32, M128, M256):
        m.release()


def test_quad_epilogue_and_d_only_leaves(ctx):
    """alpha * AB + beta * D where the band of A A is narrower than D's: C
    leaves (whole quads among them) that come from D alone."""
    print("case: quad epilogue", flush=True)
    A = synth.DecaySpec("1d", 1500, 0.5, seed=6).dense()
    D = synth.dense_from_blocks(1500, 64, *synth.random_blocks(7, 1500, 64, 0.4))
    TA = O.build(A, 64)
    MA, MD = ctx.build(dev(A), 64), ctx.build(dev(D), 64)
    for prec in (spamm.F64, spamm.F32):
        p = ctx.multiply(MA, MA, 1e-9, mode=spamm.HYBRID, prec=prec, alpha=-1.0, beta=2.0, D=MD)
        ref = O.multiply(TA, TA, 1e-9, O.HYBRID)
        want = 2.0 * D - ref.C.to_dense()
        assert rel_fro(ctx.to_dense(p.C).cpu().numpy(), want) <= TOL[prec]
        assert p.C.info.nonnull == int((ref.C.leaf_present | O.build(D, 64).leaf_present).sum())
        assert abs(p.stats["trace"] - float(np.trace(want))) <= TOL[prec] * max(1.0, abs(float(np.trace(want))))
        p.C.release()
    MA.release()
    MD.release()


def test_quad_symmetric_square(ctx):
    """The symmetric square (upper C leaves formed, the lower ones mirrored)
    on quads, against the oracle's symmetric reading."""
    from test_gpu_symmetric import _check_sym
    print("case: quad symmetric square", flush=True)
    A = synth.DecaySpec("3d", 2048, 1.0, seed=8).dense()
    T = O.build(A, 64)
    M = ctx.build(dev(A), 64, stores=ALL)
    for mode, omode in ((spamm.SPAMM_SYM, O.SPAMM), (spamm.HYBRID_SYM, O.HYBRID)):
        ref = O.multiply_symmetric(T, 3e-3, omode)
        assert not ref.stats["trunc_tie"] and not ref.stats["sym_fallback"]
        for prec in (spamm.F64, spamm.F32, spamm.BF16X3):
            p = ctx.multiply(M, M, 3e-3, mode=mode, prec=prec)
            _check_sym(ctx, p, ref, T, prec, 3e-3)
            p.C.release()
    M.release()


def test_quad_graph_replays(ctx):
    """The quad plan and GEMM captured into the batch graph: every replay
    (with eager work between) equals the eager result."""
    import torch
    print("case: quad graph", flush=True)
    A = synth.DecaySpec("3d", 2048, 1.0, seed=12).dense()
    for leaf, prec in ((64, spamm.BF16X3), (128, spamm.F64)):  # quads of siblings, of a tile's blocks
        M = ctx.build(dev(A), leaf, stores=ALL)
        eager = ctx.multiply(M, M, 1e-3, mode=spamm.HYBRID, prec=prec)
        want = ctx.to_dense(eager.C)
        ctx.set_option("graph", 1)
        try:
            for _ in range(3):
                p = ctx.multiply(M, M, 1e-3, mode=spamm.HYBRID, prec=prec)
                assert torch.equal(ctx.to_dense(p.C), want)
                p.C.release()
                torch.cuda.synchronize()
        finally:
            ctx.set_option("graph", 0)
        eager.C.release()
        M.release()


def test_automatic_choice_follows_products_per_leaf(ctx):
    """With the default (-1) a launch group runs quads when its C leaves
    average enough kept products for its precision (FP64: 32, FP32: 128,
    the BF16 forms: 16): a 3D product of 64 products per C leaf runs FP32
    on the one-leaf GEMM and FP64 and split BF16 on quads, each bit for bit
    as when forced."""
    import torch
    print("case: automatic quad choice", flush=True)
    A = synth.DecaySpec("3d", 4096, 1.0, seed=13).dense()
    M = ctx.build(dev(A), 64, stores=ALL)
    for prec, want in ((spamm.F32, 0), (spamm.F64, 1), (spamm.BF16X3, 1)):
        ctx.set_option("gemm_quad", -1)
        ctx.timing(enable=True, reset=True)
        auto = ctx.multiply(M, M, 1e-9, mode=spamm.SPAMM, prec=prec)
        tm = ctx.timing(enable=False, reset=True)
        assert auto.stats["n_kept"] == 64 ** 3  # every product: 64 per C leaf
        assert tm["gemm_launches"] == 1 and tm["gemm_quad_launches"] == want, (prec, tm)
        ctx.set_option("gemm_quad", want)
        forced = ctx.multiply(M, M, 1e-9, mode=spamm.SPAMM, prec=prec)
        assert torch.equal(ctx.to_dense(auto.C), ctx.to_dense(forced.C))
        auto.C.release()
        forced.C.release()
    ctx.set_option("gemm_quad", 1)
    M.release()


# large leaves (128, 256): every work unit (a 128 x 128 tile of a C leaf) is
# one quad of its four 64 x 64 blocks, each product bs / 64 merged steps
BIG_CASES = [
    (1500, "1d", 0.05, 1e-6, 128),   # G = 12 -> 16, ragged, banded
    (2048, "3d", 1.0, 0.7, 128),     # pruning (no mirror pair split by the truncation)
    (1500, "1d", 0.05, 1e-6, 256),   # G = 6 -> 8, ragged, four tiles per leaf
    (2048, "3d", 1.0, 3.0, 256),
    (200, "1d", 0.05, 1e-5, 256),    # a single C leaf
]


@pytest.mark.parametrize("quad", [1, 0])
@pytest.mark.parametrize("n,kind,alpha,tau,leaf", BIG_CASES)
def test_large_leaf_quads_match_the_oracle(ctx, n, kind, alpha, tau, leaf, quad):
    """Leaves 128 and 256 on the quad kernel (the default) and on the
    one-leaf kernel, every scheme and precision, against the oracle."""
    print(f"case: large-leaf quad={quad} leaf={leaf} n={n} {kind} alpha={alpha} tau={tau}", flush=True)
    ctx.set_option("gemm_quad", quad)
    A = synth.DecaySpec(kind, n, alpha, seed=3).dense()
    B = A if kind == "3d" else synth.DecaySpec(kind, n, alpha * 1.5, seed=4).dense()
    TA = O.build(A, leaf)
    TB = TA if B is A else O.build(B, leaf)
    MA = ctx.build(dev(A), leaf, stores=ALL)
    MB = MA if B is A else ctx.build(dev(B), leaf, stores=ALL)
    for mode in MODES:
        for prec in PRECS:
            ctx.timing(enable=True, reset=True)
            p, _, _ = check_product(ctx, MA, MB, TA, TB, tau, mode, prec, alias=B is A)
            tm = ctx.timing(enable=False, reset=True)
            if p.stats["n_kept"] > 0:
                assert (tm["gemm_quad_launches"] > 0) == (quad == 1), tm
            p.C.release()
    ctx.set_option("gemm_quad", 1)
    if MB is not MA:
        MB.release()
    MA.release()


@pytest.mark.parametrize("leaf", [128, 256])
def test_large_leaf_quads_epilogue_and_symmetric(ctx, leaf):
    """alpha * AB + beta * D with C leaves from D alone, and the symmetric
    square, on large-leaf quads."""
    from test_gpu_symmetric import _check_sym
    print(f"case: large-leaf quad epilogue / symmetric leaf={leaf}", flush=True)
    A = synth.DecaySpec("1d", 1500, 0.5, seed=6).dense()
    D = synth.dense_from_blocks(1500, leaf, *synth.random_blocks(7, 1500, leaf, 0.5))
    TA = O.build(A, leaf)
    MA, MD = ctx.build(dev(A), leaf), ctx.build(dev(D), leaf)
    for prec in (spamm.F64, spamm.F32):
        p = ctx.multiply(MA, MA, 1e-9, mode=spamm.HYBRID, prec=prec, alpha=-1.0, beta=2.0, D=MD)
        ref = O.multiply(TA, TA, 1e-9, O.HYBRID)
        want = 2.0 * D - ref.C.to_dense()
        assert rel_fro(ctx.to_dense(p.C).cpu().numpy(), want) <= TOL[prec]
        assert p.C.info.nonnull == int((ref.C.leaf_present | O.build(D, leaf).leaf_present).sum())
        assert abs(p.stats["trace"] - float(np.trace(want))) <= TOL[prec] * max(1.0, abs(float(np.trace(want))))
        p.C.release()
    MA.release()
    MD.release()
    S = synth.DecaySpec("3d", 2048, 1.0, seed=8).dense()
    T = O.build(S, leaf)
    M = ctx.build(dev(S), leaf, stores=ALL)
    ref = O.multiply_symmetric(T, 3e-3, O.SPAMM)
    assert not ref.stats["trunc_tie"] and not ref.stats["sym_fallback"]
    for prec in (spamm.F64, spamm.F32, spamm.BF16X3):
        p = ctx.multiply(M, M, 3e-3, mode=spamm.SPAMM_SYM, prec=prec)
        _check_sym(ctx, p, ref, T, prec, 3e-3)
        p.C.release()
    M.release()
