"""GPU parity: the library (through the C-ABI) against the CPU oracle on the
same seeded inputs -- kept products exactly (outside the 1e-12 tie band),
C within 1e-12 (FP64) / 1e-5 (FP32) relative Frobenius, norms within 1e-14."""
import numpy as np
import pytest

import oracle as O
import synth
from paper_1906_08148_amd import spamm

from parity import TOL, check_norms, check_product, compare_kept, rel_fro

pytestmark = pytest.mark.gpu
MODES = (spamm.TRUNCMUL, spamm.SPAMM, spamm.HYBRID)


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    c = spamm.Context(arena_bytes=6 << 30)
    yield c
    c.close()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def sparse_random(n, bs, fill, seed):
    coords, data = synth.random_blocks(seed, n, bs, fill)
    return synth.dense_from_blocks(n, bs, coords, data)


def test_config1_all_modes(ctx):
    """n=1024, leaf 32, 1D alpha=0.5, tau=1e-6, A = B symmetric."""
    print("case: config1 n=1024 bs=32", flush=True)
    A = synth.DecaySpec("1d", 1024, 0.5, seed=1).dense()
    T = O.build(A, 32)
    M = ctx.build(dev(A), 32)
    assert M.info.nonnull == T.nonnull_count()
    check_norms(ctx, M, T)
    for mode in MODES:
        for prec in (spamm.F64, spamm.F32):
            check_product(ctx, M, M, T, T, 1e-6, mode, prec, alias=True)


@pytest.mark.parametrize("n,bs,kind,alpha,tau,full", [
    (1000, 32, "1d", 0.3, 2e-5, True),    # ragged tail, not a power of two
    (1000, 32, "1d", 0.3, 1e-5, False),   # the same with a tie at B's truncation boundary
    (300, 16, "rand", 0.3, 1e-2, True),   # random sparse blocks
    (2100, 64, "1d", 0.2, 1e-6, True),    # several tiles + ragged
    (700, 128, "3d", 1.0, 1e-4, True),    # 3D decay, big leaves
    (17, 16, "1d", 0.5, 1e-3, True),      # G = 2 with a 1-row tail
    (20, 32, "1d", 0.5, 1e-3, True),      # single leaf (L = 0)
])
def test_shapes_and_leaf_sizes(ctx, n, bs, kind, alpha, tau, full):
    print(f"case: n={n} bs={bs} {kind}", flush=True)
    if kind == "rand":
        A = sparse_random(n, bs, alpha, 3)
        B = sparse_random(n, bs, 0.5, 4)
    elif kind == "3d":
        n = (n // 8) * 8
        A = synth.DecaySpec("3d", n, alpha, seed=2).dense()
        B = A
    else:
        A = synth.DecaySpec("1d", n, alpha, seed=5).dense()
        B = synth.DecaySpec("1d", n, alpha * 1.3, seed=6).dense()
    TA, TB = O.build(A, bs), O.build(B, bs)
    MA, MB = ctx.build(dev(A), bs), ctx.build(dev(B), bs)
    check_norms(ctx, MA, TA)
    for mode in MODES:
        for prec in (spamm.F64, spamm.F32):
            check_product(ctx, MA, MB, TA, TB, tau, mode, prec, expect_full=full or mode == spamm.SPAMM)


def test_block_list_build_matches_dense_build(ctx):
    import torch
    print("case: block build n=3000 bs=64", flush=True)
    sp = synth.DecaySpec("1d", 3000, 0.2, seed=3)
    coords, data = sp.leaf_blocks(64)
    Mb = ctx.build_blocks(3000, 64, dev(coords.astype(np.int32)), dev(data))
    Md = ctx.build(dev(sp.dense()), 64)
    assert Mb.info.nonnull == Md.info.nonnull
    assert np.array_equal(ctx.norms(Mb), ctx.norms(Md))
    assert torch.equal(ctx.to_dense(Mb), ctx.to_dense(Md))
    T = O.build_from_blocks(3000, 64, coords, data)
    check_norms(ctx, Mb, T)
    for mode in MODES:
        check_product(ctx, Mb, Mb, T, T, 1e-6, mode, spamm.F32, alias=True)


def test_block_list_batch_build(ctx):
    """Several lists in one call give the same matrices, bit for bit, as one
    call per list; an error in any list fails the whole call."""
    import torch
    print("case: batched block build", flush=True)
    lists = []
    for n, bs, a, seed in ((3000, 64, 0.2, 3), (2048, 32, 0.5, 4), (700, 16, 0.3, 5)):
        c, d = synth.DecaySpec("1d", n, a, seed=seed).leaf_blocks(bs)
        lists.append((n, bs, dev(c.astype(np.int32)), dev(d)))
    Ms = ctx.build_blocks_batch(lists)
    for (n, bs, c, d), M in zip(lists, Ms):
        S = ctx.build_blocks(n, bs, c, d)
        assert M.info.nonnull == S.info.nonnull and M.info.G == S.info.G
        assert np.array_equal(ctx.norms(M), ctx.norms(S))
        assert torch.equal(ctx.to_dense(M), ctx.to_dense(S))
        S.release()
        M.release()
    # an empty G = 2048 list beside a small one (lists of very different
    # sizes in one call)
    e_c = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
    e_d = torch.zeros((0, 64, 64), dtype=torch.float64, device="cuda")
    big, small = ctx.build_blocks_batch([(131072, 64, e_c, e_d), lists[0]])
    S = ctx.build_blocks(*lists[0])
    assert big.info.nonnull == 0 and big.info.G == 2048
    assert small.info.nonnull == S.info.nonnull
    assert np.array_equal(ctx.norms(small), ctx.norms(S))
    assert torch.equal(ctx.to_dense(small), ctx.to_dense(S))
    for M in (big, small, S):
        M.release()
    dup = lists[1][2].clone()
    dup[1] = dup[0]
    with pytest.raises(spamm.SpammError) as e:
        ctx.build_blocks_batch([lists[0], (lists[1][0], lists[1][1], dup, lists[1][3])])
    assert e.value.code == "EINVAL"


def test_tau_zero_and_huge(ctx):
    print("case: tau 0 / huge", flush=True)
    A = sparse_random(400, 32, 0.4, 8)
    T = O.build(A, 32)
    M = ctx.build(dev(A), 32)
    for mode in MODES:
        p = ctx.multiply(M, M, 0.0, mode=mode, prec=spamm.F64)
        C = ctx.to_dense(p.C).cpu().numpy()
        assert rel_fro(C, A @ A) <= 1e-14
        q = ctx.multiply(M, M, 1e30, mode=mode, prec=spamm.F64)
        assert q.stats["n_kept"] == 0 and q.stats["c_nonnull"] == 0
        assert np.all(ctx.to_dense(q.C).cpu().numpy() == 0.0)


def test_all_null_input(ctx):
    print("case: all-null", flush=True)
    Z = np.zeros((100, 100))
    M = ctx.build(dev(Z), 16)
    assert M.info.nonnull == 0
    for mode in MODES:
        p = ctx.multiply(M, M, 1e-6, mode=mode, prec=spamm.F32)
        assert p.stats["n_kept"] == 0
        assert ctx.kept(p.C).shape == (0, 3)
    assert np.all(ctx.norms(M) == 0.0)


def test_deepest_tree_and_batch_limit(ctx):
    """The deepest quadtree (G = 2048, n = 131072 at leaf 64) with no leaves:
    one multiply runs and forms nothing; a batch whose packed counts could
    overflow one int64 is refused before any launch."""
    import torch
    print("case: empty G=2048, batch limit", flush=True)
    e_c = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
    e_d = torch.zeros((0, 64, 64), dtype=torch.float64, device="cuda")
    M = ctx.build_blocks(131072, 64, e_c, e_d, stores=spamm.STORE_F32)
    assert M.info.G == 2048 and M.info.nonnull == 0
    p = ctx.multiply(M, M, 1e-6, mode=spamm.SPAMM, prec=spamm.F32)
    assert p.stats["n_kept"] == 0 and p.stats["c_nonnull"] == 0
    p.C.release()
    with pytest.raises(spamm.SpammError) as e:
        ctx.multiply_batch([dict(A=M, B=M, tau=1e-6, mode=spamm.SPAMM, prec=spamm.F32)] * 16)
    assert e.value.code == "EUNSUPPORTED"
    M.release()


def test_deepest_tree_with_leaves(ctx):
    """G = 2048 with an upper bidiagonal of leaves whose norms span three
    decades: the per-C-leaf scans run over 4 M entries (the multi-pass scan
    path), and products, bounds and C must match the oracle."""
    print("case: bidiagonal G=2048 leaf 64", flush=True)
    rng = np.random.default_rng(11)
    G, bs = 2048, 64
    I = np.r_[np.arange(G), np.arange(G - 1)]
    J = np.r_[np.arange(G), np.arange(1, G)]
    coords = np.stack([I, J], axis=1).astype(np.int32)
    scale = 10.0 ** rng.uniform(-3, 0, len(I))
    data = rng.standard_normal((len(I), bs, bs)) * scale[:, None, None]
    M = ctx.build_blocks(G * bs, bs, dev(coords), dev(data))
    T = O.build_from_blocks(G * bs, bs, coords, data)
    check_norms(ctx, M, T)
    for mode in MODES:
        check_product(ctx, M, M, T, T, 1.0, mode, spamm.F32, alias=True)
    M.release()


def test_truncation_drop_set(ctx):
    print("case: truncation", flush=True)
    A = synth.DecaySpec("1d", 4096, 0.2, seed=1).dense()
    T = O.build(A, 64)
    M = ctx.build(dev(A), 64)
    for tau in (1e-8, 1e-6, 1e-4, 1e-2):
        Mt, dropped = ctx.truncate(M, tau)
        tr = O.truncate(T, tau)
        # no tie at this boundary, so the drop set is unique
        assert not tr.tie
        assert Mt.info.nonnull == tr.tree.nonnull_count()
        assert abs(dropped - tr.dropped_sq) <= 1e-12 * max(tr.dropped_sq, 1e-300)
        check_norms(ctx, Mt, tr.tree)
        assert np.array_equal(ctx.to_dense(Mt).cpu().numpy(), tr.tree.to_dense())


def test_epilogue_alpha_beta(ctx):
    """C = -1 * A A + 2 * A (the 2X - X^2 purification step)."""
    print("case: epilogue", flush=True)
    A = synth.DecaySpec("1d", 512, 0.4, seed=9).dense() * 0.1
    T = O.build(A, 32)
    M = ctx.build(dev(A), 32)
    for prec in (spamm.F64, spamm.F32):
        p = ctx.multiply(M, M, 1e-7, mode=spamm.HYBRID, prec=prec, alpha=-1.0, beta=2.0, D=M)
        ref = O.multiply(T, T, 1e-7, O.HYBRID)
        want = 2.0 * A - ref.C.to_dense()
        C = ctx.to_dense(p.C).cpu().numpy()
        assert rel_fro(C, want) <= TOL[prec]
        # C's structure is the union of the product's and D's
        assert p.C.info.nonnull == int((ref.C.leaf_present | T.leaf_present).sum())


def test_bitwise_repeatable_and_batch_equals_alone(ctx):
    import torch
    print("case: determinism", flush=True)
    A = synth.DecaySpec("1d", 4096, 0.2, seed=4).dense()
    B = synth.DecaySpec("3d", 2048, 0.8, seed=5).dense()
    MA = ctx.build(dev(A), 64)
    MB = ctx.build(dev(B), 32)
    alone = []
    for (M, tau, mode, prec) in [(MA, 1e-6, spamm.SPAMM, spamm.F32), (MA, 1e-4, spamm.HYBRID, spamm.F64),
                                 (MB, 1e-5, spamm.TRUNCMUL, spamm.F32), (MB, 1e-6, spamm.SPAMM, spamm.F64)]:
        p1 = ctx.multiply(M, M, tau, mode=mode, prec=prec)
        p2 = ctx.multiply(M, M, tau, mode=mode, prec=prec)
        assert torch.equal(ctx.to_dense(p1.C), ctx.to_dense(p2.C))
        alone.append((M, tau, mode, prec, ctx.to_dense(p1.C)))
    batch = ctx.multiply_batch([dict(A=M, B=M, tau=t, mode=m, prec=pr) for (M, t, m, pr, _) in alone])
    for (M, t, m, pr, Cal), pb in zip(alone, batch):
        assert torch.equal(ctx.to_dense(pb.C), Cal)


def test_error_codes(ctx):
    import torch
    print("case: error codes", flush=True)
    A = synth.DecaySpec("1d", 256, 0.5, seed=1).dense()
    M = ctx.build(dev(A), 32)
    M16 = ctx.build(dev(A), 16)
    with pytest.raises(spamm.SpammError) as e:
        ctx.multiply(M, M, -1.0)
    assert e.value.code == "EINVAL"
    with pytest.raises(spamm.SpammError) as e:
        ctx.multiply(M, M, float("nan"))
    assert e.value.code == "EINVAL"
    with pytest.raises(spamm.SpammError) as e:
        ctx.multiply(M, M16, 1e-6)
    assert e.value.code == "ESHAPE"
    bad = A.copy()
    bad[3, 7] = np.nan
    with pytest.raises(spamm.SpammError) as e:
        ctx.build(dev(bad), 32)
    assert e.value.code == "ENONFINITE"
    with pytest.raises(spamm.SpammError) as e:
        ctx.build(dev(A), 48)
    assert e.value.code == "EINVAL"
    small = spamm.Context(arena_bytes=2 << 20)
    with pytest.raises(spamm.SpammError) as e:
        small.build(dev(synth.DecaySpec("1d", 2048, 0.01, seed=1).dense()), 64)
    assert e.value.code == "ENOMEM"
    small.close()


def test_config2_full(ctx):
    """n=16384, leaf 64, 1D alpha in {0.2, 0.5}, tau in {1e-4, 1e-6, 1e-8},
    three schemes, FP64 and FP32, built from block lists."""
    for alpha in (0.2, 0.5):
        print(f"case: config2 alpha={alpha}", flush=True)
        sp = synth.DecaySpec("1d", 16384, alpha, seed=1)
        coords, data = sp.leaf_blocks(64)
        T = O.build_from_blocks(16384, 64, coords, data)
        M = ctx.build_blocks(16384, 64, dev(coords.astype(np.int32)), dev(data))
        check_norms(ctx, M, T)
        for tau in (1e-4, 1e-6, 1e-8):
            for mode in MODES:
                for prec in (spamm.F64, spamm.F32):
                    check_product(ctx, M, M, T, T, tau, mode, prec, alias=True)


def test_gemm_schedules_agree_bitwise():
    """Morton slices per XCD, request-major placement, and round-robin or
    contiguous unit ranges give bitwise the same C: each C leaf is summed by
    one workgroup in the plan's order either way."""
    import os
    import torch
    print("case: schedules", flush=True)
    A = synth.DecaySpec("1d", 8192, 0.2, seed=2).dense()
    res = {}
    for mode in ("xcd", "rm", "ranges", "chunk1", "chunk7"):
        os.environ["SPAMM_GEMM_SCHED"] = "rm" if mode == "rm" else "xcd"
        try:
            c = spamm.Context(arena_bytes=2 << 30)
        finally:
            del os.environ["SPAMM_GEMM_SCHED"]
        if mode == "ranges":
            c.set_option("unit_order", 0)
        elif mode.startswith("chunk"):
            c.set_option("unit_order", int(mode[5:]))
        M = c.build(dev(A), 64)
        ps = c.multiply_batch([dict(A=M, B=M, tau=t, mode=m, prec=spamm.F32)
                               for t in (1e-4, 1e-8) for m in MODES])
        res[mode] = [c.to_dense(p.C).cpu() for p in ps]
        for p in ps:
            p.C.release()
        M.release()
        c.close()
    for other in ("rm", "ranges", "chunk1", "chunk7"):
        for a, b in zip(res["xcd"], res[other]):
            assert torch.equal(a, b)


@pytest.mark.parametrize("n,bs,kind,tau", [
    (1000, 32, "1d", 1e-5),
    (2100, 64, "1d", 1e-6),
    (700, 128, "3d", 1e-4),
    (300, 32, "rand", 1e-2),
])
def test_bf16_and_split_bf16(ctx, n, bs, kind, tau):
    """BF16 and split-BF16 products against the FP64 oracle (relative
    Frobenius 1e-2 and 1e-5)."""
    print(f"case: bf16 n={n} bs={bs} {kind}", flush=True)
    if kind == "rand":
        A = sparse_random(n, bs, 0.4, 13)
        B = sparse_random(n, bs, 0.6, 14)
    elif kind == "3d":
        n = (n // 8) * 8
        A = B = synth.DecaySpec("3d", n, 1.0, seed=7).dense()
    else:
        A = synth.DecaySpec("1d", n, 0.3, seed=8).dense()
        B = synth.DecaySpec("1d", n, 0.4, seed=9).dense()
    TA, TB = O.build(A, bs), O.build(B, bs)
    MA, MB = ctx.build(dev(A), bs), ctx.build(dev(B), bs)
    for mode in MODES:
        for prec in (spamm.BF16, spamm.BF16X3):
            check_product(ctx, MA, MB, TA, TB, tau, mode, prec)


def test_long_units_and_window_crossing(ctx):
    """C leaves with 65 products (more than one 64-product window), ragged
    tail, every precision."""
    print("case: long units", flush=True)
    A = sparse_random(1040, 16, 1.0, 21)
    B = sparse_random(1040, 16, 1.0, 22)
    TA, TB = O.build(A, 16), O.build(B, 16)
    MA, MB = ctx.build(dev(A), 16), ctx.build(dev(B), 16)
    for prec in (spamm.F64, spamm.F32):
        check_product(ctx, MA, MB, TA, TB, 0.0, spamm.SPAMM, prec)
    A = sparse_random(2100, 32, 1.0, 23)
    TA = O.build(A, 32)
    MA = ctx.build(dev(A), 32)
    for prec in (spamm.F32, spamm.BF16X3):
        check_product(ctx, MA, MA, TA, TA, 0.0, spamm.TRUNCMUL, prec, alias=True)


def test_epilogue_with_leaves_from_d_only(ctx):
    """C = alpha AB + beta D where many C leaves come from D alone (no
    products), interleaved with product leaves."""
    print("case: epilogue D-only leaves", flush=True)
    A = synth.DecaySpec("1d", 1024, 2.0, seed=3).dense()  # narrow band
    D = sparse_random(1024, 32, 0.5, 31)
    TA = O.build(A, 32)
    MA, MD = ctx.build(dev(A), 32), ctx.build(dev(D), 32)
    for prec in (spamm.F64, spamm.F32, spamm.BF16X3):
        p = ctx.multiply(MA, MA, 1e-9, mode=spamm.SPAMM, prec=prec, alpha=0.5, beta=-3.0, D=MD)
        ref = O.multiply(TA, TA, 1e-9, O.SPAMM)
        want = 0.5 * ref.C.to_dense() - 3.0 * D
        C = ctx.to_dense(p.C).cpu().numpy()
        assert rel_fro(C, want) <= TOL[prec]
        d_only = (~ref.C.leaf_present) & O.build(D, 32).leaf_present
        assert d_only.sum() > 50
        assert p.C.info.nonnull == int((ref.C.leaf_present | O.build(D, 32).leaf_present).sum())


def _fuzz_cases(count=24, seed=2024, leaves=(16, 32, 64), precs=(spamm.F64, spamm.F32), first=0):
    """Seeded random small cases: n in [1, 300] (mostly not a multiple of the
    leaf, so grids are padded and tails ragged), the given leaf sizes, 1D
    decay or random blocks, tau = 0 or 10^U[-8, 0], every mode, the given
    precisions, A = B aliased or not."""
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(first, first + count):
        n = int(rng.integers(1, 301))
        bs = int(rng.choice(leaves))
        kind = "rand" if rng.random() < 0.4 else "1d"
        tau = 0.0 if rng.random() < 0.15 else float(10.0 ** rng.uniform(-8, 0))
        mode = int(rng.integers(0, 3))
        prec = int(rng.choice(precs))
        alias = bool(rng.random() < 0.5)
        cases.append((i, n, bs, kind, tau, mode, prec, alias, float(rng.uniform(0.05, 1.0))))
    return cases


def _fuzz_matrix(kind, n, bs, a, seed):
    if kind == "rand":
        return sparse_random(n, bs, a, seed)
    return synth.DecaySpec("1d", n, a, seed=seed).dense()


@pytest.mark.parametrize("case", _fuzz_cases() + _fuzz_cases(12, 2025, (32, 64), (spamm.BF16, spamm.BF16X3), 24),
                         ids=lambda c: f"fuzz{c[0]}")
def test_fuzz_small_random(ctx, case):
    i, n, bs, kind, tau, mode, prec, alias, a = case
    print(f"case: fuzz{i} n={n} leaf={bs} {kind} tau={tau:.2e} mode={mode} prec={prec} alias={alias}", flush=True)
    A = _fuzz_matrix(kind, n, bs, a, 100 + i)
    B = A if alias else _fuzz_matrix(kind, n, bs, min(1.0, a * 1.7), 200 + i)
    TA = O.build(A, bs)
    TB = TA if alias else O.build(B, bs)
    MA = ctx.build(dev(A), bs)
    MB = MA if alias else ctx.build(dev(B), bs)
    # random thresholds may land a product inside the tie band: then the
    # agreeing C leaves are still compared
    check_product(ctx, MA, MB, TA, TB, tau, mode, prec, alias=alias, expect_full=False)
    if not alias:
        MB.release()
    MA.release()
