"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, brute force on tiny inputs, the paper's worked examples, invariants of
the definitions, metamorphic relations and the error trends of Thms 1-3.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MODES = (O.TRUNCMUL, O.SPAMM, O.HYBRID)


def rel_fro(x, y):
    d = np.linalg.norm(x - y)
    s = np.linalg.norm(y)
    return d / s if s else d


def sparse_random(n, bs, fill, seed):
    coords, data = synth.random_blocks(seed, n, bs, fill)
    return synth.dense_from_blocks(n, bs, coords, data)


# ---------------------------------------------------------------- generator

def test_splitmix64_published_outputs():
    want = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64.txt"))
            if not l.startswith("#")]
    states = np.array([(k + 0) * 0x9E3779B97F4A7C15 % 2 ** 64 for k in range(3)],
                      dtype=np.uint64)
    got = [int(x) for x in synth.splitmix64(states)]
    assert got == want


def test_generator_symmetric_and_in_range():
    sp = synth.DecaySpec("1d", 200, 0.3, seed=2)
    A = sp.dense()
    assert np.array_equal(A, A.T)
    assert np.all(np.abs(A) <= 1.0)
    assert np.all((A == 0) | (np.abs(A) >= 1e-16))
    i, j = np.meshgrid(np.arange(200), np.arange(200), indexing="ij")
    u = synth.uniform(2, i, j, 200)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01
    sp3 = synth.DecaySpec("3d", 256, 1.0, seed=3)
    B = sp3.dense()
    assert np.array_equal(B, B.T)
    # the 8 functions of one atom share a centre: distance 0, |a| <= 1 and
    # envelope 1 only inside the 8 x 8 diagonal blocks
    pos = synth.atom_positions(3, 32)
    x, y, z = synth.morton3_decode(np.arange(8))
    assert np.array_equal(np.sort(x), [0, 0, 0, 0, 1, 1, 1, 1])
    assert np.all(np.abs(pos - np.stack(synth.morton3_decode(np.arange(32)), 1)) <= 0.1)


def test_leaf_blocks_cover_dense():
    sp = synth.DecaySpec("1d", 300, 0.2, seed=1)
    coords, data = sp.leaf_blocks(32)
    assert np.array_equal(synth.dense_from_blocks(300, 32, coords, data), sp.dense())


# ---------------------------------------------------------------- layout

def test_morton_children_and_grid():
    assert O.grid_size(1024, 32) == (32, 5)
    assert O.grid_size(300, 16) == (32, 5)
    assert O.grid_size(5, 8) == (1, 0)
    I, J = np.meshgrid(np.arange(8), np.arange(8), indexing="ij")
    k = O.morton_key(I, J)
    assert sorted(k.ravel().tolist()) == list(range(64))
    for a in (0, 1):
        for b in (0, 1):
            assert np.array_equal(O.morton_key(2 * I + a, 2 * J + b), 4 * k + 2 * a + b)


def test_pyramid_matches_direct_block_sums():
    A = sparse_random(200, 16, 0.3, 5)
    T = O.build(A, 16)
    for level in range(T.L + 1):
        span = T.G >> level
        for I in range(1 << level):
            for J in range(1 << level):
                blk = np.zeros((T.G * 16, T.G * 16))
                blk[:200, :200] = A
                sub = blk[I * span * 16:(I + 1) * span * 16, J * span * 16:(J + 1) * span * 16]
                direct = sum(float(v) * float(v) for v in sub.ravel() if v != 0.0)
                got = T.sq[level][I, J]
                assert abs(got - direct) <= 1e-13 * max(direct, 1e-300)
                assert T.present[level][I, J] == bool(np.any(sub != 0))
    assert math.isclose(T.fro() ** 2, float(np.sum(A * A)), rel_tol=1e-13)


def test_null_leaves_and_padding():
    A = np.zeros((40, 40))
    A[0, 0] = 1.0
    A[39, 39] = -2.0
    T = O.build(A, 16)
    assert (T.G, T.L) == (4, 2)
    assert T.nonnull_count() == 2
    assert T.index[0, 0] >= 0 and T.index[2, 2] >= 0
    assert np.array_equal(T.to_dense(), A)
    Z = O.build(np.zeros((10, 10)), 4)
    assert Z.nonnull_count() == 0 and not Z.present[0][0, 0]


# ---------------------------------------------------------------- worked examples

def _two_by_two(flags, rng, bs=4):
    A = np.zeros((2 * bs, 2 * bs))
    for q, f in enumerate(flags):
        if f == "1":
            I, J = divmod(q, 2)
            A[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = rng.uniform(-1, 1, (bs, bs))
    return A


def test_paper_worked_examples():
    rng = np.random.default_rng(0)
    rows = [l.split() for l in open(os.path.join(GOLDEN, "worked_examples.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    for name, fa, fb, fc, prods in rows:
        A, B = _two_by_two(fa, rng), _two_by_two(fb, rng)
        TA, TB = O.build(A, 4), O.build(B, 4)
        want = [] if prods == "-" else [tuple(int(x) for x in p.split(","))
                                        for p in prods.split(";")]
        for mode in MODES:
            r = O.multiply(TA, TB, 0.0, mode)
            assert [tuple(t) for t in r.kept.tolist()] == want, name
            got_c = "".join("1" if r.C.leaf_present[I, J] else "0"
                            for I in range(2) for J in range(2))
            assert got_c == fc, name
            assert [tuple(t) for t in O.kept_recursive(TA, TB, 0.0, mode != O.TRUNCMUL).tolist()] == want
            for (I, K, J) in want:
                assert np.array_equal(r.C.leaf(I, J),
                                      A[I * 4:I * 4 + 4, K * 4:K * 4 + 4] @ B[K * 4:K * 4 + 4, J * 4:J * 4 + 4])


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("mode", MODES)
def test_tau_zero_is_exact_product(mode):
    for A, B, bs in [
        (synth.DecaySpec("1d", 256, 0.3, 1).dense(), synth.DecaySpec("1d", 256, 0.1, 2).dense(), 16),
        (sparse_random(200, 16, 0.3, 3), sparse_random(200, 16, 0.4, 4), 16),
        (synth.DecaySpec("3d", 128, 1.0, 1).dense(), synth.DecaySpec("3d", 128, 1.0, 1).dense(), 32),
    ]:
        r = O.multiply(O.build(A, bs), O.build(B, bs), 0.0, mode)
        assert rel_fro(r.C.to_dense(), A @ B) <= 1e-14


def test_exact_product_against_triple_loop():
    rng = np.random.default_rng(1)
    A, B = rng.normal(size=(9, 9)), rng.normal(size=(9, 9))
    C = np.zeros((9, 9))
    for i in range(9):
        for j in range(9):
            C[i, j] = sum(A[i, k] * B[k, j] for k in range(9))
    assert np.allclose(O.exact_product(A, B), C, rtol=1e-14, atol=1e-14)


def _brute_force(A, B, bs, tau, use_norms):
    """Element-level triple loop: c_ij gets a_ik b_kj when leaf triple
    (i//bs, k//bs, j//bs) has two non-zero blocks passing the norm test;
    block norms come from plain loops over the block's entries."""
    n = A.shape[0]
    g = -(-n // bs)

    def blk_sq(M, I, J):
        acc, nz = 0.0, False
        for i in range(I * bs, min(n, I * bs + bs)):
            for j in range(J * bs, min(n, J * bs + bs)):
                acc += M[i, j] * M[i, j]
                nz |= M[i, j] != 0.0
        return acc, nz

    sa = [[blk_sq(A, I, K) for K in range(g)] for I in range(g)]
    sb = [[blk_sq(B, K, J) for J in range(g)] for K in range(g)]
    keep = set()
    for I in range(g):
        for K in range(g):
            for J in range(g):
                (a, na), (b, nb) = sa[I][K], sb[K][J]
                if na and nb and (not use_norms or math.sqrt(a) * math.sqrt(b) >= tau):
                    keep.add((I, K, J))
    C = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            acc = 0.0
            for k in range(n):
                if (i // bs, k // bs, j // bs) in keep:
                    acc += A[i, k] * B[k, j]
            C[i, j] = acc
    return keep, C


@pytest.mark.parametrize("bs", [1, 2, 4, 8])
def test_brute_force_tiny(bs):
    n = 24 if bs > 1 else 12
    A = synth.DecaySpec("1d", n, 0.4, 7).dense()
    B = sparse_random(n, 4, 0.6, 8)
    for tau in (0.0, 1e-3, 0.05, 0.3):
        r = O.multiply(O.build(A, bs), O.build(B, bs), tau, O.SPAMM)
        keep, C = _brute_force(A, B, bs, tau, True)
        assert {tuple(t) for t in r.kept.tolist()} == keep
        assert np.allclose(r.C.to_dense(), C, rtol=0, atol=1e-13)


def _brute_truncate(A, bs, tau):
    """Independent leaf truncation: loop-computed leaf norms, bit-loop Morton
    keys, greedy drop with exactly rounded running sums (math.fsum)."""
    n = A.shape[0]
    g = -(-n // bs)
    leaves = []
    for I in range(g):
        for J in range(g):
            blk = A[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs]
            if np.any(blk != 0):
                s = 0.0
                for v in blk.ravel():
                    s += v * v
                key = 0
                for b in range(16):
                    key |= ((I >> b) & 1) << (2 * b + 1) | ((J >> b) & 1) << (2 * b)
                leaves.append((s, key, I, J))
    leaves.sort()
    out = A.copy()
    taken = []
    for s, key, I, J in leaves:
        if math.fsum(taken + [s]) <= tau * tau:
            taken.append(s)
            out[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = 0.0
        else:
            break
    return out


@pytest.mark.parametrize("mode", [O.TRUNCMUL, O.HYBRID])
def test_brute_force_truncating_modes(mode):
    n, bs = 32, 4
    A = synth.DecaySpec("1d", n, 0.35, 11).dense()
    B = synth.DecaySpec("1d", n, 0.25, 12).dense()
    for tau in (1e-6, 1e-3, 3e-2, 0.2):
        r = O.multiply(O.build(A, bs), O.build(B, bs), tau, mode)
        At, Bt = _brute_truncate(A, bs, tau), _brute_truncate(B, bs, tau)
        keep, C = _brute_force(At, Bt, bs, tau, mode == O.HYBRID)
        assert {tuple(t) for t in r.kept.tolist()} == keep
        assert np.allclose(r.C.to_dense(), C, rtol=0, atol=1e-13)
        assert np.array_equal(r.A_used.to_dense(), At)


def test_bs1_is_elementwise_spamm_bit_exact():
    """With 1 x 1 leaves the block algorithm is the element-level chi of the
    proof of Thm 2, summed over k ascending in both."""
    A = synth.DecaySpec("1d", 20, 0.5, 3).dense()
    B = synth.DecaySpec("1d", 20, 0.3, 4).dense()
    for tau in (0.0, 1e-4, 1e-2, 0.2):
        r = O.multiply(O.build(A, 1), O.build(B, 1), tau, O.SPAMM)
        assert np.array_equal(r.C.to_dense(), O.spamm_elementwise(A, B, tau))


# ---------------------------------------------------------------- truncation

@pytest.mark.parametrize("tau", [1e-8, 1e-6, 1e-4, 1e-2, 0.5])
def test_truncation_invariant_and_maximality(tau):
    A = synth.DecaySpec("1d", 512, 0.2, 1).dense()
    T = O.build(A, 16)
    tr = O.truncate(T, tau)
    # invariant: ||A - A~||_F <= tau, recomputed from the dense difference
    D = A - tr.tree.to_dense()
    dropped = float(np.sum(D * D))
    assert dropped <= tau * tau * (1 + 1e-12)
    # the dropped leaves are exactly the ones that disappeared
    assert T.nonnull_count() - tr.tree.nonnull_count() == len(tr.dropped)
    # order: every dropped leaf precedes every kept leaf in (norm, Morton)
    if len(tr.dropped):
        I, J = np.nonzero(tr.tree.index >= 0)
        kept_key = [(T.leaf_sq[a, b], int(O.morton_key(a, b))) for a, b in zip(I, J)]
        drop_key = [(T.leaf_sq[a, b], int(O.morton_key(a, b))) for a, b in tr.dropped]
        assert max(drop_key) < min(kept_key) if kept_key else True
    # maximality: dropping the next leaf too would exceed the budget
    I, J = np.nonzero(tr.tree.index >= 0)
    if len(I):
        nxt = min(zip(T.leaf_sq[I, J], O.morton_key(I, J)))
        assert math.fsum([T.leaf_sq[a, b] for a, b in tr.dropped] + [nxt[0]]) > tau * tau * (1 - 1e-12)


def test_truncation_degenerate_cases():
    A = synth.DecaySpec("1d", 128, 0.5, 1).dense()
    T = O.build(A, 16)
    assert O.truncate(T, 0.0).tree.nonnull_count() == T.nonnull_count()
    big = O.truncate(T, 2 * T.fro())
    assert big.tree.nonnull_count() == 0
    assert np.array_equal(big.tree.to_dense(), np.zeros_like(A))
    with pytest.raises(ValueError):
        O.truncate(T, -1.0)
    with pytest.raises(ValueError):
        O.truncate(T, float("nan"))


def test_elementwise_truncation_definition():
    A = np.array([[1e-3, -2e-5], [5e-7, -1.0]])
    At = O.truncate_elementwise(A, 1e-5)
    assert np.array_equal(At, np.array([[1e-3, -2e-5], [0.0, -1.0]]))


# ---------------------------------------------------------------- SpAMM bounds

@pytest.mark.parametrize("mode", MODES)
def test_error_bounds(mode):
    for A, bs, tau in [(synth.DecaySpec("1d", 512, 0.1, 1).dense(), 16, 1e-4),
                       (synth.DecaySpec("3d", 256, 1.0, 2).dense(), 16, 1e-3),
                       (sparse_random(256, 16, 0.3, 9), 16, 2.0)]:
        T = O.build(A, bs)
        r = O.multiply(T, T, tau, mode)
        E = O.exact_product(A, A) - r.C.to_dense()
        # FP64 rounding of the two product orders: a few ulps of ||A||_F^2
        slack = 1e-14 * r.stats["normA"] * r.stats["normB"]
        assert np.linalg.norm(E) <= r.stats["err_bound"] * (1 + 1e-9) + slack
        if mode == O.SPAMM:
            G = T.G
            Cfull = np.zeros((G * bs, G * bs)); Cfull[:A.shape[0], :A.shape[0]] = E
            for I in range(G):
                for J in range(G):
                    e = np.linalg.norm(Cfull[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs])
                    assert e <= r.skipped_bound[I, J] * (1 + 1e-9) + slack
            assert r.stats["B2"] <= r.stats["B1"] * (1 + 1e-15)


def test_per_product_rule():
    A = synth.DecaySpec("1d", 256, 0.15, 4).dense()
    T = O.build(A, 16)
    tau = 1e-5
    r = O.multiply(T, T, tau, O.SPAMM)
    kept = {tuple(t) for t in r.kept.tolist()}
    for I in range(T.G):
        for K in range(T.G):
            for J in range(T.G):
                if T.index[I, K] < 0 or T.index[K, J] < 0:
                    assert (I, K, J) not in kept
                    continue
                p = np.linalg.norm(T.leaf(I, K) @ T.leaf(K, J))
                bound = math.sqrt(T.leaf_sq[I, K]) * math.sqrt(T.leaf_sq[K, J])
                if (I, K, J) in kept:
                    assert bound >= tau
                else:
                    assert p < tau and bound < tau


# ---------------------------------------------------------------- recursion

@pytest.mark.parametrize("use_norms", [False, True])
def test_recursive_alg1_equals_flat(use_norms):
    cases = [(synth.DecaySpec("1d", 512, 0.2, 1).dense(), 16),
             (synth.DecaySpec("3d", 256, 0.8, 2).dense(), 16),
             (sparse_random(300, 8, 0.15, 3), 8),
             (np.eye(5), 8)]
    for A, bs in cases:
        T = O.build(A, bs)
        for tau in (0.0, 1e-8, 1e-4, 1e-2, 1.0):
            assert np.array_equal(O.kept_recursive(T, T, tau, use_norms),
                                  O.kept_flat(T, T, tau, use_norms))


def test_single_leaf_is_tested():
    A = np.full((4, 4), 1e-3)
    T = O.build(A, 8)
    assert T.L == 0
    assert len(O.multiply(T, T, 1e-1, O.SPAMM).kept) == 0     # 4e-3^... < tau
    assert len(O.multiply(T, T, 1e-6, O.SPAMM).kept) == 1


# ---------------------------------------------------------------- metamorphic

def test_nested_in_tau():
    A = synth.DecaySpec("1d", 512, 0.15, 2).dense()
    T = O.build(A, 16)
    taus = [1e-10, 1e-8, 1e-6, 1e-4, 1e-2]
    for mode in MODES:
        sets = [{tuple(t) for t in O.multiply(T, T, t, mode).kept.tolist()} for t in taus]
        for small, large in zip(sets, sets[1:]):
            assert large <= small


def test_power_of_two_scaling_bit_exact():
    A = synth.DecaySpec("1d", 256, 0.2, 3).dense()
    B = synth.DecaySpec("1d", 256, 0.3, 4).dense()
    tau = 1e-5
    r0 = O.multiply(O.build(A, 16), O.build(B, 16), tau, O.SPAMM)
    for e in (-3, 5):
        s = 2.0 ** e
        r1 = O.multiply(O.build(A * s, 16), O.build(B, 16), tau * s, O.SPAMM)
        assert np.array_equal(r0.kept, r1.kept)
        assert np.array_equal(r1.C.to_dense(), r0.C.to_dense() * s)


def test_transpose_symmetry():
    A = synth.DecaySpec("1d", 384, 0.2, 5).dense()
    B = sparse_random(384, 16, 0.5, 6) * 1e-2 + synth.DecaySpec("1d", 384, 0.3, 6).dense()
    tau = 1e-6
    TA, TB = O.build(A, 16), O.build(B, 16)
    r = O.multiply(TA, TB, tau, O.SPAMM)
    rt = O.multiply(O.build(B.T.copy(), 16), O.build(A.T.copy(), 16), tau, O.SPAMM)
    ties = {tuple(t) for t in O.tie_triples(TA, TB, tau).tolist()}
    s1 = {(I, K, J) for I, K, J in r.kept.tolist()} - ties
    s2 = {(I, K, J) for J, K, I in rt.kept.tolist()} - ties
    assert s1 == s2
    assert rel_fro(rt.C.to_dense(), r.C.to_dense().T) <= 1e-14
    # a symmetric A gives a kept set closed under (I,K,J) -> (J,K,I)
    rs = O.multiply(TA, TA, tau, O.SPAMM)
    ks = {tuple(t) for t in rs.kept.tolist()}
    assert ks == {(J, K, I) for I, K, J in ks}


def test_alias_truncates_once():
    A = synth.DecaySpec("1d", 256, 0.2, 1).dense()
    T = O.build(A, 16)
    r = O.multiply(T, T, 1e-4, O.HYBRID)
    assert r.A_used is r.B_used
    r2 = O.multiply(T, O.build(A, 16), 1e-4, O.HYBRID)
    assert np.array_equal(r.kept, r2.kept)


def test_shape_errors():
    T16 = O.build(np.eye(32), 16)
    T8 = O.build(np.eye(32), 8)
    with pytest.raises(ValueError):
        O.multiply(T16, T8, 0.0, O.SPAMM)
    with pytest.raises(ValueError):
        O.multiply(T16, T16, -1.0, O.SPAMM)


# ---------------------------------------------------------------- trends (Thms 1-3)

def _slope(x, y):
    return float(np.polyfit(np.log(x), np.log(y), 1)[0])


@pytest.mark.slow
def test_error_trends_in_n_and_tau():
    """Thms 1-3: ||E||_F = O(n^{1/2}) at fixed tau and ~ tau^{p/2}, p -> 2,
    at fixed n; the paper measures slopes ~0.5 and ~1 (Sec. 5)."""
    ns = [256, 512, 1024, 2048]
    errs = {m: [] for m in MODES}
    for n in ns:
        A = synth.DecaySpec("1d", n, 0.1, 1).dense()
        T = O.build(A, 16)
        ex = O.exact_product(A, A)
        for m in MODES:
            errs[m].append(np.linalg.norm(ex - O.multiply(T, T, 1e-6, m).C.to_dense()))
    for m in MODES:
        s = _slope(ns, errs[m])
        assert s <= 0.70, (m, s)
        if m != O.TRUNCMUL:
            assert s >= 0.35, (m, s)
    A = synth.DecaySpec("1d", 1024, 0.1, 1).dense()
    T = O.build(A, 16)
    ex = O.exact_product(A, A)
    taus = [1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9]
    for m in MODES:
        e = [np.linalg.norm(ex - O.multiply(T, T, t, m).C.to_dense()) for t in taus]
        s = _slope(taus, e)
        assert 0.85 <= s <= 1.15, (m, s)
        # element-wise O(tau): max |E_ij| / tau stays bounded
        emax = [np.max(np.abs(ex - O.multiply(T, T, t, m).C.to_dense())) / t for t in taus[::3]]
        assert max(emax) < 10.0


# ---------------------------------------------------------------- rounding bound
#
# The bound of ``precision_bound`` covers the rounding of the kept products
# formed in a lower precision.  It is pinned by forming those products the
# way each precision does (inputs rounded, sums in FP32) and measuring the
# error against the exact sum of the same products, and by invariants.

def _bf16(x32):
    """Round float32 values to BF16 (nearest, ties to even), as float32."""
    u = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


def _formed(res, prec):
    """C leaves of res summed over kept K ascending, each product and sum in
    the arithmetic of `prec` (NumPy float32 stands in for the FP32 MFMA)."""
    Au, Bu, kept = res.A_used, res.B_used, res.kept
    out = {}
    for I, K, J in kept:
        a, b = Au.leaf(int(I), int(K)), Bu.leaf(int(K), int(J))
        a32, b32 = a.astype(np.float32), b.astype(np.float32)
        if prec == O.P_F32:
            part = a32 @ b32
        elif prec == O.P_BF16:
            part = _bf16(a32) @ _bf16(b32)
        else:
            ha, hb = _bf16(a32), _bf16(b32)
            la, lb = _bf16(a32 - ha), _bf16(b32 - hb)
            part = (la @ hb + ha @ lb) + ha @ hb
        key = (int(I), int(J))
        out[key] = part if key not in out else (out[key] + part).astype(np.float32)
    return out


@pytest.mark.parametrize("prec", ["f32", "bf16", "bf16x3"])
@pytest.mark.parametrize("kind,alpha,bs", [("1d", 0.15, 8), ("3d", 1.0, 16)])
def test_rounding_bound_holds_for_formed_products(prec, kind, alpha, bs):
    n = 256 if kind == "1d" else 192
    A = synth.DecaySpec(kind, n, alpha, seed=11).dense()
    T = O.build(A, bs)
    for mode, tau in ((O.SPAMM, 1e-5), (O.HYBRID, 1e-7), (O.TRUNCMUL, 0.0)):
        res = O.multiply(T, T, tau, mode)
        formed = _formed(res, prec)
        err2 = 0.0
        for (I, J), c in formed.items():
            ref = res.C.leaf(I, J)
            err2 += float(np.sum((c.astype(np.float64) - ref) ** 2))
        bound = O.precision_bound(res, prec)
        # the FP64 oracle's own rounding is covered by the FP64 bound
        assert math.sqrt(err2) <= bound + O.precision_bound(res, O.P_F64), (mode, math.sqrt(err2), bound)
        assert math.sqrt(err2) > 0.0


def test_rounding_bound_fp64_against_exact_rationals():
    from fractions import Fraction
    A = synth.DecaySpec("1d", 24, 0.4, seed=3).dense()
    T = O.build(A, 4)
    res = O.multiply(T, T, 1e-3, O.SPAMM)
    err2 = Fraction(0)
    by_leaf = {}
    for I, K, J in res.kept:
        by_leaf.setdefault((int(I), int(J)), []).append(int(K))
    for (I, J), ks in by_leaf.items():
        exact = [[Fraction(0)] * 4 for _ in range(4)]
        for K in ks:
            a, b = T.leaf(I, K), T.leaf(K, J)
            for r in range(4):
                for c in range(4):
                    exact[r][c] += sum(Fraction(float(a[r, q])) * Fraction(float(b[q, c])) for q in range(4))
        got = res.C.leaf(I, J)
        for r in range(4):
            for c in range(4):
                err2 += (Fraction(float(got[r, c])) - exact[r][c]) ** 2
    assert float(err2) ** 0.5 <= O.precision_bound(res, O.P_F64)


def test_rounding_bound_invariants():
    A = synth.DecaySpec("1d", 128, 0.3, seed=5).dense()
    T = O.build(A, 8)
    res = O.multiply(T, T, 1e-6, O.SPAMM)
    b = {p: O.precision_bound(res, p) for p in (O.P_F64, O.P_F32, O.P_BF16X3, O.P_BF16)}
    # finer arithmetic, smaller bound
    assert 0.0 < b[O.P_F64] < b[O.P_F32] < b[O.P_BF16X3] < b[O.P_BF16]
    # linear in the operands' scale: scaling A by 2^5 scales every product
    # norm, and the bound, by exactly 2^5
    T2 = O.build(A * 32.0, 8)
    res2 = O.multiply(T2, T2, 1e-6 * 1024.0, O.SPAMM)
    assert np.array_equal(res2.kept, res.kept)
    assert O.precision_bound(res2, O.P_F32) == 1024.0 * b[O.P_F32]
    # more products per C leaf, larger coefficient; nothing kept, zero bound
    assert O.rounding_coefficient(O.P_F32, 8, 10) > O.rounding_coefficient(O.P_F32, 8, 1)
    empty = O.multiply(T, T, 1e9, O.SPAMM)
    assert len(empty.kept) == 0 and O.precision_bound(empty, O.P_F32) == 0.0


def test_elementwise_truncmul_error_grows_like_sqrt_n():
    """Thm. 1 with the element-wise truncated matrix: a fixed number of
    entries per row falls below tau on a 1D decay matrix, so ||E||_F grows
    like n^{1/2} (the paper's Truncmul trend, Sec. 5), unlike the
    leaf-level budget, whose error does not grow with n."""
    ns = [256, 512, 1024, 2048]
    errs = []
    for n in ns:
        A = synth.DecaySpec("1d", n, 0.3, seed=1).dense()
        At = O.truncate_elementwise(A, 1e-6)
        errs.append(float(np.linalg.norm(O.exact_product(At, At) - O.exact_product(A, A))))
    assert 0.4 <= _slope(ns, errs) <= 0.7


def test_spamm_kept_set_of_a_symmetric_square_is_symmetric():
    """For A = A^T, triple (I, K, J) and (J, K, I) have the same norm product
    up to rounding: leaves (I, K) and (K, I) hold the same values, summed in
    a different order, so s_IK and s_KI may differ in the last bits.  SpAMM
    therefore keeps both or neither except for triples inside the tie band,
    and C = A A is symmetric up to rounding.  (The symmetric-square reading
    takes each lower leaf's decision from its mirror, so its kept set is
    symmetric exactly.)"""
    for kind, n, alpha, bs, tau in (("1d", 512, 0.2, 16, 1e-6), ("3d", 256, 1.0, 16, 1e-4)):
        A = synth.DecaySpec(kind, n, alpha, seed=6).dense()
        assert np.array_equal(A, A.T)
        T = O.build(A, bs)
        r = O.multiply(T, T, tau, O.SPAMM)
        kept = {tuple(t) for t in r.kept.tolist()}
        ties = {tuple(t) for t in O.tie_triples(T, T, tau).tolist()}
        mirrored = {(j, k, i) for i, k, j in kept}
        assert not ((kept ^ mirrored) - ties - {(j, k, i) for i, k, j in ties})
        C = r.C.to_dense()
        assert np.allclose(C, C.T, rtol=0, atol=1e-13 * np.abs(C).max())
