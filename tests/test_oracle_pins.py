"""More pins of the CPU oracle: the parts every GPU check leans on that the
other pin files do not fix on their own.

* ``count_candidates`` against a brute-force count of leaf triples;
* ``build_from_blocks`` against ``build`` of a dense matrix assembled here
  (a repeated coordinate, ragged padding, all-zero blocks);
* ``tie_triples`` against a brute-force band test, on inputs built to sit
  on, inside and just outside the band;
* the skipped bound b_IJ (and so B1, B2 and the Hybrid bound) against a
  per-triple loop that adds only skipped non-null products, k ascending;
Each is built so that a plausible slip (swapped sum axes, a transposed
operand, a kept product added to the bound, the first rather than the last
repeated block) fails it.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth


def _present_grid(rng, G, p):
    return rng.random((G, G)) < p


def _tree_with_structure(pres, bs, rng, scale=None):
    """A tree whose non-null leaves are exactly `pres` (random entries)."""
    G = pres.shape[0]
    M = np.zeros((G * bs, G * bs))
    for I, J in zip(*np.nonzero(pres)):
        blk = rng.standard_normal((bs, bs))
        if scale is not None:
            blk *= scale[I, J]
        M[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = blk
    return O.build(M, bs), M


# ---------------------------------------------------------------- candidates

@pytest.mark.parametrize("seed", range(6))
def test_count_candidates_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    G = [1, 2, 4, 8, 8, 16][seed]
    # A and B with different, lopsided structures: a swap of the two sum
    # axes or of the operands changes the count
    pa = _present_grid(rng, G, 0.7)
    pb = _present_grid(rng, G, 0.3)
    pa[:, 0] = True          # a full first column of A
    pb[G - 1, :] = False     # an empty last row of B
    TA, _ = _tree_with_structure(pa, 2, rng)
    TB, _ = _tree_with_structure(pb, 2, rng)
    want = 0
    for I in range(G):
        for K in range(G):
            for J in range(G):
                if pa[I, K] and pb[K, J]:
                    want += 1
    assert O.count_candidates(TA, TB) == want
    # and it is the number of triples the Truncmul kept list forms at tau 0
    assert len(O.kept_flat(TA, TB, 0.0, False)) == want


def test_count_candidates_is_not_symmetric_in_operands():
    """A lopsided pair where count(A, B) != count(B, A): swapping the
    operands (or the two sum axes) is caught."""
    pa = np.array([[1, 1], [0, 0]], dtype=bool)   # row 0 full
    pb = np.array([[1, 0], [1, 0]], dtype=bool)   # column 0 full
    rng = np.random.default_rng(3)
    TA, _ = _tree_with_structure(pa, 2, rng)
    TB, _ = _tree_with_structure(pb, 2, rng)
    # A B: i = 0, k in {0, 1}, j = 0 -> 2 triples; B A: i in {0, 1}, k = 0,
    # j in {0, 1} -> 4 triples
    assert O.count_candidates(TA, TB) == 2
    assert O.count_candidates(TB, TA) == 4


# ---------------------------------------------------------------- block lists

def _assemble(n, bs, coords, data):
    """Dense n x n from a block list written here: blocks in list order
    (a later block overwrites an earlier one at the same place), then the
    part beyond n dropped."""
    g = -(-n // bs)
    full = np.zeros((g * bs, g * bs))
    for t in range(len(coords)):
        I, J = int(coords[t][0]), int(coords[t][1])
        for r in range(bs):
            for c in range(bs):
                full[I * bs + r, J * bs + c] = data[t][r][c]
    return full[:n, :n].copy()


def _same_tree(T1, T2):
    assert (T1.n, T1.bs, T1.G, T1.L) == (T2.n, T2.bs, T2.G, T2.L)
    assert np.array_equal(T1.index >= 0, T2.index >= 0)
    for I, J in zip(*np.nonzero(T1.index >= 0)):
        assert np.array_equal(T1.leaf(I, J), T2.leaf(I, J))
    for l in range(T1.L + 1):
        assert np.array_equal(T1.sq[l], T2.sq[l])
        assert np.array_equal(T1.present[l], T2.present[l])


@pytest.mark.parametrize("n,bs", [(37, 8), (64, 16), (5, 4), (100, 32)])
def test_build_from_blocks_equals_build_of_assembled_matrix(n, bs):
    rng = np.random.default_rng(n * 7 + bs)
    g = -(-n // bs)
    coords = [(int(a), int(b)) for a, b in rng.integers(0, g, size=(3 * g, 2))]
    coords.append(coords[0])              # a repeated coordinate: the last one wins
    coords.append((g - 1, g - 1))          # the ragged corner leaf
    data = rng.standard_normal((len(coords), bs, bs))
    data[1] = 0.0                          # an all-zero listed block -> null
    if (coords[1] == coords[0]):           # keep the zero block meaningful
        coords[1] = ((coords[0][0] + 1) % g, coords[0][1])
    # entries beyond n in a ragged leaf are padding and must come out zero,
    # whatever the list holds there
    T = O.build_from_blocks(n, bs, np.asarray(coords), data)
    _same_tree(T, O.build(_assemble(n, bs, coords, data), bs))
    # the repeated coordinate really took the later block
    I0, J0 = coords[0]
    last = max(t for t in range(len(coords)) if coords[t] == (I0, J0))
    want = data[last].copy()
    want[max(0, n - I0 * bs):, :] = 0.0
    want[:, max(0, n - J0 * bs):] = 0.0
    if np.any(want != 0):
        assert np.array_equal(T.leaf(I0, J0), want)


def test_build_from_blocks_rejects_outside_coordinates():
    with pytest.raises(ValueError):
        O.build_from_blocks(10, 4, np.array([[3, 0]]), np.ones((1, 4, 4)))


def test_build_from_blocks_decay_list_matches_dense():
    spec = synth.DecaySpec("1d", 300, 0.3, seed=2)
    coords, data = spec.leaf_blocks(32)
    T = O.build_from_blocks(300, 32, coords, data)
    _same_tree(T, O.build(spec.dense(), 32))


# ---------------------------------------------------------------- tie band

def test_tie_triples_brute_force():
    """Leaf norms are chosen so that some norm products fall exactly on tau,
    some inside the 1e-12 band, some just outside it, on both sides."""
    bs, G, tau = 2, 4, 1e-6
    a = 1e-3
    # a factor f moves a norm product to tau * f
    factors = [1.0, 1 + 5e-13, 1 - 5e-13, 1 + 2e-12, 1 - 2e-12, 1 + 1e-9, 0.5, 3.0]
    A = np.zeros((G * bs, G * bs))
    B = np.zeros((G * bs, G * bs))
    rng = np.random.default_rng(9)
    for I in range(G):
        for K in range(G):
            if (I + K) % 3 == 2:
                continue                   # some null leaves in A
            A[I * bs, K * bs] = a          # one entry per leaf: ||A_ik||_F = a
    for K in range(G):
        for J in range(G):
            if (K * 3 + J) % 5 == 4:
                continue                   # some null leaves in B
            f = factors[int(rng.integers(len(factors)))]
            v = tau / a * f                # ||A_ik|| ||B_kj|| = tau * f, to a few ulps
            B[K * bs, J * bs] = v
    TA, TB = O.build(A, bs), O.build(B, bs)
    band = 1e-12
    want = set()
    for I in range(G):
        for K in range(G):
            for J in range(G):
                if not (TA.leaf_present[I, K] and TB.leaf_present[K, J]):
                    continue
                p = math.sqrt(TA.leaf_sq[I, K]) * math.sqrt(TB.leaf_sq[K, J])
                if abs(p - tau) <= band * tau:
                    want.add((I, K, J))
    got = {tuple(t) for t in O.tie_triples(TA, TB, tau, band).tolist()}
    assert got == want
    # the case is not trivial: ties exist, and so do near misses outside
    assert len(want) >= 4
    outside = 0
    for I in range(G):
        for K in range(G):
            for J in range(G):
                if TA.leaf_present[I, K] and TB.leaf_present[K, J] and (I, K, J) not in want:
                    p = math.sqrt(TA.leaf_sq[I, K]) * math.sqrt(TB.leaf_sq[K, J])
                    outside += abs(p - tau) <= 1e-8 * tau
    assert outside >= 1
    # the transposed problem has the transposed ties (B^T A^T)
    gotT = {tuple(t) for t in O.tie_triples(O.build(B.T.copy(), bs), O.build(A.T.copy(), bs), tau,
                                              band).tolist()}
    assert gotT == {(j, k, i) for i, k, j in want}


def test_tie_triples_respect_null_leaves_and_band_width():
    bs, tau = 1, 0.25
    A = np.array([[0.5, 0.0], [0.5, 0.5]])
    B = np.array([[0.5, 0.5], [0.0, 0.5]])
    TA, TB = O.build(A, bs), O.build(B, bs)
    got = {tuple(t) for t in O.tie_triples(TA, TB, tau).tolist()}
    # every non-null product is exactly 0.25; null leaves form no triple
    want = {(I, K, J) for I in range(2) for K in range(2) for J in range(2)
            if A[I, K] != 0 and B[K, J] != 0}
    assert got == want
    assert len(O.tie_triples(TA, TB, tau * (1 + 1e-9))) == 0
    assert len(O.tie_triples(TA, TB, tau * (1 + 1e-9), band=1e-8)) == len(want)


# ---------------------------------------------------------------- skipped bound

def _bound_loop(Au, Bu, tau):
    """b_IJ by a loop over k ascending that adds only the products both
    non-null and skipped by the norm test."""
    G = Au.G
    b = np.zeros((G, G))
    for I in range(G):
        for J in range(G):
            acc = 0.0
            for K in range(G):
                if not (Au.leaf_present[I, K] and Bu.leaf_present[K, J]):
                    continue
                p = math.sqrt(Au.leaf_sq[I, K]) * math.sqrt(Bu.leaf_sq[K, J])
                if not (p >= tau):
                    acc += p
            b[I, J] = acc
    return b


@pytest.mark.parametrize("mode", [O.SPAMM, O.HYBRID])
@pytest.mark.parametrize("case", range(4))
def test_skipped_bound_exact_value(mode, case):
    if case == 0:
        A = synth.DecaySpec("1d", 96, 0.3, seed=4).dense()
        B, bs, taus = A, 8, (1e-6, 1e-3, 0.05)
    elif case == 1:
        A = synth.DecaySpec("3d", 128, 1.0, seed=5).dense()
        B, bs, taus = A, 16, (1e-6, 0.5, 2.0, 5.0)
    elif case == 2:   # distinct, non-symmetric operands
        rng = np.random.default_rng(8)
        A = synth.DecaySpec("1d", 80, 0.25, seed=6).dense() * rng.uniform(0.1, 2.0, size=(80, 80))
        B = synth.DecaySpec("1d", 80, 0.5, seed=7).dense()
        bs, taus = 8, (1e-5, 1e-2)
    else:             # random block structure
        A = synth.dense_from_blocks(128, 8, *synth.random_blocks(3, 128, 8, 0.5))
        B = synth.dense_from_blocks(128, 8, *synth.random_blocks(4, 128, 8, 0.5))
        bs, taus = 8, (1.0, 21.0, 22.0)
    TA, TB = O.build(A, bs), O.build(B, bs)
    skipped_somewhere = False
    for tau in taus:
        r = O.multiply(TA, TB, tau, mode)
        want = _bound_loop(r.A_used, r.B_used, tau)
        err = np.abs(r.skipped_bound - want)
        assert np.all(err <= 1e-15 * want), (tau, err.max())
        skipped_somewhere |= bool(want.sum() > 0)
        # B1 and B2 follow from the b_IJ
        assert abs(r.stats["B1"] - float(np.sum(want))) <= 1e-14 * float(np.sum(want))
        b2 = math.sqrt(float(np.sum(want * want)))
        assert abs(r.stats["B2"] - b2) <= 1e-14 * b2
        # and the scheme's bound is assembled from them as Thms 2-3 state
        if mode == O.SPAMM:
            assert r.stats["err_bound"] == r.stats["B2"]
        else:
            tr_part = r.stats["dA"] * r.stats["normB"] + r.A_used.fro() * r.stats["dB"]
            assert abs(r.stats["err_bound"] - (tr_part + b2)) <= 1e-14 * r.stats["err_bound"]
    assert skipped_somewhere, "the case skips nothing"


def test_skipped_bound_zero_for_truncmul_and_tau_zero():
    A = synth.DecaySpec("1d", 64, 0.3, seed=4).dense()
    T = O.build(A, 8)
    assert not O.multiply(T, T, 1e-3, O.TRUNCMUL).skipped_bound.any()
    r = O.multiply(T, T, 0.0, O.SPAMM)
    assert not r.skipped_bound.any() and r.stats["B1"] == 0.0


# ---------------------------------------------------------------- dense build

@pytest.mark.parametrize("kind,n,bs", [("3d", 1024, 64), ("1d", 1000, 32), ("1d", 77, 16), ("1d", 5, 8)])
def test_dense_build_equals_block_list_of_every_leaf(kind, n, bs):
    """``build`` (whole-array form) against ``build_from_blocks`` with every
    leaf listed (one leaf at a time): the same null map, leaves, slots and
    norms, bit for bit."""
    A = synth.DecaySpec(kind, n, 0.7, seed=2).dense()
    A[:bs, :bs] = 0.0  # one all-zero leaf inside the matrix
    g = -(-n // bs)
    coords = np.array([(I, J) for I in range(g) for J in range(g)])
    data = np.zeros((len(coords), bs, bs))
    for t, (I, J) in enumerate(coords):
        blk = A[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs]
        data[t, :blk.shape[0], :blk.shape[1]] = blk
    T, Tb = O.build(A, bs), O.build_from_blocks(n, bs, coords, data)
    _same_tree(T, Tb)
    assert np.array_equal(T.index, Tb.index)
    assert not T.leaf_present[0, 0] or n <= bs and not np.any(A)


# ---------------------------------------------------------------- truncation ties

def test_truncation_tie_only_where_rounding_can_move_the_boundary():
    """tau = 0 drops nothing and the empty prefix is summed exactly: no tie.
    A boundary sum equal to tau^2 after real additions is a tie."""
    # distinct leaf norms (a symmetric matrix would pair them up, and an
    # equal-norm pair split by the boundary is a tie of its own)
    A = synth.dense_from_blocks(256, 32, *synth.random_blocks(5, 256, 32, 0.6))
    A *= np.random.default_rng(2).uniform(0.5, 2.0, size=A.shape)
    T = O.build(A, 32)
    tr = O.truncate(T, 0.0)
    assert len(tr.dropped) == 0 and not tr.tie
    # tau^2 within rounding of the smallest leaf's squared norm: whether
    # that leaf goes depends on the last bit of a sum -> tie
    s_min = float(T.leaf_sq[T.leaf_present].min())
    tr = O.truncate(T, math.sqrt(s_min))
    assert len(tr.dropped) in (0, 1) and tr.tie
    # well clear of it on either side: no tie
    assert not O.truncate(T, math.sqrt(s_min) * (1 - 1e-9)).tie
    assert not O.truncate(T, math.sqrt(s_min) * (1 + 1e-9)).tie


# ---------------------------------------------------------------- symmetric square

def _brute_pair_truncate(A, bs, tau):
    """Independent mirror-pair truncation: loop-computed leaf norms, pairs
    (I <= K) of weight s_IK + s_KI, bit-loop Morton keys, greedy drop with
    exactly rounded running sums (math.fsum of the leaf norms)."""
    n = A.shape[0]
    g = -(-n // bs)

    def sq(I, K):
        blk = A[I * bs:(I + 1) * bs, K * bs:(K + 1) * bs]
        v = 0.0
        for x in blk.ravel():
            v += x * x
        return v, bool(np.any(blk != 0))

    pairs = []
    for I in range(g):
        for K in range(I, g):
            (a, na), (b, nb) = sq(I, K), sq(K, I)
            if not (na or nb):
                continue
            key = 0
            for bit in range(16):
                key |= ((I >> bit) & 1) << (2 * bit + 1) | ((K >> bit) & 1) << (2 * bit)
            terms = [a] if I == K else [a, b]
            pairs.append((a if I == K else a + b, key, I, K, terms))
    pairs.sort(key=lambda p: (p[0], p[1]))
    out = A.copy()
    taken = []
    for w, key, I, K, terms in pairs:
        if math.fsum(taken + terms) <= tau * tau:
            taken += terms
            out[I * bs:(I + 1) * bs, K * bs:(K + 1) * bs] = 0.0
            out[K * bs:(K + 1) * bs, I * bs:(I + 1) * bs] = 0.0
        else:
            break
    return out


@pytest.mark.parametrize("kind,n,alpha,bs", [("1d", 96, 0.3, 8), ("3d", 128, 1.0, 16), ("1d", 200, 0.05, 8)])
def test_pair_truncation_brute_force_and_invariants(kind, n, alpha, bs):
    A = synth.DecaySpec(kind, n, alpha, seed=11).dense()
    T = O.build(A, bs)
    for tau in (1e-8, 1e-5, 1e-3, 1e-1, 1.0):
        tr = O.truncate_pairs(T, tau)
        At = tr.tree.to_dense()
        assert np.array_equal(At, _brute_pair_truncate(A, bs, tau))
        # symmetric, within budget, and maximal: the next pair would break it
        assert np.array_equal(At, At.T)
        assert np.linalg.norm(A - At) <= tau * (1 + 1e-12)
        assert math.sqrt(tr.dropped_sq) <= tau * (1 + 1e-15)
        if tr.boundary_sq[1] < math.inf:
            assert tr.boundary_sq[1] > tau * tau or tr.tie


@pytest.mark.parametrize("mode", [O.SPAMM, O.HYBRID])
@pytest.mark.parametrize("kind,n,alpha,bs,tau", [("1d", 300, 0.2, 16, 1e-6), ("3d", 256, 1.0, 16, 1e-3),
                                                 ("1d", 200, 0.05, 8, 1e-2)])
def test_symmetric_square_reading(mode, kind, n, alpha, bs, tau):
    """Upper C leaves as the norm test decides them on the (pair-truncated)
    operand, each lower leaf the exact transpose of its mirror with the
    mirror's bound; against a loop over the upper leaves and the full
    product of the same operand."""
    A = synth.DecaySpec(kind, n, alpha, seed=6).dense()
    assert np.array_equal(A, A.T)
    T = O.build(A, bs)
    Au = O.truncate_pairs(T, tau).tree if mode == O.HYBRID else T
    full = O.multiply(Au, Au, tau, O.SPAMM)
    sym = O.multiply_symmetric(T, tau, mode)
    assert not sym.stats["sym_fallback"]
    assert np.array_equal(sym.A_used.index >= 0, Au.index >= 0)
    want = []
    for I in range(T.G):
        for J in range(I, T.G):
            for K in range(T.G):
                if Au.leaf_present[I, K] and Au.leaf_present[K, J] and \
                        math.sqrt(Au.leaf_sq[I, K]) * math.sqrt(Au.leaf_sq[K, J]) >= tau:
                    want.append((I, K, J))
    assert {tuple(t) for t in sym.kept.tolist()} == set(want)
    assert sym.stats["n_kept"] == len(want)
    for I in range(T.G):
        for J in range(T.G):
            assert sym.C.leaf_present[I, J] == sym.C.leaf_present[J, I]
            if sym.C.leaf_present[I, J]:
                if I <= J:
                    acc = np.zeros((bs, bs))
                    for (i, k, j) in want:
                        if (i, j) == (I, J):
                            acc = acc + Au.leaf(I, k) @ Au.leaf(k, J)
                    assert np.array_equal(sym.C.leaf(I, J), acc)
                else:
                    assert np.array_equal(sym.C.leaf(I, J), sym.C.leaf(J, I).T)
            assert sym.skipped_bound[I, J] == sym.skipped_bound[min(I, J), max(I, J)]
    Cf, Cs = full.C.to_dense(), sym.C.to_dense()
    assert np.linalg.norm(Cs - Cf) <= 1e-14 * max(np.linalg.norm(Cf), 1e-300)
    assert np.array_equal(Cs, Cs.T)
    if mode == O.HYBRID:  # Thm. 3's terms with the pair truncation's dA
        dA = sym.stats["dA"]
        assert dA <= tau and abs(dA - np.linalg.norm(A - Au.to_dense())) <= 1e-12 * max(dA, 1e-300) + 1e-300


def test_pair_truncation_keeps_mirror_pairs_together():
    """Leaves (0, 1) and (1, 0) have exactly equal norms and tau^2 lies between
    one and two of them: the leaf-by-leaf truncation drops (0, 1) alone,
    the pair truncation neither (their weight 0.5 is above 0.3)."""
    bs = 4
    A = np.zeros((8, 8))
    A[0:4, 0:4] = np.eye(4) * 2.0
    A[4:8, 4:8] = np.eye(4) * 3.0
    A[0, 4] = A[4, 0] = 0.5          # s = 0.25 for both off-diagonal leaves
    T = O.build(A, bs)
    tau = math.sqrt(0.3)
    assert [tuple(x) for x in O.truncate(T, tau).dropped.tolist()] == [(0, 1)]
    assert len(O.truncate_pairs(T, tau).dropped) == 0
    assert {tuple(x) for x in O.truncate_pairs(T, math.sqrt(0.5)).dropped.tolist()} == {(0, 1), (1, 0)}


def test_symmetric_square_falls_back_when_the_null_map_is_not_symmetric():
    """A whose leaf (0, 1) is non-null and (1, 0) null: the mirror
    decisions would be wrong, so every C leaf is formed by its own test."""
    bs = 4
    A = np.zeros((8, 8))
    A[0:4, 0:4] = np.eye(4) * 2.0
    A[4:8, 4:8] = np.eye(4) * 3.0
    A[0, 4] = 0.5
    T = O.build(A, bs)
    for mode in (O.SPAMM, O.HYBRID):
        sym = O.multiply_symmetric(T, 1e-9, mode)
        full = O.multiply(T, T, 1e-9, O.SPAMM)
        assert sym.stats["sym_fallback"]
        assert np.array_equal(sym.kept, full.kept)
        assert np.array_equal(sym.C.to_dense(), full.C.to_dense())
