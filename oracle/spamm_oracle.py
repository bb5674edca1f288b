"""CPU FP64 oracle for approximate products of matrices with decay.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the GPU library (no kernels, headers, helpers or tables); it reads its
inputs from the ``synth`` generators or from plain arrays.

It follows A. G. Artemov, "Approximate multiplication of nearly sparse
matrices with decay in a fully recursive distributed task-based parallel
framework" (arXiv:1906.08148):

* Sec. 2 (SpAMM algorithm): a matrix is a quadtree whose level-t node splits
  into four level-(t+1) children; every node carries its squared Frobenius
  norm, the sum of its children's squared norms.
* Alg. 1 (SpAMM): child product (i,k,j) is formed only when
  ||A_ik||_F * ||B_kj||_F >= tau; the lowest level returns the plain product.
* Alg. 2 (MatrixMultiply) and Sec. 4.2: zero sub-matrices are stored as null;
  a product with a null operand is null.
* Sec. 4.4 (leaf level library): the hierarchy stops at a dense leaf block,
  kept when it holds at least one non-zero value.
* Sec. 3, eq. (truncated_matrices) and Thms 1-3: Truncmul multiplies the
  truncated inputs, SpAMM skips small products, Hybrid applies SpAMM to the
  truncated inputs with the same tau (proof of Thm 3).

Readings where the paper is silent (each listed with its reason in the design
notes of the repository):

* Truncation drops whole leaf blocks: the leaves are ordered by (squared norm,
  Morton key) and the longest prefix whose *exact* summed squared norm is
  <= tau^2 is dropped, so ||A - A~||_F <= tau.  Element-wise truncation
  (the theorems' object) is ``truncate_elementwise``.
* The norm test is ``sqrt(sA) * sqrt(sB) >= tau`` in FP64 with correctly
  rounded square roots; null blocks never form products, also at tau = 0.
* The test is applied uniformly at leaf triples, so a single-leaf matrix is
  also tested (the task type of Sec. 4.3 checks its own operands).
* Products within one C block are summed over k ascending.
* Parent squared norms are summed as ((c00 + c01) + c10) + c11.

Everything is FP64.  Nothing here is blocked, fused or reordered beyond what
the definitions above state.
"""
from __future__ import annotations

import math
from fractions import Fraction
from dataclasses import dataclass, field

import numpy as np

TRUNCMUL, SPAMM, HYBRID = 0, 1, 2
MODE_NAMES = {TRUNCMUL: "truncmul", SPAMM: "spamm", HYBRID: "hybrid"}


# --------------------------------------------------------------------------
# Quadtree layout (Sec. 2): level 0 is the root, level L holds the G x G leaves
# --------------------------------------------------------------------------

def grid_size(n: int, bs: int):
    """G = ceil(n/bs) rounded up to a power of two, and L = log2(G)."""
    g = -(-n // bs)
    G = 1
    while G < g:
        G *= 2
    return G, G.bit_length() - 1


def morton_key(I, J):
    """Z-order key of block (I, J); the row bit sits above the column bit,
    so the children of node (I, J) are 4*key(I,J) + 2a + b for (2I+a, 2J+b)."""
    I = np.asarray(I, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    key = np.zeros(np.broadcast(I, J).shape, dtype=np.int64)
    top = int(max(I.max(initial=0), J.max(initial=0)))
    for b in range(top.bit_length()):  # higher bits of I and J are zero
        key |= ((I >> b) & 1) << (2 * b + 1)
        key |= ((J >> b) & 1) << (2 * b)
    return key


@dataclass
class Tree:
    """A matrix as a quadtree of bs x bs leaves (Sec. 2, Sec. 4.4).

    ``index[I, J]`` is the row of ``blocks`` holding leaf (I, J), or -1 when
    the leaf is null.  ``sq[l]`` is the (2^l x 2^l) array of squared Frobenius
    norms at level l (0 for null nodes) and ``present[l]`` says which nodes
    are non-null.
    """
    n: int
    bs: int
    G: int
    L: int
    index: np.ndarray
    blocks: np.ndarray
    sq: list = field(default_factory=list)
    present: list = field(default_factory=list)

    def leaf(self, I: int, J: int) -> np.ndarray:
        return self.blocks[self.index[I, J]]

    @property
    def leaf_sq(self) -> np.ndarray:
        return self.sq[self.L]

    @property
    def leaf_present(self) -> np.ndarray:
        return self.present[self.L]

    def fro(self) -> float:
        return math.sqrt(self.sq[0][0, 0])

    def to_dense(self) -> np.ndarray:
        bs, G = self.bs, self.G
        full = np.zeros((G * bs, G * bs), dtype=np.float64)
        for I, J in zip(*np.nonzero(self.index >= 0)):
            full[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = self.leaf(I, J)
        return full[:self.n, :self.n]

    def nonnull_count(self) -> int:
        return int((self.index >= 0).sum())


def pyramid(leaf_sq: np.ndarray, leaf_present: np.ndarray):
    """Squared norms of every level (Sec. 2): a parent is the FP64 sum of its
    four children, taken as ((c00 + c01) + c10) + c11."""
    sq = [leaf_sq]
    present = [leaf_present]
    while sq[0].shape[0] > 1:
        c = sq[0]
        p = present[0]
        parent = ((c[0::2, 0::2] + c[0::2, 1::2]) + c[1::2, 0::2]) + c[1::2, 1::2]
        par_p = p[0::2, 0::2] | p[0::2, 1::2] | p[1::2, 0::2] | p[1::2, 1::2]
        sq.insert(0, parent)
        present.insert(0, par_p)
    return sq, present


def _from_leaves(n, bs, G, L, coords, blocks) -> Tree:
    """Tree from candidate leaves ``blocks[t]`` at ``coords[t] = (I, J)``
    (zero-padded bs x bs each); all-zero candidates become null."""
    index = np.full((G, G), -1, dtype=np.int64)
    leaf_sq = np.zeros((G, G), dtype=np.float64)
    nonzero = np.zeros((G, G), dtype=bool)
    kept = []
    for (I, J), b in zip(coords, blocks):
        if not np.any(b != 0):
            continue
        index[I, J] = len(kept)
        kept.append(b)
        nonzero[I, J] = True
        leaf_sq[I, J] = np.sum(b * b)
    store = np.asarray(kept, dtype=np.float64).reshape(-1, bs, bs)
    sq, present = pyramid(leaf_sq, nonzero)
    return Tree(n, bs, G, L, index, store, sq, present)


def build(dense: np.ndarray, bs: int) -> Tree:
    """Pad A to bs*G, cut it into G x G leaves, null the all-zero leaves and
    compute the squared-norm pyramid (Sec. 2; Sec. 4.2; Sec. 4.4)."""
    dense = np.asarray(dense, dtype=np.float64)
    n = dense.shape[0]
    if n < 1 or dense.shape != (n, n):
        raise ValueError("need a square matrix with n >= 1")
    G, L = grid_size(n, bs)
    full = np.zeros((G * bs, G * bs), dtype=np.float64)
    full[:n, :n] = dense
    leafs4 = full.reshape(G, bs, G, bs).transpose(0, 2, 1, 3)
    # the leaves in row-major (I, J) order, all-zero ones null, as
    # _from_leaves does for a list; each leaf's squared norm is the sum of
    # its own bs * bs squares, as there
    leafs4 = np.ascontiguousarray(leafs4)
    del full
    present = np.any(leafs4 != 0, axis=(2, 3))
    store = leafs4[present]
    del leafs4
    index = np.full((G, G), -1, dtype=np.int64)
    index[present] = np.arange(len(store))
    sqs = np.empty(len(store), dtype=np.float64)
    for c0 in range(0, len(store), 4096):  # in chunks: small temporaries
        blk = store[c0:c0 + 4096]
        sqs[c0:c0 + 4096] = np.sum(blk * blk, axis=(1, 2))
    leaf_sq = np.zeros((G, G), dtype=np.float64)
    leaf_sq[present] = sqs
    sq, pres = pyramid(leaf_sq, present)
    return Tree(n, bs, G, L, index, store.reshape(-1, bs, bs), sq, pres)


def build_from_blocks(n: int, bs: int, coords: np.ndarray, data: np.ndarray) -> Tree:
    """Same as ``build`` for a list of (I, J) blocks: unlisted blocks are zero,
    a repeated coordinate keeps its last block and entries beyond row or
    column n are padding (zero)."""
    if n < 1:
        raise ValueError("n must be >= 1")
    G, L = grid_size(n, bs)
    gmax = -(-n // bs)
    last = {}
    for t, (I, J) in enumerate(np.asarray(coords).reshape(-1, 2)):
        if not (0 <= I < gmax and 0 <= J < gmax):
            raise ValueError("block coordinate outside the matrix")
        last[(int(I), int(J))] = t
    cs, bl = [], []
    for (I, J), t in sorted(last.items()):
        b = np.array(data[t], dtype=np.float64, copy=True)
        b[max(0, n - I * bs):, :] = 0.0
        b[:, max(0, n - J * bs):] = 0.0
        cs.append((I, J))
        bl.append(b)
    return _from_leaves(n, bs, G, L, cs, bl)


def with_leaves_dropped(t: Tree, drop_mask: np.ndarray) -> Tree:
    """Copy of ``t`` with the leaves in ``drop_mask`` set to null, pyramid
    recomputed from the surviving leaves."""
    index = t.index.copy()
    index[drop_mask] = -1
    present = index >= 0
    leaf_sq = np.where(present, t.leaf_sq, 0.0)
    sq, pres = pyramid(leaf_sq, present)
    return Tree(t.n, t.bs, t.G, t.L, index, t.blocks, sq, pres)


# --------------------------------------------------------------------------
# Input truncation (vector-space truncation, Sec. 3)
# --------------------------------------------------------------------------

def _exact_scaled(x: float) -> int:
    """x * 2**1074 as an exact integer (every finite double is a multiple
    of 2**-1074)."""
    num, den = float(x).as_integer_ratio()
    return num * (1 << 1074) // den


@dataclass
class Truncation:
    tree: Tree
    dropped: np.ndarray          # (r, 2) leaf coords dropped, in drop order
    dropped_sq: float            # FP64 of the exact dropped squared norm
    boundary_sq: tuple           # exact (sum up to r*, sum up to r*+1) as floats
    tie: bool                    # boundary within the 1e-12 tie band


def truncate(t: Tree, tau: float) -> Truncation:
    """Leaf-block truncation with a global Frobenius budget tau.

    Order the non-null leaves by (squared norm, Morton key) ascending and drop
    the longest prefix whose exact summed squared norm is <= tau^2; the
    Frobenius norm of what is removed is then <= tau."""
    if not (tau >= 0.0) or math.isinf(tau):
        raise ValueError("tau must be finite and >= 0")
    I, J = np.nonzero(t.index >= 0)
    s = t.leaf_sq[I, J]
    keys = morton_key(I, J)
    order = np.lexsort((keys, s))      # primary s, secondary Morton key
    tnum, tden = float(tau).as_integer_ratio()
    # compare  sum * 2^-1074 <= (tnum/tden)^2  exactly
    limit_lhs_scale = tden * tden
    limit_rhs = tnum * tnum * (1 << 1074)
    acc = 0
    r = 0
    for idx in order:
        nxt = acc + _exact_scaled(s[idx])
        if nxt * limit_lhs_scale <= limit_rhs:
            acc = nxt
            r += 1
        else:
            break
    nxt_sum = acc + (_exact_scaled(s[order[r]]) if r < len(order) else 0)
    dropped_idx = order[:r]
    drop_mask = np.zeros_like(t.index, dtype=bool)
    drop_mask[I[dropped_idx], J[dropped_idx]] = True
    tau2 = float(tau) * float(tau)
    b0 = float(Fraction(acc, 1 << 1074))
    b1 = float(Fraction(nxt_sum, 1 << 1074)) if r < len(order) else math.inf
    band = 1e-12 * tau2
    # a dropped prefix of zero squared norm (nothing dropped, or only leaves
    # whose squares underflow) is summed exactly on every side: no tie there
    tie = (b0 > 0.0 and abs(b0 - tau2) <= band) or (r < len(order) and abs(b1 - tau2) <= band)
    # equal-norm run straddling the boundary also counts as a tie
    if 0 < r < len(order) and s[order[r - 1]] == s[order[r]]:
        tie = True
    dropped = np.stack([I[dropped_idx], J[dropped_idx]], axis=1)
    return Truncation(with_leaves_dropped(t, drop_mask), dropped, b0, (b0, b1), tie)


def truncate_pairs(t: Tree, tau: float) -> Truncation:
    """Leaf-block truncation of a symmetric matrix in mirror pairs, with the
    same global budget tau (a reading for the symmetric square; the paper's
    truncation is Sec. 3's, it does not exploit symmetry).

    Each leaf (I, K) with I < K forms a pair with (K, I) of weight
    w = s_IK + s_KI (FP64 sum), each diagonal leaf is a pair of its own with
    w = s_II; pairs with a non-null leaf are ordered by (w, Morton key of
    (I, K)) and the longest prefix whose exact summed squared norms stay
    <= tau^2 is dropped, both leaves of a pair together.  The result is
    symmetric whenever the input's null map is, and ||A - A~||_F <= tau."""
    if not (tau >= 0.0) or math.isinf(tau):
        raise ValueError("tau must be finite and >= 0")
    pres, sq = t.leaf_present, t.leaf_sq
    I, K = np.nonzero(np.triu(pres | pres.T))
    w = np.where(I == K, sq[I, K], sq[I, K] + sq[K, I])
    keys = morton_key(I, K)
    order = np.lexsort((keys, w))
    tnum, tden = float(tau).as_integer_ratio()
    limit_lhs_scale = tden * tden
    limit_rhs = tnum * tnum * (1 << 1074)

    def exact(i, k):
        e = _exact_scaled(sq[i, k])
        return e if i == k else e + _exact_scaled(sq[k, i])

    acc = 0
    r = 0
    for idx in order:
        nxt = acc + exact(I[idx], K[idx])
        if nxt * limit_lhs_scale <= limit_rhs:
            acc = nxt
            r += 1
        else:
            break
    nxt_sum = acc + (exact(I[order[r]], K[order[r]]) if r < len(order) else 0)
    drop_mask = np.zeros_like(t.index, dtype=bool)
    d = order[:r]
    drop_mask[I[d], K[d]] = True
    drop_mask[K[d], I[d]] = True
    drop_mask &= pres
    tau2 = float(tau) * float(tau)
    b0 = float(Fraction(acc, 1 << 1074))
    b1 = float(Fraction(nxt_sum, 1 << 1074)) if r < len(order) else math.inf
    band = 1e-12 * tau2
    tie = (b0 > 0.0 and abs(b0 - tau2) <= band) or (r < len(order) and abs(b1 - tau2) <= band)
    if 0 < r < len(order) and w[order[r - 1]] == w[order[r]]:
        tie = True
    dI, dJ = np.nonzero(drop_mask)
    return Truncation(with_leaves_dropped(t, drop_mask), np.stack([dI, dJ], axis=1), b0, (b0, b1), tie)


def truncate_elementwise(dense: np.ndarray, tau: float) -> np.ndarray:
    """Eq. (truncated_matrices): zero every entry with |a_ij| < tau."""
    out = np.array(dense, dtype=np.float64, copy=True)
    out[np.abs(out) < tau] = 0.0
    return out


# --------------------------------------------------------------------------
# Which leaf products are formed (Alg. 1, Alg. 2)
# --------------------------------------------------------------------------

def norm_test(sa, sb, tau) -> np.ndarray:
    """Alg. 1's test: ||A_ik||_F ||B_kj||_F >= tau, from squared norms."""
    return np.sqrt(sa) * np.sqrt(sb) >= tau


def kept_flat(A: Tree, B: Tree, tau: float, use_norms: bool) -> np.ndarray:
    """All leaf triples (I, K, J) whose product is formed: both operands
    non-null and, when ``use_norms``, the norm test passes.

    Returns an int64 (m, 3) array sorted by (Morton key of (I, J), K)."""
    G = A.G
    pa, pb = A.leaf_present, B.leaf_present
    out = []
    for I in range(G):
        ks = np.nonzero(pa[I])[0]
        if len(ks) == 0:
            continue
        ok = pb[ks, :]                                   # (|ks|, G)
        if use_norms:
            ok = ok & norm_test(A.leaf_sq[I, ks][:, None], B.leaf_sq[ks, :], tau)
        kk, jj = np.nonzero(ok)
        if len(kk):
            out.append(morton_key(I, jj) * G + ks[kk])
    return _decode_sorted(out, G)


def _decode_sorted(keys_list, G) -> np.ndarray:
    """Sort keys morton(I,J)*G + K and turn them back into (I, K, J) rows."""
    if not keys_list:
        return np.zeros((0, 3), dtype=np.int64)
    keys = np.sort(np.concatenate(keys_list).astype(np.int64))
    K = keys % G
    m = keys // G
    I = np.zeros_like(m)
    J = np.zeros_like(m)
    for b in range((G - 1).bit_length()):  # coordinates are below G
        I |= ((m >> (2 * b + 1)) & 1) << b
        J |= ((m >> (2 * b)) & 1) << b
    return np.stack([I, K, J], axis=1)


def count_candidates(A: Tree, B: Tree) -> int:
    """Number of leaf triples with both operands non-null."""
    pa = A.leaf_present.astype(np.int64)
    pb = B.leaf_present.astype(np.int64)
    return int((pa.sum(axis=0) * pb.sum(axis=1)).sum())


def kept_recursive(A: Tree, B: Tree, tau: float, use_norms: bool) -> np.ndarray:
    """Alg. 1 (and, without norms, Alg. 2's null rule) run literally on the
    two quadtrees from the root, recording each leaf triple reached.

    The first call tests the root pair itself, as the SpAMM task type of
    Sec. 4.3 checks its operands; for L >= 1 that test never changes the
    result because a parent's norm is never smaller than a child's."""
    L = A.L
    found = []

    def passes(level, ia, ka, kb, jb):
        if not (A.present[level][ia, ka] and B.present[level][kb, jb]):
            return False
        if not use_norms:
            return True
        return bool(norm_test(A.sq[level][ia, ka], B.sq[level][kb, jb], tau))

    def rec(level, I, K, J):
        if level == L:
            found.append((I, K, J))
            return
        for i in (0, 1):
            for j in (0, 1):
                for k in (0, 1):
                    ci, ck, cj = 2 * I + i, 2 * K + k, 2 * J + j
                    if passes(level + 1, ci, ck, ck, cj):
                        rec(level + 1, ci, ck, cj)

    if passes(0, 0, 0, 0, 0):
        rec(0, 0, 0, 0)
    if not found:
        return np.zeros((0, 3), dtype=np.int64)
    t = np.asarray(found, dtype=np.int64)
    return _decode_sorted([morton_key(t[:, 0], t[:, 2]) * A.G + t[:, 1]], A.G)


# --------------------------------------------------------------------------
# The product and its accounting
# --------------------------------------------------------------------------

@dataclass
class Result:
    C: Tree
    kept: np.ndarray             # (m, 3) (I, K, J), C-Morton order, K ascending
    A_used: Tree                 # operand after truncation (or A itself)
    B_used: Tree
    skipped_bound: np.ndarray    # (G, G) b_IJ = sum of skipped norm products
    stats: dict


def _check_pair(A: Tree, B: Tree, tau: float):
    if A.n != B.n or A.bs != B.bs:
        raise ValueError("A and B differ in n or leaf size")
    if not (tau >= 0.0) or math.isinf(tau):
        raise ValueError("tau must be finite and >= 0")


def multiply(A: Tree, B: Tree, tau: float, mode: int, c_blocks=None) -> Result:
    """C ~= A B by Truncmul, SpAMM or Hybrid.

    Truncmul multiplies the truncated inputs and forms every non-null product
    (Sec. 5.3 notes that no gemm is skipped); SpAMM forms the products that
    pass Alg. 1's norm test; Hybrid applies SpAMM to the inputs truncated with
    the same tau.  ``c_blocks`` (optional list of (I, J)) limits which C leaves
    are computed numerically; structure and accounting are always complete.
    """
    _check_pair(A, B, tau)
    dA = dB = 0.0
    tieA = tieB = False
    if mode in (TRUNCMUL, HYBRID):
        ta = truncate(A, tau)
        tb = ta if B is A else truncate(B, tau)
        Au, Bu = ta.tree, tb.tree
        dA, dB = math.sqrt(ta.dropped_sq), math.sqrt(tb.dropped_sq)
        tieA, tieB = ta.tie, tb.tie
    elif mode == SPAMM:
        Au, Bu = A, B
    else:
        raise ValueError("unknown mode")
    use_norms = mode in (SPAMM, HYBRID)
    kept = kept_flat(Au, Bu, tau, use_norms)
    n_candidates = count_candidates(Au, Bu)

    G, bs = A.G, A.bs
    # skipped-product bound b_IJ: sum over non-null but skipped k, k ascending
    bnd = np.zeros((G, G), dtype=np.float64)
    if use_norms:
        for I in range(G):
            ks = np.nonzero(Au.leaf_present[I])[0]
            if len(ks) == 0:
                continue
            prod = np.sqrt(Au.leaf_sq[I, ks])[:, None] * np.sqrt(Bu.leaf_sq[ks, :])
            skip = Bu.leaf_present[ks, :] & ~(prod >= tau)
            # row-by-row accumulation = a sequential sum over k ascending
            bnd[I, :] = np.where(skip, prod, 0.0).sum(axis=0)

    # C leaves: sum over kept k ascending of A_IK @ B_KJ
    want = None if c_blocks is None else {(int(a), int(b)) for a, b in c_blocks}
    c_index = np.full((G, G), -1, dtype=np.int64)
    c_list = []
    c_present = np.zeros((G, G), dtype=bool)
    if len(kept):
        c_present[kept[:, 0], kept[:, 2]] = True
    rows = kept
    if want is not None and len(kept):
        wkeys = np.array([morton_key(I, J) for I, J in want], dtype=np.int64)
        rows = kept[np.isin(morton_key(kept[:, 0], kept[:, 2]), wkeys)]
    # kept is sorted by (Morton key of (I, J), K): each C leaf is one run
    if len(rows):
        rk = morton_key(rows[:, 0], rows[:, 2])
        starts = np.flatnonzero(np.r_[True, rk[1:] != rk[:-1]])
        ends = np.r_[starts[1:], len(rows)]
    else:
        starts = ends = np.zeros(0, dtype=np.int64)
    for a, b in zip(starts, ends):
        I, J = int(rows[a, 0]), int(rows[a, 2])
        acc = np.zeros((bs, bs), dtype=np.float64)
        for K in rows[a:b, 1]:
            acc = acc + Au.leaf(I, int(K)) @ Bu.leaf(int(K), J)
        c_index[I, J] = len(c_list)
        c_list.append(acc)
    blocks = np.asarray(c_list, dtype=np.float64).reshape(-1, bs, bs)
    c_sq = np.zeros((G, G), dtype=np.float64)
    for I, J in zip(*np.nonzero(c_index >= 0)):
        b = blocks[c_index[I, J]]
        c_sq[I, J] = np.sum(b * b)
    sq, pres = pyramid(c_sq, c_present)
    C = Tree(A.n, bs, G, A.L, c_index, blocks, sq, pres)

    B1 = float(np.sum(bnd)) if use_norms else 0.0
    B2 = math.sqrt(float(np.sum(bnd * bnd))) if use_norms else 0.0
    normA, normB = A.fro(), B.fro()
    normAu = Au.fro()
    if mode == SPAMM:
        bound = B2
    elif mode == TRUNCMUL:
        bound = dA * normB + normAu * dB
    else:
        bound = dA * normB + normAu * dB + B2
    stats = dict(
        mode=mode, tau=tau, bs=bs, n=A.n, G=G, L=A.L,
        n_kept=int(len(kept)), n_candidates=n_candidates,
        flops=2.0 * bs ** 3 * len(kept),
        c_nonnull=int(c_present.sum()),
        B1=B1, B2=B2, dA=dA, dB=dB, normA=normA, normB=normB,
        err_bound=bound, trunc_tie=(tieA or tieB),
    )
    return Result(C, kept, Au, Bu, bnd, stats)


def multiply_symmetric(A: Tree, tau: float, mode: int, c_blocks=None) -> Result:
    """The square of a symmetric A formed on the upper triangle of C.

    A reading the paper leaves open (it does not exploit symmetry, Sec. 5.4):
    for A = A^T the product A A is symmetric, and the leaf triple (I, K, J)
    pairs with (J, K, I), whose norm product is the same up to the rounding
    of the two leaf norms.  Hybrid truncates A in mirror pairs
    (``truncate_pairs``), so the truncated operand stays symmetric.  The
    norm test decides the C leaves with I <= J; each leaf below the
    diagonal takes its mirror's decision and is the transpose of its
    mirror, with the mirror's skipped bound.  When the operand's null map is
    not symmetric all the same (A itself was not), every C leaf is formed
    by its own test instead.  The kept list holds the formed products: the
    upper ones, or all of them in that fallback."""
    if mode not in (SPAMM, HYBRID):
        raise ValueError("symmetric square: SpAMM or Hybrid")
    want = None
    if c_blocks is not None:  # the requested leaves and their mirrors
        want = sorted({(int(a), int(b)) for a, b in c_blocks} | {(int(b), int(a)) for a, b in c_blocks})
    if mode == HYBRID:
        tr = truncate_pairs(A, tau)
        full = multiply(tr.tree, tr.tree, tau, SPAMM, c_blocks=want)
        dA = math.sqrt(tr.dropped_sq)
        full.stats.update(mode=HYBRID, dA=dA, dB=dA, normA=A.fro(), normB=A.fro(), trunc_tie=tr.tie,
                          err_bound=dA * A.fro() + tr.tree.fro() * dA + full.stats["B2"])
    else:
        full = multiply(A, A, tau, SPAMM, c_blocks=want)
    Au = full.A_used
    pres = Au.leaf_present
    if not np.array_equal(pres, pres.T):
        full.stats["sym_fallback"] = True
        return full
    G = A.G
    kept = full.kept[full.kept[:, 0] <= full.kept[:, 2]]
    bnd = full.skipped_bound.copy()
    lower = np.tril_indices(G, -1)
    bnd[lower] = full.skipped_bound.T[lower]
    c_present = full.C.leaf_present.copy()
    c_present[lower] = full.C.leaf_present.T[lower]
    c_index = np.full((G, G), -1, dtype=np.int64)
    blocks = []
    for I, J in zip(*np.nonzero(c_present)):
        a, b = (I, J) if I <= J else (J, I)
        if full.C.index[a, b] < 0:
            continue  # a leaf not computed (outside c_blocks)
        src = full.C.leaf(a, b) if I <= J else full.C.leaf(a, b).T
        c_index[I, J] = len(blocks)
        blocks.append(np.array(src))
    bs = A.bs
    blocks = np.asarray(blocks, dtype=np.float64).reshape(-1, bs, bs)
    c_sq = np.zeros((G, G), dtype=np.float64)
    for I, J in zip(*np.nonzero(c_index >= 0)):
        b = blocks[c_index[I, J]]
        c_sq[I, J] = np.sum(b * b)
    sq, pr = pyramid(c_sq, c_present)
    C = Tree(A.n, bs, G, A.L, c_index, blocks, sq, pr)
    stats = dict(full.stats)
    B2 = math.sqrt(float(np.sum(bnd * bnd)))
    dA, normB, normAu = stats["dA"], stats["normB"], Au.fro()
    stats.update(n_kept=int(len(kept)), flops=2.0 * bs ** 3 * len(kept), c_nonnull=int(c_present.sum()),
                 B1=float(np.sum(bnd)), B2=B2, sym_fallback=False,
                 err_bound=B2 if mode == SPAMM else dA * normB + normAu * dA + B2)
    # the rounding bound of a mirrored leaf is its mirror's (same products)
    return Result(C, kept, Au, Au, bnd, stats)


# Unit roundoffs: FP64, FP32 and BF16 (8 significand bits, round to nearest).
U64, U32, U16 = 2.0 ** -53, 2.0 ** -24, 2.0 ** -8
# Compute precisions of the leaf products: FP64 inputs and sums; FP32 inputs
# and sums; BF16 inputs (the FP32 value rounded to BF16) with FP32 sums;
# split BF16 (x ~ hi + lo, both BF16, products hi*hi + hi*lo + lo*hi) with
# FP32 sums.
P_F64, P_F32, P_BF16, P_BF16X3 = "f64", "f32", "bf16", "bf16x3"


def gamma(n: float, u: float) -> float:
    """gamma_n = n u / (1 - n u): the classical bound on the relative error
    accumulated by n roundings (Higham, Accuracy and Stability of Numerical
    Algorithms, Lemma 3.1)."""
    return n * u / (1.0 - n * u)


def rounding_coefficient(prec: str, bs: int, m: int) -> float:
    """c such that every entry of the computed sum of m leaf products of
    order bs differs from the exact sum of those products by at most
    c * (sum_k |A_ik| |B_kj|) entry-wise.

    Two parts: the representation error of the inputs in the compute
    precision (e_in, for a product of two represented values) and the
    roundings of the sum (gamma over the longest chain of roundings an entry
    goes through: one product rounding, bs - 1 additions inside a leaf
    product, three times that for split BF16, and m additions across
    products), scaled by the size of the represented inputs (mag).  This is
    a bound we define for the output accounting; the paper gives none.
    """
    if prec == P_F64:
        e_in, mag, u, depth = 0.0, 1.0, U64, bs + m + 1
    elif prec == P_F32:
        e = U32  # FP64 -> FP32
        e_in, mag, u, depth = 2.0 * e + e * e, (1.0 + e) ** 2, U32, bs + m + 1
    elif prec == P_BF16:
        e = U32 + U16 * (1.0 + U32)  # FP64 -> FP32 -> BF16
        e_in, mag, u, depth = 2.0 * e + e * e, (1.0 + e) ** 2, U32, bs + m + 1
    elif prec == P_BF16X3:
        e3 = U32 + U16 * U16 * (1.0 + U32)  # |hi + lo - x| <= e3 |x|
        el = (1.0 + U16) * U16 * (1.0 + U32)  # |lo| <= el |x|
        h = (1.0 + U16) * (1.0 + U32) + el  # |hi| + |lo| <= h |x|
        # (hi_a + lo_a)(hi_b + lo_b) - lo_a lo_b against a b
        e_in, mag, u, depth = 2.0 * e3 + e3 * e3 + el * el, h * h, U32, 3 * bs + m + 1
    else:
        raise ValueError("unknown precision")
    return e_in + gamma(depth, u) * mag


def precision_bound(res: "Result", prec: str) -> float:
    """Bound on ||C_computed - C_kept||_F, where C_kept is the exact sum of the
    kept products and C_computed the same sum formed in precision `prec`.

    Per C leaf (I, J) with m kept products: ||E_IJ||_F <= c(m) * sum over
    kept K of ||A_IK||_F ||B_KJ||_F, since the Frobenius norm of |A||B| is
    at most ||A||_F ||B||_F; the leaves are disjoint, so the squares add.
    Uses the operands actually multiplied.
    """
    Au, Bu, kept = res.A_used, res.B_used, res.kept
    if len(kept) == 0:
        return 0.0
    I, K, J = kept[:, 0], kept[:, 1], kept[:, 2]
    key = morton_key(I, J)  # kept is grouped by C leaf
    starts = np.flatnonzero(np.r_[True, key[1:] != key[:-1]])
    m = np.diff(np.r_[starts, len(kept)])
    prod = np.sqrt(Au.leaf_sq[I, K]) * np.sqrt(Bu.leaf_sq[K, J])
    per_leaf = np.add.reduceat(prod, starts)
    ms, inv = np.unique(m, return_inverse=True)
    coef = np.array([rounding_coefficient(prec, Au.bs, int(x)) for x in ms])[inv]
    e = coef * per_leaf
    return math.sqrt(float(np.sum(e * e)))


def exact_product(A_dense: np.ndarray, B_dense: np.ndarray) -> np.ndarray:
    """The untruncated product, the reference for the error E (Thms 1-3)."""
    return np.asarray(A_dense, dtype=np.float64) @ np.asarray(B_dense, dtype=np.float64)


def tie_triples(A: Tree, B: Tree, tau: float, band: float = 1e-12) -> np.ndarray:
    """Non-null triples whose norm product lies within band*tau of tau; either
    outcome of the test is accepted for them."""
    G = A.G
    out = []
    for I in range(G):
        ks = np.nonzero(A.leaf_present[I])[0]
        if len(ks) == 0:
            continue
        prod = np.sqrt(A.leaf_sq[I, ks])[:, None] * np.sqrt(B.leaf_sq[ks, :])
        near = B.leaf_present[ks, :] & (np.abs(prod - tau) <= band * tau)
        kk, jj = np.nonzero(near)
        if len(kk):
            out.append(np.stack([np.full(len(kk), I), ks[kk], jj], axis=1))
    if not out:
        return np.zeros((0, 3), dtype=np.int64)
    return np.concatenate(out).astype(np.int64)


# --------------------------------------------------------------------------
# Element-level SpAMM (the object of Thm 2's proof) for tiny cases
# --------------------------------------------------------------------------

def spamm_elementwise(A: np.ndarray, B: np.ndarray, tau: float) -> np.ndarray:
    """[C]_ij = sum_k chi_ikj with chi_ikj = a_ik b_kj unless
    |a_ik| |b_kj| < tau (proof of Thm 2); zero operands contribute nothing."""
    n = A.shape[0]
    C = np.zeros((n, n), dtype=np.float64)
    for i in range(n):
        for j in range(n):
            acc = 0.0
            for k in range(n):
                a, b = A[i, k], B[k, j]
                if a != 0.0 and b != 0.0 and not (abs(a) * abs(b) < tau):
                    acc += a * b
            C[i, j] = acc
    return C
