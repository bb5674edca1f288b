"""Pins of the purification oracle: Gershgorin bounds enclose the spectrum,
tau = 0 reproduces the plain dense iteration, and on a gapped spectrum the
chain converges to the spectral projector onto the lowest n_occ states."""
import numpy as np

import oracle as O
from oracle import purify as PU


def sym(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n))
    return (M + M.T) / 2


def test_gershgorin_encloses_spectrum():
    for seed in range(4):
        A = sym(40, seed)
        lo, hi = PU.gershgorin(A)
        ev = np.linalg.eigvalsh(A)
        assert lo <= ev.min() and ev.max() <= hi
    # diagonal matrix: the discs are the points themselves
    D = np.diag([3.0, -1.0, 2.5])
    assert PU.gershgorin(D) == (-1.0, 3.0)


def test_scaled_spectrum_in_unit_interval_and_reversed():
    A = sym(50, 7)
    X0, lo, hi = PU.scale_unit(A)
    ev = np.linalg.eigvalsh(X0)
    assert ev.min() >= -1e-12 and ev.max() <= 1 + 1e-12
    # the smallest eigenvalue of A maps to the largest of X0
    evA = np.linalg.eigvalsh(A)
    assert np.isclose(ev.max(), (hi - evA.min()) / (hi - lo))


def test_tau_zero_equals_dense_iteration():
    A = sym(70, 3)
    n_occ = 35
    recs, _ = PU.sp2_chain(A, 8, n_occ, 0.0, 6, O.SPAMM)
    X, lo, hi = PU.scale_unit(A)
    for r in recs:
        tr = np.trace(X)
        X2 = X @ X
        X = X2 if tr > n_occ else 2 * X - X2
        assert r["branch"] == (0 if tr > n_occ else 1)
        assert np.linalg.norm(r["X"] - X) <= 1e-12 * np.linalg.norm(X)


def test_gapped_spectrum_converges_to_projector():
    rng = np.random.default_rng(11)
    n, n_occ = 48, 20
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([rng.uniform(-2.0, -1.0, n_occ), rng.uniform(1.0, 2.0, n - n_occ)])
    A = (Q * lam) @ Q.T
    A = (A + A.T) / 2
    recs, _ = PU.sp2_chain(A, 8, n_occ, 0.0, 40, O.TRUNCMUL)
    P = Q[:, :n_occ] @ Q[:, :n_occ].T
    X = recs[-1]["X"]
    assert abs(np.trace(X) - n_occ) < 1e-8
    assert np.linalg.norm(X - P) < 1e-8
    assert np.linalg.norm(X @ X - X) < 1e-8


def _leaf_sq(X, bs):
    G = -(-X.shape[0] // bs)
    P = np.zeros((G * bs, G * bs))
    P[:X.shape[0], :X.shape[1]] = X
    return (P.reshape(G, bs, G, bs) ** 2).sum(axis=(1, 3))


def test_truncated_chain_drops_the_smallest_pairs_within_budget():
    """With tau_c each iterate is the plain dense SP2 map of the previous one
    with whole mirror pairs of leaves removed: the removed pairs are the
    lightest (weight s_IJ + s_JI, a diagonal leaf alone; none heavier than a
    kept pair), their weights sum to the recorded amount and stay within
    tau_c^2, the lightest kept pair would not fit, and the iterate's null
    map stays symmetric."""
    i = np.arange(64)
    A = sym(64, 5) * np.exp(-np.abs(i[:, None] - i[None, :]) / 3.0)  # decay away from the diagonal
    bs, n_occ, tau_c = 8, 30, 0.05
    recs, _ = PU.sp2_chain(A, bs, n_occ, 0.0, 8, O.SPAMM, tau_c=tau_c)
    X, _, _ = PU.scale_unit(A)
    dropped_any = False
    upper = np.triu(np.ones((8, 8), dtype=bool))
    for r in recs:
        X2 = X @ X
        Xn = X2 if np.trace(X) > n_occ else 2 * X - X2
        assert r["branch"] == (0 if np.trace(X) > n_occ else 1)
        Xt = r["X"]
        sq_n, sq_t = _leaf_sq(Xn, bs), _leaf_sq(Xt, bs)
        kept = sq_t > 0
        assert np.array_equal(kept, kept.T)
        # kept leaves are the map's leaves; removed leaves are whole leaves
        mask = np.kron(kept, np.ones((bs, bs)))[:64, :64].astype(bool)
        assert np.allclose(Xt[mask], Xn[mask], rtol=0, atol=1e-12)
        assert np.all(Xt[~mask] == 0)
        w = np.where(np.eye(8, dtype=bool), sq_n, sq_n + sq_n.T)  # pair weights, upper triangle
        present = upper & ((sq_n > 0) | (sq_n.T > 0))
        gone = present & ~kept
        kept_u = present & kept
        d = w[gone].sum()
        assert abs(d - r["dropped_sq"]) <= 1e-10 * max(d, 1e-300)
        assert d <= tau_c ** 2 * (1 + 1e-12)
        if gone.any():
            dropped_any = True
            assert w[gone].max() <= w[kept_u].min() * (1 + 1e-10)
        if kept_u.any():
            assert d + w[kept_u].min() > tau_c ** 2 * (1 - 1e-10)
        assert r["nonnull"] == int(kept.sum())
        assert not r["trunc_tie"]
        X = Xt
    assert dropped_any


def test_truncated_chain_with_zero_budget_is_the_plain_chain():
    A = sym(40, 9)
    plain, _ = PU.sp2_chain(A, 8, 20, 1e-3, 5, O.HYBRID)
    trunc, _ = PU.sp2_chain(A, 8, 20, 1e-3, 5, O.HYBRID, tau_c=0.0)
    for a, b in zip(plain, trunc):
        assert a["branch"] == b["branch"] and a["n_kept"] == b["n_kept"]
        assert np.array_equal(a["X"], b["X"])
