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
