"""Symmetric squares (SPAMM_SYM, HYBRID_SYM): only C leaves on and above the
diagonal are formed and the others are mirrored.  Against the oracle's
symmetric-square reading (mirror decisions, pair truncation for Hybrid,
fallback to the full product when the null map is not symmetric) and the
library's full products of the same symmetric matrix."""
import numpy as np
import pytest

import oracle as O
import synth
from paper_1906_08148_amd import spamm

from parity import PREC_NAME, TIE_BAND, TOL, compare_kept, rel_fro, rel_fro_leaves

pytestmark = pytest.mark.gpu


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("kind,n,alpha,bs,tau", [("1d", 1500, 0.2, 32, 1e-6),
                                                 ("3d", 2048, 1.0, 64, 1e-5),
                                                 ("1d", 700, 0.1, 128, 1e-4)])
def test_symmetric_square_matches_spamm(kind, n, alpha, bs, tau):
    print(f"case: symmetric square {kind} n={n} leaf={bs} tau={tau}", flush=True)
    ctx = spamm.Context(arena_bytes=1 << 30)
    A = synth.DecaySpec(kind, n, alpha, seed=6).dense()
    assert np.array_equal(A, A.T)
    T = O.build(A, bs)
    M = ctx.build(dev(A), bs, stores=spamm.STORE_F64 | spamm.STORE_F32 | spamm.STORE_BF16)
    ref = O.multiply(T, T, tau, O.SPAMM)
    assert len(O.tie_triples(T, T, tau, TIE_BAND)) == 0
    upper = int(np.sum(ref.kept[:, 0] <= ref.kept[:, 2]))
    G = T.G
    for prec in (spamm.F64, spamm.F32, spamm.BF16X3):
        p = ctx.multiply(M, M, tau, mode=spamm.SPAMM_SYM, prec=prec)
        full = ctx.multiply(M, M, tau, mode=spamm.SPAMM, prec=prec)
        st, sf = p.stats, full.stats
        # only the upper products are formed; the structure is the full one
        assert st["n_kept"] == upper < ref.stats["n_kept"]
        assert st["flops"] == 2.0 * bs ** 3 * upper
        assert st["c_nonnull"] == ref.stats["c_nonnull"] == sf["c_nonnull"]
        assert st["n_candidates"] == sf["n_candidates"]
        for k in ("B1", "B2", "err_bound", "prec_bound"):
            assert st[k] == pytest.approx(sf[k], rel=1e-12, abs=1e-300), k
        # C against the oracle and against the full product
        assert rel_fro_leaves(ctx, p.C, ref.C) <= TOL[prec]
        Cs, Cf = ctx.to_dense(p.C).cpu().numpy(), ctx.to_dense(full.C).cpu().numpy()
        assert rel_fro(Cs, Cf) <= TOL[prec]
        assert st["trace"] == pytest.approx(sf["trace"], rel=TOL[prec])
        # leaves off the diagonal are exact transposes of their mirrors
        Np = G * bs
        Cp = np.zeros((Np, Np))
        Cp[:n, :n] = Cs
        for I in range(G):
            for J in range(I + 1, G):
                a = Cp[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs]
                b = Cp[J * bs:(J + 1) * bs, I * bs:(I + 1) * bs]
                assert np.array_equal(a, b.T)
        # the norm pyramid of the mirrored leaves equals the formed ones'
        ns, nf = ctx.norms(p.C), ctx.norms(full.C)
        assert np.allclose(ns, nf, rtol=10 * TOL[prec], atol=0.0)
        p.C.release()
        full.C.release()
    # B must be the same handle as A
    M2 = ctx.build(dev(A), bs)
    for mode in (spamm.SPAMM_SYM, spamm.HYBRID_SYM):
        with pytest.raises(spamm.SpammError) as e:
            ctx.multiply_batch([dict(A=M, B=M2, tau=tau, mode=mode, prec=spamm.F32)])
        assert e.value.code == "EINVAL"
    M2.release()
    M.release()
    ctx.close()


def _mirror_kept(kept):
    """Formed (upper) triples plus the mirrored ones of the lower leaves,
    grouped by C leaf in Morton order with K ascending."""
    k = np.asarray(kept, dtype=np.int64).reshape(-1, 3)
    low = k[k[:, 0] < k[:, 2]][:, [2, 1, 0]]
    allk = np.concatenate([k, low])
    key = O.morton_key(allk[:, 0], allk[:, 2])
    return allk[np.lexsort((allk[:, 1], key))]


def _check_sym(ctx, p, ref, T, prec, tau):
    """A symmetric-square product against the oracle's reading."""
    import dataclasses
    st = p.stats
    ties = O.tie_triples(ref.A_used, ref.A_used, tau, TIE_BAND)
    assert len(ties) == 0 and not ref.stats["trunc_tie"]
    assert compare_kept(ctx.kept(p.C), ref.kept, ties, T.G) == 0
    for k in ("n_kept", "c_nonnull", "n_candidates"):
        assert st[k] == ref.stats[k], k
    for k in ("B1", "B2", "dA", "err_bound"):
        assert st[k] == pytest.approx(ref.stats[k], rel=1e-10, abs=1e-300), k
    bnd = spamm.morton_order_to_grid(ctx.skipped_bound(p.C), T.L)
    assert np.all(np.abs(bnd - ref.skipped_bound) <= 1e-13 * ref.skipped_bound)
    # the rounding bound covers both triangles: a mirrored leaf has its mirror's
    full = ref.kept if ref.stats.get("sym_fallback") else _mirror_kept(ref.kept)
    pb = O.precision_bound(dataclasses.replace(ref, kept=full), PREC_NAME[prec])
    assert st["prec_bound"] == pytest.approx(pb, rel=1e-10)
    assert rel_fro_leaves(ctx, p.C, ref.C) <= TOL[prec]
    if not ref.stats.get("sym_fallback"):
        _assert_mirrored(ctx.to_dense(p.C).cpu().numpy(), T.bs, T.G)


def _assert_mirrored(C, bs, G):
    """Leaves below the diagonal are exact transposes of their mirrors (the
    diagonal leaves are formed, so they are symmetric only to rounding)."""
    n = C.shape[0]
    Cp = np.zeros((G * bs, G * bs))
    Cp[:n, :n] = C
    for I in range(G):
        for J in range(I + 1, G):
            a = Cp[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs]
            b = Cp[J * bs:(J + 1) * bs, I * bs:(I + 1) * bs]
            assert np.array_equal(a, b.T), (I, J)
    assert np.allclose(C, C.T, rtol=0, atol=1e-5 * max(np.abs(C).max(), 1e-300))


@pytest.mark.parametrize("kind,n,alpha,bs,tau", [("1d", 1500, 0.2, 32, 1e-6),
                                                 ("3d", 2048, 1.0, 64, 1e-5),
                                                 ("3d", 4096, 1.0, 64, 1e-6),
                                                 ("1d", 2000, 0.05, 128, 1e-4)])
def test_hybrid_sym_against_oracle(kind, n, alpha, bs, tau):
    print(f"case: hybrid_sym {kind} n={n} leaf={bs} tau={tau}", flush=True)
    ctx = spamm.Context(arena_bytes=2 << 30)
    A = synth.DecaySpec(kind, n, alpha, seed=6).dense()
    T = O.build(A, bs)
    M = ctx.build(dev(A), bs, stores=spamm.STORE_F64 | spamm.STORE_F32 | spamm.STORE_BF16)
    for mode, omode in ((spamm.HYBRID_SYM, O.HYBRID), (spamm.SPAMM_SYM, O.SPAMM)):
        ref = O.multiply_symmetric(T, tau, omode)
        assert not ref.stats["sym_fallback"]
        for prec in (spamm.F64, spamm.F32, spamm.BF16X3):
            p = ctx.multiply(M, M, tau, mode=mode, prec=prec)
            _check_sym(ctx, p, ref, T, prec, tau)
            p.C.release()
    # the pair truncation drops at most what the leaf truncation would, in
    # pairs: a Hybrid-sym product forms about half the full Hybrid products
    hs = ctx.multiply(M, M, tau, mode=spamm.HYBRID_SYM, prec=spamm.F64)
    hf = ctx.multiply(M, M, tau, mode=spamm.HYBRID, prec=spamm.F64)
    assert hs.stats["n_kept"] < 0.65 * hf.stats["n_kept"]
    hs.C.release()
    hf.C.release()
    M.release()
    ctx.close()


def test_sym_falls_back_when_the_null_map_is_not_symmetric():
    """A leaf above the diagonal zeroed, its mirror kept: the caller's A is not
    symmetric, the device check sees it, and every C leaf is formed by its
    own test, as the oracle's reading prescribes."""
    print("case: sym fallback", flush=True)
    ctx = spamm.Context(arena_bytes=1 << 30)
    bs = 32
    A = synth.DecaySpec("1d", 1024, 0.2, seed=7).dense()
    A[0:bs, bs:2 * bs] = 0.0
    T = O.build(A, bs)
    M = ctx.build(dev(A), bs)
    for mode, omode in ((spamm.HYBRID_SYM, O.HYBRID), (spamm.SPAMM_SYM, O.SPAMM)):
        ref = O.multiply_symmetric(T, 1e-6, omode)
        assert ref.stats["sym_fallback"]
        for prec in (spamm.F64, spamm.F32):
            p = ctx.multiply(M, M, 1e-6, mode=mode, prec=prec)
            _check_sym(ctx, p, ref, T, prec, 1e-6)
            p.C.release()
    M.release()
    ctx.close()


def test_sym_with_symmetric_epilogue():
    """C = 2X - X X with the symmetric X as D (the purification step)."""
    print("case: sym epilogue", flush=True)
    ctx = spamm.Context(arena_bytes=1 << 30)
    A = synth.DecaySpec("3d", 2048, 1.0, seed=8).dense() * 0.05
    T = O.build(A, 64)
    M = ctx.build(dev(A), 64)
    ref = O.multiply_symmetric(T, 1e-7, O.HYBRID)
    want = 2.0 * A - ref.C.to_dense()
    for prec in (spamm.F64, spamm.F32):
        p = ctx.multiply(M, M, 1e-7, mode=spamm.HYBRID_SYM, prec=prec, alpha=-1.0, beta=2.0, D=M)
        C = ctx.to_dense(p.C).cpu().numpy()
        assert rel_fro(C, want) <= TOL[prec]
        _assert_mirrored(C, 64, T.G)
        assert p.stats["trace"] == pytest.approx(float(np.trace(want)), rel=TOL[prec])
        p.C.release()
    M.release()
    ctx.close()
