"""Symmetric squares (SPAMM_SYM): only C leaves on and above the diagonal are
formed and the others are mirrored.  Against the oracle's SpAMM product and
the library's full SpAMM product of the same symmetric matrix."""
import numpy as np
import pytest

import oracle as O
import synth
from paper_1906_08148_amd import spamm

from parity import TIE_BAND, TOL, rel_fro, rel_fro_leaves

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
    # B must be the same handle as A, and no epilogue
    M2 = ctx.build(dev(A), bs)
    for kw in (dict(A=M, B=M2), dict(A=M, B=M, alpha=2.0)):
        with pytest.raises(spamm.SpammError) as e:
            ctx.multiply_batch([dict(kw, tau=tau, mode=spamm.SPAMM_SYM, prec=spamm.F32)])
        assert e.value.code == "EINVAL"
    M2.release()
    M.release()
    ctx.close()
