"""Context options: captured-graph launches give bitwise the results of
one-by-one launches, replay after replay with other work in between; the
16 x 16 MFMA tile variant matches the oracle; the autotuner returns a
working choice; validation measures each product against its FP64 twin."""
import numpy as np
import pytest

import oracle as O
import synth
from paper_1906_08148_amd import autotune, spamm

from parity import check_product, compare_kept, TIE_BAND

pytestmark = pytest.mark.gpu


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def batch(M1, M2):
    return [dict(A=M1, B=M1, tau=1e-6, mode=spamm.HYBRID, prec=spamm.F32),
            dict(A=M2, B=M2, tau=1e-5, mode=spamm.SPAMM, prec=spamm.F64),
            dict(A=M1, B=M1, tau=1e-4, mode=spamm.TRUNCMUL, prec=spamm.BF16X3)]


def test_graph_launch_equals_eager_over_replays():
    import torch
    print("case: graph replays", flush=True)
    ctx = spamm.Context(arena_bytes=2 << 30)
    M1 = ctx.build(dev(synth.DecaySpec("1d", 4096, 0.3, seed=2).dense()), 64)
    M2 = ctx.build(dev(synth.DecaySpec("3d", 2048, 1.0, seed=3).dense()), 32)
    eager = [ctx.to_dense(p.C) for p in ctx.multiply_batch(batch(M1, M2))]
    other = [dict(A=M2, B=M2, tau=1e-7, mode=spamm.SPAMM, prec=spamm.F32)]
    ctx.set_option("graph", 1)
    assert ctx.get_option("graph") == 1
    for rep in range(4):
        ps = ctx.multiply_batch(batch(M1, M2))
        for p, e in zip(ps, eager):
            assert torch.equal(ctx.to_dense(p.C), e), rep
            p.C.release()
        # a batch of another shape (graph instantiated anew), then eager work
        q = ctx.multiply_batch(other)[0]
        ctx.set_option("graph", 0)
        r = ctx.multiply_batch(other)[0]
        assert torch.equal(ctx.to_dense(q.C), ctx.to_dense(r.C))
        q.C.release()
        r.C.release()
        ctx.set_option("graph", 1)
        torch.cuda.synchronize()
    M1.release()
    M2.release()
    ctx.close()


@pytest.mark.parametrize("prec", [spamm.F32, spamm.BF16, spamm.BF16X3])
def test_tile_variant_parity(prec):
    print(f"case: tile variant prec={prec}", flush=True)
    ctx = spamm.Context(arena_bytes=1 << 30)
    assert ctx.get_option("gemm_tile") == 1  # the default; the other parity tests run it
    ctx.set_option("gemm_tile", 0)
    A = synth.DecaySpec("1d", 2100, 0.3, seed=5).dense()
    for bs in (32, 64, 128):
        T = O.build(A, bs)
        M = ctx.build(dev(A), bs)
        for mode in (spamm.SPAMM, spamm.HYBRID):
            check_product(ctx, M, M, T, T, 1e-6, mode, prec, alias=True)
        M.release()
    ctx.close()


def test_autotuner_picks_a_candidate():
    print("case: autotune", flush=True)
    ctx = spamm.Context(arena_bytes=2 << 30)
    sp = synth.DecaySpec("3d", 4096, 1.0, seed=4)
    A = dev(sp.dense())
    tuner = autotune.Tuner(ctx, leaves=(32, 64), tiles=(0, 1), reps=2)
    sig = autotune.signature("3d", 4096, 1.0, 1e-6, spamm.HYBRID, spamm.F32)
    best = tuner.tune(lambda leaf: ctx.build(A, leaf), sig, 1e-6, spamm.HYBRID, spamm.F32)
    assert (best["leaf"], best["tile"]) in {(32, 0), (32, 1), (64, 0), (64, 1)}
    assert len(best["table"]) == 4 and all(r["seconds"] > 0 for r in best["table"])
    assert ctx.get_option("gemm_tile") == best["tile"]
    assert tuner.tune(None, sig, 1e-6, spamm.HYBRID, spamm.F32) is best  # cached
    ctx.close()


def test_validation_against_fp64_twin():
    print("case: validation", flush=True)
    ctx = spamm.Context(arena_bytes=1 << 30)
    A = synth.DecaySpec("1d", 1500, 0.3, seed=7).dense()
    T = O.build(A, 32)
    M = ctx.build(dev(A), 32)
    reqs = [dict(A=M, B=M, tau=1e-6, mode=m, prec=p)
            for m in (spamm.SPAMM, spamm.HYBRID) for p in (spamm.F32, spamm.BF16, spamm.BF16X3, spamm.F64)]
    for pr in ctx.multiply_batch(reqs):  # builds and caches M's prune views
        pr.C.release()
    base = ctx.arena_info()["used"]
    ctx.set_option("validate", 1)
    assert ctx.get_option("validate") == 1
    prods = ctx.multiply_batch(reqs)
    for q, pr in zip(reqs, prods):
        st = pr.stats
        if q["prec"] == spamm.F64:
            assert st["val_err"] == 0.0
            continue
        ref = O.multiply(T, T, q["tau"], q["mode"])
        ties = O.tie_triples(ref.A_used, ref.B_used, q["tau"], TIE_BAND)
        # no tie on this input: the kept lists are identical
        assert compare_kept(ctx.kept(pr.C), ref.kept, ties, T.G) == 0 and not ref.stats["trunc_tie"]
        d = float(np.linalg.norm(ctx.to_dense(pr.C).cpu().numpy() - ref.C.to_dense()))
        # the twin and the oracle differ only by FP64 rounding
        assert abs(st["val_err"] - d) <= 2.0 * O.precision_bound(ref, O.P_F64), (st["val_err"], d)
        assert 0.0 < st["val_err"] <= st["prec_bound"]
    for pr in prods:
        pr.C.release()
    # the twins were released with the call
    assert ctx.arena_info()["used"] == base
    ctx.set_option("validate", 0)
    p = ctx.multiply(M, M, 1e-6, prec=spamm.F32)
    assert p.stats["val_err"] == -1.0
    p.C.release()
    # operands without the FP64 copy cannot be validated
    M32 = ctx.build(dev(A), 32, stores=spamm.STORE_F32)
    ctx.set_option("validate", 1)
    with pytest.raises(spamm.SpammError) as e:
        ctx.multiply(M32, M32, 1e-6, prec=spamm.F32)
    assert e.value.code == "EUNSUPPORTED"
    M32.release()
    M.release()
    ctx.close()


def test_validation_with_epilogue_and_mixed_leaves():
    """The FP64 twin carries the request's epilogue (C = alpha A B + beta D),
    and twins of different leaf sizes share one batch: val_err equals the
    difference from the same request computed in FP64 on its own."""
    import torch
    print("case: validation epilogue", flush=True)
    ctx = spamm.Context(arena_bytes=1 << 30)
    A = synth.DecaySpec("1d", 1200, 0.4, seed=3).dense()
    M32, M64 = ctx.build(dev(A), 32), ctx.build(dev(A), 64)
    reqs = [dict(A=M32, B=M32, tau=1e-7, mode=spamm.HYBRID, prec=spamm.F32, alpha=-1.0, beta=2.0, D=M32),
            dict(A=M64, B=M64, tau=1e-6, mode=spamm.SPAMM, prec=spamm.BF16X3, alpha=0.5, beta=-3.0, D=M64),
            dict(A=M64, B=M64, tau=1e-6, mode=spamm.TRUNCMUL, prec=spamm.F32)]
    ctx.set_option("validate", 1)
    prods = ctx.multiply_batch(reqs)
    ctx.set_option("validate", 0)
    for q, pr in zip(reqs, prods):
        ref = ctx.multiply_batch([dict(q, prec=spamm.F64)])[0]
        d = float(torch.linalg.norm(ctx.to_dense(pr.C) - ctx.to_dense(ref.C)))
        # the twin is the same FP64 computation: bitwise the same C
        assert pr.stats["val_err"] == pytest.approx(d, rel=1e-12, abs=1e-300), (pr.stats["val_err"], d)
        assert pr.stats["val_err"] > 0.0
        ref.C.release()
        pr.C.release()
    M32.release()
    M64.release()
    ctx.close()
