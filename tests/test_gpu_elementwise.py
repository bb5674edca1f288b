"""Element-wise truncation on the GPU (the truncated matrix of Thm. 1)
against the oracle: the thresholded entries bit for bit, the null leaves,
the norm pyramid, the dropped squared norm, and element-wise Truncmul (the
truncated operands multiplied exactly) in several precisions."""
import numpy as np
import pytest

import oracle as O
import synth
from paper_1906_08148_amd import spamm

from parity import check_norms, check_product

pytestmark = pytest.mark.gpu

ALL_STORES = spamm.STORE_F64 | spamm.STORE_F32 | spamm.STORE_BF16


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def dropped_sq(A, tau):
    small = A[np.abs(A) < tau]
    return float(np.sum(small * small))


@pytest.mark.parametrize("kind,n,alpha,bs,tau", [("1d", 1000, 0.3, 32, 1e-6),
                                                 ("3d", 1024, 1.0, 64, 1e-4),
                                                 ("1d", 700, 0.1, 16, 1e-3)])
def test_elementwise_truncation_matches_oracle(kind, n, alpha, bs, tau):
    print(f"case: elementwise {kind} n={n} leaf={bs} tau={tau}", flush=True)
    ctx = spamm.Context(arena_bytes=1 << 30)
    A = synth.DecaySpec(kind, n, alpha, seed=4).dense()
    M = ctx.build(dev(A), bs, stores=ALL_STORES)
    Mt, dropped = ctx.truncate_elementwise(M, tau)
    At = O.truncate_elementwise(A, tau)
    assert np.array_equal(ctx.to_dense(Mt).cpu().numpy(), At)
    Tt = O.build(At, bs)
    assert Mt.info.nonnull == Tt.nonnull_count()
    assert Tt.nonnull_count() <= O.build(A, bs).nonnull_count()
    check_norms(ctx, Mt, Tt)
    want = dropped_sq(A, tau)
    assert want > 0 and abs(dropped - want) <= 1e-12 * want
    # element-wise Truncmul: the truncated operands multiplied exactly
    for prec in (spamm.F64, spamm.F32) + ((spamm.BF16X3,) if bs >= 32 else ()):  # BF16 GEMMs: leaf >= 32
        check_product(ctx, Mt, Mt, Tt, Tt, 0.0, spamm.TRUNCMUL, prec, alias=True)
    # the result is an ordinary matrix: SpAMM on it works as on any other
    check_product(ctx, Mt, Mt, Tt, Tt, tau, spamm.HYBRID, spamm.F32, alias=True)
    Mt.release()
    M.release()
    ctx.close()


def test_elementwise_truncation_edges():
    print("case: elementwise edges", flush=True)
    ctx = spamm.Context(arena_bytes=1 << 30)
    A = synth.DecaySpec("1d", 600, 0.2, seed=9).dense()
    M = ctx.build(dev(A), 32, stores=ALL_STORES)
    # tau = 0 keeps every entry
    M0, d0 = ctx.truncate_elementwise(M, 0.0)
    assert d0 == 0.0 and np.array_equal(ctx.to_dense(M0).cpu().numpy(), A)
    assert M0.info.nonnull == M.info.nonnull
    # a tau above every entry empties the matrix, and its products are empty
    big = float(np.abs(A).max()) * 2.0
    Me, de = ctx.truncate_elementwise(M, big)
    assert Me.info.nonnull == 0 and not np.any(ctx.to_dense(Me).cpu().numpy())
    assert abs(de - float(np.sum(A * A))) <= 1e-12 * float(np.sum(A * A))
    p = ctx.multiply(Me, Me, 0.0, mode=spamm.TRUNCMUL, prec=spamm.F32)
    assert p.stats["n_kept"] == 0 and p.C.info.nonnull == 0
    p.C.release()
    # a block-list build (slots of all-zero blocks stay unused)
    n, bs = 512, 32
    coords, data = synth.random_blocks(13, n, bs, 0.3)
    data = data.copy()
    data[::5] = 0.0  # some listed blocks are all zero
    Ab = synth.dense_from_blocks(n, bs, coords, data)
    Mb = ctx.build_blocks(n, bs, dev(coords.astype(np.int32)), dev(data), stores=ALL_STORES)
    tau = float(np.median(np.abs(Ab[Ab != 0])))
    Mbt, db = ctx.truncate_elementwise(Mb, tau)
    At = O.truncate_elementwise(Ab, tau)
    assert np.array_equal(ctx.to_dense(Mbt).cpu().numpy(), At)
    assert Mbt.info.nonnull == O.build(At, bs).nonnull_count()
    assert abs(db - dropped_sq(Ab, tau)) <= 1e-12 * dropped_sq(Ab, tau)
    # operands without the FP64 copy, and bad arguments, are refused
    M32 = ctx.build(dev(A), 32, stores=spamm.STORE_F32)
    with pytest.raises(spamm.SpammError) as e:
        ctx.truncate_elementwise(M32, 1e-6)
    assert e.value.code == "EUNSUPPORTED"
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(spamm.SpammError) as e:
            ctx.truncate_elementwise(M, bad)
        assert e.value.code == "EINVAL"
    for m in (M0, Me, Mb, Mbt, M32, M):
        m.release()
    ctx.close()
