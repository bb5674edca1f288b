"""The paper's own synthetic workloads against the CPU oracle, in FP64 as
there (Sec. 5): the model problem's 1D decay (alpha = 0.005, Sec. 5.3) at
leaf 64 and 256 in all three schemes, with its error against the exact
product, and the leaf-library sweep's random uniform blocks (2048 x 2048,
fill 0.1 ... 1, every product formed, Sec. 5.2) at leaf 32 ... 256.  The
model problem runs at n = 4000 here (the bench runs n = 40000; the oracle
checks every C leaf at this size)."""
import numpy as np
import pytest

import oracle as O
import synth
from paper_1906_08148_amd import spamm

from parity import check_product, rel_fro

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    c = spamm.Context(arena_bytes=4 << 30)
    yield c
    c.close()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("leaf,tau", [(64, 1e-6), (256, 1e-9)])
def test_model_problem(ctx, leaf, tau):
    """Every scheme against the oracle (kept list, C, bounds, statistics),
    and the approximation error ||A A - C||_F, the quantity the paper fixes
    (sigma = 1e-6 there), equal to the oracle's within FP64 rounding."""
    print(f"case: model problem leaf {leaf} tau {tau}", flush=True)
    A = synth.DecaySpec("1d", 4000, 0.005, seed=3).dense()
    exact = A @ A
    T = O.build(A, leaf)
    M = ctx.build(dev(A), leaf, stores=spamm.STORE_F64)
    for mode in (spamm.TRUNCMUL, spamm.SPAMM, spamm.HYBRID):
        p, ref, branch = check_product(ctx, M, M, T, T, tau, mode, spamm.F64, alias=True)
        assert branch == "full"
        err = np.linalg.norm(exact - ctx.to_dense(p.C).cpu().numpy())
        err_ref = np.linalg.norm(exact - ref.C.to_dense())
        assert abs(err - err_ref) <= 1e-12 * np.linalg.norm(exact), (mode, err, err_ref)
        assert err <= ref.stats["err_bound"] + O.precision_bound(ref, O.P_F64)  # Thm. 2 / 3 bound holds
        p.C.release()
    M.release()


@pytest.mark.parametrize("leaf", [32, 64, 128, 256])
def test_leaf_library_sweep(ctx, leaf):
    """Random uniform blocks at fill 0.1, 0.5 and 1: every product formed
    (Truncmul at tau = 0), FP64 and FP32, against the oracle in full."""
    print(f"case: leaf library leaf {leaf}", flush=True)
    for fill in (0.1, 0.5, 1.0):
        c1, d1 = synth.random_blocks(11, 2048, leaf, fill)
        c2, d2 = synth.random_blocks(12, 2048, leaf, fill)
        TA = O.build_from_blocks(2048, leaf, c1, d1)
        TB = O.build_from_blocks(2048, leaf, c2, d2)
        MA = ctx.build_blocks(2048, leaf, dev(c1.astype(np.int32)), dev(d1))
        MB = ctx.build_blocks(2048, leaf, dev(c2.astype(np.int32)), dev(d2))
        for prec in (spamm.F64, spamm.F32):
            p, ref, branch = check_product(ctx, MA, MB, TA, TB, 0.0, spamm.TRUNCMUL, prec)
            assert branch == "full"
            # every non-null product is formed at tau = 0
            assert p.stats["n_kept"] == int(np.einsum("ik,kj->", TA.leaf_present.astype(np.int64),
                                                      TB.leaf_present.astype(np.int64)))
            p.C.release()
        MA.release()
        MB.release()
