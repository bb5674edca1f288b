"""The entry point that allocates nothing (spamm_gershgorin_static) against
the allocating one (spamm_gershgorin): the same bounds, bit for bit, on two
calls in a row (the second on a smaller matrix, so stale scratch from the
first call would show), for FP64 and FP32-only leaf stores; a grid with more
leaf rows than the static scratch holds is refused before any launch, and
no arena memory is taken."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import purify as PU
from paper_1906_08148_amd import spamm

pytestmark = pytest.mark.gpu


def _static_bounds(ctx, M, bounds):
    """One call through the C-ABI: status, then the two device values."""
    import torch
    st = spamm._lib.spamm_gershgorin_static(ctx.ptr, M.handle, ctypes.c_void_p(bounds.data_ptr()))
    torch.cuda.synchronize()
    return st, bounds.cpu().numpy().copy()


def test_gershgorin_static_matches_allocating_entry_point():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    print("case: no-alloc gershgorin", flush=True)
    ctx = spamm.Context(arena_bytes=2 << 30)
    bounds = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    cases = [("3d", 4096, 1.0, 64, spamm.STORE_F64 | spamm.STORE_F32),   # 64 leaf rows
             ("1d", 16384, 0.5, 16, spamm.STORE_F64),                   # 1024 leaf rows: the limit
             ("1d", 1000, 0.3, 32, spamm.STORE_F64),                    # fewer rows: stale rows would show
             ("1d", 700, 0.5, 16, spamm.STORE_F32)]                     # FP32-only copy
    for kind, n, alpha, leaf, stores in cases:
        A = synth.DecaySpec(kind, n, alpha, seed=3).dense()
        M = ctx.build(torch.from_numpy(A).cuda(), leaf, stores=stores)
        used = ctx.arena_info()["used"]
        st, got = _static_bounds(ctx, M, bounds)
        assert st == 0, spamm._lib.spamm_last_error(ctx.ptr)
        assert ctx.arena_info()["used"] == used  # nothing taken from the arena
        lo, hi = ctx.gershgorin(M)
        assert got[0] == lo and got[1] == hi, (kind, n, got, lo, hi)
        # and both are the Gershgorin bounds of the matrix (up to the FP32
        # rounding of an FP32-only copy)
        lo_r, hi_r = PU.gershgorin(A if stores & spamm.STORE_F64 else A.astype(np.float32).astype(np.float64))
        assert abs(lo - lo_r) <= 1e-12 * abs(lo_r) and abs(hi - hi_r) <= 1e-12 * abs(hi_r)
        M.release()
    ctx.close()


def test_gershgorin_static_refuses_grids_beyond_its_scratch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    print("case: no-alloc gershgorin size limit", flush=True)
    ctx = spamm.Context(arena_bytes=4 << 30)
    bounds = torch.zeros(2, dtype=torch.float64, device="cuda")
    # 2048 leaf rows of 16 (one leaf on the diagonal), twice the limit
    coords = torch.tensor([[0, 0]], dtype=torch.int32, device="cuda")
    data = torch.ones((1, 16, 16), dtype=torch.float64, device="cuda")
    M = ctx.build_blocks(2048 * 16, 16, coords, data, stores=spamm.STORE_F64)
    assert M.info.G == 2048
    st, got = _static_bounds(ctx, M, bounds)
    assert spamm.STATUS[st] == "EUNSUPPORTED"
    assert np.all(got == 0.0)  # nothing was launched
    # the allocating entry point still serves it
    lo, hi = ctx.gershgorin(M)
    assert lo == 1.0 - 15.0 and hi == 1.0 + 15.0
    M.release()
    ctx.close()
