"""Served results equal results alone: a mixed stream of requests (1D and 3D
decay, different n, tau and schemes) through two lanes with continuous
batching gives, request by request, the same C as running each alone."""
import pytest

from paper_1906_08148_amd import serve, spamm

pytestmark = pytest.mark.gpu


def specs():
    out = []
    rid = 0
    for kind, n, alpha in (("1d", 2048, 0.3), ("3d", 2048, 0.9), ("1d", 4096, 0.5), ("3d", 4096, 1.0),
                           ("1d", 3072, 0.2), ("3d", 1024, 0.6)):
        for tau, mode in ((1e-6, spamm.SPAMM), (1e-5, spamm.HYBRID), (1e-7, spamm.TRUNCMUL)):
            out.append(serve.RequestSpec(serve.MatrixSpec(kind, n, alpha, 40 + rid // 3), tau, mode, rid=rid))
            rid += 1
    return out


def test_alone_equals_mix():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    print("case: serving alone vs mix", flush=True)
    sp = specs()
    inputs = {s.mat: serve.make_input(s.mat, s.leaf) for s in sp}
    alone_srv = serve.Server(lanes=1, arena_bytes_per_lane=4 << 30, max_batch=1, inputs=inputs, keep_C=True)
    alone = serve.run_stream(alone_srv.sched, sp, rate=0)
    alone_srv.close()
    mix_srv = serve.Server(lanes=2, arena_bytes_per_lane=4 << 30, max_batch=8, inputs=inputs, keep_C=True)
    mix = serve.run_stream(mix_srv.sched, sp, rate=2000.0, seed=3)
    log = list(mix_srv.sched.log)
    mix_srv.close()
    assert max(len(b[2]) for b in log) > 1, "the mixed run formed no batch"
    assert len({b[0] for b in log}) == 2, "the mixed run used one lane"
    for a, m in zip(alone, mix):
        assert not a.error and not m.error, (a.error, m.error)
        assert a.stats["n_kept"] == m.stats["n_kept"]
        assert torch.equal(a.C, m.C), a.rid


def test_served_results_match_the_oracle():
    """Requests of the seeded pool served through two lanes with continuous
    batching, checked against the CPU oracle: every request with n <= 8192
    among the first 64 of the pool (C in full), and two larger ones (C on
    sampled leaves); kept products and C within the FP32 tolerance."""
    import numpy as np
    import oracle as O
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    print("case: served vs oracle", flush=True)
    pool = serve.request_pool(512)
    small = [r for r in pool[:64] if r.mat.n <= 8192]
    large = [next(r for r in pool if r.mat.kind == k and 12288 <= r.mat.n <= 20480) for k in ("1d", "3d")]
    sp = small + large
    inputs = {s.mat: serve.make_input(s.mat, s.leaf) for s in sp}
    srv = serve.Server(lanes=2, arena_bytes_per_lane=24 << 30, max_batch=8, inputs=inputs, keep_C=True)
    res = serve.run_stream(srv.sched, sp, rate=500.0, seed=5)
    log = list(srv.sched.log)
    srv.close()
    assert max(len(b[2]) for b in log) > 1, "no batch formed"
    rng = np.random.default_rng(9)
    for s, r in zip(sp, res):
        assert not r.error, r.error
        src = inputs[s.mat]
        T = O.build_from_blocks(s.mat.n, s.leaf, src[1], src[2]) if src[0] == "blocks" else O.build(src[1], s.leaf)
        big = s.mat.n > 8192
        blocks = None
        if big:
            blocks = sorted({(i, i) for i in range(0, T.G, 8)} |
                            {tuple(int(v) for v in x) for x in rng.integers(0, T.G, size=(32, 2))})
        ref = O.multiply(T, T, s.tau, s.mode, c_blocks=blocks)
        ties = O.tie_triples(ref.A_used, ref.B_used, s.tau, 1e-12)
        print(f"  rid {s.rid} {s.mat.kind} n={s.mat.n} mode={s.mode} tau={s.tau:.1e} kept {ref.stats['n_kept']} "
              f"ties {len(ties)} trunc_tie {ref.stats['trunc_tie']}", flush=True)
        if len(ties) == 0 and not ref.stats["trunc_tie"]:
            assert r.stats["n_kept"] == ref.stats["n_kept"], s.rid
            assert r.stats["c_nonnull"] == ref.stats["c_nonnull"], s.rid
        C = r.C.numpy()
        if not big:
            want = ref.C.to_dense()
            got = C
        else:
            bs = s.leaf
            got = np.stack([np.pad(C[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs],
                                   ((0, bs - len(C[I * bs:(I + 1) * bs])), (0, bs - C[:, J * bs:(J + 1) * bs].shape[1])))
                            for I, J in blocks])
            want = np.stack([ref.C.leaf(I, J) if ref.C.index[I, J] >= 0 else np.zeros((bs, bs)) for I, J in blocks])
        d = np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)
        assert d <= 1e-5, (s.rid, d)
