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
