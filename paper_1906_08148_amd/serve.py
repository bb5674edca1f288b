"""Serving loop: continuous batching of approximate products.

Requests (a decay matrix spec, tau, scheme, precision) arrive at any time.
The server runs several lanes, each a library context with its own stream
and arena.  When a lane is free it takes the pending requests, in arrival
order, that fit its memory budget (by estimated arena footprint) up to a
batch size, and runs them as one `multiply_batch` -- one persistent GEMM
launch for all their leaf products.  Requests that arrive while a batch is
on the GPU go to the next free lane, so the work of consecutive batches
overlaps on the device.  Built quadtrees stay resident in their lane (an
LRU cache keyed by the matrix spec) and are evicted only for memory.

Every result is the same as the request's result alone: the library's
batched products are bitwise equal to single products.

The scheduling (`Scheduler`) is plain Python and is tested with a fake
executor; `GpuLane` is the executor on the device.
"""
from __future__ import annotations

import threading
import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field

import numpy as np

MODE_NAMES = ("truncmul", "spamm", "hybrid")


@dataclass(frozen=True)
class MatrixSpec:
    kind: str      # "1d" or "3d"
    n: int
    alpha: float
    seed: int

    def key(self, leaf):
        return (self.kind, self.n, self.alpha, self.seed, leaf)


@dataclass
class RequestSpec:
    mat: MatrixSpec
    tau: float
    mode: int      # 0 truncmul, 1 spamm, 2 hybrid
    prec: int = 1  # FP32
    leaf: int = 64
    rid: int = -1

    def grid(self):
        g = -(-self.mat.n // self.leaf)
        G = 1
        while G < g:
            G *= 2
        return g, G

    def footprint(self, nonnull=None) -> int:
        """Arena bytes the request may need: the leaf store of A in the
        request's precision (FP64 or FP32), C (FP64 or FP32), the kept pairs
        (with the quad plan of a leaf-64 product: merged steps, their
        children and the k of every pair; of an FP64 leaf-128 / 256 product:
        bs / 64 steps of 17 bytes per pair and 128-tile) and the per-leaf
        arrays.
        `nonnull` (non-null leaves of A) defaults to an upper bound for the
        kind."""
        g, G = self.grid()
        e2 = self.leaf * self.leaf
        if nonnull is None:
            nonnull = g * g if self.mat.kind == "3d" else min(g * g, g * _band_leaves(self.mat, self.leaf))
        if self.mat.kind == "3d":
            c_leaves = min(g * g, 8 * nonnull)
        else:
            c_leaves = min(g * g, 2 * nonnull + g)
        row = max(1, nonnull // max(g, 1))
        kept = min(g ** 3, c_leaves * 2 * row)
        eb = 8 if self.prec == 0 else 4
        store = nonnull * e2 * (eb if self.prec in (0, 1) else 12)  # BF16 needs FP32 plus two BF16 copies
        if self.leaf == 64:
            per_pair = 8 + 21
        elif self.leaf > 64 and self.prec == 0:
            per_pair = 8 + 17 * (self.leaf // 64) * (self.leaf // 128) ** 2
        else:
            per_pair = 8
        return int(store + c_leaves * e2 * eb + kept * per_pair + G * G * 96 + (16 << 20))


def _band_leaves(m: MatrixSpec, leaf: int) -> int:
    """Leaves per block row of a 1D decay matrix (entries below 1e-16 are zero)."""
    w = int(np.ceil(np.log(1e16) / m.alpha))
    return 2 * (w // leaf + 1) + 1


def request_pool(count=512, seed=2024, n_max=65536, n_step=2048):
    """Seeded request pool: n ~ U{n_step .. n_max step n_step}, kind ~ U{1D,
    3D}, alpha ~ U[0.2, 1.0], tau = 10^U[-8, -4], scheme ~ U{T, S, H},
    FP32, A = B."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(1, n_max // n_step + 1)) * n_step
        kind = "1d" if rng.random() < 0.5 else "3d"
        alpha = float(rng.uniform(0.2, 1.0))
        tau = float(10.0 ** rng.uniform(-8, -4))
        mode = int(rng.integers(0, 3))
        out.append(RequestSpec(MatrixSpec(kind, n, round(alpha, 4), 1000 + i), tau, mode, rid=i))
    return out


@dataclass
class Result:
    rid: int
    stats: dict
    t_arrive: float
    t_start: float
    t_done: float
    lane: int
    batch: int
    C: object = None  # optional dense copy (tests)
    error: str = ""

    @property
    def latency(self):
        return self.t_done - self.t_arrive


@dataclass
class _Pending:
    spec: RequestSpec
    t_arrive: float
    fp: int
    done: threading.Event = field(default_factory=threading.Event)
    result: Result | None = None


class Scheduler:
    """Admission and batching.  `lanes` executors each expose `budget`
    (bytes) and `run(batch_specs) -> list[Result-like dicts]`.  A free lane
    takes pending requests in arrival order that fit budget - in-use bytes;
    a request larger than every lane's budget fails at once."""

    def __init__(self, lanes, max_batch=16, clock=time.perf_counter):
        self.lanes = lanes
        self.max_batch = max_batch
        self.clock = clock
        self.pending: deque[_Pending] = deque()
        self.cv = threading.Condition()
        self.stop = False
        self.busy = [False] * len(lanes)
        self.batches = 0
        self.log = []  # (lane, batch id, rids, t_start, t_done)
        self.threads = [threading.Thread(target=self._lane_loop, args=(i,), daemon=True) for i in range(len(lanes))]
        for t in self.threads:
            t.start()

    def submit(self, spec: RequestSpec, t_arrive=None) -> _Pending:
        p = _Pending(spec, self.clock() if t_arrive is None else t_arrive, spec.footprint())
        if p.fp > max(l.budget for l in self.lanes):
            p.result = Result(spec.rid, {}, p.t_arrive, p.t_arrive, self.clock(), -1, -1,
                              error="request larger than any lane's memory budget")
            p.done.set()
            return p
        with self.cv:
            self.pending.append(p)
            self.cv.notify_all()
        return p

    def _take(self, lane):
        """Pending requests for `lane`, in arrival order, within its budget."""
        room = self.lanes[lane].budget
        batch, keep = [], deque()
        while self.pending:
            p = self.pending.popleft()
            if len(batch) < self.max_batch and p.fp <= room:
                batch.append(p)
                room -= p.fp
            else:
                keep.append(p)
        self.pending = keep
        return batch

    def _lane_loop(self, lane):
        while True:
            with self.cv:
                while not self.stop and not self.pending:
                    self.cv.wait()
                if self.stop and not self.pending:
                    return
                batch = self._take(lane)
                if not batch:  # nothing fits this lane now; wait for a change
                    self.cv.wait(timeout=0.01)
                    continue
                bid = self.batches
                self.batches += 1
                self.busy[lane] = True
            t0 = self.clock()
            try:
                outs = self.lanes[lane].run([p.spec for p in batch])
                err = ""
            except Exception as e:  # a failed batch fails its requests
                outs = [dict() for _ in batch]
                err = f"{type(e).__name__}: {e}"
            t1 = self.clock()
            for p, o in zip(batch, outs):
                p.result = Result(p.spec.rid, o.get("stats", {}), p.t_arrive, t0, t1, lane, bid, o.get("C"),
                                  error=err or o.get("error", ""))
                p.done.set()
            with self.cv:
                self.busy[lane] = False
                self.log.append((lane, bid, [p.spec.rid for p in batch], t0, t1))
                self.cv.notify_all()

    def close(self):
        with self.cv:
            self.stop = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()


def make_input(mat: MatrixSpec, leaf: int):
    """Host input of a matrix spec: a leaf-block list for 1D decay (only the
    blocks inside the decay envelope), the dense matrix for 3D decay."""
    import synth
    sp = synth.DecaySpec(mat.kind, mat.n, mat.alpha, seed=mat.seed)
    if mat.kind == "1d":
        coords, data = sp.leaf_blocks(leaf)
        return ("blocks", coords.astype(np.int32), data)
    return ("dense", sp.dense())


class GpuLane:
    """One lane on the device: a context (own stream and arena) and an LRU
    cache of built quadtrees.  `inputs` maps a MatrixSpec to its host input
    (make_input) or is None to generate on demand."""

    def __init__(self, arena_bytes, device=0, inputs=None, keep_C=False, graph=False, options=None):
        import torch
        from . import spamm as S
        self.S = S
        self.stream = torch.cuda.Stream(device=device)
        self.ctx = S.Context(arena_bytes=arena_bytes, device=device, stream=self.stream)
        for k, v in (options or {}).items():  # context options (spamm.Context.set_option)
            self.ctx.set_option(k, v)
        if graph:  # each batch's kernels after the sizing read-back as one HIP graph
            self.ctx.set_option("graph", 1)
        self.budget = arena_bytes
        self.device = device
        self.inputs = inputs
        self.keep_C = keep_C
        self.cache: OrderedDict = OrderedDict()

    def _matrix(self, spec: RequestSpec):
        import torch
        S = self.S
        k = spec.mat.key(spec.leaf) + (spec.prec == self.S.F64,)
        if k in self.cache:
            self.cache.move_to_end(k)
            return self.cache[k]
        src = self.inputs.get(spec.mat) if self.inputs is not None else None
        if src is None:
            src = make_input(spec.mat, spec.leaf)
        dev = f"cuda:{self.device}"
        # only the copy the request multiplies in (norms come from the FP64 input)
        stores = S.STORE_F64 if spec.prec == S.F64 else S.STORE_F32
        with torch.cuda.stream(self.stream):
            if src[0] == "blocks":
                c = torch.from_numpy(src[1]).to(dev, non_blocking=False)
                d = torch.from_numpy(src[2]).to(dev, non_blocking=False)
                M = self.ctx.build_blocks(spec.mat.n, spec.leaf, c, d, stores=stores)
            else:
                d = torch.from_numpy(src[1]).to(dev, non_blocking=False)
                M = self.ctx.build(d, spec.leaf, stores=stores)
            self.stream.synchronize()
            del d
        self.cache[k] = M
        return M

    def _evict(self, need, keep):
        free = self.ctx.arena_info()["free"]
        while free < need and self.cache:
            k = next((x for x in self.cache if x not in keep), None)
            if k is None:
                break
            self.cache.pop(k).release()
            free = self.ctx.arena_info()["free"]

    def run(self, specs):
        S = self.S
        keys = {s.mat.key(s.leaf) + (s.prec == self.S.F64,) for s in specs}
        need = sum(s.footprint() for s in specs)
        self._evict(need, keys)
        mats = [self._matrix(s) for s in specs]
        reqs = [dict(A=M, B=M, tau=s.tau, mode=s.mode, prec=s.prec) for s, M in zip(specs, mats)]
        try:
            prods = self.ctx.multiply_batch(reqs)
        except S.SpammError as e:
            if e.code != "ENOMEM":
                raise
            if len(specs) == 1:
                # free space can be split: drop every other cached tree, once
                if not any(x not in keys for x in self.cache):
                    raise
                self._evict(float("inf"), keys)
                prods = self.ctx.multiply_batch(reqs)
            else:
                half = len(specs) // 2  # split the batch and retry
                return self.run(specs[:half]) + self.run(specs[half:])
        import torch
        out = []
        with torch.cuda.stream(self.stream):
            for p in prods:
                o = {"stats": dict(p.stats)}
                if self.keep_C:
                    o["C"] = self.ctx.to_dense(p.C).cpu()
                p.C.release()
                out.append(o)
        return out

    def close(self):
        for M in self.cache.values():
            M.release()
        self.cache.clear()
        self.ctx.close()


class Server:
    """Continuous-batching server over `lanes` GPU lanes."""

    def __init__(self, lanes=2, arena_bytes_per_lane=32 << 30, max_batch=16, device=0, inputs=None,
                 keep_C=False, graph=False, options=None):
        self.lanes = [GpuLane(arena_bytes_per_lane, device, inputs, keep_C, graph, options) for _ in range(lanes)]
        self.sched = Scheduler(self.lanes, max_batch=max_batch)

    def submit(self, spec: RequestSpec, t_arrive=None):
        return self.sched.submit(spec, t_arrive)

    def close(self):
        self.sched.close()
        for l in self.lanes:
            l.close()


def run_stream(server_or_sched, specs, rate, seed=7, clock=time.perf_counter, sleep=time.sleep):
    """Submit `specs` with Poisson arrivals at `rate` per second; wait for all
    results.  Returns the results in submission order."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=len(specs)) if rate > 0 else np.zeros(len(specs))
    t0 = clock()
    t = t0
    handles = []
    for s, g in zip(specs, gaps):
        t += g
        d = t - clock()
        if d > 0:
            sleep(d)
        handles.append(server_or_sched.submit(s, t_arrive=t))
    for h in handles:
        h.done.wait()
    return [h.result for h in handles]


def summarize(results, t_span=None):
    lat = sorted(r.latency for r in results if not r.error)
    ok = [r for r in results if not r.error]
    if not ok:
        return {"completed": 0}
    span = t_span if t_span is not None else (max(r.t_done for r in ok) - min(r.t_arrive for r in ok))
    flops = sum(r.stats.get("flops", 0.0) for r in ok)

    def q(p):
        return lat[min(len(lat) - 1, int(round(p * (len(lat) - 1))))]
    return {"completed": len(ok), "failed": len(results) - len(ok), "p50_s": q(0.5), "p99_s": q(0.99),
            "multiplies_per_s": len(ok) / span, "gflops": flops / span / 1e9, "span_s": span}
