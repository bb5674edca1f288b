"""Thin Python binding of libspamm.so (include/spamm.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory (the arena and input tensors) and the
stream.  If the compiled library is missing this module raises; there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libspamm.so")

TRUNCMUL, SPAMM, HYBRID, SPAMM_SYM, HYBRID_SYM = 0, 1, 2, 3, 4
F64, F32, BF16, BF16X3 = 0, 1, 2, 3
STORE_F64, STORE_F32, STORE_BF16 = 1, 2, 4
MODES = {"truncmul": TRUNCMUL, "spamm": SPAMM, "hybrid": HYBRID, "spamm_sym": SPAMM_SYM, "hybrid_sym": HYBRID_SYM}
PRECS = {"f64": F64, "f32": F32, "bf16": BF16, "bf16x3": BF16X3}
STATUS = {0: "OK", 1: "EINVAL", 2: "ESHAPE", 3: "ENOMEM", 4: "ENONFINITE",
          5: "EUNSUPPORTED", 6: "EDEVICE"}


class SpammError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.code = STATUS.get(status, str(status))
        super().__init__(f"SPAMM_{self.code}: {message}")


class Stats(ctypes.Structure):
    _fields_ = [("n_kept", ctypes.c_int64), ("n_candidates", ctypes.c_int64),
                ("c_nonnull", ctypes.c_int64), ("flops", ctypes.c_double),
                ("B1", ctypes.c_double), ("B2", ctypes.c_double),
                ("dA", ctypes.c_double), ("dB", ctypes.c_double),
                ("normA", ctypes.c_double), ("normB", ctypes.c_double),
                ("normA_used", ctypes.c_double), ("err_bound", ctypes.c_double),
                ("trace", ctypes.c_double), ("normC", ctypes.c_double),
                ("prec_bound", ctypes.c_double), ("val_err", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# The same two records as numpy dtypes (C layout), so that a whole batch is
# marshalled with one array conversion instead of per-field ctypes access.
STATS_DTYPE = np.dtype([(k, np.int64 if t is ctypes.c_int64 else np.float64) for k, t in Stats._fields_])
REQUEST_DTYPE = np.dtype([("A", np.uintp), ("B", np.uintp), ("tau", np.float64), ("mode", np.int32),
                          ("prec", np.int32), ("ep", np.uintp)], align=True)


class BlockList(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("leaf", ctypes.c_int32), ("stores", ctypes.c_uint32),
                ("nblocks", ctypes.c_int64), ("coords", ctypes.c_void_p), ("data", ctypes.c_void_p)]


class Epilogue(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("D", ctypes.c_void_p)]


class Request(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("tau", ctypes.c_double),
                ("mode", ctypes.c_int32), ("prec", ctypes.c_int32), ("ep", ctypes.c_void_p)]


assert REQUEST_DTYPE.itemsize == ctypes.sizeof(Request) and STATS_DTYPE.itemsize == ctypes.sizeof(Stats)


class MatInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("leaf", ctypes.c_int32), ("G", ctypes.c_int32),
                ("L", ctypes.c_int32), ("nonnull", ctypes.c_int64), ("stores", ctypes.c_uint32),
                ("has_plan", ctypes.c_int32), ("n_kept", ctypes.c_int64),
                ("device_bytes", ctypes.c_size_t)]


class Timing(ctypes.Structure):
    _fields_ = [("build_ms", ctypes.c_double), ("trunc_ms", ctypes.c_double),
                ("prune_ms", ctypes.c_double), ("gemm_ms", ctypes.c_double),
                ("pyramid_ms", ctypes.c_double), ("build_launches", ctypes.c_int64),
                ("trunc_launches", ctypes.c_int64), ("prune_launches", ctypes.c_int64),
                ("gemm_launches", ctypes.c_int64), ("pyramid_launches", ctypes.c_int64),
                ("gemm_flops", ctypes.c_double), ("gemm_quad_launches", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

_SIGS = {
    "spamm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "spamm_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "spamm_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "spamm_ctx_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "spamm_ctx_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "spamm_ctx_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(Timing)]),
    "spamm_ctx_arena_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t),
                                            ctypes.POINTER(ctypes.c_size_t),
                                            ctypes.POINTER(ctypes.c_size_t)]),
    "spamm_build": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p)]),
    "spamm_build_blocks": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p)]),
    "spamm_truncate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_double)]),
    "spamm_truncate_symmetric": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_double)]),
    "spamm_truncate_elementwise": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_double)]),
    "spamm_multiply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Stats)]),
    "spamm_build_blocks_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                                ctypes.POINTER(ctypes.c_void_p)]),
    "spamm_multiply_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]),
    "spamm_norms": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "spamm_kept": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.POINTER(ctypes.c_int64)]),
    "spamm_skipped_bound": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_int64]),
    "spamm_to_dense": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "spamm_ctx_set_option": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64]),
    "spamm_ctx_get_option": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]),
    "spamm_gershgorin": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]),
    "spamm_gershgorin_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "spamm_leaves": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_void_p]),
    "spamm_mat_info_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MatInfo)]),
    "spamm_release": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
}


def load_library(path: str | None = None):
    """Load libspamm.so (after torch, so both share one HIP runtime).  The
    environment variable SPAMM_LIB may name another build of the library."""
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        path = os.environ.get("SPAMM_LIB", LIB_PATH)
    import torch  # noqa: F401  (binds libamdhip64 first)
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_1906_08148_amd.build_lib` (no fallback exists)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols(path: str | None = None):
    lib = load_library(path)
    return {name for name in _SIGS if hasattr(lib, name)}


class Matrix:
    """A library matrix handle (immutable)."""

    def __init__(self, ctx: "Context", handle: int):
        self.ctx = ctx
        self.handle = ctypes.c_void_p(handle)

    @property
    def info(self) -> MatInfo:
        out = MatInfo()
        self.ctx._check(_lib.spamm_mat_info_get(self.handle, ctypes.byref(out)))
        return out

    @property
    def n(self):
        return self.info.n

    def release(self):
        if self.handle is not None and self.handle.value:
            _lib.spamm_release(self.ctx.ptr, self.handle)
        self.handle = None

    def __del__(self):
        try:
            if self.handle is not None and self.ctx.ptr is not None:
                self.release()
        except Exception:
            pass


def _hval(m: Matrix) -> int:
    """The handle's address (0 for a released matrix, which the library rejects)."""
    return (m.handle.value or 0) if m.handle is not None else 0


@dataclass
class Product:
    C: Matrix
    stats: dict | None


class Context:
    """Library context over a torch-allocated device arena."""

    def __init__(self, arena_bytes: int = 1 << 30, device: int = 0, stream=None):
        import torch
        load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the spamm library needs an MI355X (gfx950)")
        self.device = device
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = s
        out = ctypes.c_void_p()
        st = _lib.spamm_ctx_create(device, ctypes.c_void_p(self.arena.data_ptr()), self.arena.numel(),
                                   ctypes.c_void_p(s.cuda_stream), ctypes.byref(out))
        if st != 0:
            raise SpammError(st, "spamm_ctx_create failed")
        self.ptr = out

    def _check(self, st):
        if st != 0:
            raise SpammError(st, _lib.spamm_last_error(self.ptr).decode())

    def close(self):
        if self.ptr is not None:
            import gc
            gc.collect()
            st = _lib.spamm_ctx_destroy(self.ptr)
            self.ptr = None
            if st == 0:
                # the context synchronised its stream and is gone: the arena
                # goes back to torch now, not when this object is collected
                self.arena = None

    def arena_info(self):
        u, f, l = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        self._check(_lib.spamm_ctx_arena_info(self.ptr, ctypes.byref(u), ctypes.byref(f), ctypes.byref(l)))
        return {"used": u.value, "free": f.value, "largest_free": l.value}

    def timing(self, enable: bool = True, reset: bool = False, read: bool = True):
        """Enable/disable per-kernel-class event timing; returns the totals
        since the last reset (synchronises) when ``read``."""
        out = Timing() if read else None
        self._check(_lib.spamm_ctx_timing(self.ptr, int(enable), int(reset),
                                          ctypes.byref(out) if read else None))
        return out.as_dict() if read else None

    def set_stream(self, stream):
        self._check(_lib.spamm_ctx_set_stream(self.ptr, ctypes.c_void_p(stream.cuda_stream)))
        self.stream = stream

    # ---- build
    def build(self, dense, leaf: int, stores: int = STORE_F64 | STORE_F32) -> Matrix:
        import torch
        assert dense.dtype == torch.float64 and dense.is_cuda and dense.dim() == 2
        assert dense.stride(1) == 1
        out = ctypes.c_void_p()
        self._check(_lib.spamm_build(self.ptr, ctypes.c_void_p(dense.data_ptr()), dense.shape[0],
                                     dense.stride(0), leaf, stores, ctypes.byref(out)))
        return Matrix(self, out.value)

    def build_blocks(self, n: int, leaf: int, coords, data, stores: int = STORE_F64 | STORE_F32) -> Matrix:
        import torch
        assert coords.dtype == torch.int32 and coords.is_cuda and coords.is_contiguous()
        assert data.dtype == torch.float64 and data.is_cuda and data.is_contiguous()
        out = ctypes.c_void_p()
        m = coords.shape[0]
        self._check(_lib.spamm_build_blocks(self.ptr, n, leaf, m, ctypes.c_void_p(coords.data_ptr() if m else 0),
                                            ctypes.c_void_p(data.data_ptr() if m else 0), stores,
                                            ctypes.byref(out)))
        return Matrix(self, out.value)

    def build_blocks_batch(self, lists, stores: int = STORE_F64 | STORE_F32):
        """Several block-list builds with one synchronisation: `lists` holds
        (n, leaf, coords, data) tuples as for build_blocks."""
        import torch
        k = len(lists)
        arr = (BlockList * k)()
        for i, (n, leaf, coords, data) in enumerate(lists):
            assert coords.dtype == torch.int32 and coords.is_cuda and coords.is_contiguous()
            assert data.dtype == torch.float64 and data.is_cuda and data.is_contiguous()
            m = coords.shape[0]
            arr[i] = BlockList(n, leaf, stores, m, coords.data_ptr() if m else 0, data.data_ptr() if m else 0)
        outs = (ctypes.c_void_p * k)()
        self._check(_lib.spamm_build_blocks_batch(self.ptr, k, arr, outs))
        return [Matrix(self, outs[i]) for i in range(k)]

    # ---- truncation / multiply
    def truncate(self, m: Matrix, tau: float, symmetric: bool = False):
        """Leaf-block truncation with budget tau (Sec. 3); symmetric: in
        mirror pairs.  Returns (matrix, dropped squared norm)."""
        out = ctypes.c_void_p()
        dropped = ctypes.c_double()
        fn = _lib.spamm_truncate_symmetric if symmetric else _lib.spamm_truncate
        self._check(fn(self.ptr, m.handle, tau, ctypes.byref(out), ctypes.byref(dropped)))
        return Matrix(self, out.value), dropped.value

    def truncate_elementwise(self, m: Matrix, tau: float):
        """Zero every entry with |a| < tau (Thm. 1); returns (matrix, dropped squared norm)."""
        out = ctypes.c_void_p()
        dropped = ctypes.c_double()
        self._check(_lib.spamm_truncate_elementwise(self.ptr, m.handle, tau, ctypes.byref(out),
                                                    ctypes.byref(dropped)))
        return Matrix(self, out.value), dropped.value

    def multiply(self, A: Matrix, B: Matrix, tau: float, mode=SPAMM, prec=F32,
                 alpha=None, beta=None, D: Matrix | None = None, stats: bool = True) -> Product:
        return self.multiply_batch([dict(A=A, B=B, tau=tau, mode=mode, prec=prec, alpha=alpha,
                                         beta=beta, D=D)], stats=stats)[0]

    def multiply_batch(self, reqs, stats: bool = True):
        n = len(reqs)
        rows = []
        eps = []  # epilogue records stay alive until the call returns
        for r in reqs:
            mode = MODES.get(r.get("mode"), r.get("mode", SPAMM))
            prec = PRECS.get(r.get("prec"), r.get("prec", F32))
            ep = 0
            if r.get("alpha") is not None or r.get("beta") is not None or r.get("D") is not None:
                e = Epilogue(1.0 if r.get("alpha") is None else float(r["alpha"]),
                             0.0 if r.get("beta") is None else float(r["beta"]),
                             r["D"].handle if r.get("D") is not None else None)
                eps.append(e)
                ep = ctypes.addressof(e)
            rows.append((_hval(r["A"]), _hval(r["B"]), float(r["tau"]), int(mode), int(prec), ep))
        arr = np.array(rows, dtype=REQUEST_DTYPE)
        outs = (ctypes.c_void_p * n)()
        st = np.zeros(n, dtype=STATS_DTYPE) if stats else None
        self._check(_lib.spamm_multiply_batch(self.ptr, n, arr.ctypes.data_as(ctypes.c_void_p), outs,
                                              st.ctypes.data_as(ctypes.c_void_p) if stats else None))
        if not stats:
            return [Product(Matrix(self, outs[i]), None) for i in range(n)]
        names = STATS_DTYPE.names
        return [Product(Matrix(self, outs[i]), dict(zip(names, row))) for i, row in enumerate(st.tolist())]

    # ---- read-back
    def norms(self, m: Matrix, level: int = -1) -> np.ndarray:
        info = m.info
        cnt = ((4 ** (info.L + 1)) - 1) // 3 if level < 0 else 4 ** level
        buf = np.zeros(cnt, dtype=np.float64)
        got = ctypes.c_int64()
        self._check(_lib.spamm_norms(self.ptr, m.handle, level, buf.ctypes.data_as(ctypes.c_void_p), cnt,
                                     ctypes.byref(got)))
        return buf

    def kept(self, C: Matrix) -> np.ndarray:
        nk = C.info.n_kept
        buf = np.zeros((max(nk, 0), 3), dtype=np.int32)
        got = ctypes.c_int64()
        self._check(_lib.spamm_kept(self.ptr, C.handle, buf.ctypes.data_as(ctypes.c_void_p), nk,
                                    ctypes.byref(got)))
        return buf.astype(np.int64)

    def skipped_bound(self, C: Matrix) -> np.ndarray:
        G = C.info.G
        buf = np.zeros(G * G, dtype=np.float64)
        self._check(_lib.spamm_skipped_bound(self.ptr, C.handle, buf.ctypes.data_as(ctypes.c_void_p), G * G))
        return buf

    def to_dense(self, m: Matrix):
        import torch
        n = m.info.n
        out = torch.empty((n, n), dtype=torch.float64, device=f"cuda:{self.device}")
        self._check(_lib.spamm_to_dense(self.ptr, m.handle, ctypes.c_void_p(out.data_ptr()), n))
        return out

    OPTIONS = {"gemm_tile": 0, "placement": 1, "graph": 2, "unit_order": 3,  # unit_order: chunk size (0: contiguous ranges)
               "validate": 4, "gemm_quad": 5}

    def set_option(self, name: str, value: int):
        """validate (1: measure ||C - C_FP64||_F into stats["val_err"]),
        gemm_tile (1: 16x16 MFMA tiles, the default; 0: 32x32), placement (0: XCD
        slices, 1: request-major), graph (1: one captured graph per batch),
        gemm_quad (1: leaf-64 products in quads of sibling C leaves, and
        leaf-128 / 256 tiles as quads of their 64 x 64 blocks; 0: one C leaf
        (or tile) per work unit; -1, the default: leaf 64 on quads where the
        C leaves average enough kept products, leaves 128 / 256 on quads in
        FP64)."""
        self._check(_lib.spamm_ctx_set_option(self.ptr, self.OPTIONS[name], int(value)))

    def get_option(self, name: str) -> int:
        v = ctypes.c_int64()
        self._check(_lib.spamm_ctx_get_option(self.ptr, self.OPTIONS[name], ctypes.byref(v)))
        return v.value

    def gershgorin(self, m: Matrix):
        """(lo, hi) Gershgorin bounds of the spectrum, FP64."""
        lo, hi = ctypes.c_double(), ctypes.c_double()
        self._check(_lib.spamm_gershgorin(self.ptr, m.handle, ctypes.byref(lo), ctypes.byref(hi)))
        return lo.value, hi.value

    def gershgorin_static(self, m: Matrix, bounds):
        """Gershgorin bounds written into the device tensor `bounds` (two
        float64 values, lo then hi), stream-ordered, with no allocation."""
        import torch
        assert bounds.dtype == torch.float64 and bounds.is_cuda and bounds.numel() >= 2 and bounds.is_contiguous()
        self._check(_lib.spamm_gershgorin_static(self.ptr, m.handle, ctypes.c_void_p(bounds.data_ptr())))

    def identity(self, n: int, leaf: int, stores: int = STORE_F64 | STORE_F32) -> Matrix:
        """The n x n identity as a quadtree (diagonal leaves only)."""
        import torch
        g = -(-n // leaf)
        coords = torch.tensor([[i, i] for i in range(g)], dtype=torch.int32, device=f"cuda:{self.device}")
        blk = np.zeros((g, leaf, leaf), dtype=np.float64)
        for i in range(g):
            m = min(leaf, n - i * leaf)
            blk[i, np.arange(m), np.arange(m)] = 1.0
        data = torch.from_numpy(blk).to(f"cuda:{self.device}")
        return self.build_blocks(n, leaf, coords, data, stores=stores)

    def leaves(self, m: Matrix, ij) -> np.ndarray:
        """FP64 copies of the leaves at block coordinates ij (k, 2): (k, bs, bs)."""
        ij = np.ascontiguousarray(np.asarray(ij, dtype=np.int32).reshape(-1, 2))
        bs = m.info.leaf
        out = np.zeros((len(ij), bs, bs), dtype=np.float64)
        self._check(_lib.spamm_leaves(self.ptr, m.handle, ij.ctypes.data_as(ctypes.c_void_p), len(ij),
                                      out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def morton_order_to_grid(vals: np.ndarray, level: int) -> np.ndarray:
    """Reshape a level's Morton-ordered values into a (2^level, 2^level) grid."""
    side = 1 << level
    m = np.arange(side * side, dtype=np.int64)
    r = np.zeros_like(m)
    c = np.zeros_like(m)
    for b in range(level):
        r |= ((m >> (2 * b + 1)) & 1) << b
        c |= ((m >> (2 * b)) & 1) << b
    out = np.zeros((side, side), dtype=vals.dtype)
    out[r, c] = vals
    return out
