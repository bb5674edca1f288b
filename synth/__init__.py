"""Seeded synthetic inputs: matrices with exponential decay.

This module only *draws inputs*.  It holds none of the approximate-product
arithmetic (no norms, no truncation, no pruning, no block products), so both
the CPU oracle and the GPU path may take their inputs from it.

Definition of the generator (the single source of truth for every input in
tests and benchmarks):

* ``splitmix64(x)``: the SplitMix64 finaliser of Steele, Lea and Flood
  (OOPSLA 2014), in the form popularised by S. Vigna: add the golden-ratio
  increment ``0x9E3779B97F4A7C15`` and apply two xor-shift-multiply rounds and
  a final xor-shift, all modulo 2**64.
* ``u(seed, i, j) = (splitmix64((seed << 40) ^ (min(i,j)*n + max(i,j))) >> 11) * 2**-53``,
  a uniform double in [0, 1) that is symmetric in (i, j).
* 1D decay (distance d(i,j) = |i-j|, the model problem of the paper's results
  section):  a_ij = (2 u_ij - 1) * exp(-alpha |i-j|).
* 3D decay (distance = Euclidean distance between basis-function centres, the
  structure of the paper's overlap matrices): atoms sit on the Z-order
  (Morton) prefix of a 32^3 unit lattice, each jittered by U[-0.1, 0.1]^3
  drawn from ``u`` with salt bit 39 set in the key; every atom carries
  ``funcs_per_atom`` (default 8) consecutive basis functions at its position;
  a_ij = (2 u_ij - 1) * exp(-alpha * dist(i, j)).
* Entries with |a_ij| < 1e-16 are set to zero, as the paper does for its model
  problem.

The integer/hash part is reproduced bit-for-bit by the NumPy and the torch
backends; ``exp``/``sqrt`` may differ by an ulp between backends, so one run
always feeds the *same* generated bits to every consumer.
"""
from __future__ import annotations

import os

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
MIX1 = np.uint64(0xBF58476D1CE4E5B9)
MIX2 = np.uint64(0x94D049BB133111EB)
TINY = 1e-16
JITTER = 0.1
JITTER_SALT = 1 << 39
LATTICE_BITS = 5  # 32^3 lattice


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied to a uint64 array (wraps mod 2**64)."""
    z = np.asarray(x, dtype=np.uint64) + GOLDEN
    z = (z ^ (z >> np.uint64(30))) * MIX1
    z = (z ^ (z >> np.uint64(27))) * MIX2
    return z ^ (z >> np.uint64(31))


def _u_from_key(key: np.ndarray) -> np.ndarray:
    return (splitmix64(key) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform(seed: int, i: np.ndarray, j: np.ndarray, n: int) -> np.ndarray:
    """Symmetric uniform u(seed, i, j) in [0, 1) (broadcasting i, j)."""
    i = np.asarray(i, dtype=np.uint64)
    j = np.asarray(j, dtype=np.uint64)
    lo = np.minimum(i, j)
    hi = np.maximum(i, j)
    key = (np.uint64(seed) << np.uint64(40)) ^ (lo * np.uint64(n) + hi)
    return _u_from_key(key)


def morton3_decode(a: np.ndarray):
    """Lattice coordinates of Z-order index a in a 2^5-per-side cube."""
    a = np.asarray(a, dtype=np.int64)
    xyz = [np.zeros_like(a) for _ in range(3)]
    for b in range(LATTICE_BITS):
        for c in range(3):
            xyz[c] |= ((a >> (3 * b + c)) & 1) << b
    return xyz[2], xyz[1], xyz[0]


def atom_positions(seed: int, n_atoms: int) -> np.ndarray:
    """(n_atoms, 3) float64 jittered lattice positions (Morton prefix)."""
    if n_atoms > 1 << (3 * LATTICE_BITS):
        raise ValueError("at most 32768 atoms")
    a = np.arange(n_atoms, dtype=np.int64)
    x, y, z = morton3_decode(a)
    pos = np.stack([x, y, z], axis=1).astype(np.float64)
    keys = (np.uint64(seed) << np.uint64(40)) ^ np.uint64(JITTER_SALT) ^ (
        np.arange(3 * n_atoms, dtype=np.uint64))
    jit = (2.0 * _u_from_key(keys) - 1.0) * JITTER
    return pos + jit.reshape(n_atoms, 3)


class DecaySpec:
    """A seeded decay matrix: kind '1d' or '3d', size n, decay rate alpha."""

    def __init__(self, kind: str, n: int, alpha: float, seed: int = 1,
                 funcs_per_atom: int = 8):
        if kind not in ("1d", "3d"):
            raise ValueError(kind)
        self.kind, self.n, self.alpha, self.seed = kind, int(n), float(alpha), int(seed)
        self.fpa = int(funcs_per_atom)
        self._pos = None
        if kind == "3d":
            if self.n % self.fpa:
                raise ValueError("n must be a multiple of funcs_per_atom")
            self._pos = atom_positions(self.seed, self.n // self.fpa)

    def __repr__(self):
        return f"DecaySpec({self.kind!r}, n={self.n}, alpha={self.alpha}, seed={self.seed})"

    def distance(self, i: np.ndarray, j: np.ndarray) -> np.ndarray:
        if self.kind == "1d":
            return np.abs(i.astype(np.float64) - j.astype(np.float64))
        pi = self._pos[i // self.fpa]
        pj = self._pos[j // self.fpa]
        d = pi - pj
        return np.sqrt((d * d).sum(axis=-1))

    def block(self, r0: int, r1: int, c0: int, c1: int) -> np.ndarray:
        """Dense entries for rows [r0, r1) x cols [c0, c1) (clipped to n)."""
        r1, c1 = min(r1, self.n), min(c1, self.n)
        i = np.arange(r0, r1, dtype=np.int64)[:, None]
        j = np.arange(c0, c1, dtype=np.int64)[None, :]
        i, j = np.broadcast_arrays(i, j)
        u = uniform(self.seed, i, j, self.n)
        if self.kind == "1d":
            env = np.exp(-self.alpha * self.distance(i, j))
        else:
            # the envelope depends on the atom pair only: the same distance
            # and exponential as per entry, evaluated once per atom pair
            ai = np.arange(r0, r1, dtype=np.int64) // self.fpa
            aj = np.arange(c0, c1, dtype=np.int64) // self.fpa
            a0, b0 = ai[0], aj[0]
            pa = self._pos[a0:ai[-1] + 1]
            pb = self._pos[b0:aj[-1] + 1]
            d = pa[:, None, :] - pb[None, :, :]
            e_atoms = np.exp(-self.alpha * np.sqrt((d * d).sum(axis=-1)))
            env = e_atoms[(ai - a0)[:, None], (aj - b0)[None, :]]
        a = (2.0 * u - 1.0) * env
        a[np.abs(a) < TINY] = 0.0
        return a

    def dense(self) -> np.ndarray:
        """The whole matrix; row blocks are generated on a thread pool (the
        values do not depend on the split)."""
        out = np.empty((self.n, self.n), dtype=np.float64)
        step = max(1, (1 << 21) // max(self.n, 1))
        starts = list(range(0, self.n, step))

        def fill(r):
            out[r:r + step] = self.block(r, r + step, 0, self.n)

        workers = min(16, os.cpu_count() or 1, len(starts))
        if workers <= 1:
            for r in starts:
                fill(r)
        else:
            from concurrent.futures import ThreadPoolExecutor
            with ThreadPoolExecutor(workers) as ex:
                list(ex.map(fill, starts))
        return out

    def leaf_blocks(self, bs: int):
        """Candidate leaf blocks for building from a block list.

        Returns (coords, data): int32 (m, 2) block coordinates (I, J) and
        float64 (m, bs, bs) zero-padded block contents, for every block whose
        decay envelope can exceed the 1e-16 cut.  Blocks may still be all
        zero; the library decides what is null.
        """
        g = -(-self.n // bs)
        coords = []
        if self.kind == "1d":
            # smallest |i-j| inside block (I,J) is max(0, |I-J|*bs - (bs-1))
            for I in range(g):
                for J in range(g):
                    dmin = max(0, abs(I - J) * bs - (bs - 1))
                    if np.exp(-self.alpha * dmin) >= TINY:
                        coords.append((I, J))
        else:
            coords = [(I, J) for I in range(g) for J in range(g)]
        coords = np.asarray(coords, dtype=np.int32).reshape(-1, 2)
        data = np.zeros((len(coords), bs, bs), dtype=np.float64)
        for t, (I, J) in enumerate(coords):
            blk = self.block(I * bs, (I + 1) * bs, J * bs, (J + 1) * bs)
            data[t, :blk.shape[0], :blk.shape[1]] = blk
        return coords, data


def dense_from_blocks(n: int, bs: int, coords: np.ndarray, data: np.ndarray) -> np.ndarray:
    """Assemble a dense n x n matrix from a block list (later blocks win)."""
    g = -(-n // bs)
    full = np.zeros((g * bs, g * bs), dtype=np.float64)
    for (I, J), blk in zip(coords, data):
        full[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = blk
    return np.ascontiguousarray(full[:n, :n])


def random_blocks(seed: int, n: int, bs: int, fill: float):
    """Random uniform non-zero blocks (the leaf-library benchmark input):
    each block of the ceil(n/bs)^2 grid is non-zero with probability
    ``fill``; entries are 2u-1 from the same hash."""
    g = -(-n // bs)
    I, J = np.meshgrid(np.arange(g), np.arange(g), indexing="ij")
    sel = uniform(seed + 7919, I, J, g) < fill
    coords = np.stack([I[sel], J[sel]], axis=1).astype(np.int32)
    data = np.zeros((len(coords), bs, bs), dtype=np.float64)
    for t, (a, b) in enumerate(coords):
        i = np.arange(a * bs, a * bs + bs, dtype=np.int64)[:, None]
        j = np.arange(b * bs, b * bs + bs, dtype=np.int64)[None, :]
        i, j = np.broadcast_arrays(i, j)
        # not symmetric on purpose: key uses (i, j) in order
        key = (np.uint64(seed) << np.uint64(40)) ^ (
            i.astype(np.uint64) * np.uint64(g * bs) + j.astype(np.uint64))
        blk = 2.0 * _u_from_key(key) - 1.0
        blk[(i >= n) | (j >= n)] = 0.0
        data[t] = blk
    return coords, data
