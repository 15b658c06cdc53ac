"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference implementations of what the HIP
library computes, written from the paper (Navarro, Bustos, Hitschfeld,
"Possibilities of Recursive GPU Mapping for Discrete Orthogonal Simplices"):

* ``maps``          -- the block-space maps (lambda2 of Sec. III-A, the lambda3
                       reading of Sec. III-C, from below, the recursive sets of
                       Sec. III-B, the 4-simplex map on the set of Sec. III-D,
                       bounding box and linear enumeration of Sec. I), integer
                       arithmetic only.
* ``edm_rows`` / ``edm_packed`` / ``edm_pairs`` -- packed squared-distance
                       matrix on the 2-simplex (Sec. I, II), FP64 loops.
* ``at_energy`` / ``at_grad`` / ``at_grad_rows`` -- Axilrod-Teller triplet
                       energy (angle form) and its analytic gradient on the
                       3-simplex (Sec. I: triple-interaction n-body).
* ``at_triplet_rows`` -- per-triplet Axilrod-Teller energies, packed.
* ``lj_energy`` / ``lj_grad`` -- Lennard-Jones pair energy and gradient.
* ``quad_contacts`` -- 4-point contacts (4-cliques of the contact graph) on
                       the 4-simplex, by neighbour-list intersection.
* ``life_step`` / ``life_window`` -- Conway's Life on the 2-simplex of cells
                       (a cellular automaton on a triangular domain, Sec. I).
* ``checksum_range`` / ``checksum_walk`` -- element-id checksums.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import maps  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_dbl = ctypes.c_double
_ptr = ctypes.c_void_p


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_edm_rows.argtypes = [_ptr, _i64, _i64, _i64, _i64, _i64, _ptr]
        L.orc_edm_pairs.argtypes = [_ptr, _i64, _i64, _ptr, _ptr, _i64, _ptr]
        L.orc_at_energy.argtypes = [_ptr, _i64, _i64, _dbl, _i64, _i64]
        L.orc_at_energy.restype = _dbl
        L.orc_at_grad.argtypes = [_ptr, _i64, _i64, _dbl, _ptr]
        L.orc_at_triplet_rows.argtypes = [_ptr, _i64, _i64, _dbl, _i64, _i64, _ptr]
        L.orc_at_grad_rows.argtypes = [_ptr, _i64, _i64, _dbl, _ptr, _i64, _ptr]
        L.orc_lj_energy.argtypes = [_ptr, _i64, _i64, _dbl, _dbl, _dbl]
        L.orc_lj_energy.restype = _dbl
        L.orc_lj_grad.argtypes = [_ptr, _i64, _i64, _dbl, _dbl, _dbl, _ptr]
        L.orc_quad_contacts.argtypes = [_ptr, _i64, _i64, _dbl]
        L.orc_quad_contacts.restype = _i64
        L.orc_mix64.argtypes = [_u64]
        L.orc_mix64.restype = _u64
        L.orc_checksum_range.argtypes = [_u64]
        L.orc_checksum_range.restype = _u64
        L.orc_checksum_walk.argtypes = [ctypes.c_int, _i64, ctypes.POINTER(_i64)]
        L.orc_checksum_walk.restype = _u64
        _lib = L
    return _lib


def _f32(X: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float32)
    assert X.ndim == 2
    return X


def set_threads(k: int) -> None:
    """Thread count of the oracle's parallel loops from now on."""
    lib().orc_set_threads(int(k))


def threads() -> int:
    return lib().orc_max_threads()


def packed_offset(i: int, n: int) -> int:
    """Index of element (i, i) in the row-major packed upper triangle."""
    return i * n - (i * (i - 1)) // 2


def edm_rows(X: np.ndarray, i0: int, i1: int) -> np.ndarray:
    X = _f32(X)
    n, d = X.shape
    out = np.empty(packed_offset(i1, n) - packed_offset(i0, n), dtype=np.float64)
    lib().orc_edm_rows(X.ctypes.data, n, d, d, i0, i1, out.ctypes.data)
    return out


def edm_packed(X: np.ndarray) -> np.ndarray:
    return edm_rows(X, 0, X.shape[0])


def edm_pairs(X: np.ndarray, I: np.ndarray, J: np.ndarray) -> np.ndarray:
    X = _f32(X)
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    out = np.empty(I.shape[0], dtype=np.float64)
    lib().orc_edm_pairs(X.ctypes.data, X.shape[1], X.shape[1], I.ctypes.data, J.ctypes.data,
                        I.shape[0], out.ctypes.data)
    return out


def at_energy(X: np.ndarray, nu: float = 1.0, i0: int = 0, i1: int | None = None) -> float:
    X = _f32(X)
    n = X.shape[0]
    return lib().orc_at_energy(X.ctypes.data, n, X.shape[1], nu, i0, n if i1 is None else i1)


def triplet_rows_len(n: int, i0: int, i1: int) -> int:
    """Elements of rows [i0, i1) of the packed triplet array: sum of C(n-1-i, 2)."""
    return sum((n - 1 - i) * (n - 2 - i) // 2 for i in range(i0, i1))


def at_triplet_rows(X: np.ndarray, nu: float = 1.0, i0: int = 0, i1: int | None = None) -> np.ndarray:
    """Per-triplet energies of rows [i0, i1), triplets i < j < k in lexicographic order."""
    X = _f32(X)
    n = X.shape[0]
    i1 = n if i1 is None else i1
    out = np.empty(triplet_rows_len(n, i0, i1), dtype=np.float64)
    lib().orc_at_triplet_rows(X.ctypes.data, n, X.shape[1], nu, i0, i1, out.ctypes.data)
    return out


def at_grad(X: np.ndarray, nu: float = 1.0) -> np.ndarray:
    X = _f32(X)
    n = X.shape[0]
    G = np.empty((n, 3), dtype=np.float64)
    lib().orc_at_grad(X.ctypes.data, n, X.shape[1], nu, G.ctypes.data)
    return G


def at_grad_rows(X: np.ndarray, idx, nu: float = 1.0) -> np.ndarray:
    X = _f32(X)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    G = np.empty((idx.shape[0], 3), dtype=np.float64)
    lib().orc_at_grad_rows(X.ctypes.data, X.shape[0], X.shape[1], nu, idx.ctypes.data,
                           idx.shape[0], G.ctypes.data)
    return G


def lj_energy(X: np.ndarray, eps: float = 1.0, sigma: float = 1.0, rc: float = 3.0) -> float:
    X = _f32(X)
    return lib().orc_lj_energy(X.ctypes.data, X.shape[0], X.shape[1], eps, sigma, rc)


def lj_grad(X: np.ndarray, eps: float = 1.0, sigma: float = 1.0, rc: float = 3.0) -> np.ndarray:
    X = _f32(X)
    G = np.empty((X.shape[0], 3), dtype=np.float64)
    lib().orc_lj_grad(X.ctypes.data, X.shape[0], X.shape[1], eps, sigma, rc, G.ctypes.data)
    return G


def quad_contacts(X: np.ndarray, rc: float) -> int:
    """Quadruplets i<j<k<l with all six pairs in contact (FP32 squared distance
    below fl(rc^2)): the 4-cliques of the contact graph."""
    X = _f32(X)
    return int(lib().orc_quad_contacts(X.ctypes.data, X.shape[0], X.shape[1], rc))


def life_step(S: np.ndarray) -> np.ndarray:
    """One generation of Conway's Life (birth on 3 neighbours, survival on 2 or
    3, Moore neighbourhood) on the discrete orthogonal 2-simplex of cells
    (i, j), 0 <= i <= j < n: cells outside it are dead and stay dead.  S is a
    dense n x n uint8 grid; the result is one too, 0 below the diagonal."""
    n = S.shape[0]
    inside = np.triu(np.ones((n, n), dtype=bool))
    alive = (S != 0) & inside
    P = np.pad(alive, 1).astype(np.uint8)
    count = np.zeros((n, n), dtype=np.uint8)
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            if di or dj:
                count += P[1 + di:1 + di + n, 1 + dj:1 + dj + n]
    new = ((count == 3) | (alive & (count == 2))) & inside
    return new.astype(np.uint8)


def life_window(S: np.ndarray, i0: int, i1: int, j0: int, j1: int) -> np.ndarray:
    """Cells [i0, i1) x [j0, j1) of life_step(S), computed from that window of S
    and a one-cell ring around it (cells past the grid count as dead)."""
    n = S.shape[0]
    a0, a1, b0, b1 = max(i0 - 1, 0), min(i1 + 1, n), max(j0 - 1, 0), min(j1 + 1, n)
    W = np.zeros((a1 - a0 + 2, b1 - b0 + 2), dtype=np.uint8)
    W[1:-1, 1:-1] = S[a0:a1, b0:b1]
    ii = np.arange(a0 - 1, a1 + 1)[:, None]
    jj = np.arange(b0 - 1, b1 + 1)[None, :]
    inside = (ii <= jj) & (ii >= 0) & (jj < n)
    alive = (W != 0) & inside
    count = np.zeros((W.shape[0] - 2, W.shape[1] - 2), dtype=np.uint8)
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            if di or dj:
                count += alive[1 + di:W.shape[0] - 1 + di, 1 + dj:W.shape[1] - 1 + dj]
    core = alive[1:-1, 1:-1]
    new = ((count == 3) | (core & (count == 2))) & inside[1:-1, 1:-1]
    return new.astype(np.uint8)[i0 - a0:i1 - a0, j0 - b0:j1 - b0]


def mix64(x: int) -> int:
    return int(lib().orc_mix64(x))


def checksum_range(v: int) -> int:
    return int(lib().orc_checksum_range(v))


KIND = {"pairs_le": 0, "pairs_lt": 1, "triplets_le": 2, "triplets_lt": 3, "quads_le": 4, "quads_lt": 5}


def checksum_walk(kind: str, n: int) -> tuple[int, int]:
    c = _i64(0)
    s = lib().orc_checksum_walk(KIND[kind], n, ctypes.byref(c))
    return int(s), int(c.value)


def simplex_volume(m: int, n: int, strict: bool) -> int:
    """Number of elements: C(n+m-1, m) (paper eq. (2)) or C(n, m) when strict."""
    from math import comb
    return comb(n, m) if strict else comb(n + m - 1, m)
