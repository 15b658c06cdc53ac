"""Seeded synthetic inputs shared by the HIP path's tests/bench and by the oracle.

This module only draws numbers.  It holds none of the simplex-map or
interaction arithmetic: neither the oracle nor the HIP library imports the
other, and both receive their inputs from here.

Recipes (all seeded with ``numpy.random.default_rng(seed)``, PCG64):

* ``uniform``  -- FP32 coordinates uniform in [0, 1)^d.
* ``normal``   -- FP32 coordinates drawn from N(0, 1).
* ``integer``  -- FP32 coordinates that are small integers; with them every
  FP32 squared distance below 2**24 is exact, so FP32 and FP64 agree bit for bit.
* ``rsa``      -- random sequential adsorption in a cube: candidates are drawn
  uniformly (FP64) in [0, side)^3 and kept only if their distance to every
  point kept so far is at least ``dmin``; the kept points are cast to FP32.

* ``bits``     -- uint8 0/1 cells of an n x n grid, each 1 with probability
  ``density`` (the initial states of the cellular automaton on the 2-simplex;
  the consumer keeps the cells of its domain).

``WORKLOADS`` lists the workloads by what they are.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["uniform", "normal", "integer", "rsa", "bits", "WORKLOADS", "workload_input"]


def uniform(n: int, d: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((n, d), dtype=np.float32)


def normal(n: int, d: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, d), dtype=np.float32)


def integer(n: int, d: int, seed: int, lo: int = -8, hi: int = 8) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi, size=(n, d)).astype(np.float32)


def bits(n: int, seed: int, density: float = 0.3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    thr = int(round(density * 256))
    return (rng.integers(0, 256, size=(n, n), dtype=np.uint8) < thr).astype(np.uint8)


def bits_flat(count: int, seed: int, density: float = 0.3) -> np.ndarray:
    """``count`` independent cells, 1 with probability ``density`` (in steps of
    1/256), as a flat uint8 vector: a cell buffer in any layout."""
    rng = np.random.default_rng(seed)
    thr = int(round(density * 256))
    return (rng.integers(0, 256, size=count, dtype=np.uint8) < thr).astype(np.uint8)


def rsa(n: int, seed: int, side: float = 20.0, dmin: float = 0.8,
        batch: int = 8192, max_tries: int = 50_000_000) -> np.ndarray:
    """Random sequential adsorption of ``n`` points in [0, side)^3.

    A candidate is accepted iff its Euclidean distance to every previously
    accepted point is >= ``dmin``.  A uniform cell grid with cells no smaller
    than ``dmin`` only accelerates the test (27 neighbouring cells hold every
    point that could be closer than ``dmin``); it does not change which points
    are kept.
    """
    rng = np.random.default_rng(seed)
    ncell = max(1, int(math.floor(side / dmin)))
    csize = side / ncell
    assert csize >= dmin
    cells: dict[tuple[int, int, int], list[tuple[float, float, float]]] = {}
    out: list[tuple[float, float, float]] = []
    d2 = dmin * dmin
    tries = 0
    while len(out) < n:
        cand = (rng.random((batch, 3)) * side).tolist()
        for p in cand:
            tries += 1
            if tries > max_tries:
                raise RuntimeError(f"rsa: {n} points at dmin={dmin} not reached in {max_tries} tries")
            cx = min(int(p[0] / csize), ncell - 1)
            cy = min(int(p[1] / csize), ncell - 1)
            cz = min(int(p[2] / csize), ncell - 1)
            ok = True
            for ax in (cx - 1, cx, cx + 1):
                if not ok:
                    break
                for ay in (cy - 1, cy, cy + 1):
                    if not ok:
                        break
                    for az in (cz - 1, cz, cz + 1):
                        lst = cells.get((ax, ay, az))
                        if lst is None:
                            continue
                        for q in lst:
                            dx = p[0] - q[0]
                            dy = p[1] - q[1]
                            dz = p[2] - q[2]
                            if dx * dx + dy * dy + dz * dz < d2:
                                ok = False
                                break
                        if not ok:
                            break
            if ok:
                t = (p[0], p[1], p[2])
                out.append(t)
                cells.setdefault((cx, cy, cz), []).append(t)
                if len(out) == n:
                    break
    return np.asarray(out, dtype=np.float64).astype(np.float32)


# The five workloads: name -> (generator, kwargs, description)
WORKLOADS = {
    "edm_n1024_d3": dict(kind="uniform", n=1024, d=3, seed=0,
                         desc="packed EDM, n=1024, d=3, FP32 uniform [0,1)^3; lambda map dump"),
    "edm_n65536_d64": dict(kind="normal", n=65536, d=64, seed=1,
                           desc="packed EDM, n=65536, d=64, FP32 N(0,1), difference form"),
    "gram_n32768_d512": dict(kind="normal", n=32768, d=512, seed=2,
                             desc="packed EDM via Gram form, n=32768, d=512, N(0,1) -> BF16 hi/lo"),
    "at_n2048": dict(kind="rsa", n=2048, d=3, seed=3,
                     desc="Axilrod-Teller energy+forces, n=2048, RSA cube side 20, dmin 0.8, nu=1"),
    "at_lj_n8192": dict(kind="rsa", n=8192, d=3, seed=4,
                        desc="Axilrod-Teller + Lennard-Jones (eps=sigma=1, rc=3), n=8192, RSA cube side 20"),
}


def workload_input(name: str, n: int | None = None) -> np.ndarray:
    """Input array of a named workload (optionally with a different n)."""
    w = WORKLOADS[name]
    nn = w["n"] if n is None else n
    if w["kind"] == "uniform":
        return uniform(nn, w["d"], w["seed"])
    if w["kind"] == "normal":
        return normal(nn, w["d"], w["seed"])
    if w["kind"] == "rsa":
        return rsa(nn, w["seed"])
    raise KeyError(w["kind"])
