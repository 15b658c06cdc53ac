"""Block-space maps, written out plainly -- TEST INFRASTRUCTURE ONLY.

Every map sends the linear index of a block of the parallel space Pi to a tile
coordinate of the data space, or to "filtered" (-1).  Tiles are blocks of
rho^m simplex elements; nb = ceil(n / rho) tiles per dimension.  Target tile
sets:

  T2 = {(x, y): 0 <= x <= y < nb}
  T3 = {(x, y, z): 0 <= x <= y <= z < nb}
  T4 = {(x1, x2, x3, x4): 0 <= x1 <= x2 <= x3 <= x4 < nb}

Block linearisation (the layout of a tile dump): x varies fastest, then y,
then z.  For the 3-simplex lambda map the linear index first runs over Pi3 and
then over the lambda2 grid that covers the plane y = z.

Integer arithmetic only (Python ints or int64 numpy), no floating point.
"""
from __future__ import annotations

import numpy as np

FILTERED = -1


def next_pow2(v: int) -> int:
    p = 1
    while p < v:
        p *= 2
    return p


def floor_log2(v: np.ndarray) -> np.ndarray:
    """floor(log2 v) for v >= 1, by counting the powers of two not above v."""
    v = np.asarray(v, dtype=np.int64)
    out = np.full(v.shape, -1, dtype=np.int64)
    p = 1
    while True:
        ge = v >= p
        if not ge.any():
            break
        out += ge
        p *= 2
    return out


# --------------------------------------------------------------------------
# lambda2 (paper Sec. III-A, the 2-simplex map).  The parallel space is the
# orthotope (nb/2) x (nb+1).  Rows 1..nb-1 follow the paper's map: with
# b = 2^floor(log2 w_y) (the recursion level of the row) and q = floor(w_x / b)
# (which sub-orthotope of that level), lambda(w) = (w_x + q b, w_y + 2 q b),
# which always lands strictly above the diagonal.  The paper leaves the
# diagonal to the extra n blocks of S_{n+1} (V(S_n) + n = V(Delta_n)); here
# row 0 carries tiles (w_x, w_x) and row nb carries (nb/2 + w_x, nb/2 + w_x).
# A grid of nb = 1 is one block mapped to (0, 0).
# Non-power-of-two nb: "approach from above" -- build the grid for
# nb' = 2^ceil(log2 nb) and filter tiles with a coordinate >= nb.
def pi2_extent(nb: int) -> tuple[int, int]:
    nbp = next_pow2(nb)
    if nbp == 1:
        return (1, 1)
    return (nbp // 2, nbp + 1)


def lambda2_tiles(nb: int) -> np.ndarray:
    nbp = next_pow2(nb)
    ex, ey = pi2_extent(nb)
    wy, wx = np.divmod(np.arange(ex * ey, dtype=np.int64), ex)
    if nbp == 1:
        t = np.zeros((1, 2), dtype=np.int64)
    else:
        t = np.empty((ex * ey, 2), dtype=np.int64)
        top = wy == 0
        bot = wy == nbp
        mid = ~(top | bot)
        t[top, 0] = wx[top]
        t[top, 1] = wx[top]
        t[bot, 0] = nbp // 2 + wx[bot]
        t[bot, 1] = nbp // 2 + wx[bot]
        b = 2 ** floor_log2(np.maximum(wy[mid], 1))
        q = wx[mid] // b
        t[mid, 0] = wx[mid] + q * b
        t[mid, 1] = wy[mid] + 2 * q * b
    bad = (t >= nb).any(axis=1)
    t[bad] = FILTERED
    return t


# --------------------------------------------------------------------------
# lambda3 (paper Sec. III-C, the alternative 3-simplex map with two recursion
# branches).  The paper's closed form for the "diagonal or outside" case is
# not recoverable from the text (its figures are lost and the printed offsets
# do not round-trip), so this is the reading kept here; it has every property
# the section states:
#   * a main orthotope (nb/2) x (nb/2) x (nb/2 + nb/4) (the paper's
#     (n/2) x (n/2) x 3(n-1)/4, read with integer extents);
#   * its first nb/2 z-slices form the main (nb/2)^3 cube, moved as one piece;
#   * the remaining z-slices reuse the 2-simplex parameters (b, q) of
#     (w_x, w_y) with z shifted down by nb/2;
#   * a two-case rule (inside / diagonal-or-outside) folds each b^3 cube of
#     blocks across its diagonal plane onto the data space;
#   * O(1) integer work and 12.5% extra volume (|Pi3| -> 9/8 |T3 minus plane|).
# Target of Pi3: T3s = {x <= y < z}.  Each level b of the recursion owns the
# cubes {o <= x < o+b <= z < o+2b}, o = 2 q b, of T3s; such a cube splits into
# the prisms {x < o+b <= y < z} and {x <= y < o+b <= z} of b^2(b-1)/2 and
# b^2(b+1)/2 tiles, together b^3.  A block (u, v, w) of a b^3 block-cube goes
#   v <  w : (o + u,  o + b + v,  o + b + w)   (first prism)
#   v >= w : (o + w,  o + v,      o + b + u)   (second prism)
# The main cube is level b = nb/2 with o = 0 and (u, v, w) = (w_x, w_y, w_z).
# A slab block has w = w_z - nb/2; it is filtered if w_y = 0 or w >= b, else
# b = 2^floor(log2 w_y), q = floor(w_x / b), u = w_x - q b, v = w_y - b.
# The plane y = z (tiles (x, y, y), x <= y) comes from a lambda2 grid over nb.
def pi3_extent(nb: int) -> tuple[int, int, int]:
    nbp = next_pow2(nb)
    return (nbp // 2, nbp // 2, nbp // 2 + nbp // 4)


def _fold(o, b, u, v, w):
    first = v < w
    x = np.where(first, o + u, o + w)
    y = np.where(first, o + b + v, o + v)
    z = np.where(first, o + b + w, o + b + u)
    return x, y, z


def lambda3_main_tiles(nb: int) -> np.ndarray:
    nbp = next_pow2(nb)
    ex, ey, ez = pi3_extent(nb)
    tot = ex * ey * ez
    idx = np.arange(tot, dtype=np.int64)
    t = np.full((tot, 3), FILTERED, dtype=np.int64)
    if tot == 0:
        return t
    wx = idx % ex
    wy = (idx // ex) % ey
    wz = idx // (ex * ey)
    half = nbp // 2
    cube = wz < half
    # main cube: level b = nb/2, o = 0
    x, y, z = _fold(0, half, wx[cube], wy[cube], wz[cube])
    t[cube, 0], t[cube, 1], t[cube, 2] = x, y, z
    # slab
    s = ~cube
    w = wz[s] - half
    wys = wy[s]
    wxs = wx[s]
    valid = wys >= 1
    b = np.where(valid, 2 ** floor_log2(np.maximum(wys, 1)), 1)
    valid &= w < b
    q = wxs // b
    u = wxs - q * b
    v = wys - b
    o = 2 * q * b
    x, y, z = _fold(o, b, u, v, w)
    ts = np.stack([x, y, z], axis=1)
    ts[~valid] = FILTERED
    t[s] = ts
    bad = (t >= nb).any(axis=1)
    t[bad] = FILTERED
    return t


def lambda3_tiles(nb: int) -> np.ndarray:
    main = lambda3_main_tiles(nb)
    plane2 = lambda2_tiles(nb)
    plane = np.full((plane2.shape[0], 3), FILTERED, dtype=np.int64)
    ok = plane2[:, 0] >= 0
    plane[ok, 0] = plane2[ok, 0]
    plane[ok, 1] = plane2[ok, 1]
    plane[ok, 2] = plane2[ok, 1]
    return np.concatenate([main, plane], axis=0)


# --------------------------------------------------------------------------
# Bounding box (paper Sec. I): the identity over nb^m blocks, keeping only the
# blocks inside the simplex.
def bbox2_tiles(nb: int) -> np.ndarray:
    y, x = np.divmod(np.arange(nb * nb, dtype=np.int64), nb)
    t = np.stack([x, y], axis=1)
    t[x > y] = FILTERED
    return t


def bbox3_tiles(nb: int) -> np.ndarray:
    idx = np.arange(nb ** 3, dtype=np.int64)
    x = idx % nb
    y = (idx // nb) % nb
    z = idx // (nb * nb)
    t = np.stack([x, y, z], axis=1)
    t[(x > y) | (y > z)] = FILTERED
    return t


# --------------------------------------------------------------------------
# Linear enumeration g: Z^1 -> Z^m (paper Sec. I): block k is the k-th tile
# when T2 is listed by y then x, and T3 by z, then y, then x.  Tri(y) =
# y(y+1)/2 tiles have a smaller y; Tet(z) = z(z+1)(z+2)/6 have a smaller z.
# The root of the quadratic / cubic is found here by exact search over the
# integer tables, not by floating point.
def linear2_tiles(nb: int) -> np.ndarray:
    k = np.arange(nb * (nb + 1) // 2, dtype=np.int64)
    yy = np.arange(nb + 1, dtype=np.int64)
    tri = yy * (yy + 1) // 2
    y = np.searchsorted(tri, k, side="right") - 1
    x = k - tri[y]
    return np.stack([x, y], axis=1)


def linear3_tiles(nb: int) -> np.ndarray:
    k = np.arange(nb * (nb + 1) * (nb + 2) // 6, dtype=np.int64)
    zz = np.arange(nb + 1, dtype=np.int64)
    tet = zz * (zz + 1) * (zz + 2) // 6
    z = np.searchsorted(tet, k, side="right") - 1
    r = k - tet[z]
    tri = zz * (zz + 1) // 2
    y = np.searchsorted(tri, r, side="right") - 1
    x = r - tri[y]
    return np.stack([x, y, z], axis=1)


# --------------------------------------------------------------------------
# "Approach n from below" (Sec. III-A, second option): cover nb with
# power-of-two orthotopes n_1 = 2^floor(log2 nb), n_i = 2^floor(log2(nb -
# sum_{k<i} n_k)) (the binary digits of nb, largest first) plus simpler maps for
# what they leave.  Segment i = [o_i, o_i + m_i).  Reading written out here:
#   2-simplex, per segment in order: the lambda2 grid of m_i on the segment's
#     diagonal triangle, then (if tiles remain above it) the rectangle
#     [o_i, o_i + m_i) x [o_i + m_i, nb) under the identity, x fastest;
#   3-simplex, per segment in order: the lambda3 grid of m_i (its tetrahedron),
#     then the prism {x <= y in segment i, z above it} = lambda2(m_i) x identity
#     (lambda2 index fastest), then the prism {x in segment i, y <= z above it}
#     = identity x (2-simplex map from below of the rest), x fastest.
# Every block of the 2-simplex cover maps to a tile (zero filtered blocks).
def segments(nb: int) -> list[tuple[int, int]]:
    out, o, rem = [], 0, nb
    while rem > 0:
        m = 1 << (rem.bit_length() - 1)
        out.append((o, m))
        o += m
        rem -= m
    return out


def below2_tiles(nb: int) -> np.ndarray:
    parts = []
    for o, m in segments(nb):
        tri = lambda2_tiles(m) + o
        parts.append(tri)
        r = nb - o - m
        if r > 0:
            y, x = np.divmod(np.arange(m * r, dtype=np.int64), m)
            parts.append(np.stack([o + x, o + m + y], axis=1))
    return np.concatenate(parts, axis=0) if parts else np.zeros((0, 2), np.int64)


def below3_tiles(nb: int) -> np.ndarray:
    parts = []
    for o, m in segments(nb):
        tet = lambda3_tiles(m)
        ok = tet[:, 0] >= 0
        tet[ok] += o
        parts.append(tet)
        r = nb - o - m
        if r > 0:
            t2 = lambda2_tiles(m)  # m a power of two: no filtered rows
            z = np.repeat(np.arange(r, dtype=np.int64), t2.shape[0])
            pa = np.concatenate([np.tile(t2 + o, (r, 1)), (o + m + z)[:, None]], axis=1)
            parts.append(pa)
            b2 = below2_tiles(r) + (o + m)
            x = np.tile(np.arange(m, dtype=np.int64), b2.shape[0])
            pb = np.concatenate([(o + x)[:, None], np.repeat(b2, m, axis=0)], axis=1)
            parts.append(pb)
    return np.concatenate(parts, axis=0) if parts else np.zeros((0, 3), np.int64)


# --------------------------------------------------------------------------
# The recursive orthotope set of Sec. III-B, in the paper's own corner
# coordinates: the simplex {p >= 0 : p_1 + ... + p_m <= nb' - 1} (eq. (1) with
# the orthogonal corner at 0).  The map of a simplex of side s whose relative
# origin is c is the cube phi(w, c) of side s/2 placed at c, followed by m maps of
# side s/2 at c + (s/2) e_d, d = 1..m (for m = 3 "the top and the sides of the
# cube"), repeated until the smallest block.  Reading kept here: the recursion
# ends at a simplex of side 1, which is one block (so the set covers the
# non-strict simplex, diagonal included).  Blocks are listed in the order of
# that recursion (depth first: the cube x fastest, then the m sub-maps in axis
# order).  A corner point p becomes the tile (p_1, p_1 + p_2[, p_1 + p_2 + p_3])
# of T2 / T3; blocks whose last tile coordinate reaches nb are filtered (points
# of a cube outside the simplex, and everything past nb when nb' > nb).
def recursive_tiles(m: int, nb: int) -> np.ndarray:
    nbp = next_pow2(nb)
    parts = []

    def rec(c, s):
        if s == 1:
            parts.append(np.array([c], dtype=np.int64))
            return
        h = s // 2
        idx = np.arange(h ** m, dtype=np.int64)
        cube = np.stack([idx // h ** d % h for d in range(m)], axis=1) + np.array(c, dtype=np.int64)
        parts.append(cube)
        for d in range(m):
            c2 = list(c)
            c2[d] += h
            rec(tuple(c2), h)

    rec((0,) * m, nbp)
    p = np.concatenate(parts, axis=0)
    t = np.cumsum(p, axis=1)
    t[t[:, -1] >= nb] = FILTERED
    return t


# --------------------------------------------------------------------------
# 4-simplex (Sec. III-D: the recursive set of orthotopes for general m with
# r = 1/2, beta = 2, V = (n^4 - n) / 14).  The paper gives the set and its
# volume, not a map; the map written out here is this implementation's
# reading.  Target T4 = {x1 <= x2 <= x3 <= x4 < nb}, split as
#   T4s = {x1 <= x2 <= x3 < x4}  (C(nb+2, 4) tiles, the paper's V(Delta_{n-1}))
#   plane {x3 = x4}              (a copy of T3, covered by a lambda3 grid over nb,
#                                 tile (X, Y, Z) -> (X, Y, Z, Z)).
# T4s splits over the binary recursion on [0, nb'): a tuple belongs to the node
# (offset o, size 2b) where x1 and x4 first fall on different halves,
# L = [o, o+b) and H = [o+b, o+2b).  The node's cross region is
#   R3 = {x1 <= x2 <= x3 in L, x4 in H},
#   R2 = {x1 <= x2 in L, x3 < x4 in H},
#   R1 = {x1 in L, x2 <= x3 < x4 in H},
# b^2 (b+1) (7b-1) / 12 tiles in all, never more than b^4.  Each node owns one
# b^4 orthotope of blocks (level l = 0, 1, ... has 2^l nodes of side
# b = nb'/2^(l+1), so the orthotopes add up to (nb'^4 - nb') / 14): its first
# blocks list R3, then R2, then R1, and the rest are filtered.  Listing order
# inside a region: R3 by the sorted triple (by x3, then x2, then x1), x4
# fastest; R2 by the pair in L (by x2, then x1), then the pair in H (by x4,
# then x3) fastest; R1 by the triple in H (by x4, then x3, then x2), x1
# fastest.  Blocks: levels in order, nodes by offset, then the plane grid.
def _sorted_tuples(b: int, r: int, strict_last: bool) -> list:
    """Non-decreasing r-tuples over [0, b) (the last step strict when asked),
    ordered by the last coordinate, then the one before, ... (colex)."""
    out = []

    def rec(prefix_rev, k, hi):
        # prefix_rev holds the chosen coordinates from the last one down
        if k == 0:
            out.append(tuple(reversed(prefix_rev)))
            return
        for v in range(hi):
            rec(prefix_rev + [v], k - 1, v + 1)

    if strict_last:
        for last in range(b):
            sub = []

            def rec2(prefix_rev, k, hi):
                if k == 0:
                    sub.append(tuple(reversed(prefix_rev)) + (last,))
                    return
                for v in range(hi):
                    rec2(prefix_rev + [v], k - 1, v + 1)
            rec2([], r - 1, last)
            # colex order on the leading coordinates within one last value
            sub.sort(key=lambda t: tuple(reversed(t[:-1])))
            out.extend(sub)
        return out
    rec([], r, b)
    out.sort(key=lambda t: tuple(reversed(t)))
    return out


def lambda4_main_tiles(nb: int) -> np.ndarray:
    nbp = next_pow2(nb)
    rows = []
    b = nbp // 2
    nodes = 1
    while b >= 1:
        r3 = _sorted_tuples(b, 3, False)
        l2 = _sorted_tuples(b, 2, False)
        h2 = _sorted_tuples(b, 2, True)
        h3 = _sorted_tuples(b, 3, True)
        for q in range(nodes):
            o = 2 * q * b
            cross = []
            for (a, c, d) in r3:
                for e in range(b):
                    cross.append((o + a, o + c, o + d, o + b + e))
            for (a, c) in l2:
                for (d, e) in h2:
                    cross.append((o + a, o + c, o + b + d, o + b + e))
            for (c, d, e) in h3:
                for a in range(b):
                    cross.append((o + a, o + b + c, o + b + d, o + b + e))
            assert len(cross) <= b ** 4
            cross += [(FILTERED,) * 4] * (b ** 4 - len(cross))
            rows += cross
        b //= 2
        nodes *= 2
    t = np.array(rows, dtype=np.int64).reshape(-1, 4)
    t[t[:, 3] >= nb] = FILTERED
    return t


def lambda4_tiles(nb: int) -> np.ndarray:
    main = lambda4_main_tiles(nb)
    p3 = lambda3_tiles(nb)
    plane = np.full((p3.shape[0], 4), FILTERED, dtype=np.int64)
    ok = p3[:, 0] >= 0
    plane[ok, :3] = p3[ok]
    plane[ok, 3] = p3[ok, 2]
    return np.concatenate([main, plane], axis=0)


def bbox4_tiles(nb: int) -> np.ndarray:
    idx = np.arange(nb ** 4, dtype=np.int64)
    t = np.stack([idx // nb ** d % nb for d in range(4)], axis=1)
    bad = (t[:, 0] > t[:, 1]) | (t[:, 1] > t[:, 2]) | (t[:, 2] > t[:, 3])
    t[bad] = FILTERED
    return t


def linear4_tiles(nb: int) -> np.ndarray:
    """Block k = the k-th tile of T4 listed by x4, then x3, x2, x1 (exact search
    over integer tables of the simplicial numbers)."""
    w = np.arange(nb + 1, dtype=np.int64)
    pen = w * (w + 1) * (w + 2) * (w + 3) // 24   # tiles with a smaller x4
    tet = w * (w + 1) * (w + 2) // 6
    tri = w * (w + 1) // 2
    k = np.arange(pen[nb], dtype=np.int64)
    x4 = np.searchsorted(pen, k, side="right") - 1
    r = k - pen[x4]
    x3 = np.searchsorted(tet, r, side="right") - 1
    r = r - tet[x3]
    x2 = np.searchsorted(tri, r, side="right") - 1
    x1 = r - tri[x2]
    return np.stack([x1, x2, x3, x4], axis=1)


def lambda4_blocks(nb: int) -> int:
    """|Pi4| = (nb'^4 - nb') / 14 orthotope blocks + the lambda3 plane grid."""
    nbp = next_pow2(nb)
    return (nbp ** 4 - nbp) // 14 + lambda3_tiles(nb).shape[0]


def recursive_sub_maps(m: int, nb: int) -> int:
    """Number of sub-orthotopes (map calls, one launch each) of the recursive
    set of side next_pow2(nb): the cube of every recursion node plus the
    single-block leaves, counted by walking the recursion."""
    def cnt(s):
        return 1 if s == 1 else 1 + m * cnt(s // 2)
    return cnt(next_pow2(nb))


MAPS = {"lambda": 0, "bbox": 1, "linear": 2, "lambda_below": 3, "recursive": 4, "recursive_launch": 5}


def tiles(m: int, nb: int, kind: str) -> np.ndarray:
    """Tile dump of map ``kind`` (a key of MAPS) for T2 (m=2) or T3 (m=3)."""
    if kind in ("recursive", "recursive_launch"):  # one set; the launches differ
        return recursive_tiles(m, nb)
    if m == 2:
        return {"lambda": lambda2_tiles, "bbox": bbox2_tiles, "linear": linear2_tiles,
                "lambda_below": below2_tiles}[kind](nb)
    if m == 3:
        return {"lambda": lambda3_tiles, "bbox": bbox3_tiles, "linear": linear3_tiles,
                "lambda_below": below3_tiles}[kind](nb)
    if m == 4:
        return {"lambda": lambda4_tiles, "bbox": bbox4_tiles, "linear": linear4_tiles}[kind](nb)
    raise ValueError(m)


def target_tiles(m: int, nb: int) -> set:
    """The target tile set, by nested loops."""
    if m == 2:
        return {(x, y) for y in range(nb) for x in range(y + 1)}
    if m == 4:
        return {(x, y, z, w) for w in range(nb) for z in range(w + 1) for y in range(z + 1) for x in range(y + 1)}
    return {(x, y, z) for z in range(nb) for y in range(z + 1) for x in range(y + 1)}


def check_bijection(t: np.ndarray, m: int, nb: int) -> tuple[bool, str]:
    """True iff the non-filtered rows of a dump are distinct and cover the target."""
    valid = t[:, 0] >= 0
    if (t[~valid] != FILTERED).any():
        return False, "partially filtered row"
    vt = t[valid]
    if (vt < 0).any() or (vt >= nb).any():
        return False, "tile out of range"
    got = set(map(tuple, vt.tolist()))
    if len(got) != vt.shape[0]:
        return False, f"{vt.shape[0] - len(got)} duplicate tiles"
    tgt = target_tiles(m, nb)
    if got != tgt:
        return False, f"missing {len(tgt - got)}, extra {len(got - tgt)}"
    return True, "ok"
