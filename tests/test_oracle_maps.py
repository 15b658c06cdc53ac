"""Pins for the oracle's block-space maps and the paper's volume formulas.

Each check ties the oracle to something other than its own code: the
hand-derived tables in tests/golden, brute-force set equality with the target
simplices, the recursive orthotope sets of Sec. III (built here by recursion,
without any log2 / clz), and the closed-form volumes of Sec. I and III.
"""
import math
import os
from fractions import Fraction
from math import comb, factorial

import numpy as np
import pytest

from oracle import maps

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    return np.array(rows, dtype=np.int64)


def test_floor_log2_matches_bit_length():
    v = np.arange(1, 5000)
    assert (maps.floor_log2(v) == np.array([int(x).bit_length() - 1 for x in v])).all()


def test_lambda2_golden_nb8():
    g = _read_golden("lambda2_nb8.txt")
    t = maps.lambda2_tiles(8)
    ex, ey = maps.pi2_extent(8)
    assert (ex, ey) == (4, 9)
    for wx, wy, X, Y in g:
        assert tuple(t[wy * ex + wx]) == (X, Y)
    assert len(g) == t.shape[0]


def test_lambda3_golden_nb4():
    g = _read_golden("lambda3_nb4.txt")
    t = maps.lambda3_main_tiles(4)
    ex, ey, ez = maps.pi3_extent(4)
    assert (ex, ey, ez) == (2, 2, 3)
    for wx, wy, wz, X, Y, Z in g:
        assert tuple(t[(wz * ey + wy) * ex + wx]) == (X, Y, Z)
    assert len(g) == t.shape[0]


@pytest.mark.parametrize("kind", ["lambda", "bbox", "linear", "lambda_below"])
@pytest.mark.parametrize("nb", [1, 2, 3, 4, 5, 7, 8, 12, 16, 33, 64, 100, 256])
def test_map2_bijection(kind, nb):
    ok, msg = maps.check_bijection(maps.tiles(2, nb, kind), 2, nb)
    assert ok, msg


@pytest.mark.parametrize("kind", ["lambda", "bbox", "linear", "lambda_below"])
@pytest.mark.parametrize("nb", [1, 2, 3, 4, 5, 6, 8, 12, 16, 32])
def test_map3_bijection(kind, nb):
    ok, msg = maps.check_bijection(maps.tiles(3, nb, kind), 3, nb)
    assert ok, msg


@pytest.mark.slow
@pytest.mark.parametrize("nb", [512, 1024])
def test_lambda2_bijection_large(nb):
    ok, msg = maps.check_bijection(maps.lambda2_tiles(nb), 2, nb)
    assert ok, msg


@pytest.mark.parametrize("nb", [64, 128])
def test_lambda3_bijection_large(nb):
    ok, msg = maps.check_bijection(maps.lambda3_tiles(nb), 3, nb)
    assert ok, msg


def _recursive_s2(n, off=0):
    """Tiles of the recursive set S2_n (Sec. III-A): one (n/2)^2 square over the
    diagonal plus two copies of S2_{n/2}; returns {level size: set of tiles}."""
    out = {}
    if n < 2:
        return out
    h = n // 2
    out.setdefault(h, set()).update((off + x, off + h + y) for x in range(h) for y in range(h))
    for sub in (_recursive_s2(h, off), _recursive_s2(h, off + h)):
        for b, s in sub.items():
            out.setdefault(b, set()).update(s)
    return out


@pytest.mark.parametrize("nb", [2, 4, 8, 32, 128])
def test_lambda2_rows_follow_recursive_set(nb):
    """Rows [b, 2b) of Pi2 map exactly onto the level-b squares of S2, and
    Pi2 has zero filtered blocks and exactly V(Delta2) blocks."""
    t = maps.lambda2_tiles(nb)
    ex, ey = maps.pi2_extent(nb)
    assert ex * ey == nb * (nb + 1) // 2
    assert (t[:, 0] >= 0).all()
    levels = _recursive_s2(nb)
    assert sum(len(s) for s in levels.values()) == nb * (nb - 1) // 2  # V(S2_n) = n(n-1)/2
    for b, sq in levels.items():
        rows = t[b * ex:(2 * b) * ex]
        assert set(map(tuple, rows.tolist())) == sq
        # within a square the map is a translation of the block grid
        wy, wx = np.divmod(np.arange(b * ex, 2 * b * ex), ex)
        o = rows[:, 0] - (wx % b)
        assert ((rows[:, 1] - wy) == o).all()


def _recursive_s3(n, off=0):
    """Cross cubes of the two-branch recursive set S3_n (Sec. III-C): the
    tiles {off <= x < off+h <= z < off+2h, x <= y < z} (h = n/2) plus two
    copies of S3_{n/2}.  Returns {level h: set of tiles}."""
    out = {}
    if n < 2:
        return out
    h = n // 2
    cube = {(x, y, z) for x in range(off, off + h) for z in range(off + h, off + n)
            for y in range(x, z)}
    out.setdefault(h, set()).update(cube)
    for sub in (_recursive_s3(h, off), _recursive_s3(h, off + h)):
        for b, s in sub.items():
            out.setdefault(b, set()).update(s)
    return out


@pytest.mark.parametrize("nb", [2, 4, 8, 16, 32])
def test_lambda3_levels_follow_two_branch_set(nb):
    """The main cube covers the level-nb/2 cross cube; slab rows w_y in [b, 2b)
    cover the level-b cubes; each cross cube holds b^3 tiles; the level sizes
    follow V(S3_n) = (n/2)^3 + 2 V(S3_{n/2}) = (n^3 - n)/6."""
    t = maps.lambda3_main_tiles(nb)
    ex, ey, ez = maps.pi3_extent(nb)
    levels = _recursive_s3(nb)
    total = 0
    for b, cubes in levels.items():
        assert len(cubes) == (nb // (2 * b)) * b ** 3
        total += len(cubes)
    assert total == (nb ** 3 - nb) // 6
    idx = np.arange(t.shape[0])
    wx, wy, wz = idx % ex, (idx // ex) % ey, idx // (ex * ey)
    half = nb // 2
    main = set(map(tuple, t[wz < half].tolist()))
    assert main == levels[half]
    for b in [bb for bb in levels if bb < half]:
        sel = (wz >= half) & (wy >= b) & (wy < 2 * b) & (t[:, 0] >= 0)
        assert set(map(tuple, t[sel].tolist())) == levels[b]


@pytest.mark.parametrize("nb", [4, 8, 16, 64, 128, 256])
def test_lambda3_extra_volume(nb):
    """|Pi3| = 3 nb^3 / 16 and |Pi3| / |T3 minus plane| -> 9/8 (12.5% extra, Sec. III-C)."""
    ex, ey, ez = maps.pi3_extent(nb)
    v = ex * ey * ez
    assert v == 3 * nb ** 3 // 16
    s = (nb ** 3 - nb) // 6
    if nb <= 128:
        t = maps.lambda3_main_tiles(nb)
        assert int((t[:, 0] >= 0).sum()) == s
    ratio = v / s
    if nb >= 128:
        assert abs(ratio - 9 / 8) < 2e-4
    assert ratio >= 9 / 8


# --------------------------------------------------------------------------
# Volume formulas of Sec. I and III, against brute-force counting.
@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 30])
def test_simplex_volume_eq2(n):
    cnt2 = sum(1 for x in range(n) for y in range(n) if x + y <= n - 1)
    cnt3 = sum(1 for x in range(n) for y in range(n) for z in range(n) if x + y + z <= n - 1)
    assert cnt2 == comb(n + 1, 2) == n * (n + 1) // 2
    assert cnt3 == comb(n + 2, 3) == n * (n + 1) * (n + 2) // 6
    # pairs / triplets form used by the build: the same counts
    assert cnt2 == sum(1 for i in range(n) for j in range(i, n))
    assert cnt3 == sum(1 for i in range(n) for j in range(i, n) for k in range(j, n))
    # stacking identity, eq. (3)
    assert comb(n + 2, 3) == sum(comb(i + 1, 2) for i in range(1, n + 1))


def test_bbox_waste_limit():
    """V(Pi)/V(Delta) - 1 -> m! - 1 for the bounding box (Sec. I)."""
    for m in (2, 3, 4):
        n = 4096
        r = Fraction(n ** m, comb(n + m - 1, m)) - 1
        assert abs(float(r) - (factorial(m) - 1)) < m * m * factorial(m) / n


def _vol_rec(n, m, beta):
    if n < 2:
        return 0
    return (n // 2) ** m + beta * _vol_rec(n // 2, m, beta)


@pytest.mark.parametrize("k", range(1, 12))
def test_recursive_set_volumes(k):
    n = 2 ** k
    assert _vol_rec(n, 2, 2) == n * (n - 1) // 2                      # Sec. III-A
    assert _vol_rec(n, 3, 2) == (n ** 3 - n) // 6                     # Sec. III-C
    assert 5 * _vol_rec(n, 3, 3) == n ** 3 - 3 ** k                   # Sec. III-B (with the /5)
    for m in (2, 3, 4, 5, 6, 7):                                      # Sec. III-D, r = 1/2, beta = 2
        assert _vol_rec(n, m, 2) * (2 ** m - 2) == n ** m - n


def test_recursive_set_limits():
    n = 2 ** 40
    # three-branch set: 20% extra over the tetrahedron
    assert abs(Fraction(n ** 3 - 3 ** 40, 5) / comb(n + 2, 3) - 1 - Fraction(1, 5)) < 1e-9
    for m, lim in ((4, Fraction(5, 7)), (5, 3), (7, 39)):
        v = Fraction(n ** m - n, 2 ** m - 2)
        a = v / comb(n - 1 + m - 1, m) - 1
        assert abs(float(a - lim)) < 1e-6
        assert Fraction(factorial(m), 2 ** m - 2) - 1 == lim


# --------------------------------------------------------------------------
# "Approach n from below" (Sec. III-A): n_1 = 2^floor(log2 n), then
# n_i = 2^floor(log2(n - sum_{k<i} n_k)).
@pytest.mark.parametrize("nb", [1, 2, 3, 5, 6, 7, 12, 13, 33, 100, 255, 1000])
def test_below_segments_follow_paper_rule(nb):
    segs = maps.segments(nb)
    rest, off = nb, 0
    for o, m in segs:
        expect = 1
        while expect * 2 <= rest:
            expect *= 2
        assert (o, m) == (off, expect)
        off += m
        rest -= m
    assert rest == 0 and off == nb


@pytest.mark.parametrize("nb", [1, 3, 5, 12, 13, 33, 100, 255])
def test_below2_has_no_filtered_blocks(nb):
    t = maps.below2_tiles(nb)
    assert t.shape[0] == nb * (nb + 1) // 2 and (t >= 0).all()


@pytest.mark.parametrize("nb", [3, 5, 12, 13, 33])
def test_below3_block_count(nb):
    """Blocks: per segment, lambda3 of m (3 m^3/16 + m(m+1)/2 blocks) plus the
    two prisms m(m+1)/2 * r and m * r(r+1)/2, r = tiles above the segment."""
    total = 0
    for o, m in maps.segments(nb):
        r = nb - o - m
        l3 = (m // 2) * (m // 2) * (m // 2 + m // 4) + (1 if m == 1 else (m // 2) * (m + 1))
        total += l3 + m * (m + 1) // 2 * r + m * r * (r + 1) // 2
    assert maps.below3_tiles(nb).shape[0] == total
    # far fewer blocks than "from above" just past a power of two
    if nb == 33:
        assert total < maps.lambda3_tiles(33).shape[0] / 5


# --------------------------------------------------------------------------
# Recursive orthotope sets of Sec. III-B (the O(log n) map and its one launch
# per sub-orthotope), in the paper's corner coordinates.
def test_recursive_golden_nb4():
    lines = [ln.split() for ln in open(os.path.join(GOLDEN, "recursive_nb4.txt"))
             if ln.strip() and not ln.startswith("#")]
    for m in (2, 3):
        rows = np.array([[int(v) for v in ln] for ln in lines if int(ln[0]) == m], dtype=np.int64)
        t = maps.recursive_tiles(m, 4)
        assert t.shape[0] == rows.shape[0] == (10 if m == 2 else 20)
        np.testing.assert_array_equal(rows[:, 1], np.arange(rows.shape[0]))
        np.testing.assert_array_equal(t, rows[:, 2 + m:])
        # the golden corner points themselves lie in the corner simplex
        assert (rows[:, 2:2 + m].sum(axis=1) <= 3).all()


@pytest.mark.parametrize("m", [2, 3])
@pytest.mark.parametrize("nb", [1, 2, 3, 4, 5, 7, 8, 9, 16, 17, 33, 64])
def test_recursive_bijection(m, nb):
    ok, msg = maps.check_bijection(maps.recursive_tiles(m, nb), m, nb)
    assert ok, msg


@pytest.mark.parametrize("k", range(0, 9))
def test_recursive_block_counts(k):
    """Blocks of the set of side n = 2^k: the paper's recursion V = (n/2)^m +
    m V(n/2) (built here by _vol_rec, which ends at V(1) = 0) plus the m^k
    single-block leaves kept by this reading; closed forms n(n+1)/2 (m = 2,
    the triangle exactly) and (n^3 + 4 * 3^k) / 5 (m = 3, eq. of Sec. III-B with
    the leaves)."""
    n = 2 ** k
    for m in (2, 3):
        got = maps.recursive_tiles(m, n).shape[0]
        assert got == _vol_rec(n, m, m) + m ** k
    assert maps.recursive_tiles(2, n).shape[0] == n * (n + 1) // 2
    assert 5 * maps.recursive_tiles(3, n).shape[0] == n ** 3 + 4 * 3 ** k
    # every 2-D block maps; 3-D blocks outside the tetrahedron are the extra volume
    assert (maps.recursive_tiles(2, n) >= 0).all()
    assert (maps.recursive_tiles(3, n)[:, 0] >= 0).sum() == comb(n + 2, 3)


@pytest.mark.parametrize("k", range(0, 10))
def test_recursive_sub_map_counts(k):
    """One map call per recursion node: (m^(k+1) - 1) / (m - 1) sub-orthotopes,
    at least (n - 1) / 2 (Sec. III-B: linear in n or worse)."""
    n = 2 ** k
    for m in (2, 3):
        c = maps.recursive_sub_maps(m, n)
        assert c == (m ** (k + 1) - 1) // (m - 1)
        assert c >= (n - 1) / 2


def test_recursive_extra_volume_tends_to_one_fifth():
    """The 3-branch set exceeds the tetrahedron by 1/5 in the limit (Sec. III-B)."""
    prev = 0.0
    for k in range(2, 9):
        n = 2 ** k
        t = maps.recursive_tiles(3, n)
        extra = t.shape[0] / comb(n + 2, 3) - 1
        assert prev <= extra < 0.2
        prev = extra
    assert prev > 0.17
    n = 2 ** 40
    assert abs(Fraction(n ** 3 + 4 * 3 ** 40, 5) / comb(n + 2, 3) - 1 - Fraction(1, 5)) < 1e-9


@pytest.mark.parametrize("m", [2, 3])
def test_recursive_first_blocks_are_the_main_cube(m):
    """The first (n/2)^m blocks are phi(w, 0): corner points with every
    coordinate below n/2, x fastest; the next blocks start the sub-map at
    (n/2) e_1."""
    n = 16
    t = maps.recursive_tiles(m, n)
    h = n // 2
    head = t[:h ** m]
    w = np.arange(h ** m)
    q = np.stack([w // h ** d % h for d in range(m)], axis=1)
    inside = q.sum(axis=1) < n
    assert (head[~inside] == maps.FILTERED).all() and (m == 3 or inside.all())
    p = np.diff(np.concatenate([np.zeros((head.shape[0], 1), np.int64), head], axis=1), axis=1)
    np.testing.assert_array_equal(p[inside], q[inside])
    nxt = t[h ** m]
    assert tuple(nxt) == ((h, h) if m == 2 else (h, h, h))


# --------------------------------------------------------------------------
# 4-simplex: the r = 1/2, beta = 2 recursive set of Sec. III-D and the lambda4
# reading built on it.
def test_lambda4_golden_nb4():
    g = _read_golden("lambda4_nb4.txt")
    t = maps.lambda4_main_tiles(4)
    np.testing.assert_array_equal(g[:, 0], np.arange(18))
    np.testing.assert_array_equal(t, g[:, 1:])


@pytest.mark.parametrize("kind", ["lambda", "bbox", "linear", "recursive"])
@pytest.mark.parametrize("nb", [1, 2, 3, 4, 5, 7, 8, 9, 16, 17])
def test_map4_bijection(kind, nb):
    ok, msg = maps.check_bijection(maps.tiles(4, nb, kind), 4, nb)
    assert ok, msg


@pytest.mark.parametrize("k", range(0, 6))
def test_lambda4_orthotopes_follow_recursive_set(k):
    """The orthotope part has the paper's volume V(S^4_n) = (n^4 - n)/14 (the
    recursion (n/2)^4 + 2 V(n/2), built by _vol_rec) and covers T4s =
    {x1 <= x2 <= x3 < x4}, whose C(n+2, 4) = (n-1)n(n+1)(n+2)/24 tiles are the
    paper's V(Delta_{n-1}); each node's cross region has b^2 (b+1)(7b-1)/12 tiles."""
    n = 2 ** k
    main = maps.lambda4_main_tiles(n)
    assert main.shape[0] == _vol_rec(n, 4, 2) == (n ** 4 - n) // 14
    valid = main[main[:, 0] >= 0]
    assert valid.shape[0] == comb(n + 2, 4) == (n - 1) * n * (n + 1) * (n + 2) // 24
    assert (valid[:, 2] < valid[:, 3]).all()
    # per level: 2^l nodes, each b^4 blocks of which the cross region maps
    off, b, nodes = 0, n // 2, 1
    while b >= 1:
        cross = b * b * (b + 1) * (7 * b - 1) // 12
        assert cross <= b ** 4
        for q in range(nodes):
            blk = main[off:off + b ** 4]
            assert (blk[:cross, 0] >= 0).all() and (blk[cross:] == maps.FILTERED).all()
            o = 2 * q * b
            assert (blk[:cross, 0] >= o).all() and (blk[:cross, 0] < o + b).all()
            assert (blk[:cross, 3] >= o + b).all() and (blk[:cross, 3] < o + 2 * b).all()
            off += b ** 4
        b //= 2
        nodes *= 2


def test_lambda4_extra_volume():
    """Sec. III-D: with r = 1/2, beta = 2 the m = 4 set exceeds the simplex by a
    fraction tending to 4!/(2^4 - 2) - 1 = 5/7; the lambda4 blocks (orthotopes +
    plane grid) over the tiles of T4 approach the same limit from below."""
    prev = 0.0
    for k in range(1, 7):
        n = 2 ** k
        a = maps.lambda4_blocks(n) / comb(n + 3, 4) - 1
        assert prev <= a < Fraction(5, 7)
        prev = a
    assert prev > 0.6
    assert Fraction(factorial(4), 2 ** 4 - 2) - 1 == Fraction(5, 7)


def test_linear4_matches_nested_loops():
    nb = 12
    want = [(x, y, z, w) for w in range(nb) for z in range(w + 1) for y in range(z + 1) for x in range(y + 1)]
    np.testing.assert_array_equal(maps.linear4_tiles(nb), np.array(want, dtype=np.int64))


@pytest.mark.parametrize("k", range(0, 6))
def test_recursive4_counts(k):
    n = 2 ** k
    assert maps.recursive_tiles(4, n).shape[0] == _vol_rec(n, 4, 4) + 4 ** k
    assert maps.recursive_sub_maps(4, n) == (4 ** (k + 1) - 1) // 3


# --------------------------------------------------------------------------
# Closed-form inverses, derived from the recursive sets rather than from the
# forward maps: a tile of T2 with X < Y belongs to the level b = 2^L where
# L = msb(X xor Y) (the highest bit where the two indices first part) and to
# the square q = X >> (L+1) of that level.
def _msb(v):
    return np.array([int(x).bit_length() - 1 for x in v], dtype=np.int64)


@pytest.mark.parametrize("nb", [2, 4, 8, 64, 256])
def test_lambda2_closed_form_inverse(nb):
    t = maps.lambda2_tiles(nb)
    ex, _ = maps.pi2_extent(nb)
    wy, wx = np.divmod(np.arange(t.shape[0], dtype=np.int64), ex)
    X, Y = t[:, 0], t[:, 1]
    off = X < Y
    L = _msb(X[off] ^ Y[off])
    b = np.int64(1) << L
    q = X[off] >> (L + 1)
    np.testing.assert_array_equal(X[off] - q * b, wx[off])
    np.testing.assert_array_equal(Y[off] - 2 * q * b, wy[off])
    diag = X == Y
    low = X[diag] < nb // 2
    np.testing.assert_array_equal(np.where(low, 0, nb), wy[diag])
    np.testing.assert_array_equal(np.where(low, X[diag], X[diag] - nb // 2), wx[diag])


@pytest.mark.parametrize("nb", [4, 8, 32, 64])
def test_lambda3_closed_form_inverse(nb):
    """Tiles X <= Y < Z of the orthotope part: level L = msb(X xor Z), offset
    o = X with the low L+1 bits cleared; Y >= o + b is the first prism."""
    t = maps.lambda3_main_tiles(nb)
    ex, ey, _ = maps.pi3_extent(nb)
    idx = np.arange(t.shape[0], dtype=np.int64)
    wx, wy, wz = idx % ex, (idx // ex) % ey, idx // (ex * ey)
    ok = t[:, 0] >= 0
    X, Y, Z = t[ok, 0], t[ok, 1], t[ok, 2]
    L = _msb(X ^ Z)
    b = np.int64(1) << L
    o = (X >> (L + 1)) << (L + 1)
    first = Y >= o + b
    u = np.where(first, X - o, Z - o - b)
    v = np.where(first, Y - o - b, Y - o)
    w = np.where(first, Z - o - b, X - o)
    half = nb // 2
    main = b == half
    q = o // (2 * b)
    np.testing.assert_array_equal(np.where(main, u, u + q * b), wx[ok])
    np.testing.assert_array_equal(np.where(main, v, v + b), wy[ok])
    np.testing.assert_array_equal(np.where(main, w, w + half), wz[ok])


# --------------------------------------------------------------------------
# Sec. III-D, choosing (r, beta): V(S_n) = (n^m - beta^(log_{1/r} n)) /
# (1/r^m - beta) (the paper's generic closed form).  With 1/r^m - beta equal to
# m! exactly, V(S_n) < n^m / m! < C(n+m-2, m) = V(Delta_{n-1}) for every n >= 2
# and m >= 4 (the simplex has a positive n^(m-1) term), so the set never covers;
# approaching m! from below, 1/r^m - beta = m! - eps, it covers from some n0,
# and n0 grows as eps shrinks.
def _vol_generic(n, m, beta, inv_rm):
    depth = math.log(n) / math.log(inv_rm ** (1.0 / m))  # log_{1/r} n
    return (n ** m - beta ** depth) / (inv_rm - beta)


def _n0(m, beta, eps, limit=2 ** 24):
    inv_rm = math.factorial(m) + beta - eps
    n0 = None
    for k in range(1, 25):
        for n in (2 ** k, 3 * 2 ** (k - 1)):
            if n > limit:
                continue
            covers = _vol_generic(n, m, beta, inv_rm) >= comb(n + m - 2, m)
            if covers and n0 is None:
                n0 = n
            if not covers:
                n0 = None
    return n0


@pytest.mark.parametrize("m", [4, 5, 6, 7])
def test_generic_set_with_exact_factorial_never_covers(m):
    for beta in (2, 3, 4):
        inv_rm = math.factorial(m) + beta
        for n in [2, 3, 5, 10, 100, 1000, 10 ** 4, 10 ** 5]:
            assert _vol_generic(n, m, beta, inv_rm) < comb(n + m - 2, m)


def test_generic_set_from_below_covers_beyond_n0():
    for m in (4, 5):
        n_prev = 0
        for eps in (4.0, 1.0, 0.25):
            n0 = _n0(m, 2, eps)
            assert n0 is not None and n0 > n_prev  # a finite n0, growing as eps -> 0
            n_prev = n0
