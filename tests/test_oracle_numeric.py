"""Pins for the FP64 oracle's arithmetic (EDM, Axilrod-Teller, Lennard-Jones,
element checksums).

The checks come from outside the oracle's code: scipy's pdist, exact integer
arithmetic, closed forms for special triangles and pair distances,
homogeneity / symmetry invariants, an independent pure-Python formula
(the squared-distance form of the Axilrod-Teller term against the oracle's
angle form), finite differences and published SplitMix64 outputs.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.spatial.distance import pdist, squareform

import oracle
import synth


# ------------------------------------------------------------------ EDM
def test_edm_matches_scipy_pdist():
    X = synth.normal(57, 7, seed=11)
    D = oracle.edm_packed(X)
    full = squareform(pdist(X.astype(np.float64), "sqeuclidean"))
    iu = np.triu_indices(57)
    assert D.shape == (57 * 58 // 2,)
    np.testing.assert_allclose(D, full[iu], rtol=1e-13, atol=0)


def test_edm_layout_and_diagonal():
    n = 33
    X = synth.uniform(n, 3, seed=5)
    D = oracle.edm_packed(X)
    for i in range(n):
        p = oracle.packed_offset(i, n)
        assert D[p] == 0.0
        for j in (i + 1, n - 1):
            if j < n and j > i:
                ref = float(np.sum((X[i].astype(np.float64) - X[j].astype(np.float64)) ** 2))
                assert D[p + (j - i)] == ref
    assert (D >= 0).all()


def test_edm_integer_inputs_exact():
    X = synth.integer(40, 5, seed=3)
    D = oracle.edm_packed(X)
    Xi = X.astype(np.int64)
    k = 0
    for i in range(40):
        for j in range(i, 40):
            assert D[k] == float(((Xi[i] - Xi[j]) ** 2).sum())
            k += 1


def test_edm_rows_and_pairs_consistent():
    X = synth.normal(50, 4, seed=7)
    D = oracle.edm_packed(X)
    for i0, i1 in ((0, 1), (3, 9), (49, 50)):
        part = oracle.edm_rows(X, i0, i1)
        a = oracle.packed_offset(i0, 50)
        np.testing.assert_array_equal(part, D[a:a + part.size])
    I = np.array([0, 5, 7, 49])
    J = np.array([0, 9, 40, 49])
    got = oracle.edm_pairs(X, I, J)
    want = [D[oracle.packed_offset(i, 50) + j - i] for i, j in zip(I, J)]
    np.testing.assert_array_equal(got, want)


# ------------------------------------------------------------------ Axilrod-Teller
def _at_sform_py(p, q, r, nu=1.0):
    """Independent squared-distance form: cos g = t / (2 r r) by the law of
    cosines, so E = nu (P - 3/8 T) P^(-5/2)."""
    s1 = sum((a - b) ** 2 for a, b in zip(q, p))
    s2 = sum((a - b) ** 2 for a, b in zip(r, q))
    s3 = sum((a - b) ** 2 for a, b in zip(p, r))
    t1, t2, t3 = s3 - s1 - s2, s1 - s2 - s3, s2 - s3 - s1
    P, T = s1 * s2 * s3, t1 * t2 * t3
    return nu * (P - 0.375 * T) * P ** -2.5


def test_at_equilateral_closed_form():
    a = 1.5
    X = np.array([[0, 0, 0], [a, 0, 0], [a / 2, a * math.sqrt(3) / 2, 0]], np.float32)
    Xd = X.astype(np.float64)
    sides = [np.linalg.norm(Xd[i] - Xd[j]) for i, j in ((0, 1), (1, 2), (0, 2))]
    # cos 60 = 1/2 -> (1 + 3/8) / r^9 for an exact equilateral triangle; use the
    # FP32-rounded geometry's side lengths (they differ from a in the 8th digit)
    r = float(np.prod(sides)) ** (1 / 3)
    assert oracle.at_energy(X, nu=2.0) == pytest.approx(2.0 * 11 / (8 * r ** 9), rel=2e-6)


def test_at_collinear_and_right_angle():
    a = 1.25  # exactly representable
    X = np.array([[0, 0, 0], [a, 0, 0], [2 * a, 0, 0]], np.float32)
    assert oracle.at_energy(X) == pytest.approx(-1.0 / (4 * a ** 9), rel=1e-14)
    # right angle at particle 0: cos = 0 -> E = 1 / (a * a * a sqrt 2)^3
    Y = np.array([[0, 0, 0], [a, 0, 0], [0, a, 0]], np.float32)
    assert oracle.at_energy(Y) == pytest.approx(1.0 / (a * a * a * math.sqrt(2)) ** 3, rel=1e-14)


def test_at_matches_independent_sform_ordered_sum():
    X = synth.rsa(9, seed=21, side=4.0, dmin=0.5)
    P = X.astype(np.float64).tolist()
    tot = 0.0
    for i, j, k in itertools.permutations(range(9), 3):  # ordered distinct triples
        tot += _at_sform_py(P[i], P[j], P[k], nu=0.7)
    assert oracle.at_energy(X, nu=0.7) == pytest.approx(tot / 6.0, rel=1e-12)


def test_at_energy_row_ranges_add_up():
    X = synth.rsa(30, seed=2, side=5.0, dmin=0.5)
    e = oracle.at_energy(X)
    parts = sum(oracle.at_energy(X, i0=a, i1=b) for a, b in ((0, 7), (7, 8), (8, 30)))
    assert parts == pytest.approx(e, rel=1e-13)


def test_at_triplet_rows_element_by_element():
    """Packed per-triplet energies: lexicographic i < j < k order, each element
    equal to the independent s-form of that triplet."""
    X = synth.rsa(11, seed=23, side=4.0, dmin=0.5)
    P = X.astype(np.float64).tolist()
    want = [_at_sform_py(P[i], P[j], P[k], nu=0.8) for i, j, k in itertools.combinations(range(11), 3)]
    got = oracle.at_triplet_rows(X, nu=0.8)
    assert got.shape == (math.comb(11, 3),)
    np.testing.assert_allclose(got, want, rtol=1e-12)


def test_at_triplet_rows_slices_and_sum():
    X = synth.rsa(40, seed=4, side=6.0, dmin=0.5)
    full = oracle.at_triplet_rows(X)
    assert full.size == math.comb(40, 3) == oracle.triplet_rows_len(40, 0, 40)
    assert full.sum() == pytest.approx(oracle.at_energy(X), rel=1e-12)
    cuts = [0, 1, 2, 17, 37, 38, 40]
    parts = [oracle.at_triplet_rows(X, i0=a, i1=b) for a, b in zip(cuts, cuts[1:])]
    np.testing.assert_array_equal(np.concatenate(parts), full)


def test_at_triplet_rows_equilateral():
    a = 1.5
    X = np.array([[0, 0, 0], [a, 0, 0], [a / 2, a * math.sqrt(3) / 2, 0]], np.float32)
    Xd = X.astype(np.float64)
    r = float(np.prod([np.linalg.norm(Xd[i] - Xd[j]) for i, j in ((0, 1), (1, 2), (0, 2))])) ** (1 / 3)
    (e,) = oracle.at_triplet_rows(X)
    assert e == pytest.approx(11 / (8 * r ** 9), rel=2e-6)


def test_at_homogeneity_and_invariance():
    X = synth.rsa(12, seed=4, side=5.0, dmin=0.5)
    e = oracle.at_energy(X)
    assert oracle.at_energy(2.0 * X) == pytest.approx(e * 2.0 ** -9, rel=1e-12)
    perm = np.random.default_rng(0).permutation(12)
    assert oracle.at_energy(X[perm]) == pytest.approx(e, rel=1e-12)
    # translation by an exactly representable offset
    assert oracle.at_energy(X + np.float32(0.5)) == pytest.approx(e, rel=1e-5)
    # rotation by 90 degrees about z is exact in floating point
    R = X[:, [1, 0, 2]].copy()
    R[:, 0] *= -1
    assert oracle.at_energy(R) == pytest.approx(e, rel=1e-12)


def test_at_gradient_finite_differences():
    X = synth.rsa(8, seed=9, side=1.9, dmin=0.3)  # coordinates < 2: h = 2^-16 is exact
    G = oracle.at_grad(X)
    h = 2.0 ** -16
    for i in range(8):
        for c in range(3):
            Xp = X.copy()
            Xm = X.copy()
            Xp[i, c] += np.float32(h)
            Xm[i, c] -= np.float32(h)
            assert float(Xp[i, c]) - float(X[i, c]) == h
            fd = (oracle.at_energy(Xp) - oracle.at_energy(Xm)) / (2 * h)
            assert fd == pytest.approx(G[i, c], rel=2e-6, abs=2e-6 * np.abs(G).max())


def test_at_gradient_invariants():
    X = synth.rsa(15, seed=13, side=5.0, dmin=0.5)
    G = oracle.at_grad(X)
    E = oracle.at_energy(X)
    Xd = X.astype(np.float64)
    scale = np.abs(G).max()
    np.testing.assert_allclose(G.sum(axis=0), 0.0, atol=1e-12 * scale * 15)       # translation
    assert float((Xd * G).sum()) == pytest.approx(-9.0 * E, rel=1e-10)              # Euler, degree -9
    np.testing.assert_allclose(np.cross(Xd, G).sum(axis=0), 0.0, atol=1e-11 * scale * 15)  # rotation


def test_at_grad_rows_matches_full():
    X = synth.rsa(20, seed=17, side=5.0, dmin=0.5)
    G = oracle.at_grad(X)
    idx = [0, 3, 19, 7]
    np.testing.assert_allclose(oracle.at_grad_rows(X, idx), G[idx], rtol=1e-11,
                               atol=1e-13 * np.abs(G).max())


def test_stored_full_gradient_n8192():
    """The stored FP64 gradient of the n = 8192 workload (written by
    tests/golden/make_golden.py from the oracle's full triple loop): it belongs
    to the workload's input, it satisfies the invariants of a translation- and
    rotation-invariant energy homogeneous of degree -9 (AT) against the stored
    energy, and its sampled rows equal those of the oracle's other loop (one
    particle against all pairs), stored independently."""
    import json
    import os

    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    gold = json.load(open(os.path.join(here, "expected.json")))
    full = np.load(os.path.join(here, "grad_n8192.npz"))
    X = synth.workload_input("at_lj_n8192")
    import hashlib
    assert str(full["input_sha256"]) == hashlib.sha256(np.ascontiguousarray(X).tobytes()).hexdigest()
    at, lj = full["at"], full["lj"]
    assert at.shape == lj.shape == (8192, 3)
    g = gold["at_lj_n8192"]
    Xd = X.astype(np.float64)
    scale = np.abs(at).max()
    np.testing.assert_allclose(at.sum(axis=0), 0.0, atol=1e-11 * scale)
    assert float((Xd * at).sum()) == pytest.approx(-9.0 * g["at_energy"], rel=1e-9)
    np.testing.assert_allclose(np.cross(Xd, at).sum(axis=0), 0.0, atol=1e-9 * scale * np.abs(Xd).max())
    rows = np.array(g["grad_rows"])
    np.testing.assert_allclose(at[rows], np.array(g["at_grad_rows"]), rtol=1e-10, atol=1e-12 * scale)
    lscale = np.abs(lj).max()
    np.testing.assert_allclose(lj[rows], np.array(g["lj_grad_rows"]), rtol=1e-12, atol=1e-14 * lscale)
    np.testing.assert_allclose(lj, oracle.lj_grad(X, 1.0, 1.0, 3.0), rtol=1e-12, atol=1e-14 * lscale)


# ------------------------------------------------------------------ Lennard-Jones
def test_lj_closed_forms():
    rmin = 2.0 ** (1 / 6)
    X = np.array([[0, 0, 0], [rmin, 0, 0]], np.float32)
    r = float(np.float32(rmin))
    assert oracle.lj_energy(X) == pytest.approx(4 * (r ** -12 - r ** -6), rel=1e-14)
    assert oracle.lj_energy(X) == pytest.approx(-1.0, rel=1e-6)
    assert np.abs(oracle.lj_grad(X)).max() < 1e-5
    Y = np.array([[0, 0, 0], [0, 1, 0]], np.float32)  # r = sigma
    assert oracle.lj_energy(Y) == 0.0
    Z = np.array([[0, 0, 0], [0, 0, 3.0001]], np.float32)  # beyond the cutoff
    assert oracle.lj_energy(Z) == 0.0 and not oracle.lj_grad(Z).any()
    W = np.array([[0, 0, 0], [0, 0, 2.9999]], np.float32)
    assert oracle.lj_energy(W) == pytest.approx(4 * (2.9999 ** -12 - 2.9999 ** -6), rel=1e-6)


def test_lj_pure_python_and_fd():
    X = synth.rsa(25, seed=8, side=4.0, dmin=0.8)
    P = X.astype(np.float64)
    e = 0.0
    for i in range(25):
        for j in range(i + 1, 25):
            r = float(np.linalg.norm(P[i] - P[j]))
            if r < 3.0:
                e += 4 * (r ** -12 - r ** -6)
    assert oracle.lj_energy(X) == pytest.approx(e, rel=1e-13)
    G = oracle.lj_grad(X)
    np.testing.assert_allclose(G.sum(axis=0), 0, atol=1e-10 * np.abs(G).max())
    # finite differences on a pair configuration far from the cutoff
    Y = np.array([[0.125, 0.25, 0.5], [1.0, 0.75, 0.25], [0.25, 1.5, 1.0]], np.float32)
    Gy = oracle.lj_grad(Y)
    h = 2.0 ** -18
    for i in range(3):
        for c in range(3):
            Yp, Ym = Y.copy(), Y.copy()
            Yp[i, c] += np.float32(h)
            Ym[i, c] -= np.float32(h)
            fd = (oracle.lj_energy(Yp) - oracle.lj_energy(Ym)) / (2 * h)
            assert fd == pytest.approx(Gy[i, c], rel=1e-6, abs=1e-7 * np.abs(Gy).max())


# ------------------------------------------------------------------ checksums
def test_splitmix64_published_outputs():
    # SplitMix64 seeded with 0: the first three outputs of the generator are the
    # finaliser applied to 1, 2 and 3 times the increment 0x9E3779B97F4A7C15.
    gamma = 0x9E3779B97F4A7C15
    assert oracle.mix64(0) == 0xE220A8397B1DCDAF
    assert oracle.mix64(gamma) == 0x6E789E6AA1B965F4
    assert oracle.mix64((2 * gamma) % 2 ** 64) == 0x06C45D188009454F


@pytest.mark.parametrize("kind,m,strict", [("pairs_le", 2, False), ("pairs_lt", 2, True),
                                           ("triplets_le", 3, False), ("triplets_lt", 3, True),
                                           ("quads_le", 4, False), ("quads_lt", 4, True)])
@pytest.mark.parametrize("n", [0, 1, 2, 3, 17, 40])
def test_checksum_ids_are_bijective(kind, m, strict, n):
    s, c = oracle.checksum_walk(kind, n)
    v = oracle.simplex_volume(m, n, strict)
    assert c == v
    assert s == oracle.checksum_range(v)


def test_checksum_walk_pure_python():
    n = 9
    M = 2 ** 64
    s = 0
    for i in range(n):
        for j in range(i, n):
            for k in range(j, n):
                s = (s + oracle.mix64(k * (k + 1) * (k + 2) // 6 + j * (j + 1) // 2 + i)) % M
    assert oracle.checksum_walk("triplets_le", n)[0] == s
    s = 0
    for i in range(n):
        for j in range(i + 1, n):
            for k in range(j + 1, n):
                for l in range(k + 1, n):
                    s = (s + oracle.mix64(l * (l - 1) * (l - 2) * (l - 3) // 24 + k * (k - 1) * (k - 2) // 6
                                          + j * (j - 1) // 2 + i)) % M
    assert oracle.checksum_walk("quads_lt", n)[0] == s


# --------------------------------------------------------------------------
# 4-point contacts (4-cliques of the contact graph) on the 4-simplex.
def _contacts_brute(X, rc2):
    """All quadruplets by four nested loops.  The inputs lie on a grid of
    step 1/4, so every squared distance is exact in FP32 and FP64 alike and
    the contact test needs no rounding."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    adj = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1) < rc2
    c = 0
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if not (adj[i, k] and adj[j, k]):
                    continue
                for l in range(k + 1, n):
                    c += bool(adj[i, l] and adj[j, l] and adj[k, l])
    return c


@pytest.mark.parametrize("n,seed", [(4, 1), (12, 2), (25, 3), (40, 4)])
def test_quad_contacts_brute_force(n, seed):
    X = synth.integer(n, 3, seed=seed, lo=0, hi=12).astype(np.float32) * np.float32(0.25)
    for m in (0, 10, 20, 40, 80, 10000):  # rc^2 = m/16 + 1/32: never equal to a squared distance
        rc2 = m / 16 + 1 / 32
        assert oracle.quad_contacts(X, rc2 ** 0.5) == _contacts_brute(X, rc2)


def test_quad_contacts_closed_forms():
    # everything in contact: C(n, 4); nothing: 0
    X = synth.uniform(30, 3, seed=9)
    assert oracle.quad_contacts(X, 10.0) == math.comb(30, 4)
    assert oracle.quad_contacts(X, 0.0) == 0
    # points 1 apart on a line, contact below 3.5: exactly the n - 3 runs of four
    L = np.zeros((50, 3), np.float32)
    L[:, 0] = np.arange(50)
    assert oracle.quad_contacts(L, 3.5) == 47
    assert oracle.quad_contacts(L, 2.5) == 0
    # cube corners, contact below 1.01 sqrt(2) (no body diagonal): one corner
    # of each antipodal pair, 2^4 = 16 (6 faces, 2 tetrahedra, 8 vertex stars)
    C = np.array([[x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)], np.float32)
    assert oracle.quad_contacts(C, 1.01 * 2 ** 0.5) == 16
    assert oracle.quad_contacts(C, 1.01) == 0
    assert oracle.quad_contacts(C, 1.8) == math.comb(8, 4)
    # invariant under a relabelling of the points
    X = synth.uniform(60, 3, seed=5) * np.float32(4.0)
    p = np.random.default_rng(0).permutation(60)
    assert oracle.quad_contacts(X[p], 1.5) == oracle.quad_contacts(X, 1.5) > 0


# --------------------------------------------------------------------------
# Conway's Life on the 2-simplex of cells (i <= j): known patterns far from the
# boundary behave as on the plane; the boundary kills what would leave the
# triangle; cells below the diagonal never live.
def _grid(n, cells):
    S = np.zeros((n, n), np.uint8)
    for i, j in cells:
        S[i, j] = 1
    return S


def _cells(S):
    return sorted(map(tuple, np.argwhere(S).tolist()))


def test_life_blinker_period_two():
    S = _grid(40, [(10, 29), (10, 30), (10, 31)])          # horizontal, inside the triangle
    S1 = oracle.life_step(S)
    assert _cells(S1) == [(9, 30), (10, 30), (11, 30)]     # vertical
    assert (oracle.life_step(S1) == S).all()


def test_life_still_lifes():
    block = _grid(40, [(5, 20), (5, 21), (6, 20), (6, 21)])
    assert (oracle.life_step(block) == block).all()
    beehive = _grid(40, [(8, 21), (8, 22), (9, 20), (9, 23), (10, 21), (10, 22)])
    assert (oracle.life_step(beehive) == beehive).all()


def test_life_glider_moves_one_cell_diagonally_every_four_steps():
    g = [(0, 1), (1, 2), (2, 0), (2, 1), (2, 2)]
    S = _grid(60, [(5 + i, 30 + j) for i, j in g])
    T = S
    for _ in range(4):
        T = oracle.life_step(T)
    assert _cells(T) == [(6 + i, 31 + j) for i, j in sorted(g)]


def test_life_boundary_cuts_patterns():
    n = 30
    # a vertical blinker on the last column: its horizontal phase would need
    # column n, so two cells remain, and they die in the next step
    S = _grid(n, [(9, n - 1), (10, n - 1), (11, n - 1)])
    S1 = oracle.life_step(S)
    assert _cells(S1) == [(10, n - 2), (10, n - 1)]
    assert oracle.life_step(S1).sum() == 0
    # a vertical blinker crossing the diagonal: its cell (11, 10) lies outside
    # the triangle and does not count, the two cells left have one neighbour
    # each and no cell has three, so everything dies at once
    S = _grid(n, [(9, 10), (10, 10), (11, 10)])
    assert oracle.life_step(S).sum() == 0
    # the same blinker one column to the right lies inside and oscillates
    S = _grid(n, [(9, 11), (10, 11), (11, 11)])
    assert _cells(oracle.life_step(S)) == [(10, 10), (10, 11), (10, 12)]
    # below the diagonal nothing ever lives, whatever the input holds there
    R = synth.bits(64, 9, 0.5)
    for _ in range(5):
        R = oracle.life_step(R)
        assert (np.tril(R, -1) == 0).all()


def test_life_window_equals_full_step():
    S = synth.bits(150, 4, 0.35)
    A = oracle.life_step(S)
    for (i0, i1, j0, j1) in [(0, 40, 0, 40), (20, 90, 60, 150), (100, 150, 100, 150), (0, 150, 0, 150)]:
        assert (oracle.life_window(S, i0, i1, j0, j1) == A[i0:i1, j0:j1]).all()
