"""Life on the 2-simplex of cells through the C ABI, against the oracle, bit
for bit: several generations on small grids over every map (ragged n, one
tile, many tiles), and one generation at n = 32768 on sampled windows (the
diagonal, the last row of tiles, the bound n, tile corners, the interior).

The kernel takes the tile-contiguous layout; the dense <-> tiled conversion
below is the test's own (tile (X, Y), X <= Y, at (Y(Y+1)/2 + X) * 4096, cell
at 64 (i mod 64) + (j mod 64)).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1610_07394_amd as smx
import synth

pytestmark = pytest.mark.gpu

KINDS = ["lambda", "bbox", "linear", "lambda_below", "recursive", "recursive_launch"]
B = 64


def offsets(ii, jj):
    ii, jj = np.asarray(ii, np.int64), np.asarray(jj, np.int64)
    ti, tj = ii // B, jj // B
    return (tj * (tj + 1) // 2 + ti) * (B * B) + (ii % B) * B + (jj % B)


def to_tiled(A, n):
    """Dense n x n grid -> tiled buffer; every byte of the upper tiles is copied,
    including the cells of diagonal tiles below the diagonal (never read)."""
    nb = -(-n // B)
    P = np.zeros((nb * B, nb * B), np.uint8)
    P[:n, :n] = A
    T = np.zeros(smx.life_len(n), np.uint8)
    for Y in range(nb):
        for X in range(Y + 1):
            r = (Y * (Y + 1) // 2 + X) * B * B
            T[r:r + B * B] = P[X * B:(X + 1) * B, Y * B:(Y + 1) * B].ravel()
    return T


def from_tiled(T, n):
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    up = ii <= jj
    A = np.zeros((n, n), np.uint8)
    A[up] = T[offsets(ii[up], jj[up])]
    return A


def tiled_zero_outside(T, n):
    """True iff every byte of the tiled buffer outside the triangle is 0."""
    nb = -(-n // B)
    ii, jj = np.meshgrid(np.arange(nb * B), np.arange(nb * B), indexing="ij")
    sel = (ii // B <= jj // B) & ~((ii <= jj) & (jj < n))
    return not np.any(T[offsets(ii[sel], jj[sel])])


class TiledView:
    """Read-only n x n view of a tiled buffer for oracle.life_window (slices only)."""

    def __init__(self, T, n):
        self.T, self.shape = T, (n, n)

    def __getitem__(self, key):
        si, sj = key
        ii = np.arange(si.start, si.stop)[:, None]
        jj = np.arange(sj.start, sj.stop)[None, :]
        ii, jj = np.broadcast_arrays(ii, jj)
        W = np.zeros(ii.shape, np.uint8)
        up = ii <= jj
        W[up] = self.T[offsets(ii[up], jj[up])]
        return W


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 130, 200])
def test_life_generations_vs_oracle(kind, n):
    A = synth.bits(n, seed=70 + n, density=0.35)  # lower triangle random too: must be ignored
    cur = torch.from_numpy(to_tiled(A, n)).cuda()
    nxt = torch.full((smx.life_len(n),), 7, dtype=torch.uint8, device="cuda")
    ref = A
    for gen in range(5):
        smx.simplex_life(cur, n, kind, out=nxt)
        ref = oracle.life_step(ref)
        got = nxt.cpu().numpy()
        assert np.array_equal(from_tiled(got, n), ref), f"generation {gen + 1} differs"
        assert tiled_zero_outside(got, n), f"generation {gen + 1}: nonzero outside the triangle"
        cur, nxt = nxt, cur


@pytest.mark.parametrize("kind", ["lambda", "linear"])
def test_life_mid_size_ragged(kind):
    """n = 1000 (16 tiles per side, the last 40 cells wide): three generations
    of a denser start, bit for bit."""
    n = 1000
    A = synth.bits(n, seed=11, density=0.45)
    cur = torch.from_numpy(to_tiled(A, n)).cuda()
    nxt = torch.empty_like(cur)
    ref = A
    for gen in range(3):
        smx.simplex_life(cur, n, kind, out=nxt)
        ref = oracle.life_step(ref)
        assert np.array_equal(from_tiled(nxt.cpu().numpy(), n), ref), f"generation {gen + 1} differs"
        cur, nxt = nxt, cur


@pytest.mark.parametrize("kind", ["lambda", "bbox", "recursive"])
def test_life_stats(kind):
    n = 517
    A = synth.bits(n, seed=5, density=0.4)
    S = torch.from_numpy(to_tiled(A, n)).cuda()
    D, st = smx.simplex_life(S, n, kind, stats=True)
    ref = oracle.life_step(A)
    st = st.cpu().numpy()
    nb = -(-n // B)
    assert np.array_equal(from_tiled(D.cpu().numpy(), n), ref)
    assert int(st[0]) == int(ref.sum())
    assert int(st[2]) == nb * (nb + 1) // 2
    assert int(st[3]) >= int(st[2])


def test_life_still_life_and_blinker_on_gpu():
    """A block stays, a blinker flips, a lone cell dies, all across tile boundaries."""
    n = 200
    A = np.zeros((n, n), np.uint8)
    A[62:64, 63:65] = 1                     # block straddling tiles (0, 0) / (0, 1)
    A[100, 127:130] = 1                     # horizontal blinker crossing tile column 2
    A[150, 190] = 1                         # lone cell
    S = torch.from_numpy(to_tiled(A, n)).cuda()
    D = from_tiled(smx.simplex_life(S, n, "lambda").cpu().numpy(), n)
    assert np.array_equal(D, oracle.life_step(A))
    assert D[62:64, 63:65].all() and D[99:102, 128].all() and D[100, 127] == 0 and D[150, 190] == 0


def test_life_empty_grid():
    S = torch.empty(0, dtype=torch.uint8, device="cuda")
    D = smx.simplex_life(S, 0, "lambda")
    assert D.numel() == 0


def test_life_full_size_windows():
    n = 32768
    T = synth.bits_flat(smx.life_len(n), seed=2024, density=0.3)
    S = torch.from_numpy(T).cuda()
    D, st = smx.simplex_life(S, n, "lambda", stats=True)
    out = D.cpu().numpy()
    nb = n // B
    assert int(st.cpu()[2]) == nb * (nb + 1) // 2
    view_in, view_out = TiledView(T, n), TiledView(out, n)
    rng = np.random.default_rng(9)
    wins = [(0, 70, 0, 70), (n - 70, n, n - 70, n), (0, 70, n - 70, n), (4090, 4160, 4090, 4160),
            (63, 129, 127, 193), (20000, 20070, 30000, 30070)]
    for _ in range(10):
        i = int(rng.integers(0, n - 64))
        j = int(rng.integers(i, n - 64 + 1))
        wins.append((i, i + 64, j, min(j + 64, n)))
    for (i0, i1, j0, j1) in wins:
        ref = oracle.life_window(view_in, i0, i1, j0, j1)
        got = view_out[slice(i0, i1), slice(j0, j1)]
        assert np.array_equal(got, ref), f"window {(i0, i1, j0, j1)} differs"
    # the live count is a property of the whole grid: the kernel's own tally
    # must agree with a count of the output buffer (zero outside the triangle)
    assert int(st.cpu()[0]) == int(out.sum(dtype=np.int64))
