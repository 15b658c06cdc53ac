"""Packed per-triplet Axilrod-Teller energies (the 3-simplex analogue of the
packed EDM) through the C ABI, against the FP64 oracle element by element.

Error metric: a single term can cancel to ~0 (1 + 3 cos cos cos = 0), so the
per-element error is taken relative to the term's own scale nu / (r1 r2 r3)^3
(|E_t| <= 4 nu / (r1 r2 r3)^3); the bar is 1e-5 of it.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1610_07394_amd as smx
import synth

pytestmark = pytest.mark.gpu

KINDS = ["lambda", "bbox", "linear", "lambda_below", "recursive", "recursive_launch"]
TOL = 1e-5


def _term_scale(X, i, j, k, nu):
    Xd = X.astype(np.float64)
    r1 = np.linalg.norm(Xd[j] - Xd[i], axis=1)
    r2 = np.linalg.norm(Xd[k] - Xd[j], axis=1)
    r3 = np.linalg.norm(Xd[k] - Xd[i], axis=1)
    return nu / (r1 * r2 * r3) ** 3


def _lex_triplets(n, i0=0, i1=None):
    i1 = n if i1 is None else i1
    idx = [(i, j, k) for i in range(i0, i1) for j in range(i + 1, n) for k in range(j + 1, n)]
    a = np.array(idx, dtype=np.int64).reshape(-1, 3)
    return a[:, 0], a[:, 1], a[:, 2]


@pytest.mark.parametrize("n", [3, 4, 5, 31, 32, 33, 64, 65, 100, 130])
def test_packed_vs_oracle_all_maps(n):
    print(f"packed n={n}", flush=True)
    nu = 0.9
    X = synth.rsa(n, seed=40 + n, side=max(2.0, 0.9 * n ** (1 / 3)), dmin=0.6)
    Xt = torch.from_numpy(X).cuda()
    E = smx.triplet_packed(Xt, nu, "lambda")
    for kind in KINDS[1:]:
        assert torch.equal(E, smx.triplet_packed(Xt, nu, kind)), kind
    torch.cuda.synchronize()
    got = E.cpu().numpy().astype(np.float64)
    ref = oracle.at_triplet_rows(X, nu=nu)
    assert got.shape == ref.shape == (math.comb(n, 3),)
    i, j, k = _lex_triplets(n)
    err = float(np.max(np.abs(got - ref) / _term_scale(X, i, j, k, nu)))
    print(f"  max error / term scale {err:.2e}")
    assert err <= TOL


@pytest.mark.parametrize("n", [0, 1, 2])
def test_packed_degenerate_sizes(n):
    X = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    E, s = smx.triplet_packed(X, 1.0, "lambda", stats=True)
    assert E.numel() == 0 and int(s[0].item()) == 0


def test_packed_counts_checksum_and_total():
    n = 300
    X = synth.rsa(n, seed=5, side=8.0, dmin=0.8)
    Xt = torch.from_numpy(X).cuda()
    for kind in KINDS:
        E, s = smx.triplet_packed(Xt, 1.0, kind, stats=True)
        s = s.cpu().numpy()
        V = math.comb(n, 3)
        assert int(s[0]) == V and int(s[1]) % (1 << 64) == oracle.checksum_range(V)
    e_tot = smx.triplet_energy(Xt, smx.Pot(nu=1.0, at=True, lj=False), "lambda")[1].item()
    assert abs(E.double().sum().item() - e_tot) <= 1e-5 * abs(e_tot)


def test_packed_strided_positions():
    n = 70
    X4 = synth.rsa(n, seed=8, side=4.0, dmin=0.6)
    Xw = np.zeros((n, 5), np.float32)
    Xw[:, :3] = X4
    E1 = smx.triplet_packed(torch.from_numpy(X4).cuda(), 1.0)
    E2 = smx.triplet_packed(torch.from_numpy(Xw).cuda()[:, :3], 1.0)
    assert torch.equal(E1, E2)


def test_packed_full_size_n2048():
    """n = 2048 (1.43e9 triplets, 5.7 GB): sampled rows against the oracle at
    tile edges; lambda and bounding box bit-identical; the sum equals the AT
    energy."""
    X = synth.workload_input("at_n2048")
    n = X.shape[0]
    Xt = torch.from_numpy(X).cuda()
    E = smx.triplet_packed(Xt, 1.0, "lambda")
    Eb = smx.triplet_packed(Xt, 1.0, "bbox")
    torch.cuda.synchronize()
    assert torch.equal(E, Eb)
    del Eb
    c3 = math.comb(n, 3)
    worst = 0.0
    for i in [0, 31, 32, 1000, n - 33, n - 4, n - 3]:
        a = c3 - math.comb(n - i, 3)
        m = math.comb(n - 1 - i, 2)
        got = E[a:a + m].cpu().numpy().astype(np.float64)
        ref = oracle.at_triplet_rows(X, i0=i, i1=i + 1)
        ii, jj, kk = _lex_triplets(n, i, i + 1)
        worst = max(worst, float(np.max(np.abs(got - ref) / _term_scale(X, ii, jj, kk, 1.0))))
    print(f"  sampled rows: max error / term scale {worst:.2e}")
    assert worst <= TOL
    e_tot = smx.triplet_energy(Xt, smx.Pot(nu=1.0, at=True, lj=False), "lambda")[1].item()
    assert abs(E.double().sum().item() - e_tot) <= 1e-5 * abs(e_tot)


def _tiled_offsets(i, j, k):
    X, Y, Z = i // 32, j // 32, k // 32
    rank = Z * (Z + 1) * (Z + 2) // 6 + Y * (Y + 1) // 2 + X
    return rank * 32768 + (i % 32) * 1024 + (j % 32) * 32 + (k % 32)


@pytest.mark.parametrize("n", [3, 5, 31, 32, 33, 64, 65, 100])
def test_tiled_layout_matches_packed_bit_for_bit(n):
    """The tile-contiguous layout holds the packed values at the documented
    offsets, bit for bit, and zeros everywhere else, on every map."""
    X = synth.rsa(n, seed=60 + n, side=max(2.0, 0.9 * n ** (1 / 3)), dmin=0.6)
    Xt = torch.from_numpy(X).cuda()
    P = smx.triplet_packed(Xt, 0.7, "lambda").cpu().numpy()
    i, j, k = _lex_triplets(n)
    off = _tiled_offsets(i, j, k)
    for kind in KINDS:
        T, s = smx.triplet_packed_tiled(Xt, 0.7, kind, stats=True)
        T = T.cpu().numpy()
        assert T.shape[0] == smx.triplet_tiled_len(n)
        np.testing.assert_array_equal(T[off], P)
        rest = np.ones(T.shape[0], bool)
        rest[off] = False
        assert (T[rest] == 0).all()
        assert int(s[0].item()) == math.comb(n, 3)


def test_tiled_layout_full_size_rows():
    """n = 2048: sampled rows of the tiled output equal the packed output."""
    X = synth.workload_input("at_n2048")
    n = X.shape[0]
    Xt = torch.from_numpy(X).cuda()
    P = smx.triplet_packed(Xt, 1.0, "lambda")
    T = smx.triplet_packed_tiled(Xt, 1.0, "lambda")
    torch.cuda.synchronize()
    c3 = math.comb(n, 3)
    for i in [0, 31, 32, 1000, n - 3]:
        a = c3 - math.comb(n - i, 3)
        m = math.comb(n - 1 - i, 2)
        ii, jj, kk = _lex_triplets(n, i, i + 1)
        off = torch.from_numpy(_tiled_offsets(ii, jj, kk)).cuda()
        assert torch.equal(T[off], P[a:a + m])
