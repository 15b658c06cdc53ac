"""GPU parity of the map kernels: tile dumps bit-exact against the oracle's
maps, element counts and checksums exact against the oracle's simplex
checksums, for the lambda, bounding-box and linear maps."""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1610_07394_amd as smx
from oracle import maps as omaps

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "expected.json")
KINDS = ["lambda", "bbox", "linear", "lambda_below", "recursive", "recursive_launch"]


def _gold():
    with open(GOLD) as f:
        return json.load(f)


def _u64(v):
    return int(v) % (1 << 64)


def _run(m, n, rho, kind, strict, tiles=True):
    print(f"map{m} n={n} rho={rho} {kind} strict={strict}", flush=True)
    fn = smx.simplex_map2 if m == 2 else smx.simplex_map3
    t, s = fn(n, rho, kind, strict=strict, tiles=tiles)
    torch.cuda.synchronize()
    return (None if t is None else t.cpu().numpy()), s.cpu().numpy()


def _check_stats(s, m, n, rho, kind, strict):
    nb = -(-n // rho)
    V = oracle.simplex_volume(m, n, strict)
    assert int(s[0]) == V
    assert _u64(s[1]) == oracle.checksum_range(V)
    ntiles = math.comb(nb + m - 1, m)
    assert int(s[2]) == ntiles
    assert int(s[3]) == smx.parallel_blocks(m, n, rho, kind)


CASES2 = [(1024, 16), (1000, 16), (1, 16), (2, 1), (5, 1), (64, 1), (300, 64), (65, 8), (4096, 256),
          (3000, 1024)]


@pytest.mark.parametrize("n,rho", CASES2)
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("strict", [False, True])
def test_map2_dump_and_counts(n, rho, kind, strict):
    t, s = _run(2, n, rho, kind, strict)
    nb = -(-n // rho)
    np.testing.assert_array_equal(t, omaps.tiles(2, nb, kind))
    _check_stats(s, 2, n, rho, kind, strict)


CASES3 = [(64, 8), (100, 8), (33, 4), (1, 8), (8, 1), (17, 1), (256, 16), (200, 32), (1024, 64)]


@pytest.mark.parametrize("n,rho", CASES3)
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("strict", [False, True])
def test_map3_dump_and_counts(n, rho, kind, strict):
    t, s = _run(3, n, rho, kind, strict)
    nb = -(-n // rho)
    np.testing.assert_array_equal(t, omaps.tiles(3, nb, kind))
    _check_stats(s, 3, n, rho, kind, strict)


KINDS4 = ["lambda", "bbox", "linear", "recursive", "recursive_launch"]
CASES4 = [(16, 1), (17, 1), (1, 4), (30, 2), (64, 4), (100, 8), (130, 16), (256, 16)]


@pytest.mark.parametrize("n,rho", CASES4)
@pytest.mark.parametrize("kind", KINDS4)
@pytest.mark.parametrize("strict", [False, True])
def test_map4_dump_and_counts(n, rho, kind, strict):
    print(f"map4 n={n} rho={rho} {kind} strict={strict}", flush=True)
    t, s = smx.simplex_map4(n, rho, kind, strict=strict)
    torch.cuda.synchronize()
    nb = -(-n // rho)
    np.testing.assert_array_equal(t.cpu().numpy(), omaps.tiles(4, nb, kind))
    _check_stats(s.cpu().numpy(), 4, n, rho, kind, strict)


@pytest.mark.parametrize("n,rho", [(2048, 16), (1000, 8), (33 * 16, 16), (7, 1)])
@pytest.mark.parametrize("kind", KINDS4)
@pytest.mark.parametrize("strict", [False, True])
def test_count4_closed_form(n, rho, kind, strict):
    """4-simplex parallel space at n = 2048, rho = 16 (nb = 128: 1.9e7 lambda4
    blocks, 2.7e8 bounding-box blocks): the closed-form tile counts add up to
    the volume."""
    if kind == "bbox" and -(-n // rho) > 215:
        pytest.skip("nb^4 blocks exceed the launch limit")
    s = smx.simplex_count(4, n, rho, kind, strict).cpu().numpy()
    nb = -(-n // rho)
    assert int(s[0]) == oracle.simplex_volume(4, n, strict)
    assert int(s[2]) == nb * (nb + 1) * (nb + 2) * (nb + 3) // 24
    assert int(s[3]) == smx.parallel_blocks(4, n, rho, kind)


@pytest.mark.parametrize("kind", KINDS)
def test_map2_full_size_counts(kind):
    """n = 65536 at the paper-like granularity rho = 16 (8.4M lambda blocks)."""
    _, s = _run(2, 65536, 16, kind, False, tiles=False)
    g = _gold()["checksums"]["pairs_le_65536"]
    assert int(s[0]) == g["volume"] and _u64(s[1]) == int(g["checksum"])
    assert int(s[2]) == 4096 * 4097 // 2


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("strict", [False, True])
def test_map3_full_size_counts(kind, strict):
    """n = 8192 triplets with 32^3 tiles: 9.2e10 elements counted exactly."""
    _, s = _run(3, 8192, 32, kind, strict, tiles=False)
    g = _gold()["checksums"]["triplets_lt_8192" if strict else "triplets_le_8192"]
    assert int(s[0]) == g["volume"] and _u64(s[1]) == int(g["checksum"])
    assert int(s[2]) == 256 * 257 * 258 // 6


def test_lambda_block_counts_match_paper_ratios():
    """|Pi2| = |T2| exactly; |Pi3| / |T3 minus plane| = 9/8 + O(1/nb) (12.5% extra)."""
    for n, rho in ((65536, 16), (8192, 32)):
        nb = n // rho
        assert smx.parallel_blocks(2, n, rho, "lambda") == nb * (nb + 1) // 2
    nb = 256
    main = smx.parallel_blocks(3, 8192, 32, "lambda") - nb * (nb + 1) // 2
    assert main == 3 * nb ** 3 // 16
    assert abs(main / ((nb ** 3 - nb) / 6) - 9 / 8) < 1e-4


@pytest.mark.parametrize("m,n,rho", [(2, 1024, 16), (2, 1000, 16), (2, 65536, 16), (2, 33 * 64 + 5, 64),
                                     (3, 8192, 8), (3, 1000, 8), (3, 33 * 32, 32), (3, 5, 1)])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("strict", [False, True])
def test_count_kernel_closed_form(m, n, rho, kind, strict):
    """Parallel space only: the per-tile closed-form counts add up to the volume."""
    s = smx.simplex_count(m, n, rho, kind, strict).cpu().numpy()
    nb = -(-n // rho)
    assert int(s[0]) == oracle.simplex_volume(m, n, strict)
    assert int(s[2]) == (nb * (nb + 1) // 2 if m == 2 else nb * (nb + 1) * (nb + 2) // 6)
    assert int(s[3]) == smx.parallel_blocks(m, n, rho, kind)


@pytest.mark.parametrize("m,nb", [(2, 1), (2, 2), (2, 13), (2, 64), (2, 1000), (2, 4096), (3, 1), (3, 5), (3, 17),
                                  (3, 128), (3, 300), (4, 1), (4, 3), (4, 8), (4, 17), (4, 64)])
@pytest.mark.parametrize("kind", KINDS)
def test_decode_lane_parallel(m, nb, kind):
    """The map decoded one lane per logical id: the mapped ids are exactly the
    tiles of T_m (count and colex-rank checksum of a bijection), and every id of
    the parallel space is decoded once."""
    if m == 4 and kind == "lambda_below":
        pytest.skip("from below is not defined for the 4-simplex")
    vol = math.comb(nb + m - 1, m)
    s = smx.simplex_decode(m, nb, kind).cpu().numpy()
    assert int(s[0]) == vol
    assert _u64(s[1]) == oracle.checksum_range(vol)
    assert int(s[3]) == smx.parallel_blocks(m, nb, 1, kind)
