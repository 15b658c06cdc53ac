"""CPU tests of the C-ABI library: it loads, exports every symbol the header
declares, validates arguments on the host before any HIP call, and its inline
map code (evaluated on the host) equals the oracle's maps.  No device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1610_07394_amd as smx
from oracle import maps as omaps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smx.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(smx_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 14
    L = ctypes.CDLL(smx.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_parallel_volume_is_parallel_blocks():
    """smx_parallel_volume (the paper's |Pi|, in blocks) is the same count as
    smx_parallel_blocks, errors included."""
    L = ctypes.CDLL(smx.LIB_PATH)
    for f in (L.smx_parallel_volume, L.smx_parallel_blocks):
        f.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int]
        f.restype = ctypes.c_int64
    for m, n, rho in ((2, 1024, 16), (2, 1000, 16), (3, 8192, 8), (3, 100, 4), (4, 1024, 8), (2, 0, 16)):
        for mp in range(6):
            if m == 4 and mp == 3:
                continue
            assert L.smx_parallel_volume(m, n, rho, mp) == L.smx_parallel_blocks(m, n, rho, mp)
    assert L.smx_parallel_volume(2, 64, 16, 0) == (4 // 2) * (4 + 1)  # Pi2 = (nb/2) x (nb+1), nb = 4
    assert L.smx_parallel_volume(5, 64, 16, 0) == -1


def test_version_and_volume():
    assert "gfx950" in smx.version()
    for n in (0, 1, 2, 3, 10, 1024, 65536):
        assert smx.volume(2, n) == n * (n + 1) // 2
        assert smx.volume(2, n, strict=True) == n * (n - 1) // 2 if n > 0 else smx.volume(2, n, True) == 0
        assert smx.volume(3, n) == n * (n + 1) * (n + 2) // 6
        assert smx.volume(3, n, strict=True) == max(0, n * (n - 1) * (n - 2) // 6)
    assert smx.volume(5, 10) == -1
    assert smx.volume(2, -1) == -1


@pytest.mark.parametrize("m,n,rho", [(2, 1024, 16), (2, 65536, 64), (2, 1000, 16), (3, 2048, 32),
                                     (3, 8192, 32), (3, 100, 8), (2, 1, 16), (3, 5, 1)])
@pytest.mark.parametrize("kind", list(smx.MAPS))
def test_parallel_blocks_match_oracle(m, n, rho, kind):
    nb = (n + rho - 1) // rho
    if m == 3 and kind == "bbox" and nb > 64:
        expect = nb ** 3
    else:
        expect = omaps.tiles(m, nb, kind).shape[0]
    assert smx.parallel_blocks(m, n, rho, kind) == expect


@pytest.mark.parametrize("nb", [1, 2, 3, 4, 7, 8, 16, 33, 64, 100, 512, 1024, 4096])
@pytest.mark.parametrize("kind", list(smx.MAPS))
def test_host_map2_equals_oracle(nb, kind):
    if kind == "bbox" and nb > 1024:
        pytest.skip("bbox dump of nb^2 blocks checked at smaller nb")
    got = smx.map_tiles_host(2, nb, 1, kind)
    want = omaps.tiles(2, nb, kind)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("nb", [1, 2, 3, 4, 5, 8, 16, 31, 64, 128, 256])
@pytest.mark.parametrize("kind", list(smx.MAPS))
def test_host_map3_equals_oracle(nb, kind):
    if kind == "bbox" and nb > 64:
        pytest.skip("bbox dump of nb^3 blocks checked at smaller nb")
    got = smx.map_tiles_host(3, nb, 1, kind)
    want = omaps.tiles(3, nb, kind)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("nb", [1, 2, 3, 4, 5, 8, 9, 16, 17, 32, 33, 64])
@pytest.mark.parametrize("kind", ["lambda", "bbox", "linear", "recursive", "recursive_launch"])
def test_host_map4_equals_oracle(nb, kind):
    if kind == "bbox" and nb > 33:
        pytest.skip("bbox dump of nb^4 blocks checked at smaller nb")
    got = smx.map_tiles_host(4, nb, 1, kind)
    want = omaps.tiles(4, nb, kind)
    np.testing.assert_array_equal(got, want)


def test_map4_limits_and_volume():
    from math import comb
    for n in (0, 1, 3, 4, 10, 1000):
        assert smx.volume(4, n) == comb(n + 3, 4) and smx.volume(4, n, True) == comb(n, 4)
    assert smx.parallel_blocks(4, 2048, 16, "lambda") == omaps.lambda4_blocks(128)
    assert smx.parallel_blocks(4, 2048, 16, "linear") == comb(131, 4)
    L = smx.lib()
    null = None
    # from below is not defined for m = 4; rho past 16; m = 5
    assert L.smx_simplex_count(4, 100, 1, 3, 0, ctypes.c_void_p(256), ctypes.c_void_p(256), 1 << 20, null) == 3
    assert L.smx_simplex_map4(100, 32, 0, 0, null, null, null, 0, null) == 1
    assert L.smx_simplex_count(5, 100, 1, 0, 0, ctypes.c_void_p(256), ctypes.c_void_p(256), 1 << 20, null) == 1
    # bounding box past 2^31 blocks; lambda4 past nb' = 256
    assert L.smx_parallel_blocks(4, 256 * 16, 16, 1) == -1
    assert L.smx_parallel_blocks(4, 257 * 16, 16, 0) == -1


def test_linear_map_exact_where_fp32_roots_are_not():
    """Block indices near 2^31 map exactly although a plain FP32 root is wrong there."""
    nb = 65535  # linear grid of nb (nb + 1) / 2 = 2,147,450,880 blocks
    # k = T(y) - 1 and T(y) around the largest rows
    ys = np.arange(nb - 3000, nb + 1, dtype=np.int64)
    ks = np.concatenate([ys * (ys + 1) // 2 - 1, ys[:-1] * (ys[:-1] + 1) // 2])
    ks = ks[(ks >= 0) & (ks < nb * (nb + 1) // 2)]
    f32 = np.floor((np.sqrt(8 * ks.astype(np.float32) + np.float32(1)) - np.float32(1)) / np.float32(2))
    y_true = np.searchsorted(np.arange(nb + 2, dtype=np.int64) * np.arange(1, nb + 3, dtype=np.int64) // 2,
                             ks, side="right") - 1
    assert (f32.astype(np.int64) != y_true).any()  # FP32 alone fails in this range
    for k, yt in zip(ks[::97], y_true[::97]):
        t = smx.map_tiles_host(2, nb, 1, "linear", first=int(k), count=1)[0]
        assert t[1] == yt and t[0] == k - yt * (yt + 1) // 2


def _call(fn, *a):
    return fn(*a)


def test_validation_errors_before_any_device_work():
    L = smx.lib()
    null = None
    st = ctypes.c_void_p(0)
    # bad map / rho / n on the map dumps
    assert L.smx_simplex_map2(16, 16, 7, 0, null, null, null, 0, null) == 1
    assert L.smx_simplex_map2(16, 3, 0, 0, null, null, null, 0, null) == 1
    assert L.smx_simplex_map2(-1, 16, 0, 0, null, null, null, 0, null) == 1
    assert L.smx_simplex_map3(16, 128, 0, 0, null, null, null, 0, null) == 1
    assert b"rho" in L.smx_last_error()
    # stats without a workspace
    assert L.smx_simplex_map2(16, 16, 0, 0, null, ctypes.c_void_p(8), null, 0, null) == 1
    # n = 0 is a no-op
    assert L.smx_simplex_map2(0, 16, 0, 0, null, null, null, 0, null) == 0
    # parallel-space count: bad m / rho / map, no stats, no workspace
    assert L.smx_simplex_count(5, 16, 1, 0, 0, ctypes.c_void_p(256), ctypes.c_void_p(256), 1 << 20, null) == 1
    assert L.smx_simplex_count(2, 16, 3, 0, 0, ctypes.c_void_p(256), ctypes.c_void_p(256), 1 << 20, null) == 1
    assert L.smx_simplex_count(2, 16, 1, 9, 0, ctypes.c_void_p(256), ctypes.c_void_p(256), 1 << 20, null) == 1
    assert L.smx_simplex_count(2, 16, 1, 0, 0, null, ctypes.c_void_p(256), 1 << 20, null) == 1
    assert L.smx_simplex_count(3, 16, 1, 0, 0, ctypes.c_void_p(256), null, 0, null) == 1
    assert b"workspace" in L.smx_last_error()
    # packed triplet energies: n past 2^21, bad ldx / map, NULL buffers, stats without workspace
    assert L.smx_triplet_packed(null, (1 << 21) + 1, 3, 1.0, 0, null, null, 0, null, null) == 2
    assert L.smx_triplet_packed(null, 10, 2, 1.0, 0, null, null, 0, null, null) == 1
    assert L.smx_triplet_packed(null, 10, 3, 1.0, 7, null, null, 0, null, null) == 1
    assert L.smx_triplet_packed(null, 10, 3, 1.0, 0, null, null, 0, null, null) == 1
    assert L.smx_triplet_packed(ctypes.c_void_p(256), 10, 3, 1.0, 0, ctypes.c_void_p(256), null, 0,
                                ctypes.c_void_p(256), null) == 1
    # 4-point contacts: n past 16384, bad ldx / map / rc, from below, NULL count, no workspace
    assert L.smx_quad_contacts(null, 16385, 3, 1.0, 0, null, null, 0, null, null) == 2
    assert L.smx_quad_contacts(null, 10, 2, 1.0, 0, null, null, 0, null, null) == 1
    assert L.smx_quad_contacts(null, 10, 3, 1.0, 9, null, null, 0, null, null) == 1
    assert L.smx_quad_contacts(null, 10, 3, 1.0, 3, null, null, 0, null, null) == 3
    assert L.smx_quad_contacts(null, 10, 3, -1.0, 0, null, null, 0, null, null) == 1
    assert L.smx_quad_contacts(null, 10, 3, float("nan"), 0, null, null, 0, null, null) == 1
    assert L.smx_quad_contacts(ctypes.c_void_p(256), 10, 3, 1.0, 0, null, null, 0, null, null) == 1
    assert L.smx_quad_contacts(ctypes.c_void_p(256), 10, 3, 1.0, 0, ctypes.c_void_p(256), null, 0, null,
                               null) == 1
    assert b"workspace" in L.smx_last_error()
    # tile-contiguous layouts share the checks of their packed forms
    assert L.smx_triplet_packed_tiled(null, (1 << 21) + 1, 3, 1.0, 0, null, null, 0, null, null) == 2
    assert L.smx_triplet_packed_tiled(null, 10, 3, 1.0, 7, null, null, 0, null, null) == 1
    assert L.smx_triplet_packed_tiled(null, 10, 3, 1.0, 0, null, null, 0, null, null) == 1
    assert L.smx_edm_tiled(null, 10, 0, 3, 0, 0, null, null, 0, null, null) == 1
    assert L.smx_edm_tiled(null, 10, 3, 3, 0, 9, null, null, 0, null, null) == 1
    assert L.smx_edm_tiled(ctypes.c_void_p(256), 10, 3, 3, 0, 1, ctypes.c_void_p(256), null, 0, null, null) == 1
    assert L.smx_edm_tiled(null, 0, 3, 3, 0, 0, null, null, 0, null, null) == 0
    # Life on the 2-simplex: n negative / past 2^24, bad map, NULL or aliased
    # buffers, statistics without a workspace; n = 0 is a no-op
    a, b = ctypes.c_void_p(256), ctypes.c_void_p(4352)
    assert L.smx_simplex_life(a, b, -1, 0, null, null, 0, null) == 1
    assert L.smx_simplex_life(a, b, (1 << 24) + 1, 0, null, null, 0, null) == 2
    assert L.smx_simplex_life(a, b, 100, 6, null, null, 0, null) == 1
    assert L.smx_simplex_life(null, b, 100, 0, null, null, 0, null) == 1
    assert L.smx_simplex_life(a, a, 100, 0, null, null, 0, null) == 1
    assert L.smx_simplex_life(a, b, 100, 0, ctypes.c_void_p(8), null, 0, null) == 1
    assert b"workspace" in L.smx_last_error()
    assert L.smx_simplex_life(null, null, 0, 0, null, null, 0, null) == 0
    # lane-parallel decode: bad m / nb / map, NULL stats, no workspace, from
    # below on the 4-simplex
    v = ctypes.c_void_p(256)
    assert L.smx_simplex_decode(5, 8, 0, v, v, 1 << 20, null) == 1
    assert L.smx_simplex_decode(2, -1, 0, v, v, 1 << 20, null) == 1
    assert L.smx_simplex_decode(2, 8, 6, v, v, 1 << 20, null) == 1
    assert L.smx_simplex_decode(2, 8, 0, null, v, 1 << 20, null) == 1
    assert L.smx_simplex_decode(3, 8, 0, v, v, 8, null) == 1
    assert b"workspace" in L.smx_last_error()
    assert L.smx_simplex_decode(4, 8, 3, v, v, 1 << 20, null) == 3
    assert L.smx_simplex_decode(2, 1 << 20, 1, v, v, 1 << 20, null) == 3  # bounding-box grid past 65535
    # probe: NULL output, block count, iterations
    assert L.smx_probe_valu(null, 1, 1, null) == 1
    assert L.smx_probe_valu(ctypes.c_void_p(256), 0, 1, null) == 1
    assert L.smx_probe_valu(ctypes.c_void_p(256), 1, 0, null) == 1
    # EDM argument checks
    assert L.smx_edm_packed(null, 10, 0, 3, 0, 0, null, null, 0, null, null) == 1
    assert L.smx_edm_packed(null, 10, 3, 2, 0, 0, null, null, 0, null, null) == 1
    assert L.smx_edm_packed(null, 10, 3, 3, 6, 0, null, null, 0, null, null) == 1  # internal map id
    assert b"map" in L.smx_last_error()
    assert L.smx_edm_packed(null, 10, 3, 3, 0, 9, null, null, 0, null, null) == 1
    assert L.smx_edm_packed(null, 10, 3, 3, 0, 0, null, null, 0, null, null) == 1  # NULL X / D
    assert L.smx_edm_packed(ctypes.c_void_p(256), 10, 3, 3, 0, 1, ctypes.c_void_p(256), null, 0, null,
                            null) == 1  # Gram without workspace
    assert b"workspace" in L.smx_last_error()
    assert L.smx_edm_packed(null, 0, 3, 3, 0, 0, null, null, 0, null, null) == 0
    assert L.smx_edm_packed(null, 1 << 31, 3, 3, 0, 0, null, null, 0, null, null) == 2
    # triplet checks
    pot = smx.Pot()._c()
    assert L.smx_triplet_energy(null, 10, 2, ctypes.byref(pot), 0, null, null, 0, null, null) == 1
    assert L.smx_triplet_energy(null, 10, 3, None, 0, null, null, 0, null, null) == 1
    assert L.smx_triplet_energy(null, 10, 3, ctypes.byref(pot), 0, null, null, 0, null, null) == 1
    bad = smx.Pot(lj=True, rc=-1.0)._c()
    assert L.smx_triplet_energy(ctypes.c_void_p(256), 10, 3, ctypes.byref(bad), 0, ctypes.c_void_p(256),
                                ctypes.c_void_p(256), 1 << 20, null, null) == 1
    assert L.smx_triplet_energy_backward(ctypes.c_void_p(256), 10, 3, ctypes.byref(pot), 0, null,
                                         ctypes.c_void_p(256), ctypes.c_void_p(256), 1 << 20, null) == 1
    # the allocation-free variant checks its arguments, and its size limit, first
    L.smx_triplet_energy_grad_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                                  ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                                  ctypes.c_void_p, ctypes.c_void_p]
    pp = ctypes.cast(ctypes.byref(pot), ctypes.c_void_p)
    assert L.smx_triplet_energy_grad_noalloc(ctypes.c_void_p(256), 65537, 3, pp, 0, null,
                                             ctypes.c_void_p(256), null) == 1
    assert b"static scratch limit" in L.smx_last_error()
    assert L.smx_triplet_energy_grad_noalloc(ctypes.c_void_p(256), -1, 3, pp, 0, null, ctypes.c_void_p(256),
                                             null) == 1
    assert L.smx_triplet_energy_grad_noalloc(ctypes.c_void_p(256), 10, 3, pp, 0, null, null, null) == 1
    assert b"gradient" in L.smx_last_error()
    assert L.smx_triplet_energy_grad_noalloc(ctypes.c_void_p(256), 10, 2, pp, 0, null, ctypes.c_void_p(256),
                                             null) == 1
    assert L.smx_triplet_energy_grad_noalloc(ctypes.c_void_p(256), 10, 3, null, 0, null, ctypes.c_void_p(256),
                                             null) == 1
    assert L.smx_scale_grad(null, -1, null, null, null) == 1
    assert L.smx_scale_grad(null, 0, null, null, null) == 0
    ms, cnt = ctypes.c_double(), ctypes.c_int64()
    assert L.smx_profile_read(99, ctypes.byref(ms), ctypes.byref(cnt)) == 1


def test_grid_overflow_is_reported():
    # lambda3 past 2^31 blocks, bounding box past the grid dimension limit
    assert smx.lib().smx_parallel_blocks(3, 1 << 22, 1, 0) == -1
    assert smx.lib().smx_parallel_blocks(2, 1 << 17, 1, 1) == -1


def test_workspace_sizes():
    assert smx.workspace_bytes(0, 100) == 256 * 128
    w_fp32 = smx.workspace_bytes(1, 1000, 64, 0)
    w_bf16 = smx.workspace_bytes(1, 1000, 64, 1)
    w_split = smx.workspace_bytes(1, 1000, 64, 2)
    assert w_fp32 < w_bf16 < w_split
    assert w_split - w_bf16 >= 1000 * 64 * 2
    assert smx.workspace_bytes(2, 8192) >= 8192 * 3 * 8


def test_binding_rejects_host_tensors():
    import torch
    X = torch.zeros((4, 3), dtype=torch.float32)
    with pytest.raises(ValueError):
        smx.edm_packed(X)
    with pytest.raises(ValueError):
        smx.triplet_energy(X)


@pytest.mark.parametrize("m,nbs", [(2, [1, 2, 3, 4, 7, 8, 16, 33, 64, 100, 512]), (3, [1, 2, 3, 4, 5, 8, 16, 31, 64])])
@pytest.mark.parametrize("kind", ["lambda", "bbox", "linear"])
def test_inverse_maps_round_trip(m, nbs, kind):
    """The library's inverse maps send every mapped tile back to the block that
    mapped it, and every tile of the simplex to a block that maps to it."""
    for nb in nbs:
        t = smx.map_tiles_host(m, nb, 1, kind)
        ok = t[:, 0] >= 0
        ids = smx.map_blocks_host(m, nb, 1, t[ok], kind)
        np.testing.assert_array_equal(ids, np.nonzero(ok)[0])
        target = np.array(sorted(omaps.target_tiles(m, nb)), dtype=np.int32)
        back = smx.map_tiles_host(m, nb, 1, kind)[smx.map_blocks_host(m, nb, 1, target, kind)]
        np.testing.assert_array_equal(back, target)


def test_inverse_maps_reject_bad_tiles():
    with pytest.raises(ValueError):
        smx.map_blocks_host(2, 8, 1, [[3, 2]])
    with pytest.raises(ValueError):
        smx.map_blocks_host(3, 8, 1, [[0, 1, 8]])
    with pytest.raises(NotImplementedError):
        smx.map_blocks_host(2, 8, 1, [[0, 1]], "recursive")
