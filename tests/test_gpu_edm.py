"""GPU parity of the packed EDM against the FP64 oracle.

Tolerances (element-wise, off the diagonal; the diagonal must be exactly 0):
* FP32 difference form: |D^ - D| / D <= 1e-5.  Every term is non-negative, so
  the rounding error is at most about (d + 2) 2^-24 D and typically
  sqrt(d) 2^-24 D (< 1e-5 for the d <= 512 used here).
* Gram forms are compared relative to the scale |x_i|^2 + |x_j|^2 (the Gram
  form cancels when x_i ~ x_j).  BF16 keeps 8 significant bits, so
  round-to-nearest has unit roundoff u = 2^-8.
  plain BF16: each product carries <= 2u relative rounding and
  sum_k |x_ik x_jk| <= (|x_i|^2 + |x_j|^2) / 2, so |D^ - D| <= 2u (|x_i|^2 +
  |x_j|^2) = 2^-7 (...) plus FP32 accumulation -> bound 8e-3;
  split BF16: hi + lo carries x to u^2 = 2^-16 and the dropped lo*lo term is
  <= u^2 |x||y|, so |D^ - D| <= 3 u^2 (...) ~ 4.6e-5 (...) plus the FP32
  accumulation of G and of the norms (<= d 2^-25 each) -> bound 1e-4.
* Integer-valued inputs make every variant exact, so there the outputs must
  equal the oracle bit for bit.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1610_07394_amd as smx
import synth

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "expected.json")
KINDS = ["lambda", "bbox", "linear", "lambda_below", "recursive", "recursive_launch"]
TOL = {"fp32": 1e-5, "bf16": 8e-3, "split_bf16": 1e-4}


def _diag_idx(n):
    i = np.arange(n, dtype=np.int64)
    return i * n - i * (i - 1) // 2


def _edm(X, kind="lambda", prec="fp32", stats=False):
    print(f"edm n={X.shape[0]} d={X.shape[1]} {kind} {prec}", flush=True)
    Xt = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    r = smx.edm_packed(Xt, kind, prec, stats=stats)
    torch.cuda.synchronize()
    return r


def _errors(D, ref, X, prec):
    n = X.shape[0]
    dg = _diag_idx(n)
    assert (D[dg] == 0).all()
    off = np.ones(D.shape[0], bool)
    off[dg] = False
    if prec == "fp32":
        return float(np.max(np.abs(D[off] - ref[off]) / ref[off])) if off.any() else 0.0
    nrm = (X.astype(np.float64) ** 2).sum(1)
    ii = np.repeat(np.arange(n), np.arange(n, 0, -1))
    jj = np.concatenate([np.arange(i, n) for i in range(n)])
    scale = nrm[ii] + nrm[jj]
    return float(np.max(np.abs(D[off] - ref[off]) / scale[off])) if off.any() else 0.0


SHAPES = [(1, 3), (2, 3), (5, 1), (63, 3), (64, 3), (65, 7), (200, 32), (129, 33), (300, 64), (1024, 3),
          (257, 100), (130, 512)]


@pytest.mark.parametrize("n,d", SHAPES)
@pytest.mark.parametrize("prec", ["fp32", "bf16", "split_bf16"])
def test_edm_vs_oracle_all_maps_bit_identical(n, d, prec):
    X = synth.normal(n, d, seed=n * 1000 + d)
    ref = oracle.edm_packed(X)
    outs = [_edm(X, k, prec).cpu().numpy() for k in KINDS]
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])  # the map changes only the schedule
    D = outs[0].astype(np.float64)
    assert (D >= 0).all()
    err = _errors(D, ref, X, prec)
    print(f"  max error {err:.3e}")
    assert err <= TOL[prec]


@pytest.mark.parametrize("n,d", [(100, 3), (129, 64), (300, 512)])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "split_bf16"])
def test_edm_integer_inputs_exact(n, d, prec):
    X = synth.integer(n, d, seed=7 + n, lo=-8, hi=8)
    ref = oracle.edm_packed(X)
    D = _edm(X, "lambda", prec).cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(D, ref)


def test_edm_uniform_workload_small():
    """n = 1024, d = 3, uniform [0,1)^3: the small correctness workload."""
    X = synth.workload_input("edm_n1024_d3")
    ref = oracle.edm_packed(X)
    for kind in KINDS:
        D, s = _edm(X, kind, "fp32", stats=True)
        D = D.cpu().numpy().astype(np.float64)
        assert _errors(D, ref, X, "fp32") <= 1e-5
        s = s.cpu().numpy()
        V = 1024 * 1025 // 2
        assert int(s[0]) == V and int(s[1]) % (1 << 64) == oracle.checksum_range(V)
        assert int(s[2]) == 16 * 17 // 2


def test_edm_strided_rows():
    base = synth.normal(150, 40, seed=5)
    Xt = torch.from_numpy(base).cuda()[:, :37]  # ldx = 40 > d = 37
    ref = oracle.edm_packed(np.ascontiguousarray(base[:, :37]))
    for prec in ("fp32", "split_bf16"):
        D = smx.edm_packed(Xt, "lambda", prec).cpu().numpy().astype(np.float64)
        assert _errors(D, ref, base[:, :37], prec) <= TOL[prec]


def _sample_rows(D, X, rows):
    n = X.shape[0]
    worst = 0.0
    for i in rows:
        a = int(i * n - i * (i - 1) // 2)
        got = D[a:a + n - i].cpu().numpy().astype(np.float64)
        ref = oracle.edm_rows(X, int(i), int(i) + 1)
        assert got[0] == 0.0
        if n - i > 1:
            worst = max(worst, float(np.max(np.abs(got[1:] - ref[1:]) / ref[1:])))
    return worst


def test_edm_full_size_fp32():
    """n = 65536, d = 64 (8.6 GB packed output): maps bit-identical, sampled
    rows within 1e-5 of the oracle, element count and checksum exact."""
    X = synth.workload_input("edm_n65536_d64")
    n = X.shape[0]
    Xt = torch.from_numpy(X).cuda()
    D = smx.edm_packed(Xt, "lambda")
    D2 = smx.edm_packed(Xt, "bbox")
    torch.cuda.synchronize()
    assert torch.equal(D, D2)
    del D2
    D3 = smx.edm_packed(Xt, "linear")
    assert torch.equal(D, D3)
    del D3
    rows = sorted({0, 1, 63, 64, 65, 4095, 32768, n - 65, n - 64, n - 2, n - 1,
                   *np.random.default_rng(1).integers(0, n, 8).tolist()})
    worst = _sample_rows(D, X, rows)
    print(f"  sampled max rel error {worst:.3e}")
    assert worst <= 1e-5
    _, s = smx.edm_packed(Xt, "lambda", stats=True, out=D)
    s = s.cpu().numpy()
    g = json.load(open(GOLD))["checksums"]["pairs_le_65536"]
    assert int(s[0]) == g["volume"] and int(s[1]) % (1 << 64) == int(g["checksum"])


@pytest.mark.parametrize("prec", ["bf16", "split_bf16", "fp32"])
def test_edm_full_size_gram(prec):
    """n = 32768, d = 512: sampled rows against the oracle, per-variant error."""
    X = synth.workload_input("gram_n32768_d512")
    n = X.shape[0]
    Xt = torch.from_numpy(X).cuda()
    D = smx.edm_packed(Xt, "lambda", prec)
    Db = smx.edm_packed(Xt, "bbox", prec)
    torch.cuda.synchronize()
    assert torch.equal(D, Db)
    del Db
    rows = sorted({0, 127, 128, 255, 256, 16383, n - 257, n - 256, n - 129, n - 128, n - 1,
                   *np.random.default_rng(2).integers(0, n, 5).tolist()})
    nrm = (X.astype(np.float64) ** 2).sum(1)
    worst = 0.0
    for i in rows:
        a = int(i * n - i * (i - 1) // 2)
        got = D[a:a + n - i].cpu().numpy().astype(np.float64)
        ref = oracle.edm_rows(X, int(i), int(i) + 1)
        assert got[0] == 0.0
        if prec == "fp32":
            e = np.abs(got[1:] - ref[1:]) / ref[1:]
        else:
            e = np.abs(got[1:] - ref[1:]) / (nrm[i] + nrm[i + 1:])
        if e.size:
            worst = max(worst, float(e.max()))
    print(f"  {prec}: sampled max error {worst:.3e}")
    assert worst <= TOL[prec]


@pytest.mark.parametrize("d", [40, 300])
@pytest.mark.parametrize("prec", ["bf16", "split_bf16"])
def test_edm_gram_large_n_ragged(prec, d):
    """n = 16484 (128-element Gram tiles, the last one ragged, 32-row operand
    blocks padded), d = 40 (K padded to 64, a partial ring of k steps; ordinary
    stores) and d = 300 (K padded to 304; streaming stores): all maps
    bit-identical; sampled rows at tile edges against the oracle."""
    n = 16484
    X = np.random.default_rng(11).standard_normal((n, d)).astype(np.float32)
    Xt = torch.from_numpy(X).cuda()
    D = smx.edm_packed(Xt, "lambda", prec)
    for kind in KINDS[1:]:
        assert torch.equal(D, smx.edm_packed(Xt, kind, prec)), kind
    torch.cuda.synchronize()
    rows = [0, 1, 127, 128, 255, 256, 8191, 8192, 16383, 16384, n - 101, n - 100, n - 2, n - 1]
    nrm = (X.astype(np.float64) ** 2).sum(1)
    worst = 0.0
    for i in rows:
        a = int(i * n - i * (i - 1) // 2)
        got = D[a:a + n - i].cpu().numpy().astype(np.float64)
        ref = oracle.edm_rows(X, i, i + 1)
        assert got[0] == 0.0 and (got >= 0).all()
        if got.size > 1:
            worst = max(worst, float((np.abs(got[1:] - ref[1:]) / (nrm[i] + nrm[i + 1:])).max()))
    print(f"  {prec}: max error {worst:.3e}")
    assert worst <= TOL[prec]


def _tiled_edm_offsets(i, j):
    X, Y = i // 128, j // 128
    return (Y * (Y + 1) // 2 + X) * 16384 + (i % 128) * 128 + (j % 128)


@pytest.mark.parametrize("n,d", [(1, 3), (5, 1), (127, 3), (128, 8), (129, 33), (300, 64), (1100, 40)])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "split_bf16"])
def test_edm_tiled_layout_matches_packed(n, d, prec):
    """The tile-contiguous layout holds the packed values at the documented
    offsets, bit for bit, and zeros elsewhere, on every map."""
    X = synth.normal(n, d, seed=3 * n + d)
    Xt = torch.from_numpy(X).cuda()
    P = smx.edm_packed(Xt, "lambda", prec).cpu().numpy()
    ii = np.concatenate([np.full(n - i, i) for i in range(n)])
    jj = np.concatenate([np.arange(i, n) for i in range(n)])
    off = _tiled_edm_offsets(ii, jj)
    for kind in KINDS:
        T = smx.edm_tiled(Xt, kind, prec).cpu().numpy()
        assert T.shape[0] == smx.edm_tiled_len(n)
        np.testing.assert_array_equal(T[off], P)
        rest = np.ones(T.shape[0], bool)
        rest[off] = False
        assert (T[rest] == 0).all()


@pytest.mark.parametrize("d", [112, 128, 240, 256])
@pytest.mark.parametrize("prec", ["bf16", "split_bf16"])
def test_edm_gram_store_kinds(d, prec):
    """The Gram kernel writes with ordinary or streaming (non-temporal) stores
    by the padded depth (plain BF16 streams from d_pad = 256, split from 128),
    so these d sit on both sides of both switches.  At n = 300 tile (0, 1) is
    interior (unmasked stores) and the rest is fringe.  Element by element
    against the oracle, every map bit-identical, and the tile-contiguous layout
    holding the same values."""
    n = 300
    X = synth.normal(n, d, seed=500 + d)
    ref = oracle.edm_packed(X)
    outs = [_edm(X, k, prec).cpu().numpy() for k in KINDS]
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    D = outs[0].astype(np.float64)
    assert (D >= 0).all()
    err = _errors(D, ref, X, prec)
    print(f"  max error {err:.3e}")
    assert err <= TOL[prec]
    ii = np.concatenate([np.full(n - i, i) for i in range(n)])
    jj = np.concatenate([np.arange(i, n) for i in range(n)])
    T = smx.edm_tiled(torch.from_numpy(X).cuda(), "lambda", prec).cpu().numpy()
    np.testing.assert_array_equal(T[_tiled_edm_offsets(ii, jj)], outs[0])


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_edm_tiled_full_size_rows(prec):
    """Full-size inputs (n = 65536, d = 64 FP32; n = 32768, d = 512 split BF16):
    sampled rows of the tiled output equal the packed output."""
    name = "edm_n65536_d64" if prec == "fp32" else "gram_n32768_d512"
    X = synth.workload_input(name)
    n = X.shape[0]
    Xt = torch.from_numpy(X).cuda()
    P = smx.edm_packed(Xt, "lambda", prec)
    T = smx.edm_tiled(Xt, "lambda", prec)
    torch.cuda.synchronize()
    for i in [0, 127, 128, n // 2 + 5, n - 1]:
        a = i * n - i * (i - 1) // 2
        jj = np.arange(i, n)
        off = torch.from_numpy(_tiled_edm_offsets(np.full(n - i, i), jj)).cuda()
        assert torch.equal(T[off], P[a:a + n - i])
