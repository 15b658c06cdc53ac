"""Every hot-path kernel and map through the checked library (device checks
compiled in): no map may produce a tile outside the simplex and no unmasked
store may leave it, at ragged sizes, on every map; the results still match the
oracle.  The checks record a flag and skip the access instead of faulting."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1610_07394_amd as smx
import synth

pytestmark = pytest.mark.gpu

MAPS = ["lambda", "bbox", "linear", "lambda_below", "recursive", "recursive_launch"]


@pytest.fixture(scope="module", autouse=True)
def checked_library():
    smx.select_library(checked=True)
    smx.check_flags(clear=True)
    yield
    smx.select_library(checked=False)


def test_unchecked_library_reports_unsupported():
    smx.select_library(checked=False)
    try:
        with pytest.raises(NotImplementedError):
            smx.check_flags()
    finally:
        smx.select_library(checked=True)


@pytest.mark.parametrize("kind", MAPS)
def test_maps_and_workloads_stay_in_the_simplex(kind):
    print(f"checked {kind}", flush=True)
    # map dumps, 2- and 3-simplex (and 4-simplex where the map is defined)
    smx.simplex_map2(1000, 16, kind)
    smx.simplex_map3(200, 8, kind, strict=True)
    if kind != "lambda_below":
        smx.simplex_map4(100, 4, kind, strict=True)
    # EDM, every precision, ragged n and tiles past the interior
    for n, d in ((300, 7), (1100, 40)):
        X = synth.normal(n, d, seed=n)
        Xt = torch.from_numpy(X).cuda()
        for prec in ("bf16", "split_bf16"):
            smx.edm_packed(Xt, kind, prec)
        got = smx.edm_packed(Xt, kind, "fp32").cpu().numpy().astype(np.float64)
        ref = oracle.edm_packed(X)
        diag = np.array([i * n - i * (i - 1) // 2 for i in range(n)])
        off = np.ones(ref.shape, bool)
        off[diag] = False
        assert (got[diag] == 0).all()
        assert np.max(np.abs(got[off] - ref[off]) / ref[off]) <= 1e-5
    # Axilrod-Teller + LJ, packed triplets, 4-point contacts
    P = synth.rsa(130, seed=3, side=6.0, dmin=0.8)
    Pt = torch.from_numpy(P).cuda()
    E, G = smx.triplet_energy_grad(Pt, smx.Pot(nu=1.0, at=True, lj=True), kind)
    Ep = smx.triplet_packed(Pt, 1.0, kind)
    torch.cuda.synchronize()
    assert abs(E[1].item() - oracle.at_energy(P)) <= 1e-5 * abs(oracle.at_energy(P))
    assert Ep.numel() == math.comb(130, 3)
    if kind != "lambda_below":
        C = synth.uniform(140, 3, seed=5) * np.float32(4.0)
        c = smx.quad_contacts(torch.from_numpy(C).cuda(), 1.5, kind)
        assert int(c.item()) == oracle.quad_contacts(C, 1.5)
    assert smx.check_flags(clear=True) == 0
