"""4-point contacts (4-cliques of the contact graph) over the 4-simplex
through the C ABI, against the oracle's neighbour-list count: the result is an
integer decided on the same FP32 squared distances, so it must match exactly
for every map."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1610_07394_amd as smx
import synth

pytestmark = pytest.mark.gpu

KINDS = ["lambda", "bbox", "linear", "recursive", "recursive_launch"]


def _gpu(X):
    return torch.from_numpy(np.ascontiguousarray(X)).cuda()


@pytest.mark.parametrize("n", [4, 5, 31, 63, 64, 65, 127, 128, 129, 200, 300])
def test_contacts_vs_oracle_all_maps(n):
    print(f"contacts n={n}", flush=True)
    X = synth.uniform(n, 3, seed=70 + n) * np.float32(max(2.0, 1.6 * n ** (1 / 3)))
    Xt = _gpu(X)
    for rc in (0.9, 1.7):
        ref = oracle.quad_contacts(X, rc)
        for kind in KINDS:
            c, s = smx.quad_contacts(Xt, rc, kind, stats=True)
            s = s.cpu().numpy()
            assert int(c.item()) == ref, (kind, rc)
            nb = -(-n // 64)
            assert int(s[0]) == math.comb(n, 4) and int(s[2]) == math.comb(nb + 3, 4)
            assert int(s[3]) == smx.parallel_blocks(4, nb, 1, kind)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_contacts_degenerate_sizes(n):
    X = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    c, s = smx.quad_contacts(X, 5.0, stats=True)
    assert int(c.item()) == 0 and int(s[0].item()) == 0


def test_contacts_dense_and_empty():
    """Radius past the diameter: every quadruplet (dense words, full popcounts);
    radius 0: none."""
    n = 150
    X = synth.uniform(n, 3, seed=3)
    Xt = _gpu(X)
    for kind in KINDS:
        assert int(smx.quad_contacts(Xt, 10.0, kind).item()) == math.comb(n, 4)
        assert int(smx.quad_contacts(Xt, 0.0, kind).item()) == 0


def test_contacts_exact_grid_and_stride():
    """Grid coordinates (every squared distance exact) and a strided input."""
    n = 190
    X = synth.integer(n, 3, seed=8, lo=0, hi=24).astype(np.float32) * np.float32(0.25)
    Xw = np.zeros((n, 6), np.float32)
    Xw[:, :3] = X
    rc = (30 / 16 + 1 / 32) ** 0.5
    ref = oracle.quad_contacts(X, rc)
    assert ref > 0
    assert int(smx.quad_contacts(_gpu(X), rc).item()) == ref
    assert int(smx.quad_contacts(_gpu(Xw)[:, :3], rc).item()) == ref


def test_contacts_full_size_n8192():
    """The n = 8192 workload (the Axilrod-Teller particle set, contact radius 2):
    1.9e14 quadruplets, exact count on every map that fits the launch limits."""
    X = synth.workload_input("at_lj_n8192")
    Xt = _gpu(X)
    ref = oracle.quad_contacts(X, 2.0)
    print(f"  oracle: {ref} 4-cliques", flush=True)
    for kind in KINDS:
        c, s = smx.quad_contacts(Xt, 2.0, kind, stats=True)
        s = s.cpu().numpy()
        print(f"  {kind}: {int(c.item())}", flush=True)
        assert int(c.item()) == ref
        assert int(s[0]) == math.comb(8192, 4) and int(s[2]) == math.comb(128 + 3, 4)


def test_contacts_max_size_n16384():
    """The largest n the entry point takes (nb = 256 tiles per dimension), a
    uniform cloud at the same contact degree as the n = 8192 set; the bounding
    box's 256^4 ids exceed the launch limit and are refused."""
    n = 16384
    X = synth.uniform(n, 3, seed=16) * np.float32(20.0 * 2 ** (1 / 3))
    Xt = _gpu(X)
    ref = oracle.quad_contacts(X, 2.0)
    print(f"  oracle: {ref} 4-cliques", flush=True)
    assert ref > 0
    for kind in ["lambda", "linear", "recursive"]:
        c, s = smx.quad_contacts(Xt, 2.0, kind, stats=True)
        s = s.cpu().numpy()
        print(f"  {kind}: {int(c.item())}", flush=True)
        assert int(c.item()) == ref
        assert int(s[0]) == math.comb(n, 4) and int(s[2]) == math.comb(256 + 3, 4)
    with pytest.raises(Exception):
        smx.quad_contacts(Xt, 2.0, "bbox")
