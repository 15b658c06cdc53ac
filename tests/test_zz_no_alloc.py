"""The allocation-free energy + gradient entry point (its workspace is the
library's static device array) against smx_triplet_energy_grad, which takes a
caller-allocated workspace: the same energies and gradients to the tolerance
of the FP32 kernels (relative 1e-5; atomic FP64 accumulation orders differ),
on consecutive calls whose second input is smaller than the first, so stale
scratch contents from the first call must not leak into the second."""
import numpy as np
import pytest
import torch

import oracle
import paper_1610_07394_amd as smx
import synth

pytestmark = pytest.mark.gpu

ATLJ = smx.Pot(nu=1.0, at=True, lj=True, eps=1.0, sigma=1.0, rc=3.0)


def _pts(n, seed):
    side = max(1.5, 20.0 * (max(n, 1) / 8192) ** (1 / 3))
    return synth.rsa(n, seed=seed, side=side, dmin=0.8)


def _fmetric(G, ref):
    return float(np.linalg.norm(G - ref, axis=1).max() / np.linalg.norm(ref, axis=1).max())


def _check_pair(Xt, kind):
    E0, G0 = smx.triplet_energy_grad(Xt, ATLJ, kind)
    E1, G1 = smx.triplet_energy_grad_noalloc(Xt, ATLJ, kind)
    torch.cuda.synchronize()
    E0, E1 = E0.cpu().numpy(), E1.cpu().numpy()
    for q in range(3):
        assert abs(E1[q] - E0[q]) <= 1e-5 * max(abs(E0[1]), abs(E0[2])), (q, E0, E1)
    err = _fmetric(G1.cpu().numpy().astype(np.float64), G0.cpu().numpy().astype(np.float64))
    print(f"  n={Xt.shape[0]} {kind}: noalloc vs workspace grad {err:.2e}", flush=True)
    assert err <= 1e-5
    return E1, G1


@pytest.mark.parametrize("kind", ["lambda", "bbox", "linear"])
def test_noalloc_matches_workspace_entry_point_twice(kind):
    print(f"noalloc {kind}: n=700 then n=150", flush=True)
    X1 = _pts(700, seed=21)
    _check_pair(torch.from_numpy(X1).cuda(), kind)
    X2 = _pts(150, seed=22)
    E, G = _check_pair(torch.from_numpy(X2).cuda(), kind)
    # the second (smaller) call against the oracle as well
    e_ref = oracle.at_energy(X2) + oracle.lj_energy(X2)
    assert abs(E[0] - e_ref) <= 1e-5 * (abs(oracle.at_energy(X2)) + abs(oracle.lj_energy(X2)))
    g_ref = oracle.at_grad(X2) + oracle.lj_grad(X2)
    assert _fmetric(G.cpu().numpy().astype(np.float64), g_ref) <= 1e-5


def test_noalloc_small_and_limit():
    X = torch.from_numpy(_pts(2, seed=5)).cuda()
    E, G = smx.triplet_energy_grad_noalloc(X, ATLJ, "lambda")
    torch.cuda.synchronize()
    E = E.cpu().numpy()
    assert E[1] == 0.0 and abs(E[2] - oracle.lj_energy(_pts(2, seed=5))) <= 1e-5 * max(1.0, abs(E[2]))
    big = torch.zeros((smx.NOALLOC_MAX_N + 1, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError, match="static scratch limit"):
        smx.triplet_energy_grad_noalloc(big, ATLJ, "lambda")
