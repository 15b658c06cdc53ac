"""The VALU issue probe the benchmark uses for its measured ceiling: it runs
through the C ABI and reports a rate between a quarter of and twice the
single-issue FP32 rate of the chip (256 CUs x 64 lanes x 2.4 GHz)."""
import numpy as np
import pytest
import torch

import paper_1610_07394_amd as smx

pytestmark = pytest.mark.gpu


def test_valu_probe_rate_and_output():
    blocks, iters = 2048, 512
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    smx._check(smx.lib().smx_probe_valu(out.data_ptr(), blocks, iters, smx._stream()))
    ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev[0].record()
    smx._check(smx.lib().smx_probe_valu(out.data_ptr(), blocks, iters, smx._stream()))
    ev[1].record()
    torch.cuda.synchronize()
    rate = blocks * 256 * iters * 64 / (ev[0].elapsed_time(ev[1]) / 1e3)
    spec = 256 * 64 * 2.4e9
    print(f"  probe: {rate:.3e} lane-ops/s ({rate / spec:.2f} of {spec:.3e})")
    assert 0.25 * spec <= rate <= 2.0 * spec
    assert np.isfinite(out.cpu().numpy()).all()
