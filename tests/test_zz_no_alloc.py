"""The allocation-free pyramid entry point against the allocating one, through the C ABI."""
import sys

import numpy as np
import pytest

from paper_2110_10156_amd import binding as bd

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def test_noalloc_pyramid_equals_allocating_entry_point_on_consecutive_calls():
    """Two calls in a row, the second on a smaller input (the scratch array keeps the first
    call's contents): each output is bit-identical to csngf_smooth_downsample's."""
    import torch
    rng = np.random.default_rng(31)
    cases = [((110, 176, 176), 3.0, 2),    # (nz, ny, nx), sigma, factor: a paper-scale pyramid level
             ((37, 50, 61), 1.5, 1)]       # smaller, ragged, no downsampling
    s = torch.cuda.Stream()
    for shape, sigma, factor in cases:
        _say("noalloc pyramid", shape, sigma, factor)
        vol = torch.from_numpy(rng.random(shape).astype(np.float32)).cuda()
        ref = bd.smooth_downsample(vol, sigma, factor)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            out = bd.smooth_downsample_noalloc(vol, sigma, factor, stream=s)
        s.synchronize()
        assert out.shape == ref.shape
        assert torch.equal(out, ref), float((out - ref).abs().max())
    # the host-pointer path of the allocating entry point agrees too
    vol_np = rng.random((20, 24, 28)).astype(np.float32)
    host = bd.smooth_downsample(vol_np, 2.0, 2)
    dev = bd.smooth_downsample_noalloc(torch.from_numpy(vol_np).cuda(), 2.0, 2)
    torch.cuda.synchronize()
    assert np.array_equal(dev.cpu().numpy(), host)
