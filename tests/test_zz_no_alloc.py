"""td_lap_decode_noalloc (the decode for callers that cannot allocate device
memory) against td_lap_decode, through the C-ABI: bit-equal on two calls in
a row, the second on a smaller region, with nothing allocated on the device
meanwhile; a region beyond the fixed scratch is refused before any launch.
"""
import numpy as np
import pytest

from gpu_common import rel_l2, require_gpu
from oracle import laplace
from synth.fbm import terrain_latent

pytestmark = pytest.mark.gpu

DEC = {"factor": 8, "sigma_low": 20.0, "sigma_res": 2.0, "blur_sigma": 5.0, "blur_radius": 15}


def _latent(torch, region, seed):
    lx0, ly0, lw, lh = laplace.required_latent(region, DEC)
    lat = terrain_latent(seed, lx0, ly0, lw, lh, 4)
    return torch.from_numpy(lat).cuda(), lx0, ly0, lat


def test_noalloc_decode_equals_decode(weights):
    require_gpu()
    import torch
    from paper_2512_08309_amd import td
    print("no-alloc decode: 8192x8192 px at (-8000, 123456), then 200x136 px at (803, -517)", flush=True)
    with td.Context(0) as ref_ctx, td.Context(0) as c:
        ref_ctx.load_weights(weights("lg"))
        c.load_weights(weights("lg"))
        cases = [((-8000, 123456, 8192, 8192), 21), ((803, -517, 200, 136), 5)]
        inputs = []
        for region, seed in cases:
            lat_dev, lx0, ly0, lat = _latent(torch, region, seed)
            X0, Y0, W, H = region
            want = torch.empty((H, W), device="cuda")
            ref_ctx.lap_decode(lat_dev, lx0, ly0, X0, Y0, W, H, want)
            inputs.append((region, lat_dev, lx0, ly0, lat, want, torch.full((H, W), np.nan, device="cuda")))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for region, lat_dev, lx0, ly0, _, _, got in inputs:      # two calls in a row, the second smaller
            X0, Y0, W, H = region
            c.lap_decode_noalloc(lat_dev, lx0, ly0, X0, Y0, W, H, got)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        for region, _, lx0, ly0, lat, want, got in inputs:
            assert torch.equal(got, want), region
            if region[2] * region[3] < 1 << 20:                  # the oracle on the small region
                ref = laplace.decode(lat.astype(np.float64), (lx0, ly0), region, DEC)
                assert rel_l2(got.cpu().numpy(), ref) <= 1e-5
        # the large region needs 2 x 1.1 M floats (9 MB) of scratch; none was allocated
        assert free0 - free1 < (2 << 20), (free0, free1)


def test_noalloc_decode_refuses_regions_beyond_its_scratch(weights):
    require_gpu()
    import torch
    from paper_2512_08309_amd import td
    with td.Context(0) as c:
        c.load_weights(weights("lg"))
        region = (0, 0, 1 << 20, 64)                  # a strip: needs 2 x 131104 x 40 floats > 2^22
        lx0, ly0, lw, lh = laplace.required_latent(region, DEC)
        zeros = torch.zeros((lh, lw, 4), device="cuda")           # refused before any launch reads it
        big = torch.empty((region[3], region[2]), device="cuda")
        with pytest.raises(td.TDError) as e:
            c.lap_decode_noalloc(zeros, lx0, ly0, *region, big)
        assert e.value.status == td.TD_E_INVAL and "scratch" in str(e.value)
        del big, zeros
        lat_dev, lx0, ly0, _ = _latent(torch, (64, 64, 8, 8), 3)
        out = torch.zeros((8, 8), device="cuda")
        c.lap_decode_noalloc(lat_dev, lx0, ly0, 64, 64, 8, 8, out)   # the context still works
        want = torch.empty((8, 8), device="cuda")
        c.lap_decode(lat_dev, lx0, ly0, 64, 64, 8, 8, want)
        torch.cuda.synchronize()
        assert torch.equal(out, want)
