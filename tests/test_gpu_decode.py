"""GPU parity of the Laplacian decode against the FP64 oracle."""
import numpy as np
import pytest

from gpu_common import rel_l2, require_gpu
from oracle import laplace
from oracle.sampler import Model, sample
from synth.fbm import terrain_latent

pytestmark = pytest.mark.gpu

DEC = {"factor": 8, "sigma_low": 20.0, "sigma_res": 2.0, "blur_sigma": 5.0, "blur_radius": 15}


@pytest.fixture(scope="module")
def ctx(weights):
    require_gpu()
    from paper_2512_08309_amd import td
    c = td.Context(0).load_weights(weights("lg"))
    yield c
    c.close()


@pytest.mark.parametrize("out_region", [(0, 0, 256, 192), (-803, 517, 203, 77), (8 * 1000001, -8 * 999, 64, 64)])
def test_decode_fbm_latent_matches_oracle(ctx, out_region):
    import torch
    lx0, ly0, lw, lh = laplace.required_latent(out_region, DEC)
    lx0, ly0 = lx0 - 3, ly0 - 2          # a larger latent than needed
    lw, lh = lw + 7, lh + 5
    lat = terrain_latent(21, lx0, ly0, lw, lh, 4)
    X0, Y0, W, H = out_region
    out = torch.empty((H, W), dtype=torch.float32, device="cuda")
    ctx.lap_decode(torch.from_numpy(lat).cuda(), lx0, ly0, X0, Y0, W, H, out)
    torch.cuda.synchronize()
    ref = laplace.decode(lat.astype(np.float64), (lx0, ly0), out_region, DEC)
    got = out.cpu().numpy()
    assert rel_l2(got, ref) <= 1e-5
    assert np.max(np.abs(got - ref)) <= 1e-4 * np.max(np.abs(ref)) + 1e-3


def test_decode_rejects_short_apron(ctx):
    import torch
    from paper_2512_08309_amd import td
    lat = torch.zeros((20, 20, 4), device="cuda")
    out = torch.empty((8, 8), device="cuda")
    with pytest.raises(td.TDError):
        ctx.lap_decode(lat, 0, 0, 64, 64, 8, 8, out)


def test_height_query_matches_oracle(weights):
    require_gpu()
    from paper_2512_08309_amd import td
    with td.Context(0) as c:
        c.load_weights(weights("lg"))
        region = (-50, 77, 48, 40)
        got = c.sample_region(3, *region, td.TD_LEVEL_HEIGHT)
        m = Model(weights("lg"))
        lx0, ly0, lw, lh = laplace.required_latent(region, DEC)
        lat = sample(m, 3, lx0, ly0, lw, lh, 0)
        ref = laplace.decode(lat, (lx0, ly0), region, DEC)
        assert got.shape == (40, 48)
        assert rel_l2(got, ref) <= 1e-4


def test_calls_on_torch_default_stream_are_ordered_with_torch(ctx):
    """A call given torch's current stream (the default stream, handle 0) is
    ordered with torch's work on it: the decode reads a latent torch writes
    just before it behind a spin, and a region query's result is not
    overwritten by a fill torch queued before it."""
    import torch
    from paper_2512_08309_amd import td
    region = (0, 0, 256, 192)
    lx0, ly0, lw, lh = laplace.required_latent(region, DEC)
    src = torch.from_numpy(terrain_latent(21, lx0, ly0, lw, lh, 4)).cuda()
    ref = torch.empty((192, 256), device="cuda")
    ctx.lap_decode(src, lx0, ly0, *region, ref)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    assert s.cuda_stream == 0
    lat = torch.zeros_like(src)
    out = torch.zeros_like(ref)
    torch.cuda._sleep(20_000_000)
    lat.copy_(src)
    ctx.lap_decode(lat, lx0, ly0, *region, out, s)
    assert float((out - ref).abs().max()) == 0.0

    want = torch.from_numpy(ctx.sample_region(5, 3, 4, 40, 24, 0)).cuda()
    got = torch.empty_like(want)
    torch.cuda._sleep(20_000_000)
    got.fill_(-1.0)
    ctx.sample_region_async(5, 3, 4, 40, 24, 0, got, s)
    assert float((got - want).abs().max()) == 0.0


@pytest.mark.parametrize("region", [(-800, 1600, 384, 320), (8 * 999991, -8 * 1000003, 296, 400)])
def test_encode_matches_oracle(ctx, region):
    """Laplacian encode of an elevation field (the oracle's decode of an fBm
    latent, rounded to float32) against the oracle's encode of the same
    float32 heights: geometry exact, values rel L2 <= 1e-5."""
    import torch
    X0, Y0, W, H = region
    lx0, ly0, lw, lh = laplace.required_latent(region, DEC)
    lat = terrain_latent(21, lx0, ly0, lw, lh, 4)
    h32 = laplace.decode(lat.astype(np.float64), (lx0, ly0), region, DEC).astype(np.float32)
    ref, origin = laplace.encode(h32.astype(np.float64), region, DEC, 4)
    geom = ctx.lap_encode(None, X0, Y0, W, H)
    assert geom == (origin[0], origin[1], ref.shape[1], ref.shape[0])
    out = torch.empty((geom[3], geom[2], 4), device="cuda")
    ctx.lap_encode(torch.from_numpy(h32).cuda(), X0, Y0, W, H, out)
    torch.cuda.synchronize()
    err = rel_l2(out.cpu().numpy(), ref)
    print("encode rel L2 %.2e" % err)
    assert err <= 1e-5


def test_encode_rejects_bad_regions(ctx):
    import torch
    from paper_2512_08309_amd import td
    h = torch.zeros((320, 384), device="cuda")
    out = torch.empty((8, 8, 4), device="cuda")
    for X0, Y0, W, H in [(4, 0, 384, 320), (0, 0, 380, 320), (0, 0, 256, 256)]:
        with pytest.raises(td.TDError):
            ctx.lap_encode(None, X0, Y0, W, H)
    with pytest.raises(td.TDError):        # output too small for (384 / 8 - 32) x (320 / 8 - 32) x 4
        ctx.lap_encode(h, 0, 0, 384, 320, out)


DEC_WIDE = dict(DEC, blur_sigma=9.0, blur_radius=30)


@pytest.fixture(scope="module")
def ctx_wide(weights):
    require_gpu()
    from paper_2512_08309_amd import td
    c = td.Context(0).load_weights(weights("lgw"))
    yield c
    c.close()


def test_decode_wide_blur_matches_oracle(ctx_wide):
    """A blur radius past the single-launch blur's limit (30 > 24): the
    decode's multi-launch path against the oracle."""
    import torch
    region = (-803, 517, 203, 77)
    lx0, ly0, lw, lh = laplace.required_latent(region, DEC_WIDE)
    lat = terrain_latent(21, lx0, ly0, lw, lh, 4)
    X0, Y0, W, H = region
    out = torch.empty((H, W), dtype=torch.float32, device="cuda")
    ctx_wide.lap_decode(torch.from_numpy(lat).cuda(), lx0, ly0, X0, Y0, W, H, out)
    torch.cuda.synchronize()
    ref = laplace.decode(lat.astype(np.float64), (lx0, ly0), region, DEC_WIDE)
    assert rel_l2(out.cpu().numpy(), ref) <= 1e-5


def test_encode_wide_blur_matches_oracle(ctx_wide):
    import torch
    region = (-800, 1600, 640, 576)
    X0, Y0, W, H = region
    lx0, ly0, lw, lh = laplace.required_latent(region, DEC_WIDE)
    lat = terrain_latent(21, lx0, ly0, lw, lh, 4)
    h32 = laplace.decode(lat.astype(np.float64), (lx0, ly0), region, DEC_WIDE).astype(np.float32)
    ref, origin = laplace.encode(h32.astype(np.float64), region, DEC_WIDE, 4)
    geom = ctx_wide.lap_encode(None, X0, Y0, W, H)
    assert geom == (origin[0], origin[1], ref.shape[1], ref.shape[0])
    out = torch.empty((geom[3], geom[2], 4), device="cuda")
    ctx_wide.lap_encode(torch.from_numpy(h32).cuda(), X0, Y0, W, H, out)
    torch.cuda.synchronize()
    assert rel_l2(out.cpu().numpy(), ref) <= 1e-5
