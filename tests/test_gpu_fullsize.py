"""Parity at the benchmark's full size, in its launch configuration.

The cold C2 elevation query the bench times (8192 x 8192 px at full-res
origin (104, -8000008), i.e. a 1024^2 latent plus the 17-px decode apron,
K = 20, seed 7, automatic batch, FP32) runs once through the C-ABI.  The
FP64 oracle cannot evaluate that cone (about 61k window-denoises), so it
checks what it can compute one by one:

* the blended Euler step J_t at sampled pixels and levels: the oracle's
  level step (the four windows over the pixel, their denoiser, the W-blend
  of Eq. 2 and the Euler update) applied to the J_{t+1} the device used,
  read back from its cache;
* a heightfield crop, decoded by the oracle from the device's J_0;

and properties that hold at any size: every output finite, and cold crop
queries on a fresh context (latent and elevation) bit-equal to the same
crops of the full run.
"""
import numpy as np
import pytest

from gpu_common import planar, rel_l2, require_gpu
from oracle import laplace
from oracle.sampler import Model, level_step
from oracle.tdw import read_tdw
from oracle.windows import kappa_list

pytestmark = pytest.mark.gpu

SEED = 7
LX, LY, SIDE = 13, -1000001, 1024


def _hwc(planar_chw):
    return np.moveaxis(np.asarray(planar_chw, dtype=np.float64), 0, -1)


def _hull(windows, H, S, O):
    xs = [ix * S + O for ix, _ in windows]
    ys = [iy * S + O for _, iy in windows]
    return (min(xs), min(ys), max(xs) - min(xs) + H, max(ys) - min(ys) + H)


@pytest.fixture(scope="module")
def full_run(weights):
    require_gpu()
    import torch
    from paper_2512_08309_amd import td
    path = weights("c2")
    ctx = td.Context(0).load_weights(path)
    region = (8 * LX, 8 * LY, 8 * SIDE, 8 * SIDE)
    out = torch.empty((region[3], region[2]), dtype=torch.float32, device="cuda")
    print("full-size query", region, flush=True)
    ctx.sample_region_async(SEED, *region, td.TD_LEVEL_HEIGHT, out, torch.cuda.current_stream())
    torch.cuda.synchronize()
    yield td, torch, ctx, path, region, out
    ctx.close()


def test_full_size_output_finite_and_cone_evaluated_once(full_run):
    td, torch, ctx, path, region, out = full_run
    assert bool(torch.isfinite(out).all())
    st = ctx.cache_stats()
    hdr, _ = read_tdw(path)
    dec = hdr["decode"]
    lat = laplace.required_latent(region, dec)
    from oracle.windows import cone_window_count
    assert st["misses"] == cone_window_count(lat, 0, 20, 64, 32)


@pytest.mark.parametrize("t", [19, 9, 0])
def test_full_size_euler_step_matches_oracle(full_run, t):
    td, torch, ctx, path, region, out = full_run
    m = Model(path)
    hdr, _ = read_tdw(path)
    lx0, ly0, lw, lh = laplace.required_latent(region, hdr["decode"])
    for px, py in ((lx0 + 517, ly0 + 301), (lx0 + lw - 3, ly0 + 7)):
        r = (px, py, 2, 2)
        wins = kappa_list(r, m.H, m.s, m.o)
        rn = _hull(wins, m.H, m.s, m.o)
        j_next = _hwc(ctx.sample_region(SEED, *rn, t + 1))       # served from the cache
        got = ctx.sample_region(SEED, *r, t)
        ref = planar(level_step(m, j_next, rn, r, wins, t))
        err = rel_l2(got, ref)
        print("level", t, "pixel", (px, py), "windows", len(wins), "rel L2 %.2e" % err)
        assert err <= 2e-5, (t, px, py, err)


def test_full_size_height_crop_matches_oracle_decode(full_run):
    td, torch, ctx, path, region, out = full_run
    hdr, _ = read_tdw(path)
    dec = hdr["decode"]
    X0, Y0 = region[0] + 4001, region[1] + 117
    crop = (X0, Y0, 24, 16)
    lat = laplace.required_latent(crop, dec)
    latent = _hwc(ctx.sample_region(SEED, *lat, 0))
    ref = laplace.decode(latent, lat[:2], crop, dec)
    got = out[Y0 - region[1]:Y0 - region[1] + 16, X0 - region[0]:X0 - region[0] + 24].cpu().numpy()
    err = rel_l2(got, ref)
    print("height crop rel L2 %.2e" % err)
    assert err <= 1e-5


def test_full_size_cold_crops_bit_equal(full_run):
    td, torch, ctx, path, region, out = full_run
    hdr, _ = read_tdw(path)
    lx0, ly0, _, _ = laplace.required_latent(region, hdr["decode"])
    lat_crop = (lx0 + 700, ly0 + 900, 48, 40)
    full_lat = ctx.sample_region(SEED, *lat_crop, 0)               # the full run's J_0 there
    crop = (region[0] + 2048, region[1] + 6000, 40, 24)
    with td.Context(0) as c2:
        c2.load_weights(path)
        c2.set_option("batch", 37)                                  # another batch composition
        cold_lat = c2.sample_region(SEED, *lat_crop, 0)
        cold_h = c2.sample_region(SEED, *crop, td.TD_LEVEL_HEIGHT)
    assert np.array_equal(cold_lat, full_lat)
    got = out[crop[1] - region[1]:crop[1] - region[1] + 24, crop[0] - region[0]:crop[0] - region[0] + 40]
    assert np.array_equal(cold_h, got.cpu().numpy())
