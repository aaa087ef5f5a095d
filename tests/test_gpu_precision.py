"""Reduced precision (BF16 convolution operands, FP32 accumulation; FP8-e4m3
weights with per-output-channel FP32 scales) against the FP64 oracle.

Every mode is held to the precision target of the workload (relative error
<= 2e-2).  BF16 meets it.  FP8-e4m3 weights do not on these random-init
networks (measured 4.2e-2 to 7.0e-2 per denoiser, 5.7e-2 at J_0 of the
128x128 crop): those cases are strict expected failures that name the
measured error.  Separate tests named as regression guards hold the FP8
mode to the level it measures (8e-2), so a further loss of accuracy still
fails.  The tests print the measured errors so they can be quoted.
"""
import numpy as np
import pytest

from gpu_common import planar, rel_l2, require_gpu
from oracle import laplace
from oracle.sampler import Model, sample_levels

pytestmark = pytest.mark.gpu

DEC = {"factor": 8, "sigma_low": 20.0, "sigma_res": 2.0, "blur_sigma": 5.0, "blur_radius": 15}


@pytest.fixture(scope="module")
def lp_ctx(weights):
    require_gpu()
    from paper_2512_08309_amd import td
    made = {}

    def get(config, precision):
        key = (config, precision)
        if key not in made:
            c = td.Context(0).load_weights(weights(config))
            c.set_option("precision", precision)
            assert c.info("precision") == precision
            made[key] = c
        return made[key]
    yield get
    for c in made.values():
        c.close()


# The workload's target: relative error vs the FP64 oracle <= 2e-2.
TARGET = 2e-2
# Regression guard of the FP8-weight mode: the level it measures (e4m3 has 3
# mantissa bits), not a precision claim.
FP8_GUARD = 8e-2
FP8_MISS = pytest.mark.xfail(strict=True, reason="FP8-e4m3 weights miss the 2e-2 target on these random-init "
                             "networks: measured 4.2e-2 to 7.0e-2 per denoiser, 5.7e-2 at J_0 of the 128x128 "
                             "C1 crop, 1.4e-1 heightfield on the 8192^2 query")
PRECS = [1, pytest.param(2, marks=FP8_MISS)]
DENOISER_CASES = [("c1", 0, 8), ("c1", 5, 8), ("c2", 0, 2), ("c2", 15, 2), ("cc", 0, 4), ("cc", 6, 4)]


def _denoiser_error(lp_ctx, weights, config, k, n, prec):
    import torch
    from oracle.tdw import read_tdw
    from oracle.unet import UNetDenoiser
    c = lp_ctx(config, prec)
    hdr, t = read_tdw(weights(config))
    m = Model(weights(config))
    H, C = m.H, m.C
    x = (m.sched[k] * np.random.default_rng(20 + k).standard_normal((n, H, H, C))).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    out = torch.empty_like(xd)
    c.denoise_windows(xd, k, out)
    ref = UNetDenoiser(hdr, t)(x.astype(np.float64), m.sched[k], None)
    err = rel_l2(out.cpu().numpy(), ref)
    print("precision %d denoiser %s sigma_%d rel L2 %.3e" % (prec, config, k, err))
    return err


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("config,k,n", DENOISER_CASES)
def test_lowp_denoiser_close_to_oracle(lp_ctx, weights, config, k, n, prec):
    assert _denoiser_error(lp_ctx, weights, config, k, n, prec) <= TARGET


@pytest.mark.parametrize("config,k,n", DENOISER_CASES)
def test_fp8_weights_denoiser_regression_guard(lp_ctx, weights, config, k, n):
    assert _denoiser_error(lp_ctx, weights, config, k, n, 2) <= FP8_GUARD


_CROP_REF = {}


def _crop_errors(lp_ctx, weights, prec):
    """128x128 C1 crop at (3, 9): error of every level J_t and of the
    heightfield; the FP32 path is checked against its own bar on the way."""
    m = Model(weights("c1"))
    region = (3, 9, 128, 128)
    if "c1" not in _CROP_REF:
        _CROP_REF["c1"] = sample_levels(m, 5, *region, 0)
    ref = _CROP_REF["c1"]
    c32 = lp_ctx("c1", 0)
    c16 = lp_ctx("c1", prec)
    errs16, errs32 = {}, {}
    for t in range(m.K, -1, -1):
        r = planar(ref[t])
        errs16[t] = rel_l2(c16.sample_region(5, *region, t), r)
        errs32[t] = rel_l2(c32.sample_region(5, *region, t), r)
    print("per-level rel L2 vs FP64 oracle, precision %d:" % prec, {t: "%.2e" % e for t, e in errs16.items()})
    print("per-level rel L2 vs FP64 oracle, fp32:", {t: "%.2e" % e for t, e in errs32.items()})
    assert errs16[m.K] < 1e-7 and errs32[m.K] < 1e-7    # the noise level (FP32 rounding of sigma_0 * G)
    assert max(errs32.values()) <= 1e-4
    # heightfield of the interior (decode needs the 17 px apron inside the crop)
    out = (8 * 20, 8 * 26, 8 * 90, 8 * 90)
    lx0, ly0, lw, lh = laplace.required_latent(out, DEC)
    assert lx0 >= 3 and ly0 >= 9 and lx0 + lw <= 131 and ly0 + lh <= 137
    lat = ref[0][ly0 - 9:ly0 - 9 + lh, lx0 - 3:lx0 - 3 + lw]
    href = laplace.decode(lat, (lx0, ly0), out, DEC)
    from paper_2512_08309_amd import td
    h16 = c16.sample_region(5, *out, td.TD_LEVEL_HEIGHT)
    h32 = c32.sample_region(5, *out, td.TD_LEVEL_HEIGHT)
    e16, e32 = rel_l2(h16, href), rel_l2(h32, href)
    print("heightfield rel RMSE vs FP64 oracle: precision %d %.3e, fp32 %.3e" % (prec, e16, e32))
    assert e32 <= 1e-4
    return errs16, e16


@pytest.mark.parametrize("prec", PRECS)
def test_lowp_c1_crop_error_every_level(lp_ctx, weights, prec):
    errs, eh = _crop_errors(lp_ctx, weights, prec)
    assert max(errs.values()) <= TARGET and eh <= TARGET


def test_fp8_weights_crop_regression_guard(lp_ctx, weights):
    errs, eh = _crop_errors(lp_ctx, weights, 2)
    assert max(errs.values()) <= FP8_GUARD and eh <= FP8_GUARD


def test_bf16_seed_consistency_bit_exact(lp_ctx):
    c = lp_ctx("c1", 1)
    c.cache_clear()
    big = c.sample_region(4, 0, 0, 96, 80, 0)
    c.cache_clear()
    c.set_option("batch", 7)
    try:
        small = c.sample_region(4, 33, 21, 29, 30, 0)
    finally:
        c.set_option("batch", 4096)
    assert np.array_equal(small, big[:, 21:51, 33:62])


@pytest.mark.parametrize("prec", [0, 1])
def test_c2_window_batch_invariant_bit_exact(lp_ctx, weights, prec):
    # C2 takes most GroupNorm statistics from the producing convolution's
    # per-tile sums, and in BF16 runs every convolution on the halo-staged
    # kernel (8x8 windows share tiles four at a time): a window's estimate
    # must not depend on the other windows of its batch.
    import torch
    c = lp_ctx("c2", prec)
    m = Model(weights("c2"))
    H, C = m.H, m.C
    x = (m.sched[3] * np.random.default_rng(41).standard_normal((5, H, H, C))).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    out5 = torch.empty_like(xd)
    c.denoise_windows(xd, 3, out5)
    one = xd[2:3].contiguous()
    out1 = torch.empty_like(one)
    c.denoise_windows(one, 3, out1)
    assert np.array_equal(out5[2].cpu().numpy(), out1[0].cpu().numpy())
