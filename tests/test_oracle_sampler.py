"""Pins of the oracle sampler (no GPU): closed form, Eq. 1 vs Eq. 2, crops."""
import math

import numpy as np
import pytest

from oracle import noise, schedule
from oracle.sampler import Model, sample
from oracle.unet import prior_mean
from oracle import windows as wn


def test_schedule_values_k8():
    s = schedule.sigmas(8, 80.0, 0.002, 7.0)
    want = [80, 34.99219, 13.69857, 4.63707, 1.28661, 0.26748, 0.03519, 0.002, 0]
    assert np.allclose(s, want, rtol=0, atol=5.1e-6)  # printed to 5 decimals
    assert all(a > b for a, b in zip(s, s[1:]))


def test_euler_product_converges_to_ode_solution():
    # dx/dsigma = (x - D)/sigma with the linear-Gaussian D has the exact
    # solution (x - mu) ~ sqrt(s^2 + sigma^2): the Euler product must approach
    # s / sqrt(s^2 + sigma_0^2) at first order in 1/K.
    s, smax = 0.5, 80.0
    exact = s / math.sqrt(s * s + smax * smax)
    errs = []
    for K in (50, 100, 200, 400):
        sig = schedule.sigmas(K, smax, 0.002, 7.0)
        p = 1.0
        for k in range(K):
            p *= 1 + (sig[k + 1] - sig[k]) * sig[k] / (s * s + sig[k] ** 2)
        errs.append(abs(p - exact) / exact)
    assert errs[-1] < 0.02
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(1.6 < r < 2.5 for r in ratios)


def brute_mu_bar(x, y, c, H, s, o, eps):
    w1 = wn.weight_1d(H, eps)
    num = den = 0.0
    for iy in range((y - o) // s - H // s - 2, (y - o) // s + 2):
        for ix in range((x - o) // s - H // s - 2, (x - o) // s + 2):
            ox, oy = ix * s + o, iy * s + o
            if ox <= x < ox + H and oy <= y < oy + H:
                wgt = w1[x - ox] * w1[y - oy]
                num += wgt * prior_mean(ix, iy, c)
                den += wgt
    return num / den


@pytest.mark.parametrize("config,seed,x0,y0,level", [("lg", 0, 0, 0, 0), ("lg", 1, -37, 1000003, 0),
                                                    ("lg", 5, 3, -4, 3), ("lgt2", 2, -9, 40, 0),
                                                    ("lgt2", 3, 100, -70, 1)])
def test_linear_gaussian_closed_form(weights, config, seed, x0, y0, level):
    m = Model(weights(config))
    w, h = 23, 17
    got = sample(m, seed, x0, y0, w, h, level)
    sp = m.header["sampler"]
    sig = schedule.sigmas(m.steps, sp["sigma_max"], sp["sigma_min"], sp["rho"])
    sd = m.header["denoiser"]["prior_std"]
    prod = 1.0
    # every window is affine in its input, so any blend schedule gives the
    # same closed form over the steps run up to the level's blend point
    for k in range(m.points[m.K - level]):
        prod *= 1 + (sig[k + 1] - sig[k]) * sig[k] / (sd * sd + sig[k] ** 2)
    g = noise.noise_region(seed, x0, y0, w, h, m.C).astype(np.float64)
    for (yy, xx, c) in [(0, 0, 0), (h - 1, w - 1, 3), (5, 11, 1), (16, 2, 2), (8, 8, 0)]:
        mu = brute_mu_bar(x0 + xx, y0 + yy, c, m.H, m.s, m.o, m.eps)
        want = mu + (sig[0] * g[yy, xx, c] - mu) * prod
        assert got[yy, xx, c] == pytest.approx(want, rel=1e-12, abs=1e-12)


def bounded_multidiffusion(m, seed, canvas, level):
    """Eq. 1 on a finite canvas: every window that lies inside the canvas."""
    X0, Y0, WW, HH = canvas
    j = m.sched[0] * noise.noise_region(seed, X0, Y0, WW, HH, m.C).astype(np.float64)
    wins = [(ix, iy) for iy in range(-(-(Y0 - m.o) // m.s), (Y0 + HH - m.H - m.o) // m.s + 1)
            for ix in range(-(-(X0 - m.o) // m.s), (X0 + WW - m.H - m.o) // m.s + 1)]
    for t in range(m.K - 1, level - 1, -1):
        xs = np.stack([j[iy * m.s + m.o - Y0:iy * m.s + m.o - Y0 + m.H,
                         ix * m.s + m.o - X0:ix * m.s + m.o - X0 + m.H] for ix, iy in wins])
        phi = xs
        for k in schedule.level_steps(m.points, t):
            sig, sig_n = m.sched[k], m.sched[k + 1]
            phi = phi + (sig_n - sig) / sig * (phi - m.denoiser(phi, sig, wins))
        A = np.zeros_like(j)
        B = np.zeros(j.shape[:2] + (1,))
        for n, (ix, iy) in enumerate(wins):
            oy, ox = iy * m.s + m.o - Y0, ix * m.s + m.o - X0
            A[oy:oy + m.H, ox:ox + m.H] += m.W[:, :, None] * phi[n]
            B[oy:oy + m.H, ox:ox + m.H] += m.W[:, :, None]
        j = np.where(B > 0, A / np.where(B > 0, B, 1), 0.0)
    return j


@pytest.mark.parametrize("config,region", [("lg", (-5, 9, 13, 7)), ("c1k2", (3, -5, 20, 12)),
                                           ("c1t2", (-7, 2, 9, 11))])
def test_lazy_equals_bounded_multidiffusion(weights, config, region):
    m = Model(weights(config))
    regions, _ = wn.cone(region, 0, m.K, m.H, m.s, m.o)
    rK = regions[m.K]
    canvas = (rK[0] - m.s, rK[1] - 2 * m.s, rK[2] + 3 * m.s, rK[3] + 2 * m.s)
    full = bounded_multidiffusion(m, 4, canvas, 0)
    x0, y0, w, h = region
    want = full[y0 - canvas[1]:y0 - canvas[1] + h, x0 - canvas[0]:x0 - canvas[0] + w]
    got = sample(m, 4, x0, y0, w, h, 0)
    assert np.allclose(got, want, rtol=1e-11, atol=1e-11)


def test_crop_independence_unet(weights):
    m = Model(weights("c1k2"))
    big = sample(m, 7, -20, 30, 40, 24, 0)
    small = sample(m, 7, -11, 37, 9, 13, 0)
    assert np.allclose(small, big[7:20, 9:18], rtol=1e-12, atol=1e-12)
    # query order does not matter either: evaluate in the other order
    again = sample(m, 7, -20, 30, 40, 24, 0)
    assert np.array_equal(again, big)


def test_noise_level_and_zero_rule(weights):
    m = Model(weights("lg"))
    z = sample(m, 3, -4, 8, 5, 6, m.K)
    assert np.allclose(z, 80.0 * noise.noise_region(3, -4, 8, 5, 6, m.C))
    # a layout with gaps (stride > size): uncovered pixels are 0 (0/0 := 0)
    hdr = dict(m.header)
    hdr["window"] = {"size": 8, "stride": 20, "offset": 0, "eps": 0.01}
    gap = Model(hdr)
    out = sample(gap, 3, 0, 0, 40, 4, 0)
    assert np.all(out[:, 8:20] == 0) and np.all(out[:, 28:40] == 0)
    assert np.all(out[:, 0:8] != 0)
    assert np.all(sample(gap, 3, 10, 0, 5, 5, 0) == 0)


def test_blend_schedule_validation_and_levels():
    assert schedule.blend_points({"steps": 4}) == [0, 1, 2, 3, 4]
    assert schedule.blend_points({"steps": 8, "blend": [0, 4, 8]}) == [0, 4, 8]
    for bad in ([1, 8], [0, 5], [0, 4, 4, 8]):
        with pytest.raises(ValueError):
            schedule.blend_points({"steps": 8, "blend": bad})
    pts = [0, 4, 8]
    assert schedule.level_steps(pts, 1) == [0, 1, 2, 3] and schedule.level_steps(pts, 0) == [4, 5, 6, 7]


def test_truncated_t_cone_is_smaller(weights):
    full, trunc = Model(weights("c1")), Model(weights("c1t2"))
    region = (0, 0, 64, 64)
    n_full = wn.cone_window_count(region, 0, full.K, full.H, full.s)
    n_trunc = wn.cone_window_count(region, 0, trunc.K, trunc.H, trunc.s)
    assert (full.K, trunc.K) == (8, 2) and n_trunc < n_full / 5
