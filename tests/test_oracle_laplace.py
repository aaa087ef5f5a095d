"""Pins of the oracle Laplacian decode / encode (no GPU)."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import laplace as L

DEC = {"factor": 8, "sigma_low": 20.0, "sigma_res": 2.0, "blur_sigma": 5.0, "blur_radius": 15}


def _latent_for(out_region, fill):
    lx0, ly0, lw, lh = L.required_latent(out_region, DEC)
    X, Y = np.meshgrid(np.arange(lx0, lx0 + lw), np.arange(ly0, ly0 + lh))
    return fill(X, Y), (lx0, ly0)


def test_apron_is_17_latent_pixels():
    assert L.required_latent((0, 0, 8192, 8192), DEC) == (-17, -17, 1058, 1058)
    assert L.required_latent((-5, 3, 1, 1), DEC)[2] == 34   # 2 bilinear taps + 2 x 16


def test_constant_low_band_decodes_to_constant():
    out = (-37, 101, 45, 30)
    lat = np.zeros(L.required_latent(out, DEC)[3:1:-1] + (4,))
    lat[..., 0] = 1.7
    lx0, ly0 = L.required_latent(out, DEC)[:2]
    e = L.decode(lat, (lx0, ly0), out, DEC)
    assert np.allclose(e, (20.0 * 1.7) ** 2, rtol=1e-12)


def test_planar_low_band_is_reproduced():
    out = (16, -40, 50, 33)
    a, bx, by = 0.3, 0.01, -0.02
    lat3, org = _latent_for(out, lambda X, Y: a + bx * X + by * Y)
    lat = np.zeros(lat3.shape + (1,))
    lat[..., 0] = lat3
    e = L.decode(lat, org, out, DEC)
    X = np.arange(out[0], out[0] + out[2])
    Y = np.arange(out[1], out[1] + out[3])
    xi = (X + 0.5) / 8 - 0.5
    yi = (Y + 0.5) / 8 - 0.5
    z = 20.0 * (a + bx * xi[None, :] + by * yi[:, None])
    assert np.allclose(e, np.sign(z) * z * z, rtol=1e-10, atol=1e-9)


def test_down_up_is_161_filter():
    g = np.random.default_rng(0).standard_normal((12, 14))
    full = L.up8(g, (0, 0), (8, 8, 8 * 12, 8 * 10), 8)   # blocks 1..12 x 1..10 need 0..13 x 0..11
    d = L.down8(full, 8)
    k = np.array([1.0, 6.0, 1.0]) / 8
    ref = ndimage.correlate1d(ndimage.correlate1d(g, k, axis=0), k, axis=1)
    assert np.allclose(d, ref[1:11, 1:13], rtol=1e-12, atol=1e-12)


def test_blur_matches_scipy_gaussian_filter():
    g = np.random.default_rng(1).standard_normal((60, 70))
    mine = L.blur_valid(g, L.gaussian_taps(5.0, 15))
    ref = ndimage.gaussian_filter(g, sigma=5.0, truncate=3.0)
    assert np.allclose(mine, ref[15:-15, 15:-15], rtol=1e-12, atol=1e-12)


def test_atoms_orthonormal_zero_mean():
    A = np.stack([a.ravel() for a in L.atoms(8)])
    assert np.allclose(A @ A.T, np.eye(3), atol=1e-14)
    assert np.allclose(A.sum(axis=1), 0, atol=1e-14)
    assert np.allclose(A @ np.full(64, 1 / 8), 0, atol=1e-14)


def test_encode_recovers_residual_of_decode():
    out = (0, 0, 8 * 40, 8 * 40)
    lx0, ly0, lw, lh = L.required_latent(out, DEC)
    rng = np.random.default_rng(2)
    lat = np.zeros((lh, lw, 4))
    lat[..., 0] = 2.5
    lat[..., 1:] = rng.standard_normal((lh, lw, 3))
    e = L.decode(lat, (lx0, ly0), out, DEC)
    enc, (ox, oy) = L.encode(e, out, DEC, 4)
    sub = lat[oy - ly0:oy - ly0 + enc.shape[0], ox - lx0:ox - lx0 + enc.shape[1]]
    assert np.allclose(enc, sub, rtol=1e-9, atol=1e-9)


def test_signed_sqrt_pair():
    h = np.array([-8000.0, -1.0, 0.0, 0.25, 123.4])
    assert np.allclose(L.signed_square(L.signed_sqrt(h)), h, rtol=1e-15)


def test_laplacian_denoising_attenuates_low_band_noise():
    # white noise on L: the re-extracted low band keeps only what the blur
    # passes; the output differs from the clean decode far less than P does.
    out = (0, 0, 8 * 48, 8 * 48)
    lx0, ly0, lw, lh = L.required_latent(out, DEC)
    rng = np.random.default_rng(3)
    clean = np.zeros((lh, lw, 1))
    clean[..., 0] = 3.0
    noisy = clean.copy()
    noisy[..., 0] += 0.05 * rng.standard_normal((lh, lw))
    z0 = np.sqrt(L.decode(clean, (lx0, ly0), out, DEC))
    z1 = np.sqrt(L.decode(noisy, (lx0, ly0), out, DEC))
    p_err = 20.0 * 0.05
    assert np.std(z1 - z0) < 0.1 * p_err
