"""Laplacian decode / encode of a terrain latent (Sec. 5.2) and the signed
square-root pair (Sec. 5.1 and its appendix).

TEST INFRASTRUCTURE (oracle).  Reading used (the paper fixes the 8x factor
and the sigma = 5 blur, not the interpolation or the residual decoder):

* Latent J_0 with C channels: L = sigma_L J_0[0] (low band, signed-sqrt
  metres); r_k = sigma_r J_0[k], k = 1..min(C-1, 3), drive the residual.
* up8: bilinear with half-pixel centres, xi = (X + 0.5)/8 - 0.5.
* down8: mean over each 8x8 block.
* G5: separable Gaussian at latent resolution, sigma 5, radius 15, taps
  normalised to sum 1.
* Residual stand-in for the learned consistency decoder (out of scope):
  H(X, Y) = sum_k r_k(X div 8, Y div 8) beta_k(X mod 8, Y mod 8) with the
  orthonormal 8x8 DCT-II atoms (1,0), (0,1), (1,1) (first index along x).
* Decode: P = up8(L) + H, L_hat = G5 * down8(P), z = up8(L_hat) + H,
  elevation = sign(z) z^2 (the text's "L_hat + H" read as up8(L_hat) + H).
* Encode (for synthetic inputs): z = sign(h) sqrt|h|, L = G5 * down8(z),
  r_k = <z - up8(L), beta_k> per block.
* The domain is unbounded: there is no padding.  A decode of a full-res
  region needs the latent on an apron of 17 latent pixels on each side
  (1 for up8, 15 for the blur, 1 for the up8 inside P).

Pins (tests/test_oracle_laplace.py): constant and planar low bands are
reproduced exactly; down8 o up8 equals the [1, 6, 1]/8 filter; the blur
equals scipy.ndimage.gaussian_filter1d (truncate 3); the atoms are
orthonormal and zero-mean; encode recovers the residual coefficients of a
decode; the signed square-root pair inverts.
"""
import numpy as np


def signed_sqrt(h):
    return np.sign(h) * np.sqrt(np.abs(h))


def signed_square(z):
    return np.sign(z) * z * z


def gaussian_taps(sigma, radius):
    j = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-0.5 * (j / sigma) ** 2)
    return g / g.sum()


def dct_1d(factor=8):
    n = np.arange(factor, dtype=np.float64)
    b0 = np.full(factor, 1.0 / np.sqrt(factor))
    b1 = np.sqrt(2.0 / factor) * np.cos(np.pi * (2 * n + 1) / (2 * factor))
    return b0, b1


def atoms(factor=8):
    """beta_k[Y mod f, X mod f] for k = 1, 2, 3: DCT atoms (1,0), (0,1), (1,1)."""
    b0, b1 = dct_1d(factor)
    return [np.outer(b0, b1), np.outer(b1, b0), np.outer(b1, b1)]


def up_axis(grid, grid_lo, X_lo, n, factor, axis):
    """Bilinear half-pixel upsampling along one axis of `grid` (latent index
    grid_lo at position 0) onto full-res coordinates X_lo..X_lo+n-1."""
    X = np.arange(X_lo, X_lo + n, dtype=np.int64)
    num = 2 * X + 1 - factor
    i0 = num // (2 * factor)
    frac = (num - i0 * 2 * factor) / (2.0 * factor)
    a = np.take(grid, i0 - grid_lo, axis=axis)
    b = np.take(grid, i0 + 1 - grid_lo, axis=axis)
    shape = [1] * grid.ndim
    shape[axis] = n
    frac = frac.reshape(shape)
    return (1.0 - frac) * a + frac * b


def up_range(X_lo, n, factor):
    """Latent indices [lo, hi] read by up8 for full-res X_lo..X_lo+n-1."""
    lo = (2 * X_lo + 1 - factor) // (2 * factor)
    hi = (2 * (X_lo + n - 1) + 1 - factor) // (2 * factor) + 1
    return lo, hi


def up8(grid, lo_xy, out_region, factor):
    """grid [ly, lx] with latent origin lo_xy=(lx0, ly0) -> full-res [H, W]."""
    X0, Y0, W, Hh = out_region
    g = up_axis(grid, lo_xy[1], Y0, Hh, factor, axis=0)
    return up_axis(g, lo_xy[0], X0, W, factor, axis=1)


def residual(r, lo_xy, out_region, factor):
    """H on a full-res region from residual coefficients r [ly, lx, k] (k = 0..2)."""
    X0, Y0, W, Hh = out_region
    X = np.arange(X0, X0 + W)
    Y = np.arange(Y0, Y0 + Hh)
    out = np.zeros((Hh, W))
    for k, beta in enumerate(atoms(factor)[:r.shape[-1]]):
        rk = r[(Y // factor - lo_xy[1])[:, None], (X // factor - lo_xy[0])[None, :], k]
        out += rk * beta[(Y % factor)[:, None], (X % factor)[None, :]]
    return out


def down8(full, factor):
    Hh, W = full.shape
    return full.reshape(Hh // factor, factor, W // factor, factor).mean(axis=(1, 3))


def blur_valid(grid, taps):
    """Separable 'valid' correlation: output shrinks by the radius on each side."""
    r = len(taps) // 2
    n0, n1 = grid.shape
    tmp = sum(taps[j] * grid[j:n0 - 2 * r + j, :] for j in range(2 * r + 1))
    return sum(taps[j] * tmp[:, j:n1 - 2 * r + j] for j in range(2 * r + 1))


def required_latent(out_region, dec):
    """Latent region (lx0, ly0, lw, lh) a decode of out_region reads."""
    f, R = dec["factor"], dec["blur_radius"]
    X0, Y0, W, Hh = out_region
    xl, xh = up_range(X0, W, f)
    yl, yh = up_range(Y0, Hh, f)
    xl, yl = min(xl, X0 // f) - R - 1, min(yl, Y0 // f) - R - 1
    xh, yh = max(xh, (X0 + W - 1) // f) + R + 1, max(yh, (Y0 + Hh - 1) // f) + R + 1
    return xl, yl, xh - xl + 1, yh - yl + 1


def decode(latent, lat_origin, out_region, dec):
    """Elevation (metres) on out_region from latent [lh, lw, C] at lat_origin."""
    f, R = dec["factor"], dec["blur_radius"]
    C = latent.shape[-1]
    need = required_latent(out_region, dec)
    lx0, ly0 = lat_origin
    lh, lw = latent.shape[:2]
    if need[0] < lx0 or need[1] < ly0 or need[0] + need[2] > lx0 + lw or need[1] + need[3] > ly0 + lh:
        raise ValueError("latent does not cover the decode apron")
    L = dec["sigma_low"] * latent[..., 0]
    r = dec["sigma_res"] * latent[..., 1:min(C, 4)]
    X0, Y0, W, Hh = out_region
    xl, xh = up_range(X0, W, f)
    yl, yh = up_range(Y0, Hh, f)
    # down8(P) on latent blocks [xl-R, xh+R] x [yl-R, yh+R]
    bx0, by0 = xl - R, yl - R
    bw, bh = xh + R - bx0 + 1, yh + R - by0 + 1
    P_region = (bx0 * f, by0 * f, bw * f, bh * f)
    P = up8(L, lat_origin, P_region, f) + residual(r, lat_origin, P_region, f)
    Lhat = blur_valid(down8(P, f), gaussian_taps(dec["blur_sigma"], R))   # blocks [xl, xh] x [yl, yh]
    z = up8(Lhat, (xl, yl), out_region, f) + residual(r, lat_origin, out_region, f)
    return signed_square(z)


def encode(height, region, dec, channels):
    """Latent [lh, lw, channels] and its latent origin from an 8-aligned
    full-res elevation field on region (X0, Y0, W, H)."""
    f, R = dec["factor"], dec["blur_radius"]
    X0, Y0, W, Hh = region
    if X0 % f or Y0 % f or W % f or Hh % f:
        raise ValueError("encode needs an 8-aligned region")
    z = signed_sqrt(height)
    L = blur_valid(down8(z, f), gaussian_taps(dec["blur_sigma"], R))
    Lx0, Ly0 = X0 // f + R, Y0 // f + R
    ox0, oy0 = Lx0 + 1, Ly0 + 1
    ow, oh = L.shape[1] - 2, L.shape[0] - 2
    out_region = (ox0 * f, oy0 * f, ow * f, oh * f)
    zz = z[oy0 * f - Y0:(oy0 + oh) * f - Y0, ox0 * f - X0:(ox0 + ow) * f - X0]
    res = zz - up8(L, (Lx0, Ly0), out_region, f)
    lat = np.zeros((oh, ow, channels))
    lat[..., 0] = L[1:-1, 1:-1] / dec["sigma_low"]
    blocks = res.reshape(oh, f, ow, f)
    for k, beta in enumerate(atoms(f)[:channels - 1]):
        lat[..., k + 1] = np.einsum("yixj,ij->yx", blocks, beta) / dec["sigma_res"]
    return lat, (ox0, oy0)
