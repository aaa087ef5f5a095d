"""Synthetic fBm-shaped terrain latents (decode inputs).

Value noise on an integer lattice (cell size `period` latent pixels at the
first octave), quintic interpolation, `octaves` octaves with lacunarity 2
and gain 2^-H (Hurst exponent H), normalised by the sum of gains.  Lattice
values are uniform in [-1, 1) from a splitmix64 hash of (seed, octave,
lattice x, lattice y), so any region of the infinite field is reproducible.

terrain_latent(): channel 0 is the signed-sqrt of an elevation field in
[-8000, 8000] m divided by the decode's sigma_low; channels 1..C-1 are
independent fBm fields (latent units) that drive the residual.
"""
import numpy as np

M64 = (1 << 64) - 1


def _splitmix(x):
    x = (x + np.uint64(0x9E3779B97F4A7C15)) & np.uint64(M64)
    x = ((x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & np.uint64(M64)
    x = ((x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & np.uint64(M64)
    return x ^ (x >> np.uint64(31))


def _lattice(seed, octave, X, Y):
    with np.errstate(over="ignore"):
        h = _splitmix(np.uint64(seed & M64) ^ np.uint64((octave * 0x1000193) & M64))
        h = _splitmix(h ^ (X.astype(np.int64).astype(np.uint64)))
        h = _splitmix(h ^ (Y.astype(np.int64).astype(np.uint64) * np.uint64(0x632BE59BD9B4E019)))
    return (h >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0


def _quintic(t):
    return t * t * t * (t * (t * 6 - 15) + 10)


def fbm(seed, x0, y0, w, h, octaves=6, hurst=0.8, period=256.0):
    xs = np.arange(x0, x0 + w, dtype=np.float64)[None, :]
    ys = np.arange(y0, y0 + h, dtype=np.float64)[:, None]
    out = np.zeros((h, w))
    norm = 0.0
    for o in range(octaves):
        f = (2.0 ** o) / period
        gx, gy = xs * f, ys * f
        ix, iy = np.floor(gx), np.floor(gy)
        tx, ty = _quintic(gx - ix), _quintic(gy - iy)
        ix = np.broadcast_to(ix, (h, w))
        iy = np.broadcast_to(iy, (h, w))
        v00 = _lattice(seed, o, ix, iy)
        v10 = _lattice(seed, o, ix + 1, iy)
        v01 = _lattice(seed, o, ix, iy + 1)
        v11 = _lattice(seed, o, ix + 1, iy + 1)
        a = v00 + (v10 - v00) * tx
        b = v01 + (v11 - v01) * tx
        g = 2.0 ** (-hurst * o)
        out += g * (a + (b - a) * ty)
        norm += g
    return out / norm


def terrain_latent(seed, lx0, ly0, lw, lh, channels=4, sigma_low=20.0, range_m=8000.0):
    """float32 [lh, lw, channels] latent with an fBm elevation low band."""
    lat = np.zeros((lh, lw, channels), dtype=np.float64)
    elev = range_m * np.clip(fbm(seed, lx0, ly0, lw, lh) * 1.6, -1.0, 1.0)
    lat[..., 0] = np.sign(elev) * np.sqrt(np.abs(elev)) / sigma_low
    for c in range(1, channels):
        lat[..., c] = fbm(seed * 7919 + c, lx0, ly0, lw, lh, period=32.0)
    return lat.astype(np.float32)
