"""Seed noise G(seed, x, y, c, step) for the initial image J_T.

TEST INFRASTRUCTURE (oracle).  The paper only requires G to be a deterministic
function of the seed and the pixel (formal appendix, "Seeds and initial
noise"); it gives no mechanism.  The reading used here (and by the HIP path,
written independently from the same specification) is:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
  key = (lo32(seed), hi32(seed)) and counter = (u32(x), u32(y), u32(step), c div 4).
  Its four 32-bit outputs r0..r3 feed two Box-Muller pairs: channels 4q, 4q+1
  use (r0, r1); channels 4q+2, 4q+3 use (r2, r3).
* Uniform from a word r:  u = (2*(r >> 9) + 1) * 2^-24, exact in float32, in (0, 1).
* Box-Muller (Box & Muller 1958) in float32 with every operation a single
  correctly-rounded IEEE binary32 operation and no fused multiply-add:
  rho = sqrt(-2 ln u_a), phi = 2 pi u_b, even channel rho cos(phi), odd rho sin(phi).
* ln, sin and cos are not library calls but fixed series so that two
  implementations agree bit for bit:
    ln u:  u = m 2^e with m in [sqrt(1/2), sqrt(2)), s = (m-1)/(m+1),
           ln m = 2 s (1 + s^2/3 + s^4/5 + s^6/7 + s^8/9 + s^10/11) (Horner),
           ln u = e*ln2 + ln m.
    angle: v = 4 u_b, q = rint(v), a = v - q, theta = a * (pi/2) with
           |theta| <= pi/4; Taylor sin to theta^11 and cos to theta^10
           (Horner), then rotation by the quadrant q mod 4.
  Constants are the float32 values nearest to the exact rationals, pi/2,
  ln 2 and sqrt(2).

Pins (tests/test_oracle_noise.py): the generic Philox round function is
checked against numpy's Philox4x64-10 bit generator (same round structure,
64-bit constants); the 32-bit instance used here runs through that same
function.  The series are checked against float64 ln/sin/cos within a few
float32 ulps, and the outputs against N(0,1) by moments, a KS test and the
analytic tail bound |z| <= sqrt(48 ln 2).  The 4x32 key-schedule increments
are pinned by their closed forms (golden ratio, sqrt 3 - 1), and the whole
4x32 instance (its two multipliers included) by known answers from an
independent implementation, rocRAND's host-callable Philox4x32-10 engine,
compiled by the test from its public header (over 2,000 seeds and counters,
zero and all-ones words, and G's counter layout).  This module neither
imports nor calls rocRAND.
"""
from fractions import Fraction

import numpy as np

# --- Philox, generic over the word width (Random123 round structure) --------

PHILOX4x32 = dict(width=32, mult=(0xD2511F53, 0xCD9E8D57), weyl=(0x9E3779B9, 0xBB67AE85))
PHILOX4x64 = dict(width=64, mult=(0xD2E7470EE14C6C93, 0xCA5A826395121157),
                  weyl=(0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B))


def philox_generic(ctr, key, width, mult, weyl, rounds=10):
    """One Philox4xW block on Python integers.  ctr: 4 words, key: 2 words."""
    mask = (1 << width) - 1
    x = [int(c) & mask for c in ctr]
    k = [int(c) & mask for c in key]
    for r in range(rounds):
        p0 = mult[0] * x[0]
        p1 = mult[1] * x[2]
        hi0, lo0 = p0 >> width, p0 & mask
        hi1, lo1 = p1 >> width, p1 & mask
        x = [hi1 ^ x[1] ^ k[0], lo1, hi0 ^ x[3] ^ k[1], lo0]
        k = [(k[0] + weyl[0]) & mask, (k[1] + weyl[1]) & mask]
    return x


def philox4x32_scalar(ctr, key):
    return philox_generic(ctr, key, **PHILOX4x32)


def philox4x32(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 over numpy arrays (uint64 holding 32-bit words)."""
    M0, M1 = (np.uint64(m) for m in PHILOX4x32["mult"])
    W0, W1 = (np.uint64(w) for w in PHILOX4x32["weyl"])
    mask = np.uint64(0xFFFFFFFF)
    sh = np.uint64(32)
    x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) & mask for c in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & mask
    k1 = np.asarray(k1, dtype=np.uint64) & mask
    for _ in range(10):
        p0 = M0 * x0          # < 2^64: exact in uint64
        p1 = M1 * x2
        hi0, lo0 = p0 >> sh, p0 & mask
        hi1, lo1 = p1 >> sh, p1 & mask
        x0, x1, x2, x3 = (hi1 ^ x1 ^ k0) & mask, lo1, (hi0 ^ x3 ^ k1) & mask, lo0
        k0 = (k0 + W0) & mask
        k1 = (k1 + W1) & mask
    return x0, x1, x2, x3


# --- float32 constants of the series -----------------------------------------

def _f32(v):
    """Nearest float32 to an exact value (Fraction or float)."""
    return np.float32(float(v))


F32 = np.float32
ONE = F32(1.0)
TWO_POW_M24 = F32(2.0 ** -24)
HALF_PI = F32(np.pi / 2)                      # 0x3fc90fdb
LN2 = F32(np.log(2.0))                        # 0x3f317218
SQRT2 = F32(np.sqrt(2.0))                     # 0x3fb504f3
LN_COEF = [_f32(Fraction(1, n)) for n in (11, 9, 7, 5, 3)]          # Horner order
SIN_COEF = [_f32(Fraction(-1, 39916800)), _f32(Fraction(1, 362880)), _f32(Fraction(-1, 5040)),
            _f32(Fraction(1, 120)), _f32(Fraction(-1, 6))]
COS_COEF = [_f32(Fraction(-1, 3628800)), _f32(Fraction(1, 40320)), _f32(Fraction(-1, 720)),
            _f32(Fraction(1, 24)), _f32(Fraction(-1, 2))]


def uniform_from_word(r):
    """u = (2*(r>>9)+1) * 2^-24, exactly representable in float32."""
    r = np.asarray(r, dtype=np.uint64)
    k = ((r >> np.uint64(9)) * np.uint64(2) + np.uint64(1)).astype(np.float32)  # < 2^24: exact
    return (k * TWO_POW_M24).astype(np.float32)


def ln_series(u):
    """ln u for u in (0, 1] by the specified atanh series, float32 ops only."""
    u = np.asarray(u, dtype=np.float32)
    bits = u.view(np.uint32)
    e = (bits >> np.uint32(23)).astype(np.int32) - 127
    m = ((bits & np.uint32(0x7FFFFF)) | np.uint32(0x3F800000)).view(np.float32)
    big = m >= SQRT2
    m = np.where(big, (m * F32(0.5)).astype(np.float32), m).astype(np.float32)
    e = e + big.astype(np.int32)
    s = ((m - ONE).astype(np.float32) / (m + ONE).astype(np.float32)).astype(np.float32)
    s2 = (s * s).astype(np.float32)
    p = np.full_like(s2, LN_COEF[0])
    for c in LN_COEF[1:]:
        p = ((p * s2).astype(np.float32) + c).astype(np.float32)
    p = ((p * s2).astype(np.float32) + ONE).astype(np.float32)
    t = (s * p).astype(np.float32)
    lnm = (t + t).astype(np.float32)
    return ((e.astype(np.float32) * LN2).astype(np.float32) + lnm).astype(np.float32)


def sincos_2pi(ub):
    """(sin(2 pi ub), cos(2 pi ub)) for ub in (0,1) by quadrant reduction + Taylor."""
    ub = np.asarray(ub, dtype=np.float32)
    v = (ub * F32(4.0)).astype(np.float32)
    q = np.rint(v).astype(np.float32)
    a = (v - q).astype(np.float32)
    th = (a * HALF_PI).astype(np.float32)
    t2 = (th * th).astype(np.float32)
    ps = np.full_like(t2, SIN_COEF[0])
    for c in SIN_COEF[1:]:
        ps = ((ps * t2).astype(np.float32) + c).astype(np.float32)
    ps = ((ps * t2).astype(np.float32) + ONE).astype(np.float32)
    sn = (ps * th).astype(np.float32)
    pc = np.full_like(t2, COS_COEF[0])
    for c in COS_COEF[1:]:
        pc = ((pc * t2).astype(np.float32) + c).astype(np.float32)
    cs = ((pc * t2).astype(np.float32) + ONE).astype(np.float32)
    quad = q.astype(np.int64) & 3
    sin_phi = np.select([quad == 0, quad == 1, quad == 2], [sn, cs, -sn], -cs).astype(np.float32)
    cos_phi = np.select([quad == 0, quad == 1, quad == 2], [cs, -sn, -cs], sn).astype(np.float32)
    return sin_phi, cos_phi


def box_muller(ra, rb):
    """Two standard normals (even, odd) from two 32-bit words."""
    ua = uniform_from_word(ra)
    ub = uniform_from_word(rb)
    rho = np.sqrt((F32(-2.0) * ln_series(ua)).astype(np.float32)).astype(np.float32)
    sn, cs = sincos_2pi(ub)
    return (rho * cs).astype(np.float32), (rho * sn).astype(np.float32)


def gaussian(seed, x, y, c, step):
    """G(seed, x, y, c, step): float32 standard normal, broadcast over x, y, c."""
    seed = int(seed) & ((1 << 64) - 1)
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    c = np.asarray(c, dtype=np.int64)
    x, y, c = np.broadcast_arrays(x, y, c)
    ux = x.astype(np.uint64) & np.uint64(0xFFFFFFFF)
    uy = y.astype(np.uint64) & np.uint64(0xFFFFFFFF)
    r0, r1, r2, r3 = philox4x32(ux, uy, np.uint64(int(step) & 0xFFFFFFFF),
                                (c // 4).astype(np.uint64),
                                np.uint64(seed & 0xFFFFFFFF), np.uint64(seed >> 32))
    second = ((c % 4) // 2) == 1
    ra = np.where(second, r2, r0)
    rb = np.where(second, r3, r1)
    z_even, z_odd = box_muller(ra, rb)
    return np.where((c % 2) == 1, z_odd, z_even).astype(np.float32)


def noise_region(seed, x0, y0, w, h, channels, step=0):
    """G on region [x0, x0+w) x [y0, y0+h) as float32 array [h, w, C] (x = column)."""
    ys = np.arange(y0, y0 + h, dtype=np.int64)[:, None, None]
    xs = np.arange(x0, x0 + w, dtype=np.int64)[None, :, None]
    cs = np.arange(channels, dtype=np.int64)[None, None, :]
    return gaussian(seed, xs, ys, cs, step)
