"""Sliding-window layout, kappa and window weights.

TEST INFRASTRUCTURE (oracle).

* Window i = (ix, iy) covers [ix*s + o, ix*s + o + H) x [iy*s + o, iy*s + o + H)
  (Sec. 3.2, square sliding windows; offset o as in the window-range
  algorithm of the formal appendix).  x is the column, y the row.
* kappa(R) for R = [a, b) per axis is the window-range algorithm of the
  formal appendix: i_min = ceil((a - o - H + 1) / s), i_max = floor((b - 1 - o) / s),
  empty if i_min > i_max on any axis.  Python integer // is mathematical
  floor, so negative coordinates are handled exactly.
* Weight map: separable linear window (Sec. 6, results setup) falling from 1
  at the centre to eps at the border: w(u) = eps + (1-eps)(1 - |2u-(H-1)|/(H-1)),
  W(u, v) = w(u) w(v), in float64.

Pins: kappa against brute-force enumeration of all windows in a box around R
(tests/test_oracle_windows.py); the weight map against its end values and
symmetry.
"""
import numpy as np


def ceil_div(a, b):
    return -((-a) // b)


def kappa_axis(a, b, size, stride, offset):
    """Inclusive window-index range [i_min, i_max] meeting pixel range [a, b)."""
    i_min = ceil_div(a - offset - size + 1, stride)
    i_max = (b - 1 - offset) // stride
    return i_min, i_max


def kappa(region, size, stride, offset=0):
    """kappa(R) as ((ix_min, ix_max), (iy_min, iy_max)) or None when empty.

    region = (x0, y0, w, h) meaning [x0, x0+w) x [y0, y0+h)."""
    x0, y0, w, h = region
    if w <= 0 or h <= 0:
        return None
    ix = kappa_axis(x0, x0 + w, size, stride, offset)
    iy = kappa_axis(y0, y0 + h, size, stride, offset)
    if ix[0] > ix[1] or iy[0] > iy[1]:
        return None
    return ix, iy


def kappa_list(region, size, stride, offset=0):
    """Windows of kappa(R) in canonical order: iy ascending, then ix ascending."""
    k = kappa(region, size, stride, offset)
    if k is None:
        return []
    (ix0, ix1), (iy0, iy1) = k
    return [(ix, iy) for iy in range(iy0, iy1 + 1) for ix in range(ix0, ix1 + 1)]


def window_origin(ix, iy, stride, offset=0):
    return ix * stride + offset, iy * stride + offset


def hull_of_windows(k, size, stride, offset=0):
    """Bounding region (x0, y0, w, h) of the union of windows in kappa range k."""
    (ix0, ix1), (iy0, iy1) = k
    x0 = ix0 * stride + offset
    y0 = iy0 * stride + offset
    return (x0, y0, (ix1 - ix0) * stride + size, (iy1 - iy0) * stride + size)


def weight_1d(size, eps):
    u = np.arange(size, dtype=np.float64)
    if size == 1:
        return np.ones(1)
    return eps + (1.0 - eps) * (1.0 - np.abs(2.0 * u - (size - 1)) / (size - 1))


def weight_map(size, eps):
    """W[v, u] = w(v) * w(u), row v, column u."""
    w = weight_1d(size, eps)
    return w[:, None] * w[None, :]


def cone(region, t_query, steps, size, stride, offset=0):
    """Per-level regions and window ranges of a query's dependency cone.

    Returns (regions, kappas): regions[t] for t = t_query..steps, kappas[t] for
    t = t_query..steps-1 (None if empty; then every deeper level is empty too).
    regions[t+1] is the bounding region of all windows of kappas[t]."""
    regions = {t_query: region}
    kappas = {}
    for t in range(t_query, steps):
        k = kappa(regions[t], size, stride, offset)
        kappas[t] = k
        if k is None:
            regions[t + 1] = None
            for u in range(t + 1, steps):
                kappas[u] = None
                regions[u + 1] = None
            break
        regions[t + 1] = hull_of_windows(k, size, stride, offset)
    return regions, kappas


def cone_window_count(region, t_query, steps, size, stride, offset=0):
    """Number of Phi evaluations a cold query needs: sum over levels of |kappa(R_t)|."""
    _, kappas = cone(region, t_query, steps, size, stride, offset)
    n = 0
    for t in range(t_query, steps):
        k = kappas[t]
        if k is not None:
            n += (k[0][1] - k[0][0] + 1) * (k[1][1] - k[1][0] + 1)
    return n
