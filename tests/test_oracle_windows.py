"""Pins of the oracle's window indexing (no GPU)."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import windows as wn


def brute_kappa(region, H, s, o):
    x0, y0, w, h = region
    out = []
    for iy in range((y0 - o - H) // s - 2, (y0 + h - o) // s + 3):
        for ix in range((x0 - o - H) // s - 2, (x0 + w - o) // s + 3):
            ox, oy = ix * s + o, iy * s + o
            if ox < x0 + w and ox + H > x0 and oy < y0 + h and oy + H > y0:
                out.append((ix, iy))
    return out


@settings(max_examples=400, deadline=None)
@given(x0=st.integers(-10 ** 6, 10 ** 6), y0=st.integers(-10 ** 6, 10 ** 6),
       w=st.integers(1, 70), h=st.integers(1, 70),
       H=st.integers(1, 40), s=st.integers(1, 45), o=st.integers(-50, 50))
def test_kappa_equals_brute_force(x0, y0, w, h, H, s, o):
    assert wn.kappa_list((x0, y0, w, h), H, s, o) == brute_kappa((x0, y0, w, h), H, s, o)


def test_kappa_empty_between_windows():
    # s > H leaves gaps: a region inside a gap meets no window.
    assert wn.kappa((10, 0, 5, 1), 8, 20, 0) is None
    assert wn.kappa_list((10, 0, 5, 1), 8, 20, 0) == []


@pytest.mark.parametrize("region,K,H,s,count", [
    ((0, 0, 64, 64), 8, 32, 16, 1320),
    ((5, -7, 64, 64), 8, 32, 16, 1520),
    ((13, -1000001, 1024, 1024), 20, 64, 32, 58840),
])
def test_cone_counts(region, K, H, s, count):
    assert wn.cone_window_count(region, 0, K, H, s) == count


def test_cone_regions_cover_window_inputs():
    regions, kappas = wn.cone((3, -9, 40, 21), 0, 5, 32, 16)
    for t in range(5):
        for ix, iy in wn.kappa_list(regions[t], 32, 16):
            x, y = wn.window_origin(ix, iy, 16)
            rx, ry, rw, rh = regions[t + 1]
            assert rx <= x and x + 32 <= rx + rw and ry <= y and y + 32 <= ry + rh


def test_cone_brute_force_small():
    # level by level: brute-force windows meeting R_t, hull of them = R_{t+1}
    H, s, K = 6, 4, 4
    region = (-3, 2, 5, 3)
    regions, _ = wn.cone(region, 0, K, H, s)
    r = region
    for t in range(K):
        ws = brute_kappa(r, H, s, 0)
        xs = [ix * s for ix, _ in ws]
        ys = [iy * s for _, iy in ws]
        r = (min(xs), min(ys), max(xs) + H - min(xs), max(ys) + H - min(ys))
        assert regions[t + 1] == r


def test_weight_map_shape_and_values():
    H, eps = 32, 0.01
    w = wn.weight_1d(H, eps)
    assert w[0] == pytest.approx(eps) and w[-1] == pytest.approx(eps)
    assert np.allclose(w, w[::-1])
    assert w.max() == pytest.approx(1 - (1 - eps) / (H - 1))
    assert np.all(np.diff(w[:H // 2]) > 0)
    W = wn.weight_map(H, eps)
    assert W.shape == (H, H) and np.allclose(W, np.outer(w, w))
