"""The C-ABI library: loads, exports every declared symbol, host-only logic
(no GPU needed)."""
import os
import re

import pytest
from hypothesis import given, settings, strategies as st

from oracle import windows as wn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _td():
    from paper_2512_08309_amd import td
    return td


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "td.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(td_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    td = _td()
    decl = declared_symbols()
    assert len(decl) >= 16
    assert sorted(td.EXPORTS) == decl
    for name in decl:
        assert hasattr(td.lib, name), name


@settings(max_examples=300, deadline=None)
@given(x0=st.integers(-2 ** 30, 2 ** 30), y0=st.integers(-2 ** 30, 2 ** 30), w=st.integers(1, 300),
       h=st.integers(1, 300), H=st.integers(1, 80), s=st.integers(1, 90), o=st.integers(-100, 100))
def test_kappa_matches_oracle(x0, y0, w, h, H, s, o):
    td = _td()
    k = wn.kappa((x0, y0, w, h), H, s, o)
    got = td.td_kappa(x0, y0, w, h, H, s, o)
    if k is None:
        assert got is None
    else:
        assert got == (k[0][0], k[0][1], k[1][0], k[1][1])


@pytest.mark.parametrize("region,level,K,H,s", [
    ((0, 0, 64, 64), 0, 8, 32, 16), ((5, -7, 64, 64), 0, 8, 32, 16), ((13, -1000001, 1024, 1024), 0, 20, 64, 32),
    ((-1000003, 999983, 64, 64), 0, 8, 32, 16), ((3, 9, 128, 128), 0, 8, 32, 16), ((0, 0, 7, 3), 5, 8, 32, 16),
    ((10, 0, 5, 5), 0, 4, 8, 20)])
def test_cone_counts_match_oracle(region, level, K, H, s):
    td = _td()
    assert td.td_cone_windows(*region, level, K, H, s) == wn.cone_window_count(region, level, K, H, s)


def test_argument_errors_without_device():
    td = _td()
    with pytest.raises(td.TDError):
        td.td_cone_windows(0, 0, 0, 5, 0, 8, 32, 16)
    assert td.td_last_error(None) == ""
    assert td.lib.td_sample_region(None, 0, 0, 0, 1, 1, 0, None, 0) == td.TD_E_INVAL
    assert td.lib.td_cache_clear(None) == td.TD_E_INVAL
    assert td.lib.td_set_conditioning(None, None) == td.TD_E_INVAL
    assert td.lib.td_denoise_windows(None, None, None, 0, 0, None) == td.TD_E_INVAL


def test_create_fails_cleanly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    td = _td()
    with pytest.raises(td.TDError):
        td.td_create(0)


def test_stream_argument_mapping():
    """None stays NULL (the call's own default); torch's default stream
    (handle 0) becomes TD_STREAM_DEFAULT, not NULL; other handles pass."""
    from paper_2512_08309_amd import td

    class S:
        def __init__(self, h):
            self.cuda_stream = h

    assert td._stream(None) is None
    assert td._stream(S(0)).value == td.TD_STREAM_DEFAULT == 1
    assert td._stream(S(0x7f00aa00)).value == 0x7f00aa00
    assert td._stream(0x1234).value == 0x1234


def test_device_buffer_arguments_refuse_host_memory():
    """A host array or CPU tensor never reaches the library as a device
    address: the binding raises before the call."""
    import numpy as np
    import torch
    from paper_2512_08309_amd import td
    for bad in (torch.zeros(16), np.zeros(16, dtype=np.float32), [0.0] * 16):
        with pytest.raises(ValueError):
            td._dev(bad, "buf")
    with pytest.raises(ValueError):
        td.td_noise_region(1, 0, 0, torch.zeros((4, 4, 1)))


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library the binding raises instead of falling back
    to anything else (there is no CPU path)."""
    from paper_2512_08309_amd import td
    monkeypatch.setattr(td, "LIB_PATH", str(tmp_path / "libtd.so"))
    with pytest.raises(ImportError, match="not built"):
        td._load()
