"""Edge cases of the region query through the C-ABI: degenerate shapes,
coordinates at the edge of the supported range, the maximum side and the
maximum area, and argument errors (which leave the context usable).

The linear-Gaussian model (closed-form denoiser) keeps the oracle fast; the
1-pixel case is also checked on the C1 UNet.  Regions whose cone is too big
for the oracle are checked through properties that hold at any size: finite
values and cold crop queries bit-equal to the big result.
"""
import numpy as np
import pytest

from gpu_common import planar, rel_l2, require_gpu
from oracle.sampler import Model, sample

pytestmark = pytest.mark.gpu

LIM = (1 << 31) - (1 << 22)      # |coordinate| bound of a region (exclusive)


@pytest.fixture(scope="module")
def lg(weights):
    require_gpu()
    from paper_2512_08309_amd import td
    c = td.Context(0).load_weights(weights("lg"))
    yield td, c, Model(weights("lg")), weights("lg")
    c.close()


@pytest.mark.parametrize("region", [(0, 0, 1, 1), (7, -3, 1, 97), (-50, 11, 97, 1), (31, 31, 2, 2),
                                    (-17, -17, 3, 50)])
@pytest.mark.parametrize("level", [0, 7])
def test_degenerate_shapes_match_oracle(lg, region, level):
    td, c, m, _ = lg
    got = c.sample_region(5, *region, level)
    assert got.shape == (4, region[3], region[2])
    assert rel_l2(got, planar(sample(m, 5, *region, level))) <= 1e-6


def test_single_pixel_unet_matches_oracle(weights):
    require_gpu()
    from paper_2512_08309_amd import td
    with td.Context(0) as c:
        c.load_weights(weights("c1"))
        got = c.sample_region(11, -1000003, 999983, 1, 1, 0)
    ref = planar(sample(Model(weights("c1")), 11, -1000003, 999983, 1, 1, 0))
    assert rel_l2(got, ref) <= 1e-4


@pytest.mark.parametrize("region", [(LIM - 65, 5, 64, 40), (-LIM + 1, -LIM + 1, 40, 64), (3, LIM - 2, 9, 1)])
def test_extreme_coordinates_match_oracle(lg, region):
    td, c, m, _ = lg
    got = c.sample_region(2, *region, 0)
    assert rel_l2(got, planar(sample(m, 2, *region, 0))) <= 1e-6


def test_maximum_side_and_area_at_the_top_level(lg):
    """A 2^20 x 1 strip and a 2^13 x 2^13 (2^26 px) square at level K - 1:
    finite, and cold crops on a fresh context are bit-equal to them."""
    import torch
    td, c, m, path = lg
    strip = (-(1 << 19), 77, 1 << 20, 1)
    square = (1000, -3000, 1 << 13, 1 << 13)
    outs = {}
    for r in (strip, square):
        c.cache_clear()
        out = torch.empty((4, r[3], r[2]), device="cuda")
        print("max-size query", r, flush=True)
        c.sample_region_async(8, *r, 7, out)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(out).all())
        outs[r] = out
    c.cache_clear()
    crops = [(strip, (strip[0] + 123457, 77, 300, 1)), (strip, (strip[0] + (1 << 20) - 40, 77, 40, 1)),
             (square, (1000 + 4000, -3000 + 8150, 70, 42)), (square, (1000, -3000, 33, 17))]
    with td.Context(0) as fresh:
        fresh.load_weights(path)
        fresh.set_option("batch", 3)
        for n, (big, (x0, y0, w, h)) in enumerate(crops):
            got = fresh.sample_region(8, x0, y0, w, h, 7)
            want = outs[big][:, y0 - big[1]:y0 - big[1] + h, x0 - big[0]:x0 - big[0] + w].cpu().numpy()
            assert np.array_equal(got, want), (x0, y0, w, h)
            if n % 2 == 0:
                assert rel_l2(got, planar(sample(m, 8, x0, y0, w, h, 7))) <= 1e-6


def test_argument_errors_leave_the_context_usable(lg):
    td, c, m, _ = lg
    before = c.sample_region(4, 10, 20, 30, 40, 0)
    bad = [(0, 0, 0, 5, 0), (0, 0, 5, 0, 0), (0, 0, (1 << 20) + 1, 1, 0), (0, 0, 1 << 14, 1 << 13, 0),
           (LIM - 10, 0, 10, 10, 0), (0, -LIM, 5, 5, 0), (0, 0, 4, 4, 9), (0, 0, 4, 4, -2)]
    for x0, y0, w, h, level in bad:
        with pytest.raises(td.TDError) as e:
            c.sample_region(4, x0, y0, w, h, level)
        assert str(e.value)
    small = np.empty((4, 3, 3), dtype=np.float32)
    assert td.lib.td_sample_region(c.ctx, 4, 0, 0, 4, 4, 0, td._fptr(small), small.size) == td.TD_E_INVAL
    after = c.sample_region(4, 10, 20, 30, 40, 0)
    assert np.array_equal(before, after)


def test_failed_query_drops_the_cache_and_the_context_recovers(weights):
    """A query that fails after planning (its batch workspace cannot be
    allocated: 2^20 windows of the 16/32 UNet is far beyond HBM) must not
    leave pinned or never-computed windows behind: the cache is dropped,
    the error is reported once, and the next query equals a fresh context's."""
    require_gpu()
    from paper_2512_08309_amd import td
    path = weights("c1")
    with td.Context(0) as c:
        c.load_weights(path)
        c.set_option("batch", 64)
        c.sample_region(3, 0, 0, 16, 16, 0)                    # warms part of the next cone
        assert c.cache_stats()["bytes_used"] > 0
        c.set_option("batch", 1 << 20)
        with pytest.raises(td.TDError) as e:
            c.sample_region(3, -8, -8, 40, 40, 0)
        assert e.value.status == td.TD_E_NOMEM, str(e.value)
        assert c.cache_stats()["bytes_used"] == 0
        c.set_option("batch", 64)
        got = c.sample_region(3, -8, -8, 40, 40, 0)
        c.cache_set_budget(1 << 20)                             # every window evictable again
        c.sample_region(3, 500, 500, 16, 16, 0)
        assert c.cache_stats()["bytes_used"] <= 1 << 20
    with td.Context(0) as f:
        f.load_weights(path)
        want = f.sample_region(3, -8, -8, 40, 40, 0)
    assert np.array_equal(got, want)


def _tdw_bytes(blob, data):
    """A TDW1 file from a raw header blob and a data section."""
    import struct
    start = (8 + len(blob) + 63) // 64 * 64
    return b"TDW1" + struct.pack("<I", len(blob)) + blob + b"\0" * (start - 8 - len(blob)) + data


def test_malformed_weight_files_are_rejected_and_keep_the_model(weights, tmp_path):
    """Every malformed file gives TD_E_FORMAT (a missing one TD_E_IO) with a
    message, and the context keeps answering with the model it had; a fresh
    context that never loaded a model refuses queries with TD_E_STATE."""
    require_gpu()
    import json
    import struct
    from paper_2512_08309_amd import td
    good = weights("c1")
    raw = open(good, "rb").read()
    n = struct.unpack("<I", raw[4:8])[0]
    hdr = json.loads(raw[8:8 + n])
    data = raw[(8 + n + 63) // 64 * 64:]

    def edited(f):
        h = json.loads(json.dumps(hdr))
        f(h)
        return _tdw_bytes(json.dumps(h).encode(), data)

    cases = {
        "empty": b"",
        "magic": b"TDW2" + raw[4:],
        "header_length": raw[:4] + struct.pack("<I", len(raw)) + raw[8:],
        "json_syntax": _tdw_bytes(b'{"denoiser": {"kind": ', data),
        "json_depth": _tdw_bytes(b"[" * 100 + b"]" * 100, data),
        "data_truncated": raw[:len(raw) - 1000],
        "integer_range": edited(lambda h: h["denoiser"].__setitem__("in_channels", 1e30)),
        "tensor_missing": edited(lambda h: h["tensors"].pop()),
        "tensor_shape": edited(lambda h: h["tensors"][0].__setitem__("shape", [3, 3])),
        "tensor_size": edited(lambda h: h["tensors"][0].__setitem__("shape", [1 << 30, 1 << 30, 4])),
        "denoiser_kind": edited(lambda h: h["denoiser"].__setitem__("kind", "transformer")),
    }
    with td.Context(0) as c:
        c.load_weights(good)
        before = c.sample_region(6, -40, 17, 24, 20, 0)
        with pytest.raises(td.TDError) as e:
            c.load_weights(str(tmp_path / "no_such_file.tdw"))
        assert e.value.status == td.TD_E_IO
        for name, content in cases.items():
            p = tmp_path / (name + ".tdw")
            p.write_bytes(content)
            with pytest.raises(td.TDError) as e:
                c.load_weights(str(p))
            assert e.value.status == td.TD_E_FORMAT, (name, str(e.value))
            assert str(e.value), name
        assert np.array_equal(c.sample_region(6, -40, 17, 24, 20, 0), before)
    with td.Context(0) as fresh:
        p = tmp_path / "magic.tdw"
        with pytest.raises(td.TDError):
            fresh.load_weights(str(p))
        with pytest.raises(td.TDError) as e:
            fresh.sample_region(6, 0, 0, 4, 4, 0)
        assert e.value.status == td.TD_E_STATE


def test_device_buffer_checks(lg):
    """Wrong dtype, strided views and wrong window shapes are refused by the
    binding (ValueError) before anything is launched; the context stays usable."""
    import torch
    td, c, m, _ = lg
    before = c.sample_region(4, 10, 20, 30, 40, 0)
    C, H = c.info("channels"), c.info("window")
    bad_outputs = [torch.empty((C, 40, 30), dtype=torch.float64, device="cuda"),
                   torch.empty((C, 40, 60), device="cuda")[:, :, ::2],
                   torch.empty((C, 40, 30), dtype=torch.float16, device="cuda")]
    for out in bad_outputs:
        with pytest.raises(ValueError):
            c.sample_region_async(4, 10, 20, 30, 40, 0, out)
    x = torch.zeros((2, H, H, C), device="cuda")
    with pytest.raises(ValueError):
        td.td_denoise_windows(c.ctx, x, 0, torch.zeros((2, H, H + 1, C), device="cuda"))
    with pytest.raises(ValueError):
        td.td_denoise_windows(c.ctx, torch.zeros((2, H, H, C + 1), device="cuda"), 0, x)
    with pytest.raises(ValueError):
        td.td_lap_decode(c.ctx, torch.zeros((50, 50, C + 1), device="cuda"), 0, 0, 0, 0, 8, 8,
                         torch.zeros((8, 8), device="cuda"))
    torch.cuda.synchronize()
    assert np.array_equal(c.sample_region(4, 10, 20, 30, 40, 0), before)
