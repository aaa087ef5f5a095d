"""Pins of the oracle UNet layers (no GPU).

The per-layer checks compare the numpy float64 oracle with torch's CPU
float64 operators (conv2d, group_norm, scaled_dot_product_attention,
avg_pool2d, interpolate), i.e. with library routines that use their own
layout conventions (OIHW weights, NCHW activations).  The whole-network
composition is checked the same way on the tiny configuration.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import unet as U
from oracle.schedule import precond
from oracle.tdw import read_tdw


def nchw(x):
    return torch.from_numpy(np.ascontiguousarray(x.transpose(0, 3, 1, 2)))


def nhwc(t):
    return t.numpy().transpose(0, 2, 3, 1)


def test_conv2d_direct_loops_and_torch():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 6, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    got = U.conv2d(x, w, b)
    ref = nhwc(F.conv2d(nchw(x), torch.from_numpy(w), torch.from_numpy(b), padding=1))
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)
    direct = np.zeros_like(got)
    for n in range(2):
        for y in range(5):
            for xx in range(6):
                for o in range(4):
                    acc = b[o]
                    for c in range(3):
                        for dy in range(3):
                            for dx in range(3):
                                yy, xs = y + dy - 1, xx + dx - 1
                                if 0 <= yy < 5 and 0 <= xs < 6:
                                    acc += w[o, c, dy, dx] * x[n, yy, xs, c]
                    direct[n, y, xx, o] = acc
    assert np.allclose(got, direct, rtol=1e-12, atol=1e-12)
    w1 = rng.standard_normal((7, 3, 1, 1))
    assert np.allclose(U.conv2d(x, w1, b[:1].repeat(7)),
                       nhwc(F.conv2d(nchw(x), torch.from_numpy(w1), torch.from_numpy(b[:1].repeat(7)))),
                       rtol=1e-12, atol=1e-12)


def test_group_norm_matches_torch():
    rng = np.random.default_rng(1)
    x = 3 + 2 * rng.standard_normal((3, 4, 4, 12))
    g, bt = rng.standard_normal(12), rng.standard_normal(12)
    got = U.group_norm(x, g, bt, 4, 1e-5)
    ref = nhwc(F.group_norm(nchw(x), 4, torch.from_numpy(g), torch.from_numpy(bt), 1e-5))
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-10)


def test_pool_and_upsample_match_torch():
    x = np.random.default_rng(2).standard_normal((2, 8, 6, 3))
    assert np.allclose(U.avgpool2(x), nhwc(F.avg_pool2d(nchw(x), 2)))
    assert np.array_equal(U.upsample2(x), nhwc(F.interpolate(nchw(x), scale_factor=2, mode="nearest")))


def _t(a):
    return torch.from_numpy(np.asarray(a))


def torch_attention(t, p, x, groups, eps, nh):
    B, C, H, W = x.shape
    h = F.group_norm(x, groups, _t(t[p + "gn.weight"]), _t(t[p + "gn.bias"]), eps)
    qkv = F.conv2d(h, _t(t[p + "qkv.weight"]), _t(t[p + "qkv.bias"])).reshape(B, 3, nh, C // nh, H * W)
    q, k, v = (qkv[:, i].transpose(-1, -2) for i in range(3))
    o = F.scaled_dot_product_attention(q, k, v)
    o = o.transpose(-1, -2).reshape(B, C, H, W)
    return x + F.conv2d(o, _t(t[p + "proj.weight"]), _t(t[p + "proj.bias"]))


def test_attention_matches_torch_sdpa():
    rng = np.random.default_rng(3)
    C, nh = 16, 4
    t = {"a.gn.weight": 1 + 0.1 * rng.standard_normal(C), "a.gn.bias": 0.1 * rng.standard_normal(C),
         "a.qkv.weight": rng.standard_normal((3 * C, C, 1, 1)) / 4, "a.qkv.bias": rng.standard_normal(3 * C),
         "a.proj.weight": rng.standard_normal((C, C, 1, 1)) / 4, "a.proj.bias": rng.standard_normal(C)}
    net = U.UNet({"gn_groups": 4, "gn_eps": 1e-5, "num_heads": nh}, t)
    x = rng.standard_normal((2, 4, 4, C))
    got = net.attention("a.", x)
    ref = nhwc(torch_attention(t, "a.", nchw(x), 4, 1e-5, nh))
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-10)


def torch_unet(hdr, t, x, c_noise):
    a = hdr["denoiser"]
    G, eps = a["gn_groups"], a["gn_eps"]

    def conv(p, h):
        w = _t(t[p + ".weight"])
        return F.conv2d(h, w, _t(t[p + ".bias"]), padding=w.shape[-1] // 2)

    def gn(p, h):
        return F.group_norm(h, G, _t(t[p + ".weight"]), _t(t[p + ".bias"]), eps)

    c0 = a["channels"][0]
    half = c0 // 2
    fr = torch.exp(-np.log(a["pe_max_period"]) * torch.arange(half, dtype=torch.float64) / half)
    pe = torch.cat([torch.cos(c_noise * fr), torch.sin(c_noise * fr)])
    e = F.silu(F.linear(pe, _t(t["emb.lin1.weight"]), _t(t["emb.lin1.bias"])))
    e = F.silu(F.linear(e, _t(t["emb.lin2.weight"]), _t(t["emb.lin2.bias"])))

    def res(p, h):
        y = conv(p + "conv1", F.silu(gn(p + "gn1", h)))
        y = y + F.linear(e, _t(t[p + "emb.weight"]), _t(t[p + "emb.bias"]))[None, :, None, None]
        y = conv(p + "conv2", F.silu(gn(p + "gn2", y)))
        return (conv(p + "skip", h) if p + "skip.weight" in t else h) + y

    nl = len(a["channels"])
    h = conv("conv_in", x)
    skips = []
    for l in range(nl):
        if l:
            h = F.avg_pool2d(h, 2)
        for j in range(a["num_res_blocks"]):
            h = res("enc.%d.%d." % (l, j), h)
            if l in a["attn_levels"]:
                h = torch_attention(t, "enc.%d.%d.attn." % (l, j), h, G, eps, a["num_heads"])
            skips.append(h)
    h = res("mid.0.", h)
    if a["mid_attn"]:
        h = torch_attention(t, "mid.attn.", h, G, eps, a["num_heads"])
    h = res("mid.1.", h)
    for l in reversed(range(nl)):
        for j in range(a["num_res_blocks"]):
            h = res("dec.%d.%d." % (l, j), torch.cat([h, skips.pop()], 1))
            if l in a["attn_levels"]:
                h = torch_attention(t, "dec.%d.%d.attn." % (l, j), h, G, eps, a["num_heads"])
        if l:
            h = F.interpolate(h, scale_factor=2, mode="nearest")
    return conv("out.conv", F.silu(gn("out.gn", h)))


@pytest.mark.parametrize("config", ["c1", "c2"])
def test_whole_unet_matches_torch_composition(weights, config):
    hdr, t = read_tdw(weights(config))
    H = hdr["window"]["size"]
    x = np.random.default_rng(4).standard_normal((1, H, H, hdr["denoiser"]["in_channels"]))
    got = U.UNet(hdr["denoiser"], t).forward(x, -0.3)
    ref = nhwc(torch_unet(hdr, t, nchw(x), -0.3))
    assert np.allclose(got, ref, rtol=1e-9, atol=1e-9)
    assert 0.05 < np.std(got) < 20   # fan-in init keeps activations O(1)


def test_preconditioning_limits(weights):
    hdr, t = read_tdw(weights("c1"))
    D = U.UNetDenoiser(hdr, t)
    x = np.random.default_rng(5).standard_normal((2, 32, 32, 1))
    d = D(x, 1e-6, None)
    assert np.allclose(d, x, atol=1e-5)
    c_skip, c_out, c_in, _ = precond(80.0, 0.5)
    assert c_skip + (c_out / 0.5) ** 2 == pytest.approx(1.0)   # c_skip + c_out^2/sd^2 = 1
    assert c_in * np.sqrt(80.0 ** 2 + 0.25) == pytest.approx(1.0)
