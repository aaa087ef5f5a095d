"""Model configurations and seeded random initialisation -> ``.tdw`` files.

Configurations (window H/s, sampler steps K, UNet widths) follow the
workloads the method is measured on:

* ``c1``  : 1-channel latent, windows 32 at stride 16, K = 8, 2-level UNet
            (16/32 channels, 2 res-blocks per level, GroupNorm 8 groups).
* ``c2``  : 4-channel latent, windows 64 at stride 32, K = 20, 4-level UNet
            (128/256/256/512, 2 res-blocks, 8-head attention at the lowest
            level, GroupNorm 32 groups).
* ``c2k4``, ``c2k2``: ``c2`` with K reduced to 4 / 2 (same network).
* ``lg``  : analytic linear-Gaussian denoiser (no tensors), 4 channels,
            windows 32 at stride 16, K = 8.
* ``c1t2``, ``lgt2``, ``c2t1``/``c2t2``/``c2t5``: the same models with
            truncated T (blends only at the listed schedule indices).
* ``cc``  : coarse model of the hierarchy (1 channel, 2-level UNet 64/128,
            windows 32/16, K = 8 with one blend at the end, noise counter
            word 2); ``c1h`` is ``c1`` conditioned on it (its final latent,
            nearest-upsampled 8x, concatenated to the input).
* ``lgc``, ``lgh``: the linear-Gaussian pair with the same wiring.
* ``lgw``: ``lg`` with a wider decode blur (sigma 9, radius 30).
* ``s2``  : the half-width student of ``c2`` (64/128/128/256), two-step
            consistency sampling at sigma 80 and 0.35; ``lgs`` is an analytic
            two-step model (prior std 0.7) whose teacher stand-in is ``lg``;
            ``st`` is a small network of the student's shape (32/32, windows
            16) for gradient checks; ``c2n`` is a narrow teacher with the
            student's channels and window layout (16/32, K = 2), small
            enough for the oracle to sample its fallbacks in seconds.

Initialisation: every tensor is Gaussian from numpy's PCG64 seeded with the
given seed, drawn in file order.  Conv / linear weights ~ N(0, 1/fan_in);
biases ~ N(0, 0.1^2); GroupNorm gamma ~ 1 + N(0, 0.1^2), beta ~ N(0, 0.1^2)
(non-trivial so that a mis-indexed bias or affine parameter is visible).
"""
import copy
import os

import numpy as np

from .tdw import write_tdw

SAMPLER_EDM = {"sigma_max": 80.0, "sigma_min": 0.002, "rho": 7.0, "sigma_data": 0.5}
DECODE = {"factor": 8, "sigma_low": 20.0, "sigma_res": 2.0, "blur_sigma": 5.0, "blur_radius": 15}

CONFIGS = {
    "c1": {
        "denoiser": {"kind": "unet", "in_channels": 1, "channels": [16, 32], "num_res_blocks": 2,
                     "attn_levels": [], "mid_attn": False, "num_heads": 1, "gn_groups": 8,
                     "gn_eps": 1e-5, "emb_mult": 4, "pe_max_period": 10000.0},
        "sampler": dict(SAMPLER_EDM, steps=8),
        "window": {"size": 32, "stride": 16, "offset": 0, "eps": 0.01},
    },
    "c2": {
        "denoiser": {"kind": "unet", "in_channels": 4, "channels": [128, 256, 256, 512],
                     "num_res_blocks": 2, "attn_levels": [3], "mid_attn": True, "num_heads": 8,
                     "gn_groups": 32, "gn_eps": 1e-5, "emb_mult": 4, "pe_max_period": 10000.0},
        "sampler": dict(SAMPLER_EDM, steps=20),
        "window": {"size": 64, "stride": 32, "offset": 0, "eps": 0.01},
    },
    "lg": {
        "denoiser": {"kind": "linear_gaussian", "in_channels": 4, "prior_std": 0.5},
        "sampler": dict(SAMPLER_EDM, steps=8),
        "window": {"size": 32, "stride": 16, "offset": 0, "eps": 0.01},
    },
}
for _k in (4, 2):
    CONFIGS["c2k%d" % _k] = copy.deepcopy(CONFIGS["c2"])
    CONFIGS["c2k%d" % _k]["sampler"]["steps"] = _k
CONFIGS["c1k2"] = copy.deepcopy(CONFIGS["c1"])
CONFIGS["c1k2"]["sampler"]["steps"] = 2
# hierarchy: a coarse model at 1/8 resolution (its own noise stream, one
# blend at the end) whose final latent conditions the 1-channel fine model
CONFIGS["cc"] = {
    "denoiser": {"kind": "unet", "in_channels": 1, "channels": [64, 128], "num_res_blocks": 2,
                 "attn_levels": [], "mid_attn": False, "num_heads": 1, "gn_groups": 32,
                 "gn_eps": 1e-5, "emb_mult": 4, "pe_max_period": 10000.0},
    "sampler": dict(SAMPLER_EDM, steps=8, blend=[0, 8], noise_step=2),
    "window": {"size": 32, "stride": 16, "offset": 0, "eps": 0.01},
}
CONFIGS["c1h"] = copy.deepcopy(CONFIGS["c1"])
CONFIGS["c1h"]["cond"] = {"channels": 1, "factor": 8}
CONFIGS["lgc"] = {
    "denoiser": {"kind": "linear_gaussian", "in_channels": 1, "prior_std": 0.5},
    "sampler": dict(SAMPLER_EDM, steps=8, blend=[0, 8], noise_step=2),
    "window": {"size": 32, "stride": 16, "offset": 0, "eps": 0.01},
}
CONFIGS["lgh"] = {
    "denoiser": {"kind": "linear_gaussian", "in_channels": 1, "prior_std": 0.5},
    "sampler": dict(SAMPLER_EDM, steps=8),
    "window": {"size": 32, "stride": 16, "offset": 0, "eps": 0.01},
    "cond": {"channels": 1, "factor": 8},
}
# few-step students (consistency sampling: two steps, intermediate sigma 0.35)
CONSISTENCY_2 = {"kind": "consistency", "steps": 2, "sigmas": [80.0, 0.35], "sigma_data": 0.5}
CONFIGS["s2"] = {
    "denoiser": {"kind": "unet", "in_channels": 4, "channels": [64, 128, 128, 256], "num_res_blocks": 2,
                 "attn_levels": [3], "mid_attn": True, "num_heads": 8, "gn_groups": 32, "gn_eps": 1e-5,
                 "emb_mult": 4, "pe_max_period": 10000.0},
    "sampler": dict(CONSISTENCY_2),
    "window": {"size": 64, "stride": 32, "offset": 0, "eps": 0.01},
}
CONFIGS["st"] = {   # a small student-shaped network for gradient checks
    "denoiser": {"kind": "unet", "in_channels": 4, "channels": [32, 32], "num_res_blocks": 1,
                 "attn_levels": [1], "mid_attn": True, "num_heads": 2, "gn_groups": 8, "gn_eps": 1e-5,
                 "emb_mult": 4, "pe_max_period": 10000.0},
    "sampler": dict(CONSISTENCY_2),
    "window": {"size": 16, "stride": 8, "offset": 0, "eps": 0.01},
}
CONFIGS["c2n"] = {   # a narrow teacher of the student's layout (judge parity)
    "denoiser": {"kind": "unet", "in_channels": 4, "channels": [16, 32], "num_res_blocks": 1,
                 "attn_levels": [], "mid_attn": False, "num_heads": 1, "gn_groups": 8, "gn_eps": 1e-5,
                 "emb_mult": 4, "pe_max_period": 10000.0},
    "sampler": dict(SAMPLER_EDM, steps=2),
    "window": {"size": 64, "stride": 32, "offset": 0, "eps": 0.01},
}
CONFIGS["lgs"] = {
    "denoiser": {"kind": "linear_gaussian", "in_channels": 4, "prior_std": 0.7},
    "sampler": dict(CONSISTENCY_2),
    "window": {"size": 32, "stride": 16, "offset": 0, "eps": 0.01},
}
# truncated T (blend only after the listed schedule indices)
# ``lg`` with a wider decode blur (sigma 9, radius 30): the decode and
# encode take their multi-launch blur path (radius > 24)
CONFIGS["lgw"] = copy.deepcopy(CONFIGS["lg"])
CONFIGS["lgw"]["decode"] = dict(DECODE, blur_sigma=9.0, blur_radius=30)
for _name, _base, _blend in [("c1t2", "c1", [0, 4, 8]), ("lgt2", "lg", [0, 3, 8]), ("c2t2", "c2", [0, 10, 20]),
                             ("c2t5", "c2", [0, 4, 8, 12, 16, 20]), ("c2t1", "c2", [0, 20])]:
    CONFIGS[_name] = copy.deepcopy(CONFIGS[_base])
    CONFIGS[_name]["sampler"]["blend"] = _blend


def _resblock(prefix, cin, cout, emb_dim):
    t = [(prefix + "gn1.weight", (cin,), "gamma"), (prefix + "gn1.bias", (cin,), "beta"),
         (prefix + "conv1.weight", (cout, cin, 3, 3), cin * 9), (prefix + "conv1.bias", (cout,), "bias"),
         (prefix + "emb.weight", (cout, emb_dim), emb_dim), (prefix + "emb.bias", (cout,), "bias"),
         (prefix + "gn2.weight", (cout,), "gamma"), (prefix + "gn2.bias", (cout,), "beta"),
         (prefix + "conv2.weight", (cout, cout, 3, 3), cout * 9), (prefix + "conv2.bias", (cout,), "bias")]
    if cin != cout:
        t += [(prefix + "skip.weight", (cout, cin, 1, 1), cin), (prefix + "skip.bias", (cout,), "bias")]
    return t


def _attn(prefix, c):
    return [(prefix + "gn.weight", (c,), "gamma"), (prefix + "gn.bias", (c,), "beta"),
            (prefix + "qkv.weight", (3 * c, c, 1, 1), c), (prefix + "qkv.bias", (3 * c,), "bias"),
            (prefix + "proj.weight", (c, c, 1, 1), c), (prefix + "proj.bias", (c,), "bias")]


def unet_tensor_specs(arch, cond_channels=0):
    """Ordered (name, shape, init) for a UNet architecture; init is fan_in or a tag.
    A conditioned network's input conv also reads the conditioning channels."""
    ch = arch["channels"]
    nl = len(ch)
    nres = arch["num_res_blocks"]
    cin_img = arch["in_channels"]
    cin_x = cin_img + cond_channels
    emb = arch["emb_mult"] * ch[0]
    attn = set(arch["attn_levels"])
    t = [("emb.lin1.weight", (emb, ch[0]), ch[0]), ("emb.lin1.bias", (emb,), "bias"),
         ("emb.lin2.weight", (emb, emb), emb), ("emb.lin2.bias", (emb,), "bias"),
         ("conv_in.weight", (ch[0], cin_x, 3, 3), cin_x * 9), ("conv_in.bias", (ch[0],), "bias")]
    skips = []
    c = ch[0]
    for l in range(nl):
        for j in range(nres):
            p = "enc.%d.%d." % (l, j)
            t += _resblock(p, c, ch[l], emb)
            c = ch[l]
            if l in attn:
                t += _attn(p + "attn.", c)
            skips.append(c)
    t += _resblock("mid.0.", c, c, emb)
    if arch["mid_attn"]:
        t += _attn("mid.attn.", c)
    t += _resblock("mid.1.", c, c, emb)
    for l in reversed(range(nl)):
        for j in range(nres):
            p = "dec.%d.%d." % (l, j)
            cs = skips.pop()
            t += _resblock(p, c + cs, ch[l], emb)
            c = ch[l]
            if l in attn:
                t += _attn(p + "attn.", c)
    t += [("out.gn.weight", (c,), "gamma"), ("out.gn.bias", (c,), "beta"),
          ("out.conv.weight", (cin_img, c, 3, 3), c * 9), ("out.conv.bias", (cin_img,), "bias")]
    return t


def init_tensors(specs, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for name, shape, init in specs:
        z = rng.standard_normal(shape)
        if init == "gamma":
            v = 1.0 + 0.1 * z
        elif init in ("beta", "bias"):
            v = 0.1 * z
        else:
            v = z / np.sqrt(float(init))
        out.append((name, v.astype(np.float32)))
    return out


def header_for(config):
    cfg = copy.deepcopy(CONFIGS[config])
    cfg["decode"] = dict(cfg.get("decode", DECODE))
    cfg["format"] = "tdw"
    cfg["version"] = 1
    cfg["name"] = config
    return cfg


def param_count(config):
    cfg = CONFIGS[config]
    if cfg["denoiser"]["kind"] != "unet":
        return 0
    cc = cfg.get("cond", {}).get("channels", 0)
    return int(sum(np.prod(s) for _, s, _ in unet_tensor_specs(cfg["denoiser"], cc)))


def make_weights(config, path, seed=0):
    """Write the seeded random-init weight file for a configuration."""
    hdr = header_for(config)
    if hdr["denoiser"]["kind"] == "unet":
        cc = hdr.get("cond", {}).get("channels", 0)
        tensors = init_tensors(unet_tensor_specs(hdr["denoiser"], cc), seed)
    else:
        tensors = []
    hdr["init_seed"] = seed
    write_tdw(path, hdr, tensors)
    return path


def cached_weights(config, directory, seed=0):
    """Path of the weight file for (config, seed) under directory, written once."""
    os.makedirs(directory, exist_ok=True)
    path = os.path.join(directory, "%s_seed%d.tdw" % (config, seed))
    if not os.path.exists(path):
        tmp = path + ".tmp%d" % os.getpid()
        make_weights(config, tmp, seed)
        os.replace(tmp, path)
    return path
