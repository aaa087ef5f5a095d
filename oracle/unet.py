"""FP64 UNet F(x; c_noise) and the denoisers D(x; sigma).

TEST INFRASTRUCTURE (oracle).  The paper's networks (EDM2 backbone with sCM
changes, Sec. 5.3 and the implementation-details appendix) are trained
models and are not reproduced; the workloads instead fix a plain UNet whose
layout is read as follows (activations NHWC, float64):

* conv_in 3x3 (zero padding at the window border).
* Encoder level l = 0..L-1 at resolution H/2^l: 2x2 average pool before
  every level but the first, then n_res ResBlocks, each followed by
  attention at the attention levels; every block output is kept as a skip.
* Middle: ResBlock, attention (if enabled), ResBlock.
* Decoder level l = L-1..0: n_res ResBlocks on concat(h, popped skip)
  (h channels first), each followed by attention at attention levels;
  nearest 2x upsample after every level but level 0.
* Output: GroupNorm, SiLU, conv 3x3.
* ResBlock(x): h = conv1(SiLU(GN1(x))) + Lin_emb(emb);
  h = conv2(SiLU(GN2(h))); out = skip(x) + h, skip = 1x1 conv when the
  channel count changes, identity otherwise.
* Attention(x): GN, 1x1 qkv (q, k, v = consecutive channel thirds, head h =
  channels h*d..h*d+d-1 of each), softmax(q k^T / sqrt(d)) v per head, 1x1
  proj, residual add.
* GroupNorm: biased variance over (pixels, channels of the group), eps from
  the header, then per-channel gamma, beta.
* emb = SiLU(Lin2(SiLU(Lin1(pe(c_noise))))), pe = [cos(c w_j), sin(c w_j)],
  w_j = P^(-j/(c0/2)), j < c0/2, P = pe_max_period (positional embedding
  in place of Fourier features, as in sCM).
* Conditioning (hierarchy, Sec. 5.1; DAGs of infinite tensors in the
  infinite-tensor appendix): a conditioned network's input conv reads
  concat(c_in x, y), the window's conditioning channels y appended after
  the scaled input and not scaled themselves.  The linear-Gaussian stand-in
  adds y (channel c mod C_y) to its prior mean.

Pins (tests/test_oracle_unet.py): conv against a direct seven-loop sum and
against scipy.signal.correlate; GroupNorm output moments; attention against
a per-head loop with scipy.special.softmax; avgpool/upsample identities; a
ResBlock with zero conv weights reduces to its skip path; the whole
network is translation-equivariant away from the border.  Beyond these
per-layer pins the network composition is "parity unpinned" (no paper
numbers exist for a random-init network).
"""
import numpy as np

from .schedule import precond


def silu(x):
    with np.errstate(over="ignore"):
        return x / (1.0 + np.exp(-x))


def conv2d(x, w, b, max_bytes=1 << 28):
    """Cross-correlation with zero padding; x [B,H,W,Ci], w [Co,Ci,k,k], b [Co]."""
    B, H, W, Ci = x.shape
    Co, _, k, _ = w.shape
    p = k // 2
    wm = w.transpose(2, 3, 1, 0).reshape(k * k * Ci, Co)
    out = np.empty((B, H, W, Co), dtype=np.float64)
    per = max(1, int(max_bytes // (H * W * k * k * Ci * 8)))
    for b0 in range(0, B, per):
        xb = x[b0:b0 + per]
        if p:
            xb = np.pad(xb, ((0, 0), (p, p), (p, p), (0, 0)))
        cols = np.stack([xb[:, dy:dy + H, dx:dx + W, :] for dy in range(k) for dx in range(k)], axis=3)
        out[b0:b0 + per] = (cols.reshape(-1, k * k * Ci) @ wm).reshape(-1, H, W, Co) + b
    return out


def group_norm(x, gamma, beta, groups, eps):
    B, H, W, C = x.shape
    g = x.reshape(B, H * W, groups, C // groups)
    mu = g.mean(axis=(1, 3), keepdims=True)
    var = ((g - mu) ** 2).mean(axis=(1, 3), keepdims=True)
    y = ((g - mu) / np.sqrt(var + eps)).reshape(B, H, W, C)
    return y * gamma + beta


def avgpool2(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def upsample2(x):
    return x.repeat(2, axis=1).repeat(2, axis=2)


def linear(v, w, b):
    return w @ v + b


def positional_embedding(c_noise, dim, max_period):
    half = dim // 2
    freqs = max_period ** (-np.arange(half, dtype=np.float64) / half)
    a = c_noise * freqs
    return np.concatenate([np.cos(a), np.sin(a)])


class UNet:
    def __init__(self, arch, tensors):
        self.a = arch
        self.t = tensors
        self.groups = arch["gn_groups"]
        self.eps = arch["gn_eps"]

    def gn(self, prefix, x):
        return group_norm(x, self.t[prefix + ".weight"], self.t[prefix + ".bias"], self.groups, self.eps)

    def conv(self, prefix, x):
        return conv2d(x, self.t[prefix + ".weight"], self.t[prefix + ".bias"])

    def embedding(self, c_noise):
        c0 = self.a["channels"][0]
        pe = positional_embedding(c_noise, c0, self.a["pe_max_period"])
        e = silu(linear(pe, self.t["emb.lin1.weight"], self.t["emb.lin1.bias"]))
        return silu(linear(e, self.t["emb.lin2.weight"], self.t["emb.lin2.bias"]))

    def resblock(self, p, x, emb):
        h = self.conv(p + "conv1", silu(self.gn(p + "gn1", x)))
        h = h + linear(emb, self.t[p + "emb.weight"], self.t[p + "emb.bias"])
        h = self.conv(p + "conv2", silu(self.gn(p + "gn2", h)))
        skip = self.conv(p + "skip", x) if (p + "skip.weight") in self.t else x
        return skip + h

    def attention(self, p, x):
        B, H, W, C = x.shape
        nh = self.a["num_heads"]
        d = C // nh
        qkv = self.conv(p + "qkv", self.gn(p + "gn", x)).reshape(B, H * W, 3 * C)
        q, k, v = (qkv[:, :, i * C:(i + 1) * C].reshape(B, H * W, nh, d).transpose(0, 2, 1, 3)
                   for i in range(3))
        s = q @ k.transpose(0, 1, 3, 2) / np.sqrt(d)
        s = np.exp(s - s.max(axis=-1, keepdims=True))
        s = s / s.sum(axis=-1, keepdims=True)
        o = (s @ v).transpose(0, 2, 1, 3).reshape(B, H, W, C)
        return x + self.conv(p + "proj", o)

    def forward(self, x, c_noise):
        a = self.a
        nl = len(a["channels"])
        attn = set(a["attn_levels"])
        emb = self.embedding(c_noise)
        h = self.conv("conv_in", x)
        skips = []
        for l in range(nl):
            if l > 0:
                h = avgpool2(h)
            for j in range(a["num_res_blocks"]):
                p = "enc.%d.%d." % (l, j)
                h = self.resblock(p, h, emb)
                if l in attn:
                    h = self.attention(p + "attn.", h)
                skips.append(h)
        h = self.resblock("mid.0.", h, emb)
        if a["mid_attn"]:
            h = self.attention("mid.attn.", h)
        h = self.resblock("mid.1.", h, emb)
        for l in reversed(range(nl)):
            for j in range(a["num_res_blocks"]):
                p = "dec.%d.%d." % (l, j)
                h = np.concatenate([h, skips.pop()], axis=-1)
                h = self.resblock(p, h, emb)
                if l in attn:
                    h = self.attention(p + "attn.", h)
            if l > 0:
                h = upsample2(h)
        return self.conv("out.conv", silu(self.gn("out.gn", h)))


class UNetDenoiser:
    """D(x; sigma) = c_skip x + c_out F(c_in x; c_noise) (EDM preconditioning)."""

    def __init__(self, header, tensors, batch=64):
        self.net = UNet(header["denoiser"], tensors)
        self.sigma_data = header["sampler"]["sigma_data"]
        self.batch = batch

    def __call__(self, x, sigma, windows, cond=None):
        c_skip, c_out, c_in, c_noise = precond(sigma, self.sigma_data)
        out = np.empty_like(x)
        for b0 in range(0, x.shape[0], self.batch):
            xb = x[b0:b0 + self.batch]
            inp = c_in * xb
            if cond is not None:
                inp = np.concatenate([inp, cond[b0:b0 + self.batch]], axis=-1)
            out[b0:b0 + self.batch] = c_skip * xb + c_out * self.net.forward(inp, c_noise)
        return out


def prior_mean(ix, iy, c):
    """Per-window prior mean of the analytic linear-Gaussian denoiser."""
    return 0.1 * ((ix % 7) - 3) - 0.05 * ((iy % 5) - 2) + 0.01 * c


class LinearGaussianDenoiser:
    """Exact posterior mean for a window prior N(mu_i, s^2) under noise sigma:
    D_i(x; sigma) = mu_i + s^2/(s^2+sigma^2) (x - mu_i).  An analytic stand-in
    for the network used to pin the sampler in closed form."""

    def __init__(self, header):
        self.s = header["denoiser"]["prior_std"]

    def __call__(self, x, sigma, windows, cond=None):
        C = x.shape[-1]
        a = self.s ** 2 / (self.s ** 2 + sigma ** 2)
        mu = np.array([[prior_mean(ix, iy, c) for c in range(C)] for ix, iy in windows],
                      dtype=np.float64)[:, None, None, :]
        if cond is not None:
            mu = mu + cond[..., [c % cond.shape[-1] for c in range(C)]]
        return mu + a * (x - mu)


def make_denoiser(header, tensors):
    kind = header["denoiser"]["kind"]
    if kind == "unet":
        return UNetDenoiser(header, tensors)
    if kind == "linear_gaussian":
        return LinearGaussianDenoiser(header)
    raise ValueError("unknown denoiser kind %r" % kind)
