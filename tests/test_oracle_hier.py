"""Pins of the hierarchy (a parent model's final latent conditions a child).

* Closed form: with the linear-Gaussian pair (parent ``lgc``: own noise
  counter word 2, one blend after 8 steps; child ``lgh``: prior mean plus
  the conditioning), the child's latent is
      J_0(p) = m(p) + y(p) + (sigma_0 G(p) - m(p) - y(p)) * Pi_child
  with y(p) = parent J_0 at (floor(x/8), floor(y/8)) given by the same
  closed form of the parent on its own noise; m are brute-force weighted
  window means.  Negative coordinates exercise the floor division.
* The conditioned UNet's input conv reads (c_in x, y) in that order: zeroing
  either half of the conv_in weights reduces it to an unconditioned network.
* Crop independence holds for the child, and the conditioning changes it.
"""
import numpy as np
import pytest

from oracle import noise, schedule
from oracle.sampler import Model, sample
from oracle.tdw import read_tdw
from oracle.unet import UNetDenoiser
from test_oracle_sampler import brute_mu_bar


def _prod(m, steps):
    sp = m.header["sampler"]
    sig = schedule.sigmas(m.steps, sp["sigma_max"], sp["sigma_min"], sp["rho"])
    sd = m.header["denoiser"]["prior_std"]
    p = 1.0
    for k in range(steps):
        p *= 1 + (sig[k + 1] - sig[k]) * sig[k] / (sd * sd + sig[k] ** 2)
    return sig[0], p


@pytest.mark.parametrize("seed,x0,y0,level", [(0, -37, -21, 0), (4, 1000003, -999985, 0), (2, -5, 9, 3)])
def test_linear_gaussian_hierarchy_closed_form(weights, seed, x0, y0, level):
    parent = Model(weights("lgc"))
    child = Model(weights("lgh"), parent=parent)
    assert parent.noise_step == 2 and parent.K == 1 and child.cond["factor"] == 8
    w, h = 23, 17
    got = sample(child, seed, x0, y0, w, h, level)
    s0c, pc = _prod(parent, parent.steps)
    s0f, pf = _prod(child, child.points[child.K - level])
    gf = noise.noise_region(seed, x0, y0, w, h, 1).astype(np.float64)
    for yy, xx in [(0, 0), (h - 1, w - 1), (5, 11), (16, 2), (8, 8), (3, 20)]:
        X, Y = x0 + xx, y0 + yy
        PX, PY = X // 8, Y // 8
        gc = float(noise.noise_region(seed, PX, PY, 1, 1, 1, step=2)[0, 0, 0])
        mc = brute_mu_bar(PX, PY, 0, parent.H, parent.s, parent.o, parent.eps)
        y = mc + (s0c * gc - mc) * pc
        mf = brute_mu_bar(X, Y, 0, child.H, child.s, child.o, child.eps) + y
        want = mf + (s0f * gf[yy, xx, 0] - mf) * pf
        assert got[yy, xx, 0] == pytest.approx(want, rel=1e-12, abs=1e-12)


def test_child_without_parent_is_refused(weights):
    child = Model(weights("lgh"))
    with pytest.raises(ValueError):
        sample(child, 0, 0, 0, 8, 8, 0)


def test_conditioned_unet_input_order(weights):
    hdr_c, t_c = read_tdw(weights("c1h"))
    hdr_u, t_u = read_tdw(weights("c1"))
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 32, 32, 1)) * 2.0
    y = rng.standard_normal((2, 32, 32, 1))
    sig = 1.3
    w = t_c["conv_in.weight"]
    assert w.shape[1] == 2
    # the conditioning half zeroed: the x half acts alone
    tc = dict(t_c, **{"conv_in.weight": np.concatenate([w[:, :1], 0 * w[:, 1:]], axis=1)})
    tu = dict(t_c, **{"conv_in.weight": w[:, :1]})
    a = UNetDenoiser(hdr_c, tc)(x, sig, None, cond=y)
    b = UNetDenoiser(hdr_u, tu)(x, sig, None)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)
    # the x half zeroed and y = c_in x: the conditioning half acts alone on c_in x
    c_in = 1.0 / np.sqrt(sig ** 2 + 0.25)
    tc = dict(t_c, **{"conv_in.weight": np.concatenate([0 * w[:, :1], w[:, 1:]], axis=1)})
    tu = dict(t_c, **{"conv_in.weight": w[:, 1:]})
    a = UNetDenoiser(hdr_c, tc)(x, sig, None, cond=c_in * x)
    b = UNetDenoiser(hdr_u, tu)(x, sig, None)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)
    del hdr_u, t_u


def test_hierarchy_crop_independence_and_effect(weights):
    import copy
    parent = Model(weights("lgc"))
    child = Model(weights("c1h"), parent=parent)
    big = sample(child, 5, -24, 8, 40, 24, 5)
    small = sample(child, 5, -11, 13, 17, 9, 5)
    assert np.allclose(small, big[5:14, 13:30], rtol=0, atol=1e-12)
    hdr = copy.deepcopy(parent.header)
    hdr["sampler"]["noise_step"] = 3          # another parent latent
    other = Model(weights("c1h"), parent=Model(hdr))
    diff = sample(other, 5, -11, 13, 17, 9, 5)
    assert np.abs(diff - small).max() > 1e-3
