"""Pins of few-step consistency sampling (the student's sampler) and of the
teacher fallback judge.

* Closed form with the analytic linear-Gaussian model ``lgs`` (prior std
  s = 0.7, sigmas 80 and 0.35): J_1(p) = m(p) + a_0 (80 G_0(p) - m(p)) +
  0.35 G_1(p) and J_0(p) = m(p) + a_1 (J_1(p) - m(p)) with a_k = s^2 /
  (s^2 + sigma_k^2), G_1 the noise on counter word 1, m the brute-force
  weighted window mean.
* The judge at threshold 0 replaces every window by the teacher's plain
  sampler from the student's noise level (``lg``, s = 0.5, 8 EDM steps: all
  of them from 80, then 0.35 -> the teacher's levels below 0.35 -> 0), at an
  infinite threshold by none: both closed forms.
"""
import math

import numpy as np
import pytest

from oracle import noise, schedule
from oracle.sampler import Model, sample
from test_oracle_sampler import brute_mu_bar


def euler_product(seq, s):
    """Factor on (x - mu) of Euler steps through the noise levels seq for a
    linear-Gaussian window prior of std s."""
    p = 1.0
    for a, b in zip(seq, seq[1:]):
        p *= 1 + (b - a) / a * (1 - s * s / (s * s + a * a))
    return p


def closed_form(m, seed, x0, y0, w, h, level, s, teacher_sched=None):
    sig = m.sched
    if teacher_sched is None:   # the student's own estimates
        f = [s * s / (s * s + v * v) for v in sig[:2]]
    else:                       # the teacher's plain sampler from each of the student's levels
        f = [euler_product([v] + [u for u in teacher_sched[:-1] if u < v] + [0.0], s) for v in sig[:2]]
    g0 = noise.noise_region(seed, x0, y0, w, h, 4, step=0).astype(np.float64)
    g1 = noise.noise_region(seed, x0, y0, w, h, 4, step=1).astype(np.float64)
    out = {}
    for yy, xx, c in [(0, 0, 0), (h - 1, w - 1, 3), (5, 11, 1), (16, 2, 2), (8, 8, 0)]:
        mu = brute_mu_bar(x0 + xx, y0 + yy, c, m.H, m.s, m.o, m.eps)
        j1 = mu + f[0] * (sig[0] * g0[yy, xx, c] - mu) + sig[1] * g1[yy, xx, c]
        out[(yy, xx, c)] = j1 if level == 1 else mu + f[1] * (j1 - mu)
    return out


@pytest.mark.parametrize("seed,x0,y0,level", [(0, 0, 0, 0), (3, -37, 1000003, 0), (5, 3, -4, 1)])
def test_consistency_linear_gaussian_closed_form(weights, seed, x0, y0, level):
    m = Model(weights("lgs"))
    assert m.consistency and m.K == 2 and m.sched == [80.0, 0.35, 0.0]
    got = sample(m, seed, x0, y0, 23, 17, level)
    for (yy, xx, c), want in closed_form(m, seed, x0, y0, 23, 17, level, 0.7).items():
        assert got[yy, xx, c] == pytest.approx(want, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("thr,s", [(0.0, 0.5), (math.inf, 0.7)])
def test_judge_extremes(weights, thr, s):
    m = Model(weights("lgs"))
    teacher = Model(weights("lg"))
    m.judge = (teacher, thr)
    got = sample(m, 2, -9, 40, 23, 17, 0)
    ts = teacher.sched if thr == 0 else None
    for (yy, xx, c), want in closed_form(m, 2, -9, 40, 23, 17, 0, s, ts).items():
        assert got[yy, xx, c] == pytest.approx(want, rel=1e-12, abs=1e-12)
    assert (m.fallbacks == m.phi_calls) if thr == 0 else m.fallbacks == 0


def test_consistency_schedule_validation():
    base = {"kind": "consistency", "steps": 2, "sigmas": [80.0, 0.35]}
    assert schedule.sampler_sigmas(base) == [80.0, 0.35, 0.0]
    for bad in [dict(base, sigmas=[0.35, 80.0]), dict(base, sigmas=[80.0, -1.0]), dict(base, steps=3),
                dict(base, blend=[0, 2])]:
        with pytest.raises(ValueError):
            schedule.sampler_sigmas(bad)
