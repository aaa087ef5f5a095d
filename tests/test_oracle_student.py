"""Pins of few-step consistency sampling (the student's sampler) and of the
teacher fallback judge.

* Closed form with the analytic linear-Gaussian model ``lgs`` (prior std
  s = 0.7, sigmas 80 and 0.35): J_1(p) = m(p) + a_0 (80 G_0(p) - m(p)) +
  0.35 G_1(p) and J_0(p) = m(p) + a_1 (J_1(p) - m(p)) with a_k = s^2 /
  (s^2 + sigma_k^2), G_1 the noise on counter word 1, m the brute-force
  weighted window mean.
* The judge at threshold 0 replaces every window's estimate by the
  teacher's plain sample J_0 on the window's region (``lg``, s = 0.5, 8 EDM
  steps), at an infinite threshold by none: both closed forms.  At
  threshold 0 the judged student's J_0 is the teacher's plain J_0 (the
  linear-Gaussian closed form of the 8-step EDM sampler) and its J_1 that
  plus s_1 G_1, since the blend of position-consistent fields returns them.
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
    """J_level of two-step consistency sampling with a linear-Gaussian prior
    of std s; with teacher_sched, every estimate is the teacher's plain J_0
    (EDM Euler through teacher_sched, which starts at the student's s_0)."""
    sig = m.sched
    g0 = noise.noise_region(seed, x0, y0, w, h, 4, step=0).astype(np.float64)
    g1 = noise.noise_region(seed, x0, y0, w, h, 4, step=1).astype(np.float64)
    out = {}
    for yy, xx, c in [(0, 0, 0), (h - 1, w - 1, 3), (5, 11, 1), (16, 2, 2), (8, 8, 0)]:
        mu = brute_mu_bar(x0 + xx, y0 + yy, c, m.H, m.s, m.o, m.eps)
        if teacher_sched is None:   # the student's own estimates
            f = [s * s / (s * s + v * v) for v in sig[:2]]
            j1 = mu + f[0] * (sig[0] * g0[yy, xx, c] - mu) + sig[1] * g1[yy, xx, c]
            out[(yy, xx, c)] = j1 if level == 1 else mu + f[1] * (j1 - mu)
        else:                       # the teacher's plain J_0 at both steps
            assert teacher_sched[0] == sig[0]
            j0t = mu + (sig[0] * g0[yy, xx, c] - mu) * euler_product(teacher_sched, s)
            out[(yy, xx, c)] = j0t + sig[1] * g1[yy, xx, c] if level == 1 else j0t
    return out


@pytest.mark.parametrize("seed,x0,y0,level", [(0, 0, 0, 0), (3, -37, 1000003, 0), (5, 3, -4, 1)])
def test_consistency_linear_gaussian_closed_form(weights, seed, x0, y0, level):
    m = Model(weights("lgs"))
    assert m.consistency and m.K == 2 and m.sched == [80.0, 0.35, 0.0]
    got = sample(m, seed, x0, y0, 23, 17, level)
    for (yy, xx, c), want in closed_form(m, seed, x0, y0, 23, 17, level, 0.7).items():
        assert got[yy, xx, c] == pytest.approx(want, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("level", [0, 1])
@pytest.mark.parametrize("thr,s", [(0.0, 0.5), (math.inf, 0.7)])
def test_judge_extremes(weights, thr, s, level):
    m = Model(weights("lgs"))
    teacher = Model(weights("lg"))
    m.judge = (teacher, thr)
    got = sample(m, 2, -9, 40, 23, 17, level)
    ts = teacher.sched if thr == 0 else None
    for (yy, xx, c), want in closed_form(m, 2, -9, 40, 23, 17, level, s, ts).items():
        assert got[yy, xx, c] == pytest.approx(want, rel=1e-12, abs=1e-12)
    assert (m.fallbacks == m.phi_calls) if thr == 0 else m.fallbacks == 0


def test_judge_at_threshold_zero_is_the_teachers_plain_sample(weights):
    """Every pixel, not only the closed-form probes: the judged student's J_0
    equals the teacher's own plain sample of the same region and seed."""
    m = Model(weights("lgs"))
    teacher = Model(weights("lg"))
    m.judge = (teacher, 0.0)
    got = sample(m, 6, 1000001, -33, 41, 19, 0)
    want = sample(Model(weights("lg")), 6, 1000001, -33, 41, 19, 0)
    assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))
    assert m.fallbacks == m.phi_calls > 0


def test_consistency_schedule_validation():
    base = {"kind": "consistency", "steps": 2, "sigmas": [80.0, 0.35]}
    assert schedule.sampler_sigmas(base) == [80.0, 0.35, 0.0]
    for bad in [dict(base, sigmas=[0.35, 80.0]), dict(base, sigmas=[80.0, -1.0]), dict(base, steps=3),
                dict(base, blend=[0, 2])]:
        with pytest.raises(ValueError):
            schedule.sampler_sigmas(bad)
