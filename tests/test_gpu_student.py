"""GPU parity of two-step consistency sampling (the student's sampler) and
of the teacher fallback judge, through the C-ABI, against the FP64 oracle.

Bars: analytic model rel L2 <= 1e-6; the half-width UNet student <= 1e-4;
judge decisions equal the oracle's (thresholds are placed in gaps of the
oracle's residuals, so FP32 vs FP64 rounding cannot flip one); crops
bit-exact.
"""
import math

import numpy as np
import pytest

from gpu_common import planar, rel_l2, require_gpu
from oracle.sampler import Model, sample

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctxs(weights):
    require_gpu()
    from paper_2512_08309_amd import td
    made = {}

    def get(config):
        if config not in made:
            made[config] = td.Context(0).load_weights(weights(config))
        return made[config]
    yield get
    for c in made.values():
        c.close()


@pytest.mark.parametrize("seed,region,level", [(0, (0, 0, 23, 17), 0), (3, (-37, 1000003, 40, 8), 0),
                                               (5, (3, -4, 31, 29), 1)])
def test_consistency_linear_gaussian_matches_oracle(ctxs, weights, seed, region, level):
    c = ctxs("lgs")
    c.set_judge(None, 0.0)
    assert c.info("steps") == 2 and c.info("levels") == 2
    got = c.sample_region(seed, *region, level)
    assert rel_l2(got, planar(sample(Model(weights("lgs")), seed, *region, level))) <= 1e-6


def gap_threshold(residuals):
    """A threshold in the widest relative gap of the residuals."""
    r = sorted(residuals)
    best, thr = 0.0, r[0] * 0.5
    for a, b in zip(r, r[1:]):
        if a > 0 and b / a > 1 + best:
            best, thr = b / a - 1, math.sqrt(a * b)
    assert best > 1e-3, "no usable gap"
    return thr


def judged_reference(weights, student, teacher, seed, region):
    """Oracle run with a threshold that no residual of that same run comes
    within 0.1% of (later steps' residuals depend on earlier decisions, so
    the threshold is re-placed until it is stable)."""
    m = Model(weights(student))
    m.judge = (Model(weights(teacher)), math.inf)
    sample(m, seed, *region, 0)
    thr = gap_threshold(m.residuals)
    for _ in range(4):
        m = Model(weights(student))
        m.judge = (Model(weights(teacher)), thr)
        ref = planar(sample(m, seed, *region, 0))
        if min(abs(math.log(r / thr)) for r in m.residuals if r > 0) > 1e-3:
            return m, thr, ref
        thr = gap_threshold(m.residuals)
    raise AssertionError("no stable threshold")


@pytest.mark.parametrize("mode", ["all", "none", "mixed"])
def test_linear_gaussian_judge_matches_oracle(ctxs, weights, mode):
    c, t = ctxs("lgs"), ctxs("lg")
    region = (-9, 40, 47, 33)
    if mode == "mixed":
        m, thr, ref = judged_reference(weights, "lgs", "lg", 2, region)
    else:
        thr = {"all": 0.0, "none": 1e30}[mode]
        m = Model(weights("lgs"))
        m.judge = (Model(weights("lg")), thr)
        ref = planar(sample(m, 2, *region, 0))
    c.set_judge(t, thr)
    c.cache_clear()                 # counters from zero
    try:
        got = c.sample_region(2, *region, 0)
        st = c.cache_stats()
    finally:
        c.set_judge(None, 0.0)
    assert rel_l2(got, ref) <= 1e-6
    assert st["judge_fallbacks"] == m.fallbacks and st["misses"] == m.phi_calls
    if mode == "mixed":
        assert 0 < m.fallbacks < m.phi_calls


def test_unet_student_matches_oracle(ctxs, weights):
    c = ctxs("s2")
    got = c.sample_region(4, -20, 33, 40, 24, 0)
    assert rel_l2(got, planar(sample(Model(weights("s2")), 4, -20, 33, 40, 24, 0))) <= 1e-4


def test_unet_student_with_teacher_judge_matches_oracle(ctxs, weights):
    """Mixed fallbacks: the flagged windows take the narrow teacher's plain
    J_0 on their regions (the oracle samples each one)."""
    c, t = ctxs("s2"), ctxs("c2n")
    m2, thr, ref = judged_reference(weights, "s2", "c2n", 1, (7, 7, 16, 16))
    c.set_judge(t, thr)
    c.cache_clear()
    try:
        got = c.sample_region(1, 7, 7, 16, 16, 0)
        st = c.cache_stats()
    finally:
        c.set_judge(None, 0.0)
    assert rel_l2(got, ref) <= 1e-4
    assert st["judge_fallbacks"] == m2.fallbacks
    assert 0 < m2.fallbacks < m2.phi_calls


@pytest.mark.parametrize("student,teacher,region", [("s2", "c2", (-40, 77, 70, 52)),
                                                    ("lgs", "lg", (1000003, -29, 41, 37))])
def test_threshold_zero_is_teacher_plain_sample(ctxs, student, teacher, region):
    """Threshold 0: every window falls back at both steps, so the judged
    student's J_0 is the teacher's plain J_0 (the 20-step C2 sampler for s2)
    and its J_1 that plus 0.35 G on counter word 1."""
    from oracle import noise as onoise
    c, t = ctxs(student), ctxs(teacher)
    want0 = t.sample_region(6, *region, 0)
    c.set_judge(t, 0.0)
    c.cache_clear()
    try:
        got0 = c.sample_region(6, *region, 0)
        st = c.cache_stats()
        c.cache_clear()
        got1 = c.sample_region(6, *region, 1)
    finally:
        c.set_judge(None, 0.0)
    assert st["judge_fallbacks"] == st["misses"] > 0
    assert rel_l2(got0, want0) <= 1e-6
    g1 = planar(onoise.noise_region(6, region[0], region[1], region[2], region[3], 4, step=1))
    assert rel_l2(got1, want0 + np.float32(0.35) * g1) <= 1e-6


def test_student_seed_consistency_bit_exact(ctxs):
    c = ctxs("s2")
    c.cache_clear()
    big = c.sample_region(8, -50, -30, 120, 90, 0)
    c.cache_clear()
    c.set_option("batch", 3)
    try:
        small = c.sample_region(8, -21, 1, 45, 38, 0)
    finally:
        c.set_option("batch", 4096)
    assert np.array_equal(small, big[:, 31:69, 29:74])


def test_judge_errors(ctxs, weights):
    from paper_2512_08309_amd import td
    c1 = ctxs("c1")
    with pytest.raises(td.TDError) as e:
        c1.set_judge(ctxs("c2"), 0.05)                   # not a consistency model
    assert e.value.status == td.TD_E_INVAL
    s = ctxs("lgs")
    with pytest.raises(td.TDError):
        s.set_judge(s, 0.05)
    with pytest.raises(td.TDError) as e:
        s.set_judge(ctxs("c1"), 0.05)                    # 1 channel vs 4
    assert e.value.status == td.TD_E_INVAL
    s.cache_clear()
    assert s.sample_region(0, 0, 0, 8, 8, 0).shape == (4, 8, 8)   # the failed call left no judge
    assert s.cache_stats()["judge_fallbacks"] == 0
    # a teacher reloaded with another layout is refused at query time
    with td.Context(0) as t:
        t.load_weights(weights("lg"))
        s.set_judge(t, 0.05)
        try:
            t.load_weights(weights("c1"))
            with pytest.raises(td.TDError) as e:
                s.sample_region(0, 0, 0, 8, 8, 0)
            assert e.value.status == td.TD_E_STATE
        finally:
            s.set_judge(None, 0.0)


def test_window_local_steps_match_oracle(ctxs, weights):
    """td_denoise_steps: the plain sampler on independent windows (the teacher
    output of distillation)."""
    import torch
    from oracle.schedule import euler_factor
    from oracle.tdw import read_tdw
    from oracle.unet import UNetDenoiser
    c = ctxs("c1k2")
    hdr, t = read_tdw(weights("c1k2"))
    m = Model(weights("c1k2"))
    x = (80.0 * np.random.default_rng(12).standard_normal((3, 32, 32, 1))).astype(np.float32)
    out = torch.empty((3, 32, 32, 1), device="cuda")
    c.denoise_steps(torch.from_numpy(x).cuda(), 0, 2, out)
    ref = x.astype(np.float64)
    den = UNetDenoiser(hdr, t)
    for k in range(2):
        ref = ref + euler_factor(m.sched[k], m.sched[k + 1]) * (ref - den(ref, m.sched[k], None))
    assert rel_l2(out.cpu().numpy(), ref) <= 1e-5


def test_noise_region_any_counter_word():
    require_gpu()
    import torch
    from oracle import noise as onoise
    from paper_2512_08309_amd import td
    out = torch.empty((9, 13, 4), device="cuda")
    td.td_noise_region(77, -5, 1000, out, step=1, scale=0.35)
    torch.cuda.synchronize()
    want = np.float32(0.35) * onoise.noise_region(77, -5, 1000, 13, 9, 4, step=1)
    assert np.array_equal(out.cpu().numpy(), want)


def test_noise_region_accumulate():
    """accumulate = 1 adds scale * G to the buffer (the re-noising of
    distillation): one float32 multiply and one add per value, bit-exact."""
    require_gpu()
    import torch
    from oracle import noise as onoise
    from paper_2512_08309_amd import td
    base = np.random.default_rng(4).standard_normal((9, 13, 4)).astype(np.float32)
    out = torch.from_numpy(base).cuda()
    td.td_noise_region(77, -5, 1000, out, step=1, scale=0.35, accumulate=True)
    torch.cuda.synchronize()
    want = base + np.float32(0.35) * onoise.noise_region(77, -5, 1000, 13, 9, 4, step=1)
    assert np.array_equal(out.cpu().numpy(), want)
