"""EDM noise schedule, preconditioning and the per-level Euler step.

TEST INFRASTRUCTURE (oracle).  The paper leaves Phi abstract ("a pretrained
diffusion model", Sec. 3.1; "an arbitrary denoising function", Sec. 3.4).
The reading used here is the EDM sampler of Karras et al. (2022):

* sigma_k = (smax^(1/rho) + k/(K-1) (smin^(1/rho) - smax^(1/rho)))^rho for
  k = 0..K-1 and sigma_K = 0; level t holds the state at sigma_{K-t}.
* D(x; sigma) = c_skip x + c_out F(c_in x; c_noise) with
  c_skip = sd^2/(sigma^2+sd^2), c_out = sigma sd / sqrt(sigma^2+sd^2),
  c_in = 1/sqrt(sigma^2+sd^2), c_noise = ln(sigma)/4.
* Phi for the step t+1 -> t is one deterministic Euler step of the window:
  Phi(x) = x + (sigma' - sigma)/sigma (x - D(x; sigma)), sigma = sigma_{K-t-1},
  sigma' = sigma_{K-t}.  At the last step sigma' = 0 and Phi(x) = D(x).

* Truncated T (Sec. 3.4): blends happen only after the schedule indices in
  the header's "blend" list; level t then holds the state at
  sigma_{b_{T-t}} and its Phi runs the Euler steps b_{T-t-1} .. b_{T-t}-1
  on the window alone.
* Few-step consistency sampling (Sec. 3.4 lets Phi be a few-step
  consistency model; the paper's core model takes two steps with the
  intermediate sigma 0.35, implementation-details table): the header gives
  "kind": "consistency" and the noise levels "sigmas" [s_0 > ... > s_{K-1}],
  with s_K = 0.  Step k maps x to D(x; s_k) + s_{k+1} G(seed, ., ., c,
  step = k + 1): the denoised estimate re-noised to the next level with
  fresh coordinate-hashed noise (multistep consistency sampling, Song et al.
  2023).  Every step is blended (T = K).

Pins: the schedule's end points and monotonicity; the linear-Gaussian
closed form of the whole sampler (tests/test_oracle_sampler.py) fixes the
level indexing, the Euler factor and the preconditioning-free path, for
every blend schedule.
"""
import math


def sampler_sigmas(sampler):
    """[sigma_0, ..., sigma_{K-1}, 0] of either sampler kind."""
    if sampler.get("kind", "edm") == "consistency":
        s = [float(v) for v in sampler["sigmas"]]
        if not s or any(v <= 0 for v in s) or any(a <= b for a, b in zip(s, s[1:])):
            raise ValueError("consistency sigmas must be positive and decreasing")
        if len(s) != sampler["steps"] or "blend" in sampler:
            raise ValueError("consistency sampling blends every one of its steps")
        return s + [0.0]
    return sigmas(sampler["steps"], sampler["sigma_max"], sampler["sigma_min"], sampler["rho"])


def sigmas(steps, sigma_max, sigma_min, rho):
    """[sigma_0, ..., sigma_{K-1}, 0] in float64."""
    if steps == 1:
        return [float(sigma_max), 0.0]
    a = sigma_max ** (1.0 / rho)
    b = sigma_min ** (1.0 / rho)
    s = [(a + k / (steps - 1) * (b - a)) ** rho for k in range(steps)]
    return s + [0.0]


def sigma_pair(sched, steps, t):
    """(sigma, sigma') used by the step that produces level t from level t+1."""
    return sched[steps - t - 1], sched[steps - t]


def blend_points(sampler):
    """Schedule indices b_0 = 0 < b_1 < ... < b_T = K after which the windows
    are blended.  Default: after every step (T = K).  With T < K, Phi of a
    level runs several window-local Euler steps (truncated T, Sec. 3.4)."""
    K = sampler["steps"]
    b = list(sampler.get("blend", range(K + 1)))
    if b[0] != 0 or b[-1] != K or any(x >= y for x, y in zip(b, b[1:])):
        raise ValueError("blend points must rise strictly from 0 to K")
    return b


def level_steps(points, t):
    """Schedule indices k of the Euler steps Phi runs to produce blend level t."""
    T = len(points) - 1
    return list(range(points[T - t - 1], points[T - t]))


def precond(sigma, sigma_data):
    s2 = sigma * sigma + sigma_data * sigma_data
    c_skip = sigma_data * sigma_data / s2
    c_out = sigma * sigma_data / math.sqrt(s2)
    c_in = 1.0 / math.sqrt(s2)
    c_noise = 0.25 * math.log(sigma)
    return c_skip, c_out, c_in, c_noise


def euler_factor(sigma, sigma_next):
    return (sigma_next - sigma) / sigma
