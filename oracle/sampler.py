"""The sampled latent J_t[R] by its definition (no cache).

TEST INFRASTRUCTURE (oracle).

* J_T(p, c) = sigma_0 G(seed, x, y, c, step=0) (seeds paragraph of the formal
  appendix; G in oracle.noise).
* For t < T, J_t on a region R is the InfiniteDiffusion update (Eq. 2): the
  windows kappa(R) are run through Phi on J_{t+1}[R_i], each output is
  weighted by W_i and placed at R_i (U_i), the placed sums are divided
  pixel by pixel by the placed weights, with 0/0 := 0 (formal appendix).
  Phi is one Euler step of the window (oracle.schedule).
* The recursion is unrolled into the query's dependency cone (Alg. 1 is a
  memoised evaluation of the same definition; the Parallelization theorem
  gives one batched round per level): R_t = query, I_t = kappa(R_t),
  R_{t+1} = bounding region of the windows of I_t; then levels are evaluated
  on finite canvases from t = T-1 down to the query level.
* Summation over the windows covering a pixel runs in canonical order
  (iy ascending, then ix ascending).
* Levels are blend levels: T = K unless the header truncates T (Phi then
  runs several window-local Euler steps, oracle.schedule.level_steps).
* J_T uses the noise counter word the header names ("noise_step", default
  0), so that the stages of a hierarchy draw independent noise.
* Consistency sampling (oracle.schedule): Phi of step k is D(x; s_k) plus
  s_{k+1} G(step = k + 1) on the window's pixels.  With a judge (Model.judge
  = (teacher, threshold)), a window whose denoised estimate differs from the
  teacher's one-step estimate D_teacher(x; s_k) by more than the threshold
  in RMS over the window takes, instead of its estimate, the teacher's plain
  sample J_0 on the window's region (same seed; read from one teacher sample
  over the flagged windows' bounding region): the plain sampler as the
  fallback (Sec. 3.4 lets Phi be a few-step model; Sec. 5.3 and the
  distillation appendix distil the core model into two steps).  With
  threshold 0 every window falls back at both steps, and J_0 of the judged
  student is the teacher's plain J_0 (J_1 is it plus s_1 G(step = 1)).
* Hierarchy (Sec. 5.1; DAGs of infinite tensors, infinite-tensor appendix):
  a model whose header has "cond" = {channels, factor f} is the child of a
  parent model (Model.parent).  Window i of the child receives, besides
  J_{t+1}[R_i], the parent's final latent J_0 nearest-upsampled by f:
  child pixel (X, Y) reads parent pixel (floor(X/f), floor(Y/f)).  The
  parent is sampled (same seed) on the region that covers every window of
  the child's cone.

Outputs are float64 arrays [h, w, C] (row y, column x, channel).

Pins (tests/test_oracle_sampler.py): closed form of the whole sampler under
the linear-Gaussian denoiser; equality with brute-force bounded
MultiDiffusion (Eq. 1) over a canvas holding the whole cone; crop and
query-order independence.
"""
import numpy as np

from .noise import noise_region
from .schedule import blend_points, euler_factor, level_steps, sampler_sigmas
from .tdw import read_tdw
from .unet import make_denoiser
from .windows import cone, kappa_list, weight_map


class Model:
    """A weight file opened by the oracle: header, float64 tensors, denoiser."""

    def __init__(self, path_or_header, tensors=None, parent=None):
        if isinstance(path_or_header, str):
            self.header, self.tensors = read_tdw(path_or_header)
        else:
            self.header, self.tensors = path_or_header, (tensors or {})
        h = self.header
        self.C = h["denoiser"]["in_channels"]
        self.steps = h["sampler"]["steps"]
        self.noise_step = h["sampler"].get("noise_step", 0)
        self.cond = h.get("cond")
        self.parent = parent
        if self.cond and parent is not None and parent.C != self.cond["channels"]:
            raise ValueError("parent channels do not match the conditioning channels")
        self.points = blend_points(h["sampler"])
        self.K = len(self.points) - 1          # blend levels T
        win = h["window"]
        self.H, self.s, self.o, self.eps = win["size"], win["stride"], win["offset"], win["eps"]
        sp = h["sampler"]
        self.consistency = sp.get("kind", "edm") == "consistency"
        self.sched = sampler_sigmas(sp)
        self.judge = None          # (teacher Model, RMS threshold) for consistency sampling
        self.fallbacks = 0
        self.residuals = []        # the judge's RMS differences, in evaluation order
        self.W = weight_map(self.H, self.eps)
        self.denoiser = make_denoiser(h, self.tensors)
        self.phi_calls = 0


def _crop(canvas, canvas_region, sub):
    cx, cy = canvas_region[0], canvas_region[1]
    x0, y0, w, h = sub
    return canvas[y0 - cy:y0 - cy + h, x0 - cx:x0 - cx + w]


def conditioning(model, seed, region):
    """Conditioning source of a child model for windows inside `region`:
    the parent's J_0 on the parent-resolution cover of the region."""
    if model.parent is None:
        raise ValueError("a conditioned model needs its parent model")
    f = model.cond["factor"]
    x0, y0, w, h = region
    cx0, cy0 = x0 // f, y0 // f
    cw, ch = (x0 + w - 1) // f - cx0 + 1, (y0 + h - 1) // f - cy0 + 1
    return f, (cx0, cy0), sample(model.parent, seed, cx0, cy0, cw, ch, 0)


def cond_windows(src, windows, model):
    """[n, H, H, C_y]: the nearest-upsampled conditioning of each window."""
    f, (cx0, cy0), J = src
    out = []
    for ix, iy in windows:
        ox, oy = ix * model.s + model.o, iy * model.s + model.o
        rows = np.arange(oy, oy + model.H, dtype=np.int64) // f - cy0
        cols = np.arange(ox, ox + model.H, dtype=np.int64) // f - cx0
        out.append(J[rows[:, None], cols[None, :]])
    return np.stack(out)


def judged(model, D, x, sigma, windows, cond, seed):
    """The student's estimate per window, or the teacher's plain sample J_0 on
    the window's region where the student differs from the teacher's one-step
    estimate by more than the threshold (RMS over the window)."""
    teacher, thr = model.judge
    DT = teacher.denoiser(x, sigma, windows, cond if teacher.cond else None)
    r = np.sqrt(((D - DT) ** 2).mean(axis=(1, 2, 3)))
    model.residuals.extend(float(v) for v in r)
    use = r > thr
    model.fallbacks += int(use.sum())
    if not use.any():
        return D
    # J_0 of the teacher on each flagged window's region, read from one
    # sample over their bounding region: the same values, since a region's
    # sample is the crop of any larger region's (seed consistency theorem of
    # the formal appendix; pinned by the crop-independence tests)
    idx = np.nonzero(use)[0]
    ox = np.array([windows[i][0] * model.s + model.o for i in idx], dtype=np.int64)
    oy = np.array([windows[i][1] * model.s + model.o for i in idx], dtype=np.int64)
    bx, by = int(ox.min()), int(oy.min())
    big = sample(teacher, seed, bx, by, int(ox.max()) + model.H - bx, int(oy.max()) + model.H - by, 0)
    out = D.copy()
    for i, px, py in zip(idx, ox - bx, oy - by):
        out[i] = big[py:py + model.H, px:px + model.H]
    return out


def level_step(model, j_next, region_next, region, windows, t, cond_src=None, seed=None):
    """J_t on `region` from J_{t+1} on `region_next` using the given windows."""
    H = model.H
    x0, y0, w, h = region
    A = np.zeros((h, w, model.C))
    B = np.zeros((h, w, 1))
    if windows:
        xs = np.stack([_crop(j_next, region_next, (ix * model.s + model.o, iy * model.s + model.o, H, H))
                       for ix, iy in windows])
        cond = None
        if model.cond:
            if cond_src is None:
                raise ValueError("conditioned model stepped without its conditioning")
            cond = cond_windows(cond_src, windows, model)
        phi = xs
        for k in level_steps(model.points, t):
            sig, sig_next = model.sched[k], model.sched[k + 1]
            D = model.denoiser(phi, sig, windows, cond)
            if not model.consistency:
                phi = phi + euler_factor(sig, sig_next) * (phi - D)
                continue
            if model.judge is not None:
                D = judged(model, D, phi, sig, windows, cond, seed)
            phi = D
            if sig_next > 0:
                phi = phi + sig_next * np.stack([
                    noise_region(seed, ix * model.s + model.o, iy * model.s + model.o, H, H, model.C, k + 1)
                    for ix, iy in windows]).astype(np.float64)
        model.phi_calls += len(windows)
        for n, (ix, iy) in enumerate(windows):
            ox, oy = ix * model.s + model.o, iy * model.s + model.o
            ax0, ax1 = max(ox, x0), min(ox + H, x0 + w)
            ay0, ay1 = max(oy, y0), min(oy + H, y0 + h)
            if ax0 >= ax1 or ay0 >= ay1:
                continue
            wv = model.W[ay0 - oy:ay1 - oy, ax0 - ox:ax1 - ox, None]
            A[ay0 - y0:ay1 - y0, ax0 - x0:ax1 - x0] += wv * phi[n, ay0 - oy:ay1 - oy, ax0 - ox:ax1 - ox]
            B[ay0 - y0:ay1 - y0, ax0 - x0:ax1 - x0] += wv
    out = np.zeros_like(A)
    np.divide(A, B, out=out, where=B > 0)
    return out


def sample(model, seed, x0, y0, w, h, level):
    """J_level on [x0, x0+w) x [y0, y0+h): float64 [h, w, C]."""
    K = model.K
    if not 0 <= level <= K:
        raise ValueError("level out of range")
    region = (x0, y0, w, h)
    if level == K:
        return model.sched[0] * noise_region(seed, x0, y0, w, h, model.C, model.noise_step).astype(np.float64)
    regions, kappas = cone(region, level, K, model.H, model.s, model.o)
    top = level
    while top < K and kappas[top] is not None:
        top += 1
    if top == K:
        rK = regions[K]
        j = model.sched[0] * noise_region(seed, rK[0], rK[1], rK[2], rK[3], model.C,
                                          model.noise_step).astype(np.float64)
    else:
        j = np.zeros((regions[top][3], regions[top][2], model.C))
    # every window of the cone lies inside the top region
    src = conditioning(model, seed, regions[top]) if (model.cond and top > level) else None
    for t in range(top - 1, level - 1, -1):
        j = level_step(model, j, regions[t + 1], regions[t], kappa_list(regions[t], model.H, model.s, model.o), t,
                       src, seed)
    return j


def sample_levels(model, seed, x0, y0, w, h, level=0):
    """{t: J_t on [x0, x0+w) x [y0, y0+h)} for t = level..K from one evaluation
    of the cone (each level's canvas contains the query region)."""
    K = model.K
    region = (x0, y0, w, h)
    regions, kappas = cone(region, level, K, model.H, model.s, model.o)
    if any(kappas[t] is None for t in range(level, K)):
        raise ValueError("sample_levels needs a layout without gaps")
    rK = regions[K]
    j = model.sched[0] * noise_region(seed, rK[0], rK[1], rK[2], rK[3], model.C,
                                      model.noise_step).astype(np.float64)
    out = {K: _crop(j, rK, region).copy()}
    src = conditioning(model, seed, rK) if model.cond else None
    for t in range(K - 1, level - 1, -1):
        j = level_step(model, j, regions[t + 1], regions[t], kappa_list(regions[t], model.H, model.s, model.o), t,
                       src, seed)
        out[t] = _crop(j, regions[t], region).copy()
    return out
