"""Throughput benchmark of lazy windowed sampling on one MI355X.

A step is one cold query through the C-ABI: the decoded elevation of a
full-resolution region (default 8192 x 8192 px, i.e. a 1024 x 1024 latent
region plus the 17-pixel decode apron) of the 4-channel latent plane, with
the 4-level UNet (128/256/256/512, 8-head attention at 8x8), windows 64 at
stride 32 and 20 EDM steps: noise, every window of the dependency cone
through the batched denoiser, blend + Euler per level, the device cache,
the Laplacian decode and the result in device memory.  The cache is cleared
before every step, so every step does the full cold work.

Reported: window-denoises/s (denoiser evaluations per second of the timed
steps), the roofline of the dominant kernel (the FP32 MFMA 3x3 convolution)
from event timing of every launch inside the timed steps, the other kernel
classes, and, as further legs: reduced precision with its error against the
FP64 oracle, p50/p99 latency of tile streams (first tile and its
neighbour, as in time-to-first/second-tile), the distilled student, the
serving loop, a truncated blend schedule, and the FP64 oracle timed on the
host cores.

Run-time budget: the warm-up and timed steps always run; the further legs
run in a fixed priority order while their estimated cost fits the wall-clock
budget (--budget-s, counted from the start of the process), and a leg that
does not fit is recorded as skipped with its estimate.  The oracle legs run
on the host cores in a child process during the untimed warm-up steps and
are joined before the timed steps start.
"""
import argparse
import json
import os
import subprocess
import sys
import tempfile
import time

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
# Precision crop of the reduced-precision comparison: C1 model, 128 x 128
# latent at (3, 9), seed 5, every level; heightfield of its interior.
CROP = (3, 9, 128, 128)
CROP_SEED = 5
CROP_HEIGHT = (8 * 20, 8 * 26, 8 * 90, 8 * 90)


def parse(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--config", default="c2")
    p.add_argument("--size", type=int, default=1024, help="latent side of the query (full-res = 8x)")
    p.add_argument("--workload", choices=["height", "latent"], default="height")
    p.add_argument("--batch", type=int, default=0)
    p.add_argument("--seed", type=int, default=7)
    p.add_argument("--budget-s", type=float, default=470.0,
                   help="wall-clock budget of the whole run; legs after the timed steps that do not fit are skipped")
    p.add_argument("--latency-pairs", type=int, default=1000, help="tile pairs of the C1 latency stream")
    p.add_argument("--c2-latency-pairs", type=int, default=4, help="tile pairs of the C2 latency stream")
    p.add_argument("--cpu-windows", type=int, default=64, help="C2 windows of the timed oracle sample")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--bf16-steps", type=int, default=1,
                   help="cold steps timed again per reduced-precision mode (0 = skip)")
    p.add_argument("--lowp-modes", default="1,2", help="precision modes to time: 1 bf16, 2 bf16 + fp8 weights")
    p.add_argument("--truncated", default="c2t2", help="truncated-T config timed cold ('' = skip)")
    p.add_argument("--serve-queries", type=int, default=256, help="queries of the serving stream (0 = skip)")
    p.add_argument("--serve-rate", type=float, default=256.0, help="Poisson arrival rate, queries/s")
    p.add_argument("--serve-rate-sustained", type=float, default=32.0,
                   help="a second, lower arrival rate the server keeps up with (0 = skip)")
    p.add_argument("--student-steps", type=int, default=150,
                   help="AdamW steps of the in-bench student distillation (0 = skip the student leg)")
    p.add_argument("--student-pairs", type=int, default=2048, help="teacher pairs of the in-bench distillation")
    p.add_argument("--judge-thresholds", default="0.35,0.5,1",
                   help="further fallback thresholds of the judged student, timed while the budget allows")
    p.add_argument("--query-only", type=int, default=-1, metavar="PRECISION",
                   help="only one cold query of the workload at this precision (0 FP32, 1 BF16, 2 FP8 weights), "
                        "for profiler runs")
    p.add_argument("--micro-only", action="store_true",
                   help="only the decode / noise micro-benchmarks (8192^2 heightfield, 8192^2 x 4 noise)")
    p.add_argument("--calib-copy-mib", type=int, default=0,
                   help="run one plain elementwise copy (read N MiB, write N MiB) before the steps, as the "
                        "reference dispatch that scales hardware byte counters")
    p.add_argument("--cpu-legs", default="", help=argparse.SUPPRESS)
    p.add_argument("--c1-weights", default="", help=argparse.SUPPRESS)
    p.add_argument("--c2-weights", default="", help=argparse.SUPPRESS)
    return p.parse_args(argv)


class Budget:
    """Wall-clock budget counted from the start of the process."""

    def __init__(self, total):
        self.total = total

    def left(self):
        return self.total - (time.perf_counter() - T_START)

    def skip(self, est):
        """None if a leg of estimated cost `est` seconds fits, else the record
        that says why it was skipped."""
        if est <= self.left():
            return None
        return {"skipped": "run-time budget: needs ~%.0f s, %.0f s left of %.0f s" % (est, max(self.left(), 0.0),
                                                                                       self.total)}


# ----------------------------------------------------------------- host leg
# The cpu_baseline leg: the oracle (FP64 NumPy) on the host cores, in a child
# process that never touches the GPU, started before the warm-up steps and
# joined before the timed steps.  It times the oracle, and writes the oracle's
# values of the precision crop that the reduced-precision legs compare with.

def _nproc():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(a):
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import laplace
    from oracle.sampler import Model, sample, sample_levels
    ncores = _nproc()
    res = {"nproc": ncores}
    with threadpool_limits(limits=ncores, user_api="blas"):
        threads = max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
        res["blas_threads"] = threads
        if not a.no_cpu_baseline:
            m = Model(a.c2_weights)
            x = 80.0 * np.random.default_rng(0).standard_normal((a.cpu_windows, m.H, m.H, m.C))
            m.denoiser(x[:1], m.sched[0], None)          # warm BLAS
            t0 = time.perf_counter()
            m.denoiser(x, m.sched[0], None)
            dt = time.perf_counter() - t0
            res["c2_sample"] = {"windows": a.cpu_windows, "s": dt}
            print("[cpu] C2 oracle sample %.1f s" % dt, file=sys.stderr, flush=True)
            m1 = Model(a.c1_weights)
            t0 = time.perf_counter()
            sample(m1, 0, 0, 0, 64, 64, 0)
            dt1 = time.perf_counter() - t0
            res["c1_cold_query"] = {"windows": m1.phi_calls, "s": dt1}
            print("[cpu] C1 oracle cold query %.1f s" % dt1, file=sys.stderr, flush=True)
        if a.bf16_steps > 0:
            m1 = Model(a.c1_weights)
            t0 = time.perf_counter()
            lv = sample_levels(m1, CROP_SEED, *CROP, 0)
            dec = m1.header["decode"]
            lx0, ly0, lw, lh = laplace.required_latent(CROP_HEIGHT, dec)
            x0, y0 = CROP[0], CROP[1]
            lat = lv[0][ly0 - y0:ly0 - y0 + lh, lx0 - x0:lx0 - x0 + lw]
            href = laplace.decode(lat, (lx0, ly0), CROP_HEIGHT, dec)
            np.savez(os.path.join(a.cpu_legs, "crop_ref.npz"), height=href,
                     **{"level_%d" % t: v for t, v in lv.items()})
            print("[cpu] oracle precision crop %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    with open(os.path.join(a.cpu_legs, "cpu.json"), "w") as f:
        json.dump(res, f)


def start_cpu_legs(a, c1_path, c2_path, workdir):
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-legs", workdir, "--c1-weights", c1_path,
           "--c2-weights", c2_path, "--cpu-windows", str(a.cpu_windows), "--bf16-steps", str(a.bf16_steps)]
    if a.no_cpu_baseline:
        cmd.append("--no-cpu-baseline")
    return subprocess.Popen(cmd, cwd=ROOT)


def counter_traffic():
    """HBM bytes per launch of the dominant kernel (FP32 3x3 conv) from the
    committed counter summary, while the kernel source still matches the one
    the counters were taken on; else None."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "conv3x3_f32_and_bf16_halo_hbm_counters.md")
    src = os.path.join(ROOT, "paper_2512_08309_amd", "csrc", "k_conv.hip")
    try:
        rec = None
        for line in open(prof):
            if line.startswith("traffic_f32_conv3x3:"):
                rec = json.loads(line.split(":", 1)[1])
        if not rec:
            return None
        with open(src, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest()[:16] != rec["k_conv_sha256_16"]:
                return None
        return rec
    except (OSError, ValueError, KeyError):
        return None


def cpu_baseline_entry(cpu):
    """The bench line's cpu_baseline: the oracle's C2 window-denoises/s."""
    s = cpu.get("c2_sample")
    if not s:
        return None
    c1 = cpu.get("c1_cold_query", {})
    return {"value": s["windows"] / s["s"], "unit": "window-denoises/s", "cores": cpu["blas_threads"],
            "nproc": cpu["nproc"], "kind": "oracle",
            "sample": "%d windows of the 4-channel C2 model through the FP64 oracle denoiser at sigma_0 (one batched "
                      "level round; the blend/Euler is <0.1%% of the sampler's work), %.1f s; run on the host cores "
                      "during the GPU's untimed warm-up steps" % (s["windows"], s["s"]),
            "c1_cold_query": {"s": c1.get("s"), "windows": c1.get("windows"),
                              "window_denoises_per_s": (c1["windows"] / c1["s"]) if c1 else None,
                              "note": "the oracle's full cold 64x64 query of the 1-channel model at (0, 0), seed 0 "
                                      "(every level of its cone), timed in full"}}


# ----------------------------------------------------------------- GPU legs

def rel(torch, got, ref):
    return float(torch.linalg.vector_norm((got - ref).double()) / torch.linalg.vector_norm(ref.double()))


def precision_errors(td, torch, c1_path, ref_path, modes):
    """Error of every level of the precision crop and of its heightfield
    against the FP64 oracle, per precision mode (0 = FP32)."""
    import numpy as np
    ref = np.load(ref_path)
    out = {}
    for prec in [0] + modes:
        with td.Context(0) as c:
            c.load_weights(c1_path)
            c.set_option("precision", prec)
            K = c.info("levels")
            lv = {}
            for t in range(K, -1, -1):
                got = c.sample_region(CROP_SEED, *CROP, t)
                r = np.moveaxis(ref["level_%d" % t], -1, 0)
                lv[str(t)] = float(np.linalg.norm(got - r) / np.linalg.norm(r))
            h = c.sample_region(CROP_SEED, *CROP_HEIGHT, td.TD_LEVEL_HEIGHT)
            eh = float(np.linalg.norm(h - ref["height"]) / np.linalg.norm(ref["height"]))
        out[prec] = {"crop": "1-channel C1 model (K=8), 128x128 latent at (3, 9), seed 5; heightfield of the "
                             "720x720 px interior at (160, 208)",
                     "rel_l2_vs_fp64_oracle_by_level": lv, "rel_l2_vs_fp64_oracle_max_level": max(lv.values()),
                     "rel_rmse_heightfield_vs_fp64_oracle": eh}
    return out


def latency_stream(td, torch, weights_path, pairs, seed, deadline, precision=0, label="C1", ctx=None):
    """TTFT/TTST-style stream: 512x512 px elevation tiles (64x64 latent, the
    paper's tile at 8x) at random tile-aligned positions in [-1e6, 1e6)
    latent px and their right neighbours; end-to-end through
    td_sample_region_async (planning, every level of the cone, decode).
    Stops early at `deadline` (perf_counter time); n says how many ran.
    ctx: an already used context of the model (else a new one is made and
    warmed on one tile)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    xs = rng.integers(-10 ** 6 // 64, 10 ** 6 // 64, size=(pairs, 2)) * 64
    first, second = [], []
    out = torch.empty((512, 512), dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    own = ctx is None
    c = td.Context(0) if own else ctx
    try:
        if own:
            c.load_weights(weights_path)
            c.set_option("precision", precision)
            c.sample_region_async(seed, 0, 0, 512, 512, td.TD_LEVEL_HEIGHT, out, st)   # kernels, workspace
            torch.cuda.synchronize()
        c.cache_clear()
        for x, y in xs:
            if time.perf_counter() > deadline:
                break
            for dx, sink in ((0, first), (64, second)):
                t0 = time.perf_counter()
                c.sample_region_async(seed, 8 * (int(x) + dx), 8 * int(y), 512, 512, td.TD_LEVEL_HEIGHT, out, st)
                torch.cuda.synchronize()
                sink.append(1e3 * (time.perf_counter() - t0))
        cs = c.cache_stats()
        c.cache_clear()
    finally:
        if own:
            c.close()

    def pct(v):
        if not v:
            return {"n": 0}
        return {"p50_ms": float(np.percentile(v, 50)), "p99_ms": float(np.percentile(v, 99)),
                "max_ms": float(np.max(v)), "n": len(v)}
    return {"workload": "%s model, %s; %d random 512x512 px elevation tiles (64x64 latent + decode apron) at "
                        "tile-aligned positions in [-1e6,1e6) latent px, seed %d, each followed by its right "
                        "neighbour; end-to-end through td_sample_region_async (planning, cone, decode), default "
                        "cache budget" % (label, "FP32" if precision == 0 else "BF16", len(first), seed),
            "first": pct(first), "neighbour": pct(second), "windows_evaluated": cs["misses"],
            "planned_pairs": pairs}


def serving_stream(td, torch, weights_path, parent_path, n, rate, seed=17, budget=64 << 30, inflight=64,
                   precision=1):
    """Poisson stream of region queries through the continuous-batching server:
    sides uniform in [64, 512] latent px, coordinates uniform in [-1e6, 1e6),
    30% revisits of an earlier region (shifted by up to half its size).  The
    fine model is conditioned on a coarse model at 1/8 resolution when
    parent_path is given."""
    import numpy as np
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n))
    qs = []
    for i in range(n):
        if qs and rng.random() < 0.3:
            b = qs[rng.integers(len(qs))]
            dx, dy = (int(v) for v in rng.integers(-(b[2] // 2), b[2] // 2 + 1, size=2))
            qs.append((b[0] + dx, b[1] + dy, b[2], b[3]))
        else:
            w, h = (int(v) for v in rng.integers(64, 513, size=2))
            x, y = (int(v) for v in rng.integers(-10 ** 6, 10 ** 6, size=2))
            qs.append((x, y, w, h))
    with td.Context(0) as c, td.Context(0) as parent:
        c.load_weights(weights_path)
        c.set_option("precision", precision)
        if parent_path:
            parent.load_weights(parent_path)
            parent.set_option("precision", precision)
            c.set_conditioning(parent)
        C = c.info("channels")
        warm = torch.empty((C, 64, 64), device="cuda")
        c.sample_region_async(seed, 0, 0, 64, 64, 0, warm)     # kernels, workspaces
        torch.cuda.synchronize()
        c.cache_clear()
        outs, tick, lat = {}, {}, []
        with td.Server(c, budget, inflight) as srv:
            t0 = time.perf_counter()
            i = 0
            while len(lat) < n:
                now = time.perf_counter() - t0
                while i < n and arrivals[i] <= now:
                    x, y, w, h = qs[i]
                    outs[i] = torch.empty((C, h, w), device="cuda")
                    tick[i] = srv.submit(seed, x, y, w, h, 0, outs[i])
                    i += 1
                if srv.progress(1) == 0 and i < n:
                    time.sleep(max(0.0, min(1e-3, arrivals[i] - (time.perf_counter() - t0))))
                for j in list(tick):
                    ok, ms = srv.poll(tick[j])
                    if ok:
                        lat.append(ms)
                        del tick[j]
                        del outs[j]
            wall = time.perf_counter() - t0
            st = srv.stats()
        cs = c.cache_stats()
        ps = parent.cache_stats() if parent_path else None
    lat = np.array(lat)
    hier = ("conditioned on a coarse 2-level UNet (64/128, windows 32/16 at 1/8 resolution, K=8, one blend)"
            if parent_path else "no coarse conditioning model")
    return {"workload": "fine 1-channel model (2-level UNet 16/32, windows 32/16, K=8) %s, %s denoisers; "
                        "%d queries, Poisson %.0f q/s, sides U[64,512], coords U[-1e6,1e6), 30%% revisits; HBM "
                        "admission budget %d GB, <= %d in flight"
                        % (hier, "BF16" if precision == 1 else "FP32", n, rate, budget >> 30, inflight),
            "queries_per_s": n / wall, "window_denoises_per_s": st["batched_windows"] / wall,
            "coarse_window_denoises_per_s": (ps["denoiser_evals"] / wall) if ps else None,
            "latency_p50_ms": float(np.percentile(lat, 50)), "latency_p99_ms": float(np.percentile(lat, 99)),
            "rounds": st["rounds"], "mean_batch": st["batched_windows"] / max(st["rounds"], 1),
            "cache_hits": cs["hits"], "windows_evaluated": cs["misses"], "wall_s": wall}


def paper_context(lat):
    """The paper's own speed figure, quoted as context (other hardware, its
    trained models, a 512^2 tile at 90 m per pixel), and the same traversal
    arithmetic applied to the neighbour-tile latency of the C1 stream here
    (512^2 px elevation tiles of synthetic random-init models): not a
    like-for-like comparison."""
    tile_m = 512 * 90.0
    ctx = {"paper": "generation 9x faster than orbital velocity (7,700 m/s): time to second tile 0.66 s for a "
                    "512^2 tile at 90 m per pixel (46 km), consumer GPU, the paper's trained models"}
    if lat and lat.get("neighbour", {}).get("n"):
        t = lat["neighbour"]["p50_ms"] * 1e-3
        ctx["here"] = {"neighbour_tile_p50_s": t, "traversal_m_per_s": tile_m / t,
                       "x_orbital_velocity": tile_m / t / 7700.0,
                       "note": "C1 neighbour elevation tile (512^2 px) of the latency stream; synthetic 2-level "
                               "UNet, not the paper's models"}
    return ctx


def micro_bench(td, torch, ctx, reps=5):
    """HBM-bound kernels on their own: the Laplacian decode of a 1058^2 x 4 fBm
    terrain latent (seed 21) to an 8192^2 heightfield, the seed noise G on
    8192^2 x 4 values (counter word 0), and the Laplacian encode of that
    heightfield back to a latent; achieved GB/s of the bytes each must write
    (decode, noise) or read (encode)."""
    from synth.fbm import terrain_latent
    lx, ly = 13 - 17, -1000001 - 17
    lat = torch.from_numpy(terrain_latent(21, lx, ly, 1058, 1058)).cuda().contiguous()
    out = torch.empty((8192, 8192), device="cuda")
    noise = torch.empty((8192, 8192, 4), device="cuda")
    ctx.lap_decode(lat, lx, ly, 8 * 13, 8 * -1000001, 8192, 8192, out)     # first use: scratch
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    e0.record()
    for _ in range(reps):
        ctx.lap_decode(lat, lx, ly, 8 * 13, 8 * -1000001, 8192, 8192, out, stream)
    e1.record()
    torch.cuda.synchronize()
    dec_ms = e0.elapsed_time(e1) / reps
    e0.record()
    for _ in range(reps):
        td.td_noise_region(7, 0, 0, noise, step=0, scale=80.0)
    e1.record()
    torch.cuda.synchronize()
    noise_ms = e0.elapsed_time(e1) / reps
    X0, Y0 = 8 * 13, 8 * -1000001
    gx, gy, gw, gh = ctx.lap_encode(None, X0, Y0, 8192, 8192)
    lat_out = torch.empty((gh, gw, lat.shape[2]), device="cuda")
    ctx.lap_encode(out, X0, Y0, 8192, 8192, lat_out, stream)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        ctx.lap_encode(out, X0, Y0, 8192, 8192, lat_out, stream)
    e1.record()
    torch.cuda.synchronize()
    enc_ms = e0.elapsed_time(e1) / reps
    return {"decode_8192": {"ms": dec_ms, "GB_per_s_written": 8192 * 8192 * 4 / (dec_ms * 1e-3) / 1e9,
                            "note": "the decode's three kernels (block means, both blur passes in one LDS-tiled "
                                    "launch, full resolution); 268 MB of heightfield written"},
            "encode_8192": {"ms": enc_ms, "GB_per_s_read": 8192 * 8192 * 4 / (enc_ms * 1e-3) / 1e9,
                            "note": "the encode's three kernels on the decoded 8192^2 heightfield (268 MB read "
                                    "once algorithmically; the kernels read it twice) to a %dx%d latent" % (gw, gh)},
            "noise_8192x4": {"ms": noise_ms, "GB_per_s_written": noise.numel() * 4 / (noise_ms * 1e-3) / 1e9,
                             "note": "Philox + bit-exact IEEE Box-Muller per pair: ALU-bound"}}


def timed_cold(ctx, torch, a, region, level, out, stream):
    """First use on a small query (kernels, workspace), then one timed cold
    query of the region; returns (seconds, cache stats)."""
    ctx.sample_region_async(a.seed, 0, 0, 64, 64, 0, torch.empty((ctx.info("channels"), 64, 64), device="cuda"),
                            stream)
    torch.cuda.synchronize()
    ctx.cache_clear()
    t0 = time.perf_counter()
    ctx.sample_region_async(a.seed, *region, level, out, stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, ctx.cache_stats()


def student_leg(td, torch, teacher, teacher_path, student_init, a, region, level, out, ref32, stream, ms32, budget):
    """Distil the half-width two-step student from the 20-step teacher (a short
    run: a.student_pairs pairs, a.student_steps AdamW steps at batch 64, lr
    2e-4), then time the same cold query with it: alone, judged by the FP32
    teacher (fallback above 0.05 RMS), and with BF16 convolutions.  ms32 is
    the FP32 plain sampler's time per query (ms_per_step)."""
    from paper_2512_08309_amd import distill
    t0 = time.perf_counter()
    x, y, e = distill.make_pairs(td, torch, teacher_path, a.student_pairs, precision=1)
    xh, yh, eh = distill.make_pairs(td, torch, teacher_path, 256, seed0=1 + a.student_pairs, precision=1)
    t1 = time.perf_counter()
    P, hist = distill.train(td, torch, student_init, x, y, e, a.student_steps, batch=64, lr=2e-4, log_every=50)
    t2 = time.perf_counter()
    held = distill.evaluate(td, torch, student_init, P, xh, yh, eh)
    del x, y, e
    res = {"student": "half-width UNet 64/128/128/256 (14.0 M parameters, 8.67 GFLOP per window), two-step "
                      "consistency sampling at sigma 80 and 0.35, T = 2",
           "distillation": {"pairs": a.student_pairs, "steps": a.student_steps, "batch": 64, "lr": 2e-4,
                            "teacher": "20-step plain sampler of the bench model, BF16 convolutions",
                            "pair_s": round(t1 - t0, 1), "train_s": round(t2 - t1, 1),
                            "ms_per_train_step": round(1e3 * (t2 - t1) / a.student_steps, 1),
                            "loss_first_last": [hist[0][1], hist[-1][1]],
                            "heldout_window_rel_rmse_vs_teacher": held},
           "fp32_plain_ms_per_query": ms32}
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "student.tdw")
        distill.save(td, student_init, P, path)
        with td.Context(0) as s:
            s.load_weights(path)
            for name, judge, prec in (("student_fp32", None, 0), ("student_bf16", None, 1),
                                      ("student_judged_fp32", teacher, 0)):
                s.set_option("precision", prec)
                s.set_judge(judge, 0.05)
                dts, st = timed_cold(s, torch, a, region, level, out, stream)
                res[name] = {"ms_per_query": 1e3 * dts, "query_speedup_vs_fp32_plain": ms32 / (1e3 * dts),
                             "window_denoises_per_s": st["denoiser_evals"] / dts, "windows": st["misses"],
                             "judge_fallbacks": st["judge_fallbacks"],
                             "rel_rmse_heightfield_vs_fp32_plain": rel(torch, out, ref32)}
                print("[bench] %s done" % name, file=sys.stderr, flush=True)
            # the threshold -> (fallback rate, error, speed) curve of the judge
            curve = []
            for thr in [float(v) for v in a.judge_thresholds.split(",") if v]:
                sk = budget.skip(1.3 * ms32 * 1e-3 + 2.0)
                if sk:
                    curve.append(dict(sk, threshold=thr))
                    continue
                s.set_judge(teacher, thr)
                dts, st = timed_cold(s, torch, a, region, level, out, stream)
                curve.append({"threshold": thr, "ms_per_query": 1e3 * dts,
                              "query_speedup_vs_fp32_plain": ms32 / (1e3 * dts),
                              "fallback_rate": st["judge_fallbacks"] / max(st["misses"], 1),
                              "rel_rmse_heightfield_vs_fp32_plain": rel(torch, out, ref32)})
                print("[bench] judge threshold %g done" % thr, file=sys.stderr, flush=True)
            res["student_judged_fp32_threshold_curve"] = curve
            s.set_judge(None, 0.0)
    res["note"] = ("random-init teacher and a short distillation: the student does not reach the 2e-2 heightfield "
                   "RMSE; its speed is measured at the error it has")
    return res


def main():
    a = parse()
    if a.cpu_legs:
        cpu_baseline(a)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU and measures the per-GPU share of the sampling path "
              "(sharding across GPUs is not built); got --gpus %d" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    budget = Budget(a.budget_s)
    from synth.models import cached_weights
    wdir = os.path.join(ROOT, ".td_weights")
    wpath = cached_weights(a.config, wdir, 0)
    c1_path = cached_weights("c1", wdir, 0)
    c2_path = cached_weights("c2", wdir, 0)
    tmp = tempfile.TemporaryDirectory()
    cpu_proc = None
    if not a.micro_only and a.query_only < 0 and (not a.no_cpu_baseline or a.bf16_steps > 0):
        cpu_proc = start_cpu_legs(a, c1_path, c2_path, tmp.name)

    import torch

    from paper_2512_08309_amd import td

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = td.Context(0).load_weights(wpath)
    if a.micro_only:
        print(json.dumps({"micro": micro_bench(td, torch, ctx)}))
        ctx.close()
        return
    if a.query_only >= 0:
        ctx.set_option("precision", a.query_only)
        out = torch.empty((8 * a.size, 8 * a.size), dtype=torch.float32, device="cuda")
        dtq, stq = timed_cold(ctx, torch, a, (8 * 13, 8 * -1000001, 8 * a.size, 8 * a.size), td.TD_LEVEL_HEIGHT, out,
                              torch.cuda.current_stream())
        print(json.dumps({"query_only": {"precision": a.query_only, "s": dtq, "windows": stq["misses"],
                                         "window_denoises_per_s": stq["misses"] / dtq}}))
        ctx.close()
        return
    if a.batch:
        ctx.set_option("batch", a.batch)
    K, C = ctx.info("steps"), ctx.info("channels")
    H, S = ctx.info("window"), ctx.info("stride")
    lx, ly = 13, -1000001
    if a.workload == "height":
        region = (8 * lx, 8 * ly, 8 * a.size, 8 * a.size)
        level = td.TD_LEVEL_HEIGHT
        out = torch.empty((region[3], region[2]), dtype=torch.float32, device="cuda")
    else:
        region = (lx, ly, a.size, a.size)
        level = 0
        out = torch.empty((C, a.size, a.size), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        ctx.cache_clear()
        ctx.sample_region_async(a.seed, *region, level, out, stream)
        torch.cuda.synchronize()
        return ctx.cache_stats()["misses"]

    if a.calib_copy_mib:
        src = torch.ones(a.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    for i in range(a.warmup):
        print("[bench] warmup step %d" % i, file=sys.stderr, flush=True)
        step()
    cpu = {}
    if cpu_proc is not None:
        print("[bench] joining the host (oracle) legs", file=sys.stderr, flush=True)
        rc = cpu_proc.wait()
        if rc == 0:
            with open(os.path.join(tmp.name, "cpu.json")) as f:
                cpu = json.load(f)
        else:
            cpu = {"error": "oracle child process exited with %d" % rc}
    ctx.set_option("timing", 1)
    ctx.kernel_stats(reset=True)
    torch.cuda.synchronize()
    windows = 0
    t0 = time.perf_counter()
    for i in range(a.steps):
        windows += step()
        print("[bench] step %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ks = ctx.kernel_stats()
    ctx.set_option("timing", 0)
    step_s = dt / a.steps
    finite = bool(torch.isfinite(out).all().item())
    ref32 = out.clone()
    legs = ["micro", "reduced_precision", "latency", "student", "serving", "truncated_T", "latency_c2"]
    done = {}

    done["micro"] = budget.skip(2.0) or micro_bench(td, torch, ctx)

    lowp = None
    if a.bf16_steps > 0:
        lowp = {}
        names = {1: "bf16", 2: "bf16_fp8w"}
        descr = {1: "BF16 convolution operands (activations and weights), FP32 accumulation",
                 2: "BF16 activations, FP8 e4m3 weights with per-output-channel FP32 scales, FP32 accumulation"}
        modes = [int(v) for v in a.lowp_modes.split(",") if v]
        est = 2.0 + a.bf16_steps * step_s / 3.0
        for mode in modes:
            sk = budget.skip(est)
            if sk:
                lowp[names[mode]] = sk
                continue
            ctx.set_option("precision", mode)
            ctx.sample_region_async(a.seed, 0, 0, 64, 64, 0, torch.empty((C, 64, 64), device="cuda"), stream)
            torch.cuda.synchronize()                   # first use: converted weights, kernels
            ctx.set_option("timing", 1)
            ctx.kernel_stats(reset=True)
            w16 = 0
            t1 = time.perf_counter()
            for i in range(a.bf16_steps):
                w16 += step()
                print("[bench] precision %d step %d done" % (mode, i), file=sys.stderr, flush=True)
            dt16 = time.perf_counter() - t1
            est = 2.0 + dt16
            ks16 = ctx.kernel_stats()
            ctx.set_option("timing", 0)
            c16 = ks16.get("conv3x3_mfma_bf16", {"ms": 0.0, "flops": 0.0, "launches": 0})
            lowp[names[mode]] = {
                "precision": descr[mode] + "; GN statistics, attention, input/output layers, blend/Euler and "
                                           "decode FP32",
                "value": w16 / dt16, "ms_per_step": 1e3 * dt16 / a.bf16_steps,
                "speedup_vs_fp32": (w16 / dt16) / (windows / dt),
                "rel_rmse_heightfield_vs_fp32_gpu": rel(torch, out, ref32),
                "conv3x3_TFLOP/s": round(c16["flops"] / (c16["ms"] * 1e-3) / 1e12, 1) if c16["ms"] else None,
                "conv3x3_frac_of_bf16_peak": round(c16["flops"] / (c16["ms"] * 1e-3) / 1e12 /
                                                   PEAK_BF16_MFMA_TFLOPS, 4) if c16["ms"] else None,
                "kernels_ms": {k: round(v["ms"], 1) for k, v in sorted(ks16.items(), key=lambda kv: -kv[1]["ms"])}}
        ctx.set_option("precision", 0)
        ref_path = os.path.join(tmp.name, "crop_ref.npz")
        if os.path.exists(ref_path):
            sk = budget.skip(5.0)
            if sk:
                lowp["vs_fp64_oracle"] = sk
            else:
                errs = precision_errors(td, torch, c1_path, ref_path,
                                        [m for m in modes if names[m] in lowp and "skipped" not in lowp[names[m]]])
                lowp["fp32_vs_fp64_oracle"] = errs.pop(0)
                for m, e in errs.items():
                    lowp[names[m]]["vs_fp64_oracle"] = e
        else:
            lowp["vs_fp64_oracle"] = {"skipped": "no oracle reference (host legs failed)"}
    done["reduced_precision"] = lowp

    if a.latency_pairs > 0:
        sk = budget.skip(8.0)
        if sk:
            done["latency"] = sk
        else:
            print("[bench] latency stream (C1)", file=sys.stderr, flush=True)
            deadline = time.perf_counter() + min(25.0, budget.left() - 5.0)
            done["latency"] = latency_stream(td, torch, c1_path, a.latency_pairs, 11, deadline)

    if a.student_steps > 0 and a.config == "c2":
        est = 0.0025 * (a.student_pairs + 256) + 0.09 * a.student_steps + 6.0 + 0.7 * step_s
        sk = budget.skip(est)
        if sk:
            done["student"] = sk
        else:
            print("[bench] student distillation", file=sys.stderr, flush=True)
            done["student"] = student_leg(td, torch, ctx, wpath, cached_weights("s2", wdir, 0), a, region, level,
                                          out, ref32, stream, 1e3 * step_s, budget)

    if a.serve_queries > 0:
        sk = budget.skip(5.0 + (a.serve_queries / a.serve_rate_sustained if a.serve_rate_sustained > 0 else 0))
        if sk:
            done["serving"] = sk
        else:
            print("[bench] serving stream", file=sys.stderr, flush=True)
            srv = serving_stream(td, torch, cached_weights("c1h", wdir, 0), cached_weights("cc", wdir, 0),
                                 a.serve_queries, a.serve_rate)
            if a.serve_rate_sustained > 0:
                print("[bench] serving stream (sustained rate)", file=sys.stderr, flush=True)
                srv = {"offered_%g_qps" % a.serve_rate: srv,
                       "offered_%g_qps" % a.serve_rate_sustained:
                           serving_stream(td, torch, cached_weights("c1h", wdir, 0), cached_weights("cc", wdir, 0),
                                          a.serve_queries, a.serve_rate_sustained)}
            done["serving"] = srv

    if a.truncated:
        # cost of the same query when the windows are blended at T < K levels
        # (Sec. 3.4): analytic cone counts, and one timed cold step
        def cone(size, T):
            return td.td_cone_windows(lx, ly, size, size, 0, T, H, S)
        trunc = {"cone_windows_by_T": {str(T): {str(sz): cone(sz, T) for sz in (128, 512, 1024)}
                                       for T in (1, 2, 5, 20)},
                 "note": "window evaluations of a cold latent query of side 128/512/1024 at (13,-1000001); "
                         "each evaluation runs K/T = 20/T Euler steps of the network"}
        sk = budget.skip(2.0 + 0.5 * step_s)
        if sk:
            trunc["timed"] = sk
        else:
            with td.Context(0) as tctx:
                tctx.load_weights(cached_weights(a.truncated, wdir, 0))
                dtt, stt = timed_cold(tctx, torch, a, region, level, out, stream)
                trunc["timed"] = {"config": a.truncated, "T": tctx.info("levels"), "ms_per_step": 1e3 * dtt,
                                  "windows": stt["misses"], "denoiser_evals": stt["denoiser_evals"],
                                  "denoiser_evals_per_s": stt["denoiser_evals"] / dtt,
                                  "speedup_vs_T20_step": step_s / dtt,
                                  "rel_rmse_heightfield_vs_T20": rel(torch, out, ref32)}
        done["truncated_T"] = trunc

    if a.c2_latency_pairs > 0:
        sk = budget.skip(3.0 + 0.6 * step_s)
        if sk:
            done["latency_c2"] = sk
        else:
            print("[bench] latency stream (C2)", file=sys.stderr, flush=True)
            deadline = time.perf_counter() + budget.left() - 3.0 - 0.6 * step_s
            done["latency_c2"] = latency_stream(td, torch, wpath, a.c2_latency_pairs, 13, deadline, label="C2",
                                                ctx=ctx)
    ctx.close()

    conv = ks.get("conv3x3_mfma_f32", {"launches": 0, "ms": 0.0, "flops": 0.0})
    traffic = counter_traffic()
    achieved = conv["flops"] / (conv["ms"] * 1e-3) / 1e12 if conv["ms"] else 0.0
    kernels = {}
    for name, v in sorted(ks.items(), key=lambda kv: -kv[1]["ms"]):
        e = {"launches": v["launches"], "ms_total": round(v["ms"], 3),
             "avg_us": round(1e3 * v["ms"] / max(v["launches"], 1), 2)}
        if v["ms"] > 0:
            e["TFLOP/s"] = round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 2)
            e["GB/s"] = round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1)
        kernels[name] = e

    res = {
        "metric": "window-denoises/s",
        "value": windows / dt,
        "unit": "window-denoises/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * step_s,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("cold %s query, full-res %dx%d px (latent %d^2 + 17 px apron) at latent (%d, %d), seed %d"
                         % ("elevation", region[2], region[3], a.size, lx, ly, a.seed))
            if level == td.TD_LEVEL_HEIGHT else
            ("cold latent query %dx%d at (%d, %d), seed %d" % (a.size, a.size, lx, ly, a.seed)),
            "latent_channels": C, "steps_K": K, "window": H, "stride": S,
            "unet": "4-level 128/256/256/512, 2 res-blocks, 8-head attention at 8x8, random init"
            if a.config.startswith("c2") else a.config,
            "windows_per_step": windows // max(a.steps, 1),
            "batch": a.batch or "auto",
        },
        "roofline": {
            "kernel": "conv3x3_mfma_f32",
            "bound": "mfma",
            "achieved": round(achieved, 2),
            "peak": PEAK_FP32_MFMA_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_MFMA_TFLOPS, 4),
            "traffic": traffic["bytes_per_launch"] if traffic else None,
            "traffic_note": ("HBM bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1, scaled by a plain copy "
                             "kernel) of the %s launch, profiles/conv3x3_f32_and_bf16_halo_hbm_counters.md; the "
                             "launches averaged in 'achieved' mix all four UNet levels" % traffic["shape"])
            if traffic else "no counter record for the current kernel source",
            "avg_launch_us": round(1e3 * conv["ms"] / max(conv["launches"], 1), 2),
            "launches": conv["launches"],
        },
        "kernels": kernels,
        "cpu_baseline": cpu_baseline_entry(cpu) if cpu else None,
        "output_finite": finite,
        "run_budget": {"budget_s": a.budget_s, "elapsed_s": round(time.perf_counter() - T_START, 1),
                       "leg_order": legs,
                       "note": "legs after the timed steps run in this order while their estimated cost fits the "
                               "budget; skipped legs say so"},
    }
    for k in legs:
        res[k] = done.get(k)
    res["paper_context"] = paper_context(done.get("latency"))
    if cpu and "error" in cpu:
        res["cpu_baseline_error"] = cpu["error"]
    tmp.cleanup()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
