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
classes, p50/p99 latency of a stream of small queries (first query and its
neighbour, as in time-to-first/second-tile), and the FP64 oracle timed on
the host cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--config", default="c2")
    p.add_argument("--size", type=int, default=1024, help="latent side of the query (full-res = 8x)")
    p.add_argument("--workload", choices=["height", "latent"], default="height")
    p.add_argument("--batch", type=int, default=0)
    p.add_argument("--seed", type=int, default=7)
    p.add_argument("--latency-pairs", type=int, default=100)
    p.add_argument("--cpu-windows", type=int, default=16)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--bf16-steps", type=int, default=1,
                   help="cold steps timed again per reduced-precision mode (0 = skip)")
    p.add_argument("--lowp-modes", default="1,2", help="precision modes to time: 1 bf16, 2 bf16 + fp8 weights")
    p.add_argument("--truncated", default="c2t2", help="truncated-T config timed cold ('' = skip)")
    p.add_argument("--serve-queries", type=int, default=256, help="queries of the serving stream (0 = skip)")
    p.add_argument("--serve-rate", type=float, default=256.0, help="Poisson arrival rate, queries/s")
    p.add_argument("--serve-rate-sustained", type=float, default=32.0,
                   help="a second, lower arrival rate the server keeps up with (0 = skip)")
    p.add_argument("--student-steps", type=int, default=300,
                   help="AdamW steps of the in-bench student distillation (0 = skip the student leg)")
    p.add_argument("--student-pairs", type=int, default=4096, help="teacher pairs of the in-bench distillation")
    p.add_argument("--micro-only", action="store_true",
                   help="only the decode / noise micro-benchmarks (8192^2 heightfield, 8192^2 x 4 noise)")
    p.add_argument("--calib-copy-mib", type=int, default=0,
                   help="run one plain elementwise copy (read N MiB, write N MiB) before the steps, as the "
                        "reference dispatch that scales hardware byte counters")
    return p.parse_args()


def cpu_baseline(weights_path, n):
    """Oracle (FP64 NumPy) denoiser on n windows at sigma_0, timed on host cores."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle.sampler import Model
    m = Model(weights_path)
    x = 80.0 * np.random.default_rng(0).standard_normal((n, m.H, m.H, m.C))
    m.denoiser(x[:1], m.sched[0], None)          # warm BLAS
    t0 = time.perf_counter()
    m.denoiser(x, m.sched[0], None)
    dt = time.perf_counter() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
    return {"value": n / dt, "unit": "window-denoises/s", "cores": threads, "kind": "oracle",
            "sample": "%d windows of the same model through the FP64 oracle denoiser at sigma_0 (one batched "
                      "level round; the sampler's blend/Euler is <0.1%% of its work), %.1f s" % (n, dt)}


def latency_stream(td, torch, weights_path, pairs, seed=11):
    """TTFT/TTST-style stream: random 64x64 queries in [-1e6, 1e6) and their right neighbours."""
    import numpy as np
    rng = np.random.default_rng(seed)
    xs = rng.integers(-10 ** 6, 10 ** 6, size=(pairs, 2))
    first, second = [], []
    with td.Context(0) as c:
        c.load_weights(weights_path)
        C = c.info("channels")
        out = torch.empty((C, 64, 64), dtype=torch.float32, device="cuda")
        st = torch.cuda.current_stream()
        c.sample_region_async(seed, 0, 0, 64, 64, 0, out, st)      # warm kernels / workspace
        torch.cuda.synchronize()
        for x, y in xs:
            for dx, sink in ((0, first), (64, second)):
                t0 = time.perf_counter()
                c.sample_region_async(seed, int(x) + dx, int(y), 64, 64, 0, out, st)
                torch.cuda.synchronize()
                sink.append(1e3 * (time.perf_counter() - t0))
    def pct(v):
        return {"p50_ms": float(np.percentile(v, 50)), "p99_ms": float(np.percentile(v, 99)), "n": len(v)}
    return {"workload": "1-channel model, windows 32/16, K=8, 2-level UNet 16/32; %d random 64x64 latent queries "
                        "in [-1e6,1e6) seed %d, each followed by its right neighbour; end-to-end through "
                        "td_sample_region_async incl. planning" % (pairs, seed),
            "first": pct(first), "neighbour": pct(second)}


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
    arithmetic applied to the neighbour-query latency of the C1 stream here
    (a 64^2 latent = 512^2 px tile of synthetic random-init models): not a
    like-for-like comparison."""
    tile_m = 512 * 90.0
    ctx = {"paper": "generation 9x faster than orbital velocity (7,700 m/s): time to second tile 0.66 s for a "
                    "512^2 tile at 90 m per pixel (46 km), consumer GPU, the paper's trained models"}
    if lat:
        t = lat["neighbour"]["p50_ms"] * 1e-3
        ctx["here"] = {"neighbour_query_p50_s": t, "traversal_m_per_s": tile_m / t,
                       "x_orbital_velocity": tile_m / t / 7700.0,
                       "note": "C1 neighbour latent query (64^2 latent, 512^2 px at 8x) of the latency stream; "
                               "synthetic 2-level UNet, not the paper's models"}
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
                            "note": "all four decode kernels; 268 MB of heightfield written"},
            "encode_8192": {"ms": enc_ms, "GB_per_s_read": 8192 * 8192 * 4 / (enc_ms * 1e-3) / 1e9,
                            "note": "all four encode kernels on the decoded 8192^2 heightfield (268 MB read "
                                    "once algorithmically; the kernels read it twice) to a %dx%d latent" % (gw, gh)},
            "noise_8192x4": {"ms": noise_ms, "GB_per_s_written": noise.numel() * 4 / (noise_ms * 1e-3) / 1e9,
                             "note": "Philox + bit-exact IEEE Box-Muller per pair: ALU-bound"}}


def student_leg(td, torch, teacher, teacher_path, student_init, a, region, level, out, ref32, stream, wps32, dt32):
    """Distil the half-width two-step student from the 20-step teacher (a short
    run: a.student_pairs pairs, a.student_steps AdamW steps at batch 64, lr
    2e-4), then time the same cold query with it: alone, judged by the FP32
    teacher (fallback above 0.05 RMS), and with BF16 convolutions."""
    import tempfile
    from paper_2512_08309_amd import distill
    t0 = time.perf_counter()
    x, y, e = distill.make_pairs(td, torch, teacher_path, a.student_pairs, precision=1)
    xh, yh, eh = distill.make_pairs(td, torch, teacher_path, 256, seed0=1 + a.student_pairs, precision=1)
    t1 = time.perf_counter()
    P, hist = distill.train(td, torch, student_init, x, y, e, a.student_steps, batch=64, lr=2e-4, log_every=100)
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
                            "heldout_window_rel_rmse_vs_teacher": held}}
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "student.tdw")
        distill.save(td, student_init, P, path)
        with td.Context(0) as s:
            s.load_weights(path)
            for name, judge, prec in (("student_fp32", None, 0), ("student_judged_fp32", teacher, 0),
                                      ("student_bf16", None, 1)):
                s.set_option("precision", prec)
                s.set_judge(judge, 0.05)
                s.sample_region_async(a.seed, *region, level, out, stream)      # first use
                torch.cuda.synchronize()
                s.cache_clear()
                t0 = time.perf_counter()
                s.sample_region_async(a.seed, *region, level, out, stream)
                torch.cuda.synchronize()
                dts = time.perf_counter() - t0
                st = s.cache_stats()
                rel = float(torch.linalg.vector_norm((out - ref32).double()) /
                            torch.linalg.vector_norm(ref32.double()))
                res[name] = {"ms_per_step": 1e3 * dts, "query_speedup_vs_fp32_plain": dt32 / dts,
                             "window_denoises_per_s": st["denoiser_evals"] / dts, "windows": st["misses"],
                             "judge_fallbacks": st["judge_fallbacks"],
                             "rel_rmse_heightfield_vs_fp32_plain": rel}
                print("[bench] %s done" % name, file=sys.stderr, flush=True)
            s.set_judge(None, 0.0)
    res["note"] = ("random-init teacher and a short distillation: the student does not reach the 2e-2 heightfield "
                   "RMSE; its speed is measured at the error it has")
    return res


def main():
    a = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build measures the per-GPU share of the sampling path "
              "(sharding across GPUs is described in DESIGN.md but not built); got --gpus %d" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2512_08309_amd import td
    from synth.models import cached_weights

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    wdir = os.path.join(ROOT, ".td_weights")
    wpath = cached_weights(a.config, wdir, 0)
    ctx = td.Context(0).load_weights(wpath)
    if a.micro_only:
        print(json.dumps({"micro": micro_bench(td, torch, ctx)}))
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
    finite = bool(torch.isfinite(out).all().item())
    ref32 = out.clone()
    micro = micro_bench(td, torch, ctx)

    lowp = None
    if a.bf16_steps > 0:
        lowp = {}
        names = {1: "bf16", 2: "bf16_fp8w"}
        descr = {1: "BF16 convolution operands (activations and weights), FP32 accumulation",
                 2: "BF16 activations, FP8 e4m3 weights with per-output-channel FP32 scales, FP32 accumulation"}
        for mode in [int(v) for v in a.lowp_modes.split(",") if v]:
            ctx.set_option("precision", mode)
            step()                                   # first use: workspace and kernels
            ctx.set_option("timing", 1)
            ctx.kernel_stats(reset=True)
            w16 = 0
            t0 = time.perf_counter()
            for i in range(a.bf16_steps):
                w16 += step()
                print("[bench] precision %d step %d done" % (mode, i), file=sys.stderr, flush=True)
            dt16 = time.perf_counter() - t0
            ks16 = ctx.kernel_stats()
            ctx.set_option("timing", 0)
            rel = float(torch.linalg.vector_norm((out - ref32).double()) / torch.linalg.vector_norm(ref32.double()))
            c16 = ks16.get("conv3x3_mfma_bf16", {"ms": 0.0, "flops": 0.0, "launches": 0})
            lowp[names[mode]] = {
                "precision": descr[mode] + "; GN statistics, attention, input/output layers, blend/Euler and "
                                           "decode FP32",
                "value": w16 / dt16, "ms_per_step": 1e3 * dt16 / a.bf16_steps,
                "speedup_vs_fp32": (w16 / dt16) / (windows / dt),
                "rel_rmse_heightfield_vs_fp32_gpu": rel,
                "conv3x3_TFLOP/s": round(c16["flops"] / (c16["ms"] * 1e-3) / 1e12, 1) if c16["ms"] else None,
                "conv3x3_frac_of_bf16_peak_2500": round(c16["flops"] / (c16["ms"] * 1e-3) / 2.5e15, 4)
                if c16["ms"] else None,
                "kernels_ms": {k: round(v["ms"], 1) for k, v in sorted(ks16.items(), key=lambda kv: -kv[1]["ms"])}}
        ctx.set_option("precision", 0)
    student = None
    if a.student_steps > 0 and a.config == "c2":
        print("[bench] student distillation", file=sys.stderr, flush=True)
        student = student_leg(td, torch, ctx, wpath, cached_weights("s2", wdir, 0), a, region, level, out, ref32,
                              stream, windows / dt, dt)
    ctx.close()

    conv = ks.get("conv3x3_mfma_f32", {"launches": 0, "ms": 0.0, "flops": 0.0})
    achieved = conv["flops"] / (conv["ms"] * 1e-3) / 1e12 if conv["ms"] else 0.0
    kernels = {}
    for name, v in sorted(ks.items(), key=lambda kv: -kv[1]["ms"]):
        e = {"launches": v["launches"], "ms_total": round(v["ms"], 3),
             "avg_us": round(1e3 * v["ms"] / max(v["launches"], 1), 2)}
        if v["ms"] > 0:
            e["TFLOP/s"] = round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 2)
            e["GB/s"] = round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1)
        kernels[name] = e

    trunc = None
    if a.truncated:
        # cost of the same query when the windows are blended at T < K levels
        # (Sec. 3.4): analytic cone counts, and one timed cold step for a.truncated
        def cone(size, T):
            return td.td_cone_windows(lx, ly, size, size, 0, T, H, S)
        trunc = {"cone_windows_by_T": {str(T): {str(sz): cone(sz, T) for sz in (128, 512, 1024)}
                                       for T in (1, 2, 5, 20)},
                 "note": "window evaluations of a cold latent query of side 128/512/1024 at (13,-1000001); "
                         "each evaluation runs K/T = 20/T Euler steps of the network"}
        tctx = td.Context(0).load_weights(cached_weights(a.truncated, wdir, 0))
        tctx.set_option("timing", 1)
        tctx.sample_region_async(a.seed, *region, level, out, stream)     # first use
        torch.cuda.synchronize()
        tctx.cache_clear()
        t0 = time.perf_counter()
        tctx.sample_region_async(a.seed, *region, level, out, stream)
        torch.cuda.synchronize()
        dtt = time.perf_counter() - t0
        stt = tctx.cache_stats()
        trunc["timed"] = {"config": a.truncated, "T": tctx.info("levels"), "ms_per_step": 1e3 * dtt,
                          "windows": stt["misses"], "denoiser_evals": stt["denoiser_evals"],
                          "denoiser_evals_per_s": stt["denoiser_evals"] / dtt,
                          "speedup_vs_T20_step": (1e3 * dt / a.steps) / (1e3 * dtt),
                          "rel_rmse_heightfield_vs_T20": float(torch.linalg.vector_norm((out - ref32).double()) /
                                                               torch.linalg.vector_norm(ref32.double()))}
        tctx.close()

    lat = None
    if a.latency_pairs > 0:
        print("[bench] latency stream", file=sys.stderr, flush=True)
        lat = latency_stream(td, torch, cached_weights("c1", wdir, 0), a.latency_pairs)
    serve = None
    if a.serve_queries > 0:
        print("[bench] serving stream", file=sys.stderr, flush=True)
        serve = serving_stream(td, torch, cached_weights("c1h", wdir, 0), cached_weights("cc", wdir, 0),
                               a.serve_queries, a.serve_rate)
        if a.serve_rate_sustained > 0:
            print("[bench] serving stream (sustained rate)", file=sys.stderr, flush=True)
            serve = {"offered_%g_qps" % a.serve_rate: serve,
                     "offered_%g_qps" % a.serve_rate_sustained:
                         serving_stream(td, torch, cached_weights("c1h", wdir, 0), cached_weights("cc", wdir, 0),
                                        a.serve_queries, a.serve_rate_sustained)}
    cpu = None
    if not a.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wpath, a.cpu_windows)

    res = {
        "metric": "window-denoises/s",
        "value": windows / dt,
        "unit": "window-denoises/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * dt / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("cold %s query, full-res %dx%d px (latent %d^2 + 17 px apron) at latent (%d, %d), seed %d"
                         % ("elevation" if level == td.TD_LEVEL_HEIGHT else "latent", region[2], region[3],
                            a.size, lx, ly, a.seed)) if level == td.TD_LEVEL_HEIGHT else
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
            "traffic": None,
            "avg_launch_us": round(1e3 * conv["ms"] / max(conv["launches"], 1), 2),
            "launches": conv["launches"],
        },
        "kernels": kernels,
        "latency": lat,
        "reduced_precision": lowp,
        "truncated_T": trunc,
        "serving": serve,
        "student": student,
        "micro": micro,
        "cpu_baseline": cpu,
        "output_finite": finite,
        "paper_context": paper_context(lat),
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
