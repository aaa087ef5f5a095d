"""Distil a two-step student from the plain sampler (the learned part).

Teacher: a UNet weight file with the EDM Euler sampler (e.g. the 20-step
4-channel model).  For seed i the pair is (x_i, y_i) with x_i = sigma_0 G(i)
on the window at the origin (the seed noise, counter word 0) and y_i the
teacher's plain sampler run on that window alone (td_denoise_steps, all K
steps).  The student (a consistency-sampled weight file with noise levels
[s_0, s_1]) is trained so that both of its steps land on y:

    L = 1/2 mean((D_S(x; s_0) - y)^2) + 1/2 mean((D_S(y + s_1 e; s_1) - y)^2)

with e = G(i) on counter word 1 (the noise its second step re-draws when
sampling).  Forward and backward are the library's hand-written kernels
(td_train_*): BF16 convolution operands by default, FP32 master weights,
weight gradients and AdamW.  Usage:

    python -m paper_2512_08309_amd.distill TEACHER.tdw STUDENT_INIT.tdw OUT.tdw \\
        [--pairs 50000] [--steps 800] [--batch 64] [--lr 2e-4]
"""
import argparse
import json
import sys
import time

import numpy as np


def make_pairs(td, torch, teacher_path, n, seed0=1, chunk=1024, precision=0):
    """(x, y, seeds): device tensors [n][H][H][C] of teacher inputs and
    outputs, and the pair seeds seed0 .. seed0 + n - 1 (the re-noise of pair i
    is G(seed_i) on counter word 1, drawn by the library when it is used)."""
    with td.Context(0) as t:
        t.load_weights(teacher_path)
        t.set_option("precision", precision)
        H, C, K = t.info("window"), t.info("channels"), t.info("steps")
        sigma0 = 80.0
        x = torch.empty((n, H, H, C), device="cuda")
        y = torch.empty_like(x)
        seeds = np.arange(seed0, seed0 + n, dtype=np.int64)
        for i in range(n):
            td.td_noise_region(int(seeds[i]), 0, 0, x[i], step=0, scale=sigma0)
        torch.cuda.synchronize()
        for i0 in range(0, n, chunk):
            i1 = min(n, i0 + chunk)
            t.denoise_steps(x[i0:i1], 0, K, y[i0:i1])
            print("[distill] teacher pairs %d / %d" % (i1, n), file=sys.stderr, flush=True)
        torch.cuda.synchronize()
    return x, y, seeds


def renoise(td, base, seeds, sigma):
    """base[b] + sigma * G(seeds[b]) on counter word 1 for every window b, in
    place (the noise kernel's accumulate mode): multistep consistency
    sampling's re-noising of an estimate at the next noise level."""
    for b, sd in enumerate(seeds):
        td.td_noise_region(int(sd), 0, 0, base[b], step=1, scale=sigma, accumulate=True)
    return base


def train(td, torch, student_path, x, y, seeds, steps, batch=64, lr=2e-4, seed=0, log_every=50,
          sigmas=(80.0, 0.35), precision=1):
    """AdamW on the student's flat FP32 master parameters (BF16 convolution
    operands with precision 1); returns (params, loss history)."""
    tr = td.Trainer(student_path).set_precision(precision)
    P = tr.load_params(student_path)
    G, m, v = torch.zeros_like(P), torch.zeros_like(P), torch.zeros_like(P)
    n = x.shape[0]
    rng = np.random.default_rng(seed)
    D = torch.empty((batch,) + tuple(x.shape[1:]), device="cuda")
    dD = torch.empty_like(D)
    hist = []
    perm = rng.permutation(n)
    pos = 0
    for step in range(1, steps + 1):
        if pos + batch > n:
            perm, pos = rng.permutation(n), 0
        sel = perm[pos:pos + batch]
        idx = torch.from_numpy(sel).cuda()
        pos += batch
        xb, yb = x.index_select(0, idx), y.index_select(0, idx)
        x2 = renoise(td, yb.clone(), seeds[sel], sigmas[1])
        G.zero_()
        tr.forward(P, xb, sigmas[0], D)
        l1 = tr.mse(D, yb, dD, weight=0.5, want_loss=(step % log_every == 0 or step == 1))
        tr.backward(P, dD, G)
        tr.forward(P, x2, sigmas[1], D)
        l2 = tr.mse(D, yb, dD, weight=0.5, want_loss=(step % log_every == 0 or step == 1))
        tr.backward(P, dD, G)
        tr.adamw(P, G, m, v, lr=lr, step=step)
        if l1 is not None:
            hist.append((step, l1 + l2))
            print("[distill] step %d loss %.5f" % (step, l1 + l2), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tr.close()
    return P, hist


def student_windows(td, torch, student_path, P, x, seeds, sigmas=(80.0, 0.35), chunk=256):
    """The student's two-step sample of independent windows: D(x; s0), re-noised
    with s1 G(seed) on counter word 1, then D(.; s1) (consistency sampling
    without blending)."""
    tr = td.Trainer(student_path)
    out = torch.empty_like(x)
    for i0 in range(0, x.shape[0], chunk):
        xb = x[i0:i0 + chunk].contiguous()
        d1 = torch.empty_like(xb)
        tr.forward(P, xb, sigmas[0], d1)
        x2 = renoise(td, d1, seeds[i0:i0 + chunk], sigmas[1])
        tr.forward(P, x2, sigmas[1], out[i0:i0 + chunk])
    torch.cuda.synchronize()
    tr.close()
    return out


def evaluate(td, torch, student_path, P, x, y, seeds):
    """Relative RMSE of the student's two-step windows against the teacher's."""
    s = student_windows(td, torch, student_path, P, x, seeds)
    return float(torch.linalg.norm((s - y).flatten()) / torch.linalg.norm(y.flatten()))


def save(td, student_path, P, out_path):
    head, data = td.read_tdw_data(student_path)
    data = data.copy()
    data[:P.numel()] = P.cpu().numpy()
    td.write_tdw_data(out_path, head, data)


def main():
    import torch
    from paper_2512_08309_amd import td
    ap = argparse.ArgumentParser()
    ap.add_argument("teacher")
    ap.add_argument("student_init")
    ap.add_argument("out")
    ap.add_argument("--pairs", type=int, default=50000)
    ap.add_argument("--steps", type=int, default=800)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=2e-4)
    ap.add_argument("--teacher-precision", type=int, default=0)
    ap.add_argument("--holdout", type=int, default=512, help="held-out pairs (seeds after the training seeds)")
    ap.add_argument("--precision", type=int, default=1, help="1: BF16 convolution operands, 0: FP32")
    a = ap.parse_args()
    t0 = time.perf_counter()
    x, y, seeds = make_pairs(td, torch, a.teacher, a.pairs + a.holdout, precision=a.teacher_precision)
    t1 = time.perf_counter()
    xt, yt, et = x[:a.pairs], y[:a.pairs], seeds[:a.pairs]
    xh, yh, eh = x[a.pairs:], y[a.pairs:], seeds[a.pairs:]
    P0 = td.Trainer(a.student_init).load_params(a.student_init)
    before = evaluate(td, torch, a.student_init, P0, xh, yh, eh)
    P, hist = train(td, torch, a.student_init, xt, yt, et, a.steps, a.batch, a.lr, precision=a.precision)
    t2 = time.perf_counter()
    after = evaluate(td, torch, a.student_init, P, xh, yh, eh)
    save(td, a.student_init, P, a.out)
    print(json.dumps({"pairs": a.pairs, "holdout": a.holdout, "pair_s": t1 - t0, "steps": a.steps,
                      "batch": a.batch, "lr": a.lr, "train_s": t2 - t1, "ms_per_step": 1e3 * (t2 - t1) / a.steps,
                      "holdout_rel_rmse_before": before, "holdout_rel_rmse_after": after, "loss": hist}))


if __name__ == "__main__":
    main()
