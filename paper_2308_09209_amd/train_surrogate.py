"""Train the learned flow surrogate on the GPU.

Training pairs are synthesised on the device: a random texture (16 random
sinusoids plus flat rectangles, the recipe of the scene generator at its
density: the generator's 40 rectangles over a 6144 x 1200 ring texture put 1-5
of them on a strip) as the template, the same texture displaced by a smooth
random field (maximum displacement U[0.5, 8] px) and given the small
photometric residual that remains after the colour transfer (gain U[0.97,
1.03], offset U[-3, 3]) as the moving image, both 256 x 1080 (a strip pair of
the 4 x 1080p rig) and rounded to integer luma.  Labels are the flows of the library's plain estimator on each pair
(vs_flow_run); the network sees pyramid level 2 of both images and learns the
label average-pooled to level 2.  Every forward, backward and optimiser step
runs in the library's kernels.

    python -m paper_2308_09209_amd.train_surrogate --pairs 20000 --steps 3000 --out weights.vsnn
"""
from __future__ import annotations

import argparse
import math
import sys
import time

import torch
import torch.nn.functional as F

from . import surrogate as S
from . import vstitch as V


def synth_pairs(n, H, W, max_disp, gen, device="cuda"):
    """n template / moving luma pairs (float32, integer valued, [n, H, W]).
    Scalar draws come from a CPU generator (no device synchronisation)."""
    ys = torch.arange(H, device=device, dtype=torch.float32).view(H, 1).expand(H, W)
    xs = torch.arange(W, device=device, dtype=torch.float32).view(1, W).expand(H, W)
    out_t, out_m = [], []
    for _ in range(n):
        r = lambda *s: torch.rand(*s, generator=gen)
        th = r(16) * math.pi
        lam = torch.exp(math.log(8.0) + r(16) * (math.log(128.0) - math.log(8.0)))
        ph = (r(16) * 2 * math.pi).to(device).view(16, 1, 1)
        amp = (r(16) / 16.0).to(device).view(16, 1, 1)
        kx = (2 * math.pi * torch.cos(th) / lam).to(device).view(16, 1, 1)
        ky = (2 * math.pi * torch.sin(th) / lam).to(device).view(16, 1, 1)
        n_rect = 1 + int(float(r(1)) * 5) % 5
        rects = [(float(a) * W, float(b) * H, 16 + float(c) * (300 - 16), 16 + float(d) * (300 - 16), float(e))
                 for a, b, c, d, e in r(n_rect, 5)]

        def texture(X, Y):
            v = 0.5 + (amp * torch.sin(kx * X + ky * Y + ph)).sum(0)
            v = (v - v.min()) / (v.max() - v.min() + 1e-6)
            for (x0, y0, rw, rh, val) in rects:
                inside = (X >= x0) & (X < x0 + rw) & (Y >= y0) & (Y < y0 + rh)
                v = torch.where(inside, torch.full_like(v, val), v)
            return v

        # smooth displacement: coarse random field, bicubic upsampled, scaled
        coarse = torch.randn(1, 2, max(2, H // 64), max(2, W // 64), generator=gen).to(device)
        d = F.interpolate(coarse, size=(H, W), mode="bicubic", align_corners=True)[0]
        scale = 0.5 + float(r(1)) * (max_disp - 0.5)
        d = d * (scale / d.norm(dim=0).max().clamp_min(1e-6))
        t = texture(xs, ys)
        # moving image: m(x + d(x)) = t(x), i.e. m(y) = t(y - d) to first order
        m = texture(xs - d[0], ys - d[1])
        gain = 0.97 + 0.06 * float(r(1))
        off = -3.0 + 6.0 * float(r(1))
        out_t.append(torch.round(t * 255.0).clamp(0, 255))
        out_m.append(torch.round((m * 255.0) * gain + off).clamp(0, 255))
    return torch.stack(out_t), torch.stack(out_m)


def pool_label(flow, w, h, f):
    """level-0 flow [h][w][2] -> its f x f block means in level pixels (vs_nn_pool_flow)"""
    out = torch.empty(((h + f - 1) // f, (w + f - 1) // f, 2), dtype=torch.float32, device=flow.device)
    V.check(V.lib().vs_nn_pool_flow(S._p(flow), w, h, f, S._p(out), S._s()), "vs_nn_pool_flow")
    return out


def build_dataset(n_pairs, H=1080, W=256, max_disp=8.0, seed=0, chunk=64, log=print, label_flow=1):
    """(level-2 template, level-2 moving, level-2 label, level-0 label) tensors;
    label_flow 1: labels from the pyramidal Lucas-Kanade estimator, 2: from
    the variational estimator (the library's vs_flow_* context either way)"""
    gen = torch.Generator().manual_seed(seed)
    pf = V.PlainFlow(W, H, flow=label_flow)
    t2l, m2l, lab2, lab0 = [], [], [], []
    t0 = time.time()
    for start in range(0, n_pairs, chunk):
        n = min(chunk, n_pairs - start)
        T, M = synth_pairs(n, H, W, max_disp, gen)
        for i in range(n):
            ftm, _ = pf(T[i].contiguous(), M[i].contiguous())
            yt2, ym2 = pf.level(S.LEVEL)
            t2l.append(yt2)
            m2l.append(ym2)
            lab2.append(pool_label(ftm, W, H, 1 << S.LEVEL))
            if len(lab0) < 64:
                lab0.append(ftm)
        if start == 0 or (start // chunk) % 20 == 0:
            log(f"# dataset {start + n}/{n_pairs} pairs ({time.time() - t0:.1f} s)")
    return torch.stack(t2l), torch.stack(m2l), torch.stack(lab2), lab0


def split(data, val=256):
    """(training pairs, held-out pairs): the last min(val, n / 10) pairs are held out"""
    n = data[0].shape[0]
    n_val = max(1, min(val, n // 10))
    return n - n_val, n


def evaluate(net, data, first, last):
    """mean level-2 end-point error of the network against the labels of pairs
    first..last-1"""
    T2, M2, L2, _ = data
    h2, w2 = T2.shape[1], T2.shape[2]
    vimgs = V.nn_images([(h2, w2)])
    sums = torch.zeros(max(1, last - first), dtype=torch.float32, device=T2.device)
    for i in range(first, last):
        x = S.pack(T2[i:i + 1], M2[i:i + 1])
        net.forward(x, vimgs)
        net.loss(L2[i].reshape(-1, 2), out=sums[i - first])
    # per-pair mean errors (library sums over each pair's pixels), averaged on the host
    per_pair = sums.cpu().double().numpy() / (h2 * w2)
    return float(per_pair[:last - first].mean()) if last > first else 0.0


def train(net, data, steps, batch=16, lr=2e-3, log=print, val=256):
    """Adam with a cosine learning rate on random batches of the training
    pairs; returns ([(step, mean training EPE of the last logging interval)],
    held-out EPE after training), both in level-2 px."""
    T2, M2, L2, _ = data
    n_tr, n = split(data, val)
    h2, w2 = T2.shape[1], T2.shape[2]
    imgs = V.nn_images([(h2, w2)] * batch)
    gen = torch.Generator(device="cuda").manual_seed(1)
    t0 = time.time()
    hist = []
    interval = 100
    sums = torch.zeros(interval, dtype=torch.float32, device=T2.device)
    run_n = 0
    for step in range(1, steps + 1):
        idx = torch.randint(0, n_tr, (batch,), generator=gen, device="cuda")
        x = S.pack(T2[idx], M2[idx])
        lab = L2[idx].reshape(-1, 2).contiguous()
        net.forward(x, imgs)
        sums[run_n].copy_(net.backward(lab))
        cur_lr = lr * 0.5 * (1 + math.cos(math.pi * step / steps))
        net.adam(lr=cur_lr)
        run_n += 1
        if step % interval == 0 or step == steps:
            # mean training error of the interval's batches (library sums per batch)
            loss = float(sums[:run_n].cpu().double().numpy().mean()) / lab.shape[0]
            hist.append((step, loss))
            run_n = 0
            log(f"# step {step}/{steps} train EPE(level 2) {loss:.4f} px ({time.time() - t0:.1f} s)")
    val_epe = evaluate(net, data, n_tr, n)
    log(f"# held-out EPE(level 2) {val_epe:.4f} px = {4 * val_epe:.4f} px at level 0")
    return hist, val_epe


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--labels", choices=("lk", "variational"), default="lk",
                    help="label source: the pyramidal Lucas-Kanade or the variational estimator")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    log = lambda s: print(s, file=sys.stderr, flush=True)
    data = build_dataset(a.pairs, seed=a.seed, log=log, label_flow=1 if a.labels == "lk" else 2)
    net = S.Net(seed=a.seed)
    n_tr, n = split(data)
    log(f"# held-out EPE(level 2) before training {evaluate(net, data, n_tr, n):.4f} px")
    hist, val = train(net, data, a.steps, batch=a.batch, lr=a.lr, log=log)
    net.save(a.out)
    log(f"# saved {a.out}")
    print(f'{{"pairs": {a.pairs}, "steps": {a.steps}, "batch": {a.batch}, "val_epe_level2": {val:.5f}, '
          f'"first_loss": {hist[0][1]:.5f}, "last_loss": {hist[-1][1]:.5f}}}', flush=True)


if __name__ == "__main__":
    main()
