"""Train the learned first-guess U-Net on one GPU with the library's kernels.

Samples: ``gen.training_sample(64, seed)`` for consecutive seeds (the 256^3
holes recipe drawn at 64^3 with the same physical radii and widths,
Dirichlet value 0).  Labels: the library's FP64 multigrid solve of each
sample (relative residual ``--label-tol``).  Training: ``mg_unet_train_step``
(AdamW; linear warm-up then cosine decay of the learning rate), batches
drawn from the device-resident set; a held-out set (seeds from
``--val-seed``) is scored each epoch.  The weights and the optimizer state go
to a safetensors file.

Usage:
  python -m paper_1104_1703_amd.train_unet --count 4096 --epochs 8 \
      --out paper_1104_1703_amd/weights/unet_holes64.safetensors
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time
from multiprocessing import get_context

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _draw(seed_n):
    from paper_1104_1703_amd import gen
    seed, n = seed_n
    p = gen.training_sample(n=n, seed=seed)
    return p.rho, p.mask


def draw_samples(seeds, n, workers):
    """(rho, mask) arrays for the given seeds, drawn on host cores."""
    rho = np.empty((len(seeds), n, n, n), np.float64)
    mask = np.empty((len(seeds), n, n, n), np.int8)
    with get_context("fork").Pool(workers) as pool:
        for i, (r, m) in enumerate(pool.imap(_draw, [(s, n) for s in seeds], chunksize=8)):
            rho[i], mask[i] = r, m
    return rho, mask


def label(rho_d, mask_d, h, tol, log_every=512):
    """FP64 multigrid solutions of every sample (device tensors)."""
    import torch

    from paper_1104_1703_amd import mg
    phi = torch.zeros_like(rho_d)
    cycles = []
    t0 = time.time()
    stream = torch.cuda.Stream(rho_d.device)
    for i in range(rho_d.shape[0]):
        H = mg.Hierarchy(mask_d[i], h, stream=stream, use_graph=0)
        _, info = H.solve(rho_d[i], phi[i], None, tol=tol)
        if info["status"] != 0:
            raise RuntimeError(f"label solve {i} did not converge: {info['status']}")
        cycles.append(info["cycles"])
        H.close()
        if (i + 1) % log_every == 0:
            print(f"  labelled {i + 1}/{rho_d.shape[0]} ({time.time() - t0:.1f} s, "
                  f"mean cycles {np.mean(cycles):.1f})", flush=True)
    return phi, cycles


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=10000)
    ap.add_argument("--val-count", type=int, default=64)
    ap.add_argument("--val-seed", type=int, default=30000)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--weight-decay", type=float, default=1e-4)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--label-tol", type=float, default=1e-10)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--resume", default=None)
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_1104_1703_amd", "weights",
                                                  "unet_holes64.safetensors"))
    args = ap.parse_args(argv)

    t0 = time.time()
    seeds = list(range(args.seed, args.seed + args.count))
    vseeds = list(range(args.val_seed, args.val_seed + args.val_count))
    rho, mask = draw_samples(seeds + vseeds, args.n, args.workers)
    print(f"drew {len(seeds)} + {len(vseeds)} samples at {args.n}^3 in {time.time() - t0:.1f} s", flush=True)

    import torch

    from paper_1104_1703_amd import mg
    dev = torch.device("cuda:0")
    rho_d = torch.from_numpy(rho).to(dev)
    mask_d = torch.from_numpy(mask).to(dev)
    del rho, mask
    h = 1.0 / args.n
    t1 = time.time()
    phi_d, cyc = label(rho_d, mask_d, h, args.label_tol)
    print(f"labelled in {time.time() - t1:.1f} s (cycles {min(cyc)}..{max(cyc)})", flush=True)
    nt = len(seeds)
    tr = (rho_d[:nt], mask_d[:nt], phi_d[:nt])
    va = (rho_d[nt:], mask_d[nt:], phi_d[nt:])

    net = mg.UNet(seed=args.init_seed)
    if args.resume:
        net.load(args.resume)
    steps_per_epoch = nt // args.batch
    total = steps_per_epoch * args.epochs
    gen_t = torch.Generator(device="cpu").manual_seed(args.init_seed)

    def lr_at(k):
        if k < args.warmup:
            return args.lr * (k + 1) / args.warmup
        q = (k - args.warmup) / max(1, total - args.warmup)
        return args.lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * q)))

    def val_loss():
        tot = 0.0
        for i in range(0, va[0].shape[0], args.batch):
            sl = slice(i, i + args.batch)
            tot += net.loss_grad(va[0][sl], va[1][sl], va[2][sl]) * va[0][sl].shape[0]
        return tot / va[0].shape[0]

    print(f"training: {total} steps of {args.batch} samples, {net.num_params} parameters; "
          f"validation loss {val_loss():.4e} before", flush=True)
    k = 0
    t2 = time.time()
    for ep in range(args.epochs):
        perm = torch.randperm(nt, generator=gen_t).to(dev)
        run = 0.0
        for s in range(steps_per_epoch):
            idx = perm[s * args.batch:(s + 1) * args.batch]
            loss = net.train_step(tr[0].index_select(0, idx), tr[1].index_select(0, idx),
                                  tr[2].index_select(0, idx), lr=lr_at(k), weight_decay=args.weight_decay,
                                  sync=(s % 50 == 49))
            if loss is not None:
                run = loss
            k += 1
            if s % 250 == 249:
                print(f"  epoch {ep} step {s + 1}/{steps_per_epoch} loss {run:.4e} lr {lr_at(k):.2e} "
                      f"({time.time() - t2:.1f} s)", flush=True)
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        net.save(args.out)
        print(f"epoch {ep}: validation loss {val_loss():.4e} ({time.time() - t2:.1f} s) -> {args.out}", flush=True)
    print(f"done in {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
