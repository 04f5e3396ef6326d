"""Benchmark: time to a 1e-10 relative residual on the 256^3 masked workload.

One step is one whole solve from a zero guess: Dirichlet fold, multigrid
cycles (2 pre + 2 post red-black passes, boundary order chosen at run time)
and the residual norm after every cycle, until ||r|| <= 1e-10 ||f||.  Inputs
are resident in HBM before the timed region.

Also measured here, for the dominant kernel (the finest-level smoother):
its average launch duration inside the timed solves, from HIP event pairs on
the solver's stream, and the oracle (plain FP64 C, host cores) on a bounded
sample of the same workload.

Beside it (not part of `value`): the same solve with FP32 inner cycles in
FP64 iterative refinement, from an interpolated (coarse-solve) guess and from
the learned U-Net guess, each timed whole (guess included).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       [--variants mixed,interp,learned,learned_mixed] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0       # MI355X HBM3E
# Algorithmic bytes of one FP64 V(2,2) cycle per active finest cell: four
# passes of 25 B, the residual with restriction (18 B) and the prolongation
# (18 B) on the finest level, times 8/7 for the coarser levels (each about an
# eighth of the one above).
VCYCLE_BYTES_FP64 = 155
SMOOTH_BYTES_FP64 = 25.0    # per active cell per pass: x read + x write + f read (8 B each) + code (1 B)
SMOOTH_BYTES_FP32 = 13.0


# algorithmic bytes per active finest cell of each kind of finest-level FP64
# pass in a cycle: the plain pass; the pass that also forms the residual and
# writes the restricted right-hand side (1/8 x 8 B); the pass that reads the
# coarse iterate for the prolongation (1/8 x 8 B); the pass that also forms
# the input's residual norm (no extra bytes)
FINEST_BYTES = {"plain": 25.0, "residual": 26.0, "prolong": 26.0, "norm": 25.0}
FINEST_KERNELS = {"plain": "k_rbgs<double, true, D, false>", "residual": "k_rbgs_res<double, D>",
                  "prolong": "k_rbgs<double, true, D, true>", "norm": "k_rbgs_norm<D>"}


def finest_kernels(timed, n_act):
    """Event-timed average launch and algorithmic rate of each kind of
    finest-level pass of a cycle ((summed ms, launches) per kind)."""
    out = {}
    for kind, (ms, n) in timed.items():
        if n == 0:
            out[kind] = {"kernel": FINEST_KERNELS[kind], "launches_timed": 0}
            continue
        us = ms / n * 1e3
        b = FINEST_BYTES[kind] * n_act
        out[kind] = {"kernel": FINEST_KERNELS[kind], "avg_launch_us": round(us, 3), "launches_timed": n,
                     "algorithmic_bytes_per_launch": b, "achieved": round(b / (us * 1e-6) / 1e9, 1),
                     "frac": round(b / (us * 1e-6) / 1e9 / PEAK_HBM_GBS, 4)}
    return out


def measured_traffic():
    """HBM bytes per launch of the finest smoother from the committed counter
    runs (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size), or
    None when the kernel's sources changed since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "smoother_traffic_holes256.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
        h = hashlib.sha256()
        for f in rec["sources"]:
            with open(os.path.join(ROOT, f), "rb") as src:
                h.update(src.read())
        if h.hexdigest() != rec["sources_sha256"]:
            return None
        return float(rec["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--variants", default="mixed,interp,learned,learned_s1,learned_s2,learned_mixed",
                    help="comma list of extra variants timed beside fp64: mixed (FP32 inner / FP64 outer), "
                         "interp (coarse-solve guess), learned (U-Net guess at --learned-stride), learned_sK "
                         "(U-Net at stride K), learned_mixed")
    ap.add_argument("--learned-stride", type=int, default=4, help="U-Net runs on the 1/stride grid")
    ap.add_argument("--no-learned-eval", dest="learned_eval", action="store_false",
                    help="skip the sphere-geometry evaluation of the learned guess at strides 1, 2, 4")
    ap.add_argument("--batch-patches", type=int, default=512,
                    help="patches of the batched workload timed beside the main line (0: skip)")
    ap.add_argument("--large-n", type=int, default=512,
                    help="edge of the porous mixed-precision workload timed beside the main line (0: skip)")
    ap.add_argument("--weights", default=None, help="U-Net weights (default: the package's trained file)")
    ap.add_argument("--smoother-launches", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-solves", type=int, default=2, help="complete oracle solves timed for cpu_baseline")
    ap.add_argument("--profile-smoother", type=int, default=0, metavar="N",
                    help="counter runs: build the 256^3 hierarchy, launch only the finest smoother N times, exit")
    ap.add_argument("--profile-workload", choices=("holes", "porous"), default="holes",
                    help="workload of --profile-smoother: the --n holes box or the --large-n porous box")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="counter runs: 4 plain device copies of MIB MiB (known bytes), exit")
    ap.add_argument("--schedules", type=int, default=0, metavar="N",
                    help="study: the sphere at N^3 to 1e-10 with N_cycles 1, 2, 3 in each boundary order "
                         "(cycles, mean rate, ms), exit")
    ap.add_argument("--schedules-workload", choices=("sphere", "holes"), default="sphere",
                    help="domain of --schedules: the sphere or the holes workload (adds AUTO order)")
    ap.add_argument("--amr", default="", metavar="N,N,...",
                    help="study: one-way nested levels (3 refinements) of the ln profile at these base sizes: "
                         "errors, orders and time, exit")
    ap.add_argument("--profile-solves", type=int, default=0, metavar="N",
                    help="counter runs: N complete FP64 solves and N mixed-precision solves of the main workload "
                         "after one warm-up each, exit")
    ap.add_argument("--profile-batch", type=int, default=0, metavar="N",
                    help="kernel runs: N batch solves of the --batch-patches workload after one warm-up, exit")
    ap.add_argument("--profile-unet", type=int, default=0, metavar="N",
                    help="kernel runs: N U-Net inferences (256^3 holes, --learned-stride) and N training steps "
                         "(batch 8 of 64^3), exit")
    return ap.parse_args()


def profile_smoother(args):
    """Finest-level smoother launches alone, for hardware-counter runs."""
    import torch

    from paper_1104_1703_amd import gen, mg
    if args.profile_workload == "porous":
        p = gen.porous_problem(args.large_n, seed=4)
    else:
        p = gen.holes_problem(n=args.n, seed=args.seed)
    H = mg.Hierarchy(torch.from_numpy(p.mask).cuda(), p.h)
    n = args.profile_smoother + (args.profile_smoother % 2)
    H.time_smoother(n)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "profile-smoother", "workload": p.name, "launches": n, "active_cells": H.n_active(0),
                      "algorithmic_bytes_per_launch": SMOOTH_BYTES_FP64 * H.n_active(0)}), flush=True)
    H.close()


def copy_calibration(args):
    """Plain copies of a known number of bytes (reference for FETCH_SIZE/WRITE_SIZE)."""
    import torch
    n = args.copy_calibration * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy-calibration", "bytes_read_per_copy": n * 8, "bytes_written_per_copy": n * 8,
                      "copies": 4}), flush=True)


def profile_solves(args):
    """Whole solves of the main workload, FP64 then mixed precision, for
    counter runs that attribute HBM traffic to every kernel of a cycle."""
    import torch

    from paper_1104_1703_amd import gen, mg
    p = gen.holes_problem(n=args.n, seed=args.seed)
    mask = torch.from_numpy(p.mask).cuda()
    rho = torch.from_numpy(p.rho).cuda()
    out = {}
    for prec in ("fp64", "mixed"):
        H = mg.Hierarchy(mask, p.h, precision=prec)
        phi = torch.zeros_like(rho)
        H.solve(rho, phi, tol=args.tol)
        cycles = []
        for _ in range(args.profile_solves):
            phi.zero_()
            _, info = H.solve(rho, phi, tol=args.tol)
            cycles.append(info["cycles"])
        torch.cuda.synchronize()
        out[prec] = cycles
        H.close()
    print(json.dumps({"mode": "profile-solves", "solves": args.profile_solves, "cycles": out,
                      "active_cells": int((p.mask > 0).sum())}), flush=True)


def profile_unet(args):
    import torch

    from paper_1104_1703_amd import gen, mg
    net = mg.UNet(seed=0)
    p = gen.holes_problem(n=args.n, seed=args.seed)
    rho = torch.from_numpy(p.rho).cuda()
    mask = torch.from_numpy(p.mask).cuda()
    out = net.infer(rho, mask, stride=args.learned_stride)
    tr = [gen.training_sample(64, 10000 + i) for i in range(8)]
    r8 = torch.from_numpy(np.stack([t.rho for t in tr])).cuda()
    m8 = torch.from_numpy(np.stack([t.mask for t in tr])).cuda()
    for _ in range(args.profile_unet):
        net.infer(rho, mask, stride=args.learned_stride, out=out)
    for _ in range(args.profile_unet):
        net.train_step(r8, m8, r8 * 1e-3, lr=1e-4, sync=False)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "profile-unet", "inferences": args.profile_unet, "stride": args.learned_stride,
                      "train_steps": args.profile_unet}), flush=True)


UNET_CONV = ("dec1a", 32, 16, 16)  # layer, up-sampled channels, skip channels, output channels
PEAK_BF16_TFLOPS = 2500.0


def unet_conv_roofline():
    """The widest convolution of a training step (dec1a: 32 up-sampled + 16
    skip channels -> 16, on 8 x 64^3 voxels), timed with HIP events on the
    stream it is launched on, against the dense BF16 matrix-core peak."""
    import torch

    from paper_1104_1703_amd import mg
    name, ca, cb, cout = UNET_CONV
    n, d = 8, 64
    g = torch.Generator(device="cpu").manual_seed(0)
    a = torch.randn((n, d // 2, d // 2, d // 2, ca), generator=g).to(torch.bfloat16).cuda()
    b = torch.randn((n, d, d, d, cb), generator=g).to(torch.bfloat16).cuda()
    w = (torch.randn((27, cout, ca + cb), generator=g) * 0.05).to(torch.bfloat16).cuda()
    bias = torch.zeros(cout, dtype=torch.float32).cuda()
    for _ in range(5):
        mg.nn.conv3d(a, w, bias, b=b, up_a=True)
    launches = 50
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(launches):
        mg.nn.conv3d(a, w, bias, b=b, up_a=True)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / launches
    flops = 2.0 * 27 * (ca + cb) * cout * n * d ** 3
    tf = flops / (ms * 1e-3) / 1e12
    return {"bound": "mfma", "kernel": f"k_conv_tile ({name}: {ca} up-sampled + {cb} skip -> {cout} channels, "
                                       f"{n} x {d}^3 voxels)",
            "achieved": round(tf, 1), "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s", "frac": round(tf / PEAK_BF16_TFLOPS, 4),
            "traffic": None, "avg_launch_us": round(ms * 1e3, 2), "algorithmic_flops_per_launch": flops}


def vcycle_rate(n_act, ms_solve, cycles):
    """Whole-cycle throughput: VCYCLE_BYTES_FP64 per active finest cell over
    the solve's time per cycle (the fold and norm readbacks included)."""
    us = ms_solve * 1e3 / max(1, cycles)
    gbs = VCYCLE_BYTES_FP64 * n_act / (us * 1e-6) / 1e9
    return {"bound": "hbm", "algorithmic_bytes_per_cycle": VCYCLE_BYTES_FP64 * n_act, "us_per_cycle": round(us, 2),
            "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4)}


def large_measurement(args):
    """The porous workload at --large-n^3 (seed 4: 4096 holes with radii
    U[0.005, 0.02), k^-2 random-field rho, Dirichlet 0): time to 1e-10 from a
    zero guess in FP64 and in mixed precision (median of 3 after one warm-up,
    wall time with inputs resident), the mixed solution's largest difference
    from the FP64 one, and the finest smoother pass at this size, where the
    working set far exceeds the 256 MB MALL."""
    import torch

    from paper_1104_1703_amd import gen, mg
    t0 = time.perf_counter()
    p = gen.porous_problem(args.large_n, seed=4)
    t_gen = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    mask = torch.from_numpy(p.mask).to(dev)
    rho = torch.from_numpy(p.rho).to(dev)
    phi = torch.zeros(p.shape, dtype=torch.float64, device=dev)
    res, phi64 = {}, None
    for prec in ("fp64", "mixed"):
        H = mg.Hierarchy(mask, p.h, precision=prec, tune=1)
        walls, info = [], None
        for rep in range(4):
            phi.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = H.solve(rho, phi, None, tol=args.tol)[1]
            torch.cuda.synchronize()
            if rep:
                walls.append(time.perf_counter() - t0)
        r = {"ms": round(float(np.median(walls)) * 1e3, 3), "cycles": info["cycles"],
             "switched_at": info["switched_at"], "final_rel_residual": info["r_final"] / info["r_ref"],
             "item_depths": H.item_depths()}
        if prec == "fp64":
            n_act = H.n_active(0)
            H.time_smoother(4)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(H.stream)
            H.time_smoother(20)
            e1.record(H.stream)
            e1.synchronize()
            us = e0.elapsed_time(e1) / 20 * 1e3
            gbs = SMOOTH_BYTES_FP64 * n_act / (us * 1e-6) / 1e9
            r["smoother_us"] = round(us, 2)
            r["smoother_algorithmic_gbs"] = round(gbs, 1)
            r["smoother_frac"] = round(gbs / PEAK_HBM_GBS, 4)
            r["vcycle"] = vcycle_rate(n_act, r["ms"], info["cycles"])
            phi64 = phi.clone()
        else:
            r["max_rel_diff_vs_fp64_solution"] = float((phi - phi64).abs().max() / phi64.abs().max())
        res[prec] = r
        H.close()
    res["mixed"]["speedup_vs_fp64"] = round(res["fp64"]["ms"] / res["mixed"]["ms"], 3)
    return {"workload": f"porous{args.large_n}: {args.large_n}^3 box minus 4096 seeded spheres (seed 4), "
                        f"{p.n_active} active, k^-2 random-field rho, Dirichlet 0, zero guess, tol {args.tol:g}",
            **res, "generate_s": round(t_gen, 1)}


def amr_study(args):
    """One-way nested levels (the accuracy tests of Sec. 5.1 in 3D): the ln
    profile (r0 = 0.1) on a base n^3 box plus 3 refined n^3 levels around the
    centre, each solved to 1e-12 with Dirichlet values interpolated from the
    level above; composite-grid errors of the potential and of the 5-point
    gradient, their orders between successive n, and the GPU time of the whole
    chain (one warm-up chain first); the same from the interpolated first
    guess on the refined levels."""
    from paper_1104_1703_amd import amr
    ns = [int(v) for v in args.amr.split(",") if v]
    amr.solve_nested(ns[0], 3)  # warm-up
    rows = []
    for n in ns:
        levels, ms = amr.solve_nested(n, 3)
        e = composite_errors(levels)
        li, ms_i = amr.solve_nested(n, 3, guess="interp")
        ei = composite_errors(li)
        rows.append({"n": n, "finest_h": levels[-1].h, "ms": round(ms, 3),
                     "cycles": [L.info["cycles"] for L in levels], **e,
                     "interp_guess": {"ms": round(ms_i, 3), "cycles": [L.info["cycles"] for L in li],
                                      "phi_linf": ei["phi_linf"], "grad_linf": ei["grad_linf"]}})
    for a, b in zip(rows, rows[1:]):
        b["orders"] = {k: round(float(np.log2(a[k] / b[k])), 3) for k in ("phi_linf", "phi_l2", "grad_linf", "grad_l2")}
    print(json.dumps({"mode": "amr", "workload": "ln profile r0 = 0.1, base n^3 box + 3 nested n^3 levels "
                      "(central 1/2, 1/4, 1/8), tol 1e-12", "rows": rows}), flush=True)


def composite_errors(levels, r0: float = 0.1):
    """Measurement of a nested solve against the closed form (not part of the
    solve): over the composite grid (each point on the finest level that
    covers it; level-0 cells whose 5-point stencil leaves the array left
    out), the largest and the volume-weighted RMS error of the potential and
    of the gradient's Euclidean length, the latter relative to the largest
    exact gradient length."""
    from paper_1104_1703_amd import gen
    ep, eg, vol, gmax = [], [], [], 0.0
    for k, L in enumerate(levels):
        ctr = gen.level_centres(L.shape, L.h, L.origin)
        phi_e, _, grad_e = gen.ln_profile(ctr, r0)
        use = gen.frame_mask(L.shape) == 1
        if k + 1 < len(levels):
            N = levels[k + 1]
            lo = np.array(N.origin) + N.h
            hi = np.array(N.origin) + (np.array(N.shape[::-1]) - 1) * N.h
            use &= ~np.all((ctr > lo) & (ctr < hi), axis=-1)
        if k == 0:
            core = np.zeros(L.shape, dtype=bool)
            core[2:-2, 2:-2, 2:-2] = True
            use &= core
        phi = L.phi.cpu().numpy()
        g = np.moveaxis(L.grad.cpu().numpy(), 0, -1)
        ep.append(np.abs(phi - phi_e)[use])
        eg.append(np.linalg.norm(g - grad_e, axis=-1)[use])
        vol.append(np.full(int(use.sum()), L.h ** 3))
        gmax = max(gmax, float(np.linalg.norm(grad_e, axis=-1)[use].max()))
    ep, eg, vol = np.concatenate(ep), np.concatenate(eg), np.concatenate(vol)
    return {"phi_linf": float(ep.max()), "phi_l2": float(np.sqrt((vol * ep ** 2).sum() / vol.sum())),
            "grad_linf": float(eg.max() / gmax), "grad_l2": float(np.sqrt((vol * eg ** 2).sum() / vol.sum()) / gmax)}


def schedules(args):
    """Multigrid schedules on the sphere (the domain where second order
    converges): N_cycles = 1 (V), 2 (W) and 3 in first and second order, each
    to 1e-10 from a zero guess (median of 3 solves after one warm-up)."""
    import torch

    from paper_1104_1703_amd import gen, mg
    p = gen.holes_problem(args.schedules, seed=2) if args.schedules_workload == "holes" else \
        gen.sphere_problem(args.schedules)
    dev = torch.device("cuda:0")
    mask = torch.from_numpy(p.mask).to(dev)
    rho = torch.from_numpy(p.rho).to(dev)
    phi = torch.zeros(p.shape, dtype=torch.float64, device=dev)
    rows = []
    orders = ("second", "first", "auto") if args.schedules_workload == "holes" else ("second", "first")
    for nc in (1, 2, 3):
        for bo in orders:
            H = mg.Hierarchy(mask, p.h, n_cycles=nc, bc_order=bo, tune=1)
            walls, info = [], None
            for rep in range(4):
                phi.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = H.solve(rho, phi, None, tol=args.tol, check=False)[1]
                torch.cuda.synchronize()
                if rep:
                    walls.append(time.perf_counter() - t0)
            h = info["history"]
            rows.append({"n_cycles": nc, "order": bo, "status": info["status"], "cycles": info["cycles"],
                         "mean_rate": (h[-1] / h[0]) ** (1.0 / max(1, info["cycles"])),
                         "ms": round(float(np.median(walls)) * 1e3, 3)})
            H.close()
    what = (f"holes{args.schedules} (seed 2; AUTO: the untimed first solve switches order, the timed ones "
            f"start held in first order)"
            if args.schedules_workload == "holes" else
            f"sphere{args.schedules}: R = 0.4 Dirichlet 0, rho = 1 inside r = 0.2")
    print(json.dumps({"mode": "schedules", "workload": f"{what}, tol {args.tol:g}", "rows": rows}), flush=True)


def profile_batch(args):
    """Batch solves alone, for kernel-trace runs: one warm-up, then N solves."""
    r = batch_measurement(args, solves=args.profile_batch)
    print(json.dumps({"mode": "profile-batch", "solves": args.profile_batch, **r}), flush=True)


def batch_measurement(args, solves=3):
    """The batched workload: `--batch-patches` masked patches (edges log-uniform
    in 16..128, multiples of 8, seed 3), FP64, V(2,2), each to 1e-10; the
    wall time of one mg_solve_batch call (inputs resident), median of
    `solves` timed solves after one warm-up, on each engine; the patch
    hierarchies are built untimed."""
    import torch

    from paper_1104_1703_amd import gen, mg
    t0 = time.perf_counter()
    probs = gen.patch_problems(count=args.batch_patches, seed=3)
    t_gen = time.perf_counter() - t0
    masks = [torch.from_numpy(p.mask).cuda() for p in probs]
    rhos = [torch.from_numpy(p.rho).cuda() for p in probs]
    dirs = [torch.from_numpy(p.dirichlet).cuda() for p in probs]
    phis = [torch.zeros(p.shape, dtype=torch.float64, device="cuda") for p in probs]

    def timed(engine):
        """A fresh batch on `engine`: its build time, the median wall of the
        timed solves, their infos and the warm-up solve's.  Patches that
        switch order in the warm-up solve keep first order in the timed ones
        (the hold of Sec. 4), on either engine alike."""
        t0 = time.perf_counter()
        B = mg.Batch(masks, [p.h for p in probs])
        torch.cuda.synchronize()
        t_build = time.perf_counter() - t0
        if B.phases(2) == 0:
            raise RuntimeError("the batch has no phase programs for the default options")
        B.set_engine(engine)
        walls, infos, first = [], None, None
        for rep in range(solves + 1):
            for x in phis:
                x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, infos, _ = B.solve(rhos, phis, dirs, tol=1e-10)
            torch.cuda.synchronize()
            if rep > 0:
                walls.append(time.perf_counter() - t0)
            else:
                first = infos
        B_phases = B.phases(2)
        B.close()
        return float(np.median(walls)) * 1e3, infos, first, t_build, B_phases

    ms, infos, first, t_build, B_phases = timed("phased")
    ms_p, infos_p, _, _, _ = timed("persistent")
    active = sum(p.n_active for p in probs)
    cycles = [i["cycles"] for i in infos]
    return {"workload": f"{len(probs)} masked patches (seed 3), {sum(p.mask.size for p in probs)} cells, "
                        f"{active} active, Dirichlet data, tol 1e-10",
            "engine": f"phase programs: one launch per cycle phase over all patches' work items "
                      f"({B_phases} launches per cycle); the first finest pass also forms the norm of its "
                      f"input, then one norm copy and synchronisation per cycle",
            "ms": round(ms, 3), "active_cells_per_s": round(active / (ms * 1e-3), 1),
            "persistent_ms": round(ms_p, 3),
            "persistent_engine": "the same programs as phases of one cooperative launch per V-cycle (grid-wide "
                                 "barriers between phases), same results bit for bit",
            "persistent_all_converged": all(i["status"] == 0 for i in infos_p),
            "cycles_min": min(cycles), "cycles_max": max(cycles), "cycles_total": int(sum(cycles)),
            "warmup_cycles_total": int(sum(i["cycles"] for i in first)),
            "warmup_switched": int(sum(i["switched_at"] > 0 for i in first)),
            "all_converged": all(i["status"] == 0 for i in infos),
            "build_s": round(t_build, 2), "generate_s": round(t_gen, 2)}


def cpu_baseline(p, repeats):
    """The oracle as it stands: its complete solve of the same workload (same
    recipe, zero guess, same 1e-10 target, its own order switch), repeated
    `repeats` times on the host cores; the mean wall time per solve."""
    import numpy as np

    from oracle import oracle as O
    threads = min(os.cpu_count() or 1, 16)
    O.set_threads(threads)
    orc = O.Oracle(p.mask, p.h)
    times, cycles = [], []
    for _ in range(max(1, repeats)):
        t0 = time.perf_counter()
        _, info = orc.solve(p.rho, np.zeros(p.shape), None, tol=1e-10)
        times.append(time.perf_counter() - t0)
        cycles.append(info["cycles"])
    cpu = ""
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": float(np.mean(times)) * 1e3,
        "unit": "ms",
        "cores": O.num_threads(),
        "host_cpu": f"{cpu}, {os.cpu_count()} logical CPUs visible",
        "kind": "oracle",
        "sample": f"{len(times)} complete oracle solves of the {p.shape[0]}^3 holes workload to 1e-10 "
                  f"({cycles} cycles, {sum(times):.1f} s in all); value = mean wall time per solve",
    }


def main():
    args = parse()
    if args.profile_smoother:
        return profile_smoother(args)
    if args.copy_calibration:
        return copy_calibration(args)
    if args.profile_unet:
        return profile_unet(args)
    if args.profile_batch:
        return profile_batch(args)
    if args.profile_solves:
        return profile_solves(args)
    if args.schedules:
        return schedules(args)
    if args.amr:
        return amr_study(args)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path "
              "(its domain decomposition over GPUs is not implemented).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1104_1703_amd import gen, mg

    dev = torch.device("cuda:0")
    p = gen.holes_problem(n=args.n, seed=args.seed)
    mask = torch.from_numpy(p.mask).to(dev)
    rho = torch.from_numpy(p.rho).to(dev)
    phi = torch.zeros(p.shape, dtype=torch.float64, device=dev)

    def time_solves(H, make_guess=None, prho=None, pphi=None):
        """W warm-up then K timed solves on one fresh hierarchy, each solve
        timed alone (wall clock, synchronised) and recorded with its regime:
        a solve that starts in second order and switches, or one that starts
        held in first order by an earlier switch (Sec. 4), take different
        cycle counts, so both the mean over the K solves (`value`) and the
        per-regime figures are reported.  Every variant runs the same
        schedule on its own fresh hierarchy.  No kernel timing is on: its
        event pairs would add a few microseconds around each launch timed."""
        prho = rho if prho is None else prho
        pphi = phi if pphi is None else pphi

        def step():
            if make_guess is None:
                pphi.zero_()
            else:
                make_guess(pphi)
            return H.solve(prho, pphi, None, tol=args.tol)[1]
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        infos, walls = [], []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            t1 = time.perf_counter()
            infos.append(step())
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t1)
        wall = time.perf_counter() - t0
        return wall / max(1, args.steps) * 1e3, infos, walls

    def regimes(infos, walls):
        out = {}
        for info, w in zip(infos, walls):
            key = ("switching" if info["switched_at"] >= 0 else
                   "held_first_order" if info["order_used"] == 1 else "second_order")
            r = out.setdefault(key, {"solves": 0, "ms": [], "cycles": [], "switched_at": []})
            r["solves"] += 1
            r["ms"].append(w * 1e3)
            r["cycles"].append(info["cycles"])
            r["switched_at"].append(info["switched_at"])
        for r in out.values():
            r["ms_mean"] = round(float(np.mean(r.pop("ms"))), 4)
            r["cycles"] = sorted(set(r["cycles"]))
            r["switched_at"] = sorted(set(r["switched_at"]))
        return out

    # hierarchy build, reported apart from the solves: with the default work
    # items (the second of two builds: the first also loads the library's
    # code objects), then with the autotuner timing its candidates (when no
    # MG_TUNE_CACHE file holds them)
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Hd = mg.Hierarchy(mask, p.h, precision="fp64")
        torch.cuda.synchronize()
        build_default_ms = (time.perf_counter() - t0) * 1e3
        Hd.close()
    t0 = time.perf_counter()
    H = mg.Hierarchy(mask, p.h, precision="fp64", tune=1)
    torch.cuda.synchronize()
    build_tuned_ms = (time.perf_counter() - t0) * 1e3
    n_act = H.n_active(0)
    depths64 = H.item_depths()
    ms_wall, infos64, walls64 = time_solves(H)
    # after the timed region, each kind of finest-level pass of a cycle timed
    # inside more solves of the same schedule by the HIP event pairs the
    # library records around its launches (one kind per set of solves)
    finest = {}
    for kind, solves in (("plain", 4), ("residual", 2), ("prolong", 2), ("norm", 2)):
        H.kernel_timing(True, kind)
        for _ in range(solves):
            phi.zero_()
            H.solve(rho, phi, None, tol=args.tol)
        finest[kind] = H.kernel_timing_read()
        H.kernel_timing(False)
    k_ms, k_launches = finest["plain"]
    last = infos64[-1]
    reg64 = regimes(infos64, walls64)
    ms_events = float(np.median([i["ms"] for i in infos64]))
    cycles_mean = float(np.mean([i["cycles"] for i in infos64]))

    # dominant kernel: the finest-level plain red-black pass, its average
    # launch duration from the HIP event pairs that the library's launches of
    # it record inside solves of the benchmark's schedule run after the timed
    # ones (the kernel's own start and end, on the solver's stream)
    if k_launches == 0:
        raise RuntimeError("no finest-level smoother launch was timed")
    smooth_ms = k_ms / k_launches
    # beside it: the same kernel back to back, in batches of 20 launches (an
    # unbroken run of a few hundred passes shows a stretch of launches 10-15%
    # slower than inside the solves, where lighter kernels come between them)
    launches = args.smoother_launches - (args.smoother_launches % 20)
    H.time_smoother(8)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    total_ms = 0.0
    for _ in range(launches // 20):
        e0.record(H.stream)
        H.time_smoother(20)
        e1.record(H.stream)
        e1.synchronize()
        total_ms += e0.elapsed_time(e1)
    b2b_ms = total_ms / max(1, launches)
    bytes_per = SMOOTH_BYTES_FP64 * n_act
    achieved = bytes_per / (smooth_ms * 1e-3) / 1e9
    phi64 = phi.clone()
    H.close()

    net_box = {}

    def network():
        from paper_1104_1703_amd import guess
        if "net" not in net_box:
            net_box["net"] = guess.load_network(args.weights or guess.WEIGHTS)
        return net_box["net"]

    def measure_variants(names, prob, pmask, prho, base_reg, base_ms, base_phi):
        """Each variant on its own fresh (tuned) hierarchy with the same
        schedule as the FP64 zero-guess line, guess included in the time."""
        out_v = {}
        for v in names:
            precision = "mixed" if v in ("mixed", "learned_mixed") else "fp64"
            make_guess, extra, ig = None, {}, None
            if v == "interp":
                from paper_1104_1703_amd import guess
                ig = guess.InterpolatedGuess(pmask, prob.h, tune=1)
                make_guess = lambda out: ig(prho, out=out)
                extra["guess"] = "problem coarsened by 2 per axis, FP64 multigrid to 1e-4, linear up-sampling"
            elif v.startswith("learned"):
                try:
                    net = network()
                except FileNotFoundError as e:
                    out_v[v] = {"skipped": str(e)}
                    continue
                stride = int(v[len("learned_s"):]) if v.startswith("learned_s") else args.learned_stride
                make_guess = lambda out, stride=stride: net.infer(prho, pmask, stride=stride, out=out)
                for _ in range(3):
                    make_guess(phi_v)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(10):
                    make_guess(phi_v)
                torch.cuda.synchronize()
                extra["guess"] = f"U-Net at 1/{stride} resolution, linear up-sampling"
                extra["guess_ms"] = round((time.perf_counter() - t0) / 10 * 1e3, 4)
            elif v != "mixed":
                raise SystemExit(f"unknown variant {v}")
            Hv = mg.Hierarchy(pmask, prob.h, precision=precision, tune=1)
            v_wall, v_infos, v_walls = time_solves(Hv, make_guess, prho, phi_v)
            v_last = v_infos[-1]
            v_reg = regimes(v_infos, v_walls)
            for k, r in v_reg.items():
                if k in base_reg:
                    r["speedup_vs_fp64"] = round(base_reg[k]["ms_mean"] / r["ms_mean"], 3)
            diff = float((phi_v - base_phi).abs().max() / base_phi.abs().max())
            out_v[v] = {"ms": round(v_wall, 4), "speedup_vs_fp64": round(base_ms / v_wall, 3),
                        "regimes": v_reg, "cycles_mean": float(np.mean([i["cycles"] for i in v_infos])),
                        "final_rel_residual": v_last["r_final"] / v_last["r_ref"],
                        "initial_rel_residual": v_last["r0"] / v_last["r_ref"],
                        "max_rel_diff_vs_fp64_solution": diff, "item_depths": Hv.item_depths(), **extra}
            Hv.close()
            if ig is not None:
                ig.close()
        return out_v

    phi_v = phi
    variants = measure_variants([x for x in args.variants.split(",") if x], p, mask, rho, reg64, ms_wall, phi64)

    # Learned guess on both readings of "applied at 256^3 like config 1":
    # the 256^3 sphere geometry (config 1's domain) next to the zero and
    # interpolated starts, at network strides 1, 2 and 4
    learned_eval = None
    if args.learned_eval:
        ps = gen.sphere_problem(args.n)
        smask = torch.from_numpy(ps.mask).to(dev)
        srho = torch.from_numpy(ps.rho).to(dev)
        phi_v = torch.zeros(ps.shape, dtype=torch.float64, device=dev)
        Hs = mg.Hierarchy(smask, ps.h, precision="fp64", tune=1)
        s_wall, s_infos, s_walls = time_solves(Hs, None, srho, phi_v)
        s_reg = regimes(s_infos, s_walls)
        s_phi = phi_v.clone()
        Hs.close()
        learned_eval = {
            "workload": f"sphere{args.n}: R = 0.4 Dirichlet 0, rho = 1 inside r = 0.2, tol {args.tol:g}",
            "zero": {"ms": round(s_wall, 4), "regimes": s_reg},
            **measure_variants(["interp", "learned_s1", "learned_s2", "learned_s4"], ps, smask, srho, s_reg,
                               s_wall, s_phi)}
        phi_v = phi

    traffic = measured_traffic() if args.n == 256 and args.seed == 2 else None
    out = {
        "metric": "time-to-1e-10 residual & smoother HBM GB/s at 256^3 masked; learned/mixed vs FP64",
        "value": round(ms_wall, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_wall, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"holes{args.n}: {args.n}^3 unit cube, outer sphere R=0.45 minus 64 seeded spheres "
                        f"(seed {args.seed}), rho = 32 Gaussians, Dirichlet 0, zero guess, V(2,2), tol {args.tol:g}",
            "active_cells": n_act,
            "precision": "fp64",
            "cycles_mean": cycles_mean,
            "regimes": reg64,
            "item_depths": depths64,
            "final_rel_residual": last["r_final"] / last["r_ref"],
            "ms_events_median": round(ms_events, 4),
            "hierarchy_build_ms": {"default": round(build_default_ms, 2), "tuned": round(build_tuned_ms, 2)},
        },
        "variants": variants,
        "learned_eval": learned_eval,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_rbgs<double,true> (finest-level red-black pass)",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_gbs": round(traffic / (smooth_ms * 1e-3) / 1e9, 1) if traffic else None,
            "avg_launch_us": round(smooth_ms * 1e3, 3),
            "launches_timed": k_launches,
            "timing": "HIP event pair (the kernel's start and end, hipExtLaunchKernel) on each plain "
                      "finest-level pass of 4 solves of the same schedule after the timed ones",
            "algorithmic_bytes_per_launch": bytes_per,
            "back_to_back_us": round(b2b_ms * 1e3, 3),
            "back_to_back_frac": round(bytes_per / (b2b_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            "finest_kernels": finest_kernels(finest, n_act),
        },
        "vcycle": vcycle_rate(n_act, ms_wall, cycles_mean),
    }
    if args.large_n > 0:
        out["large"] = large_measurement(args)
    if args.batch_patches > 0:
        out["batch"] = batch_measurement(args)
    try:
        out["unet_conv_roofline"] = unet_conv_roofline()
    except Exception as e:  # reported, never hidden
        out["unet_conv_roofline"] = {"error": str(e)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_solves)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
