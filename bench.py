"""Throughput of the splat renderer on one MI355X.

Default workload: 300k points (30% on a bumpy surface), SH degree 2, four
800x800 views per step, FP32, trained for 100 Adam steps (positions, SH,
opacity logits) against renders of a ground-truth scene.  One timed step is
the whole hot path over one batch -- projection + SH colour, depth sort, tile
binning, compositing (forward), the L2-loss gradient and the compositing +
per-point backward -- measured with HIP events on the stream; the Adam update
runs between the timed steps and is reported with them as the training-step
rate.  Inputs (scene, cameras, target images) are resident in HBM before
timing starts.

Prints ONE JSON line:  metric/value = forward+backward Mpix/s (stored-T mode),
plus forward-only and recompute-T rates, the same-run parity of step 0 and of
the last step against the FP64 oracle (all views in full, gradients in both
backward modes), the roofline of the dominant kernel (HIP events on the
library's stream around that kernel in the timed loop, and the committed
rocprofv3 figures of the same kernel), a per-stage breakdown, the FP64 CPU
oracle timed on step 0, and the serving leg (a 60 s Poisson trace at 200
req/s and a short overload trace, continuous batching against one view per
launch).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s fwd & fwd+bwd (300k pts, 800x800) at 1e-4 err; served p50/p99 latency"
PEAK_HBM = 8.0e12                 # B/s
# FP32 VALU lane-ops/s: 256 CUs x 4 SIMDs x 32 lanes per clock x 2.4 GHz = 78.6 T, the published
# 157.3 TFLOP/s FP32 vector rate with an FMA counted as one lane-op.  Plain (non-packed) FP32
# instructions with VGPR operands issue a wave64 every two clocks per SIMD, so this rate needs no
# packed instructions.
PEAK_LANE_OPS = 256 * 4 * 32 * 2.4e9
FWD_OPS_PER_BLEND = 20            # lane-ops per blended (pixel, splat), forward composite
BWD_OPS_PER_BLEND = 50            # lane-ops per blended (pixel, splat), backward composite
EMIT_BYTES_PER_ITEM = 32          # bytes tile emission reads per depth-sorted item


def load_profile(workload: str):
    """Per-kernel rocprofv3 figures of the committed summary
    profiles/kernels_<workload>.json (average duration of the step's launches,
    VALU busy share) if taken on the current kernel sources; else None."""
    from paper_2205_14330_amd.profiling import kernel_source_hash
    if workload is None:
        return None
    p = os.path.join(ROOT, "profiles", f"kernels_{workload}.json")
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("kernels")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` (rocprofv3 FETCH_SIZE + WRITE_SIZE of
    the training steps' launches) from the committed profile of `workload`,
    if it was taken on the current kernel sources; else None."""
    e = (load_profile(workload) or {}).get(kernel)
    return None if not e else e.get("bytes_per_launch")


def copy_calibration(torch, dev, mib):
    """One device copy of `mib` MiB: the reference the HBM counters are scaled by."""
    src = torch.empty(mib * (1 << 20) // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: {mib} MiB read + written")


TRAIN_STEPS = 100                 # Adam steps of the training trajectory (at least)
# Adam learning rates: positions and SH as Sec. 3.3 sets them; the opacity
# logit's rate is this benchmark's own (the paper learns no opacity)
LR_XYZ, LR_SH, LR_LOGIT = 8e-4, 3e-3, 1e-2
GRAD_RTOL = 1e-3                  # per element, relative to max(|g*|, 1e-2 ||g*||_inf)
GRAD_L2 = 1e-3                    # ||g - g*||_2 / ||g*||_2
IMG_TOL = 1e-4                    # max-abs per pixel and channel, image and transmittance


class Trainer:
    """Adam on the positions, SH coefficients and opacity logits of one scene
    (o = sigmoid(l), so dL/dl = dL/do o (1 - o)).  The scene tensors are
    updated in place on the current stream after each backward."""

    def __init__(self, init):
        import torch
        from paper_2205_14330_amd import SceneTensors
        self.init = init
        self.scene = SceneTensors(init.xyz.clone(), init.sh.clone(), init.opacity.clone(), init.radius)
        o = init.opacity.double()
        self.logit0 = torch.log(o / (1.0 - o)).float()
        self.logit = self.logit0.clone()
        self.grads = (torch.empty_like(init.xyz), torch.empty_like(init.sh), torch.empty_like(init.opacity))
        self.glogit = torch.empty_like(init.opacity)
        self.params = (self.scene.xyz, self.scene.sh, self.logit)
        self.m = [torch.zeros_like(x) for x in self.params]
        self.v = [torch.zeros_like(x) for x in self.params]
        self.t = 0

    def reset(self):
        self.scene.xyz.copy_(self.init.xyz)
        self.scene.sh.copy_(self.init.sh)
        self.scene.opacity.copy_(self.init.opacity)
        self.logit.copy_(self.logit0)
        for a in self.m + self.v:
            a.zero_()
        self.t = 0

    def update(self):
        import torch
        from paper_2205_14330_amd.chamfer import adam_step
        self.t += 1
        gx, gs, go = self.grads
        o = self.scene.opacity
        torch.mul(go, o, out=self.glogit)
        self.glogit.addcmul_(self.glogit, o, value=-1.0)          # go o (1 - o)
        for p_, g_, m_, v_, lr in zip(self.params, (gx, gs, self.glogit), self.m, self.v, (LR_XYZ, LR_SH, LR_LOGIT)):
            adam_step(p_, g_, m_, v_, self.t, lr)
        torch.sigmoid(self.logit, out=o)

    def numpy_scene(self):
        import workloads
        s = self.scene
        return workloads.Scene(s.xyz.cpu().numpy(), s.sh.cpu().numpy(), s.opacity.cpu().numpy(),
                               s.radius.cpu().numpy())


def grad_margin(g, ref):
    """(worst element error as a fraction of its bound, rel-L2) of a gradient
    against the oracle's, bound |g - g*| <= 1e-3 max(|g*|, 1e-2 ||g*||_inf)."""
    g = np.asarray(g, np.float64).reshape(-1)
    r = np.asarray(ref, np.float64).reshape(-1)
    gmax = np.abs(r).max()
    bound = GRAD_RTOL * np.maximum(np.abs(r), 1e-2 * gmax)
    return float(np.max(np.abs(g - r) / bound)), float(np.linalg.norm(g - r) / np.linalg.norm(r))


def parity_weights(views, size):
    """Seeded N(0, 1) weights w[v] [H][W][3]: the parity checks use the linear
    loss L = sum w I, so dL/dI = w is the same input on both sides."""
    rng = np.random.default_rng(np.random.SeedSequence(0, spawn_key=(3, 2)))
    return [rng.standard_normal((size, size, 3)).astype(np.float32) for _ in range(views)]


def gpu_step_outputs(dpr, scene, cams, weights, variant):
    """One step's forward and, with dL/dI = weights, the backward in both
    modes, on the current cloud (nothing is updated): the values the parity
    check compares with the oracle."""
    import torch
    out = {}
    w = [torch.from_numpy(x).cuda() for x in weights]
    for mode in ("stored", "recompute"):
        plan = dpr.Plan([scene], [(0, c) for c in cams], dpr.RenderParams(bwd_mode=mode, **variant))
        plan.forward()
        g = plan.backward(w, None)[0]
        torch.cuda.synchronize()
        if mode == "stored":
            out["images"] = [t.cpu().numpy() for t in plan.images]
            out["trans"] = [t.cpu().numpy() for t in plan.trans]
        out[mode] = [t.cpu().numpy() for t in g]
        plan.free()
    return out


def oracle_step(scene_np, cams, weights, max_splats, kernel_norm, threads):
    """The FP64 oracle on one full step: forward of every view and the
    backward with dL/dI = weights.  Returns (seconds, renders, gradients)."""
    import oracle
    op = oracle.Params(max_splats=max_splats, kernel_norm=kernel_norm)
    t0 = time.perf_counter()
    renders = [oracle.render(scene_np, cam, op, threads=threads) for cam in cams]
    g = oracle.backward(scene_np, cams, [w.astype(np.float64) for w in weights], None, params=op, threads=threads)
    return time.perf_counter() - t0, renders, g


def near_tie_masks(scene_np, cams, max_splats, kernel_norm, threads):
    """Under a cap (max_splats > 0), the pixels whose n-th splat rests on a
    predicate within a relative 1e-4 of alpha_min (the oracle's near_tie flag):
    an FP32 and an FP64 evaluation may each take one of two valid results
    there, a whole splat apart.  The parity check leaves them out (their
    weight in the linear loss is 0 on both sides).  None without a cap."""
    if not max_splats:
        return None
    import oracle
    op = oracle.Params(max_splats=max_splats, kernel_norm=kernel_norm)
    return [oracle.render(scene_np, cam, op, threads=threads).near_tie for cam in cams]


def masked(weights, masks):
    if masks is None:
        return weights
    return [np.where(m[..., None], np.float32(0.0), w).astype(np.float32) for w, m in zip(weights, masks)]


def parity_report(gpu, renders, g, masks=None):
    def err(a, r, m):
        d = np.abs(a.astype(np.float64) - r)
        if m is not None:
            d = d[~m]
        return float(d.max()) if d.size else 0.0
    ms = masks or [None] * len(renders)
    img = max(err(a, r.image, m) for a, r, m in zip(gpu["images"], renders, ms))
    tr = max(err(a, r.trans, m) for a, r, m in zip(gpu["trans"], renders, ms))
    rep = {"img_max_err": img, "trans_max_err": tr, "grads": {}}
    if masks is not None:
        rep["near_tie_pixels"] = int(sum(int(m.sum()) for m in masks))
    ok = img <= IMG_TOL and tr <= IMG_TOL
    for mode in ("stored", "recompute"):
        d = {}
        for name, got, want in zip(("xyz", "sh", "opacity"), gpu[mode], (g.xyz, g.sh, g.opacity)):
            worst, l2 = grad_margin(got, want)
            d[name] = {"worst_over_bound": round(worst, 4), "rel_l2": float(f"{l2:.3e}")}
            ok = ok and worst <= 1.0 and l2 <= GRAD_L2
        rep["grads"][mode] = d
    rep["grad_worst_over_bound"] = max(e["worst_over_bound"] for m in rep["grads"].values() for e in m.values())
    rep["grad_rel_l2"] = max(e["rel_l2"] for m in rep["grads"].values() for e in m.values())
    rep["pass"] = bool(ok)
    return rep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--points", type=int, default=300_000)
    ap.add_argument("--size", type=int, default=800)
    ap.add_argument("--views", type=int, default=4)
    ap.add_argument("--train-steps", type=int, default=TRAIN_STEPS,
                    help="length of the Adam trajectory (at least warmup + steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle (CPU baseline and the parity checks at both ends of the trajectory)")
    ap.add_argument("--persistent", action="store_true")
    ap.add_argument("--main-only", action="store_true",
                    help="time only the forward + backward metric (skip the forward-only and recompute legs)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after timing, run one device copy of this many MiB (reference for HBM counters)")
    ap.add_argument("--workload", choices=["train", "paper", "dynamic", "serve", "hull", "warmstart", "hybrid"],
                    default="train",
                    help="train: the default step; paper: the same step with the paper-literal renderer "
                         "(n = 15 splats per pixel, normalised Eq. 5) and the L2 + 0.01 TV loss")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the serving trace (train: a leg of the same JSON line; 0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--overload-rate", type=float, default=3000.0,
                    help="train: rate of the short overload trace of the serving leg (0 = skip)")
    ap.add_argument("--overload-seconds", type=float, default=2.0)
    ap.add_argument("--profile", action="store_true",
                    help="for rocprofv3: set-up, then only `warmup + steps` training steps (no timing events, "
                         "parity, other legs or serving), then the copy calibration if asked")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this renderer runs on one GPU; --gpus above 1 is not supported "
                                   "(multi-GPU sharding is a design note only)"}))
        sys.exit(2)

    import torch
    import workloads
    import paper_2205_14330_amd as dpr

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    dpr.load()
    dev = torch.device("cuda:0")
    if args.workload == "dynamic":
        return bench_dynamic(args)
    if args.workload == "hull":
        return bench_hull(args)
    if args.workload == "warmstart":
        return bench_warmstart(args)
    if args.workload == "hybrid":
        return bench_hybrid(args)
    if args.workload == "serve":
        out = {"metric": "served p50/p99 latency and Mpix/s (16 resident scenes, Poisson requests)",
               "n_gpus": 1, "dtype": "f32", "data": "synthetic"}
        out.update(bench_serving(args.serve_seconds if args.serve_seconds > 0 else 60.0, args.serve_rate))
        print(json.dumps(out), flush=True)
        return
    V, S = args.views, args.size
    W_, K = args.warmup, args.steps
    n_traj = max(args.train_steps, W_ + K)
    scene_np, cams, gt_np = workloads.surface300k_4x800(n=args.points, size=S, views_per_step=V, steps=100)
    init = dpr.SceneTensors.from_numpy(scene_np, dev)
    gt = dpr.SceneTensors.from_numpy(gt_np, dev)
    step_views = [cams[(k % 100) * V:(k % 100) * V + V] for k in range(n_traj)]

    # targets: renders of the ground-truth scene from each step's views (untimed)
    targets = []
    for k in range(min(n_traj, 100)):
        p = dpr.Plan([gt], [(0, c) for c in step_views[k]], dpr.RenderParams(bwd_mode="recompute"))
        p.forward()
        targets.append(torch.stack(p.images).clone())
        p.free()
    torch.cuda.synchronize()
    log(f"setup done: {args.points} points, {V} x {S}x{S}, trajectory of {n_traj} Adam steps, "
        f"timed steps {W_}..{W_ + K - 1}")

    trainer = Trainer(init)
    # two live plans at a time (one being inspected while the next runs), so two
    # workspaces, each reused every other step
    wss = [dpr.Workspace(dev), dpr.Workspace(dev)]
    paper = args.workload == "paper"
    lam = 0.01 if paper else 0.0
    variant = dict(max_splats=15, kernel_norm=True) if paper else {}
    # the loss gradient of a step is consumed by that step's backward on the same
    # stream before the next step's loss kernel overwrites it
    grads = [torch.empty((S, S, 3), dtype=torch.float32, device=dev) for _ in range(V)]
    loss_ws = dpr.Workspace(dev)

    def step(k, params, train=True, ev=None):
        """Step k of the trajectory: forward, Eq. (8) loss gradient, backward,
        Adam update (train), or the forward alone.  ev: a pair of events
        recorded on the stream before the plan and after the backward (or the
        forward alone), i.e. around everything but the Adam update."""
        if ev is not None:
            ev[0].record()
        plan = dpr.Plan([trainer.scene], [(0, c) for c in step_views[k]], params, workspace=wss[k % 2],
                        forward_now=True)
        plan.forward()
        if train:
            tgt = targets[k % len(targets)]
            dpr.loss_l2_tv(plan.images, [tgt[v] for v in range(V)], lam, grads=grads, workspace=loss_ws)
            plan.backward(grads, None, out=[trainer.grads])
        if ev is not None:
            ev[1].record()
        if train:
            trainer.update()
        return plan

    def run(params, train, warmup, steps, after=0, collect=None, reset=None):
        """From the step-0 cloud: `warmup` steps, then `steps` timed steps,
        then `after` more untimed.  At most two plans are alive, on the two
        workspaces; a plan is inspected and freed once the next plan's host
        sync has passed its work.  The warmup runs the same loop, inspection
        included (its first calls load torch's kernels), then `reset` clears
        what the inspection accumulated.  Returns (wall seconds of the timed
        steps, seconds of their forward + loss + backward from events)."""
        trainer.reset()
        prev = None
        evs = []

        def advance(k, inspect=True, timed=False):
            nonlocal prev
            ev = None
            if timed:
                ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                evs.append(ev)
            plan = step(k, params, train, ev)
            if prev is not None:
                if collect and inspect:
                    collect(prev)
                prev.free()
            prev = plan

        for k in range(warmup):
            advance(k)
        if prev is not None:
            if collect:
                collect(prev)
            prev.free()
            prev = None
        torch.cuda.synchronize()
        if reset:
            reset()
        n_alloc = torch.cuda.memory_stats().get("num_device_alloc", 0)
        host = []
        t0 = time.perf_counter()
        for k in range(warmup, warmup + steps):
            ts = time.perf_counter()
            advance(k, timed=True)
            host.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        dt_ev = sum(a.elapsed_time(b) for a, b in evs) / 1e3
        n_alloc = torch.cuda.memory_stats().get("num_device_alloc", 0) - n_alloc
        log(f"  timed loop: {steps} steps, host ms/step median {1e3 * float(np.median(host)):.2f} "
            f"max {1e3 * max(host):.2f} (step {int(np.argmax(host))}), device allocations {n_alloc}")
        if collect:
            collect(prev)
        prev.free()
        prev = None
        for k in range(warmup + steps, warmup + steps + after):
            advance(k, inspect=False)
        if prev is not None:
            prev.free()
        torch.cuda.synchronize()
        return dt, dt_ev

    pix_step = V * S * S
    base = dict(persistent=args.persistent, **variant)
    stage_ms = {s: 0.0 for s in dpr.STAGES}
    pair_acc = [0]
    item_acc = [0]

    def collect(p):
        for s_, v in p.stage_times().items():
            if v > 0:
                stage_ms[s_] += v
        pair_acc[0] += p.info().pairs
        item_acc[0] += p.info().items

    def reset():
        for s_ in stage_ms:
            stage_ms[s_] = 0.0
        pair_acc[0] = 0
        item_acc[0] = 0

    if args.profile:
        dt, _ = run(dpr.RenderParams(**base), True, W_, K)
        log(f"profile run: {W_} + {K} training steps, {dt / K * 1e3:.3f} ms/step")
        if args.copy_calibration_mib > 0:
            copy_calibration(torch, dev, args.copy_calibration_mib)
        print(json.dumps({"profile_run": True, "ms_per_step": round(dt / K * 1e3, 4)}), flush=True)
        return

    # parity at step 0: the GPU's outputs on the initial cloud (compared with
    # the oracle below, together with the CPU baseline)
    weights = parity_weights(V, S)
    trainer.reset()
    cores = len(os.sched_getaffinity(0))
    ms, kn = (15, 1) if paper else (0, 0)
    masks0 = None if args.no_cpu_baseline else near_tie_masks(scene_np, step_views[0], ms, kn, cores)
    weights0 = masked(weights, masks0)
    gpu0 = gpu_step_outputs(dpr, trainer.scene, step_views[0], weights0, variant)

    # stage breakdown: every stage timed.  Each timed stage records two HIP
    # events on the stream, which stretch the step, so this loop is short and
    # only names the dominant kernel and splits the step into stages.
    KB = min(K, 10)
    run(dpr.RenderParams(timing=True, **base), True, W_, KB, collect=collect, reset=reset)
    breakdown = {s_: v / KB for s_, v in stage_ms.items()}
    dom = max(breakdown, key=lambda s_: breakdown[s_])
    log("stage ms/step (every stage timed): " + ", ".join(f"{s_}={v:.3f}" for s_, v in breakdown.items()))

    # main metric: the training trajectory, forward + backward (stored T) +
    # Adam; HIP events around the dominant kernel only (its live launch
    # duration for the roofline); the trajectory runs on to its last step
    t_train, t_fb = run(dpr.RenderParams(timing=True, timing_stages=(dom,), **base), True, W_, K,
                        after=n_traj - W_ - K, collect=collect, reset=reset)
    pairs = pair_acc[0]
    items = item_acc[0]
    mpix_fb = pix_step * K / t_fb / 1e6
    mpix_train = pix_step * K / t_train / 1e6
    log(f"fwd+bwd: {t_fb / K * 1e3:.3f} ms/step, {mpix_fb:.1f} Mpix/s; with the Adam update (wall clock): "
        f"{t_train / K * 1e3:.3f} ms/step, {mpix_train:.1f} Mpix/s; {dom} {stage_ms[dom] / K:.3f} ms/launch")
    # parity at the last step: the trained cloud
    final_np = trainer.numpy_scene()
    k_last = n_traj - 1
    masks_last = None if args.no_cpu_baseline else near_tie_masks(final_np, step_views[k_last], ms, kn, cores)
    weights_last = masked(weights, masks_last)
    gpu_last = gpu_step_outputs(dpr, trainer.scene, step_views[k_last], weights_last, variant)

    # blended (pixel, splat) pairs of the timed steps, from the forward's
    # per-pixel counters, in a replay of the same trajectory (the forward is
    # bitwise deterministic; the replay's clouds differ from the timed run's
    # only by the order of the backward's float atomics)
    blend_acc = torch.zeros((), dtype=torch.int64, device=dev)
    overheads = {}

    def count(p):
        inf = p.info()
        nu = p.ws[inf.stats_off: inf.stats_off + 4 * inf.pixels].view(torch.int32)
        blend_acc.add_(nu.sum())
        rng = p.plan_ws[inf.range_off: inf.range_off + 4 * (inf.tiles + 1)].view(torch.int32).long()
        lens = (rng[1:] - rng[:-1]).float()
        nuf = nu.float()
        overheads.update({"pairs": int(inf.pairs), "n_u_mean": round(float(nuf.mean()), 1),
                          "n_u_p99": float(torch.quantile(nuf[:: max(1, nuf.numel() // 1000000)], 0.99)),
                          "n_u_max": int(nu.max()), "list_len_mean": round(float(lens.mean()), 1),
                          "list_len_max": int(lens.max())})

    run(dpr.RenderParams(stats=True, **base), True, W_, K, collect=count, reset=lambda: blend_acc.zero_())
    blends = int(blend_acc.item())

    mpix_f = mpix_r = None
    if not args.main_only:
        _, t_f = run(dpr.RenderParams(**base), False, W_, K)
        mpix_f = round(pix_step * K / t_f / 1e6, 2)
        _, t_r = run(dpr.RenderParams(bwd_mode="recompute", **base), True, W_, K)
        mpix_r = round(pix_step * K / t_r / 1e6, 2)
        log(f"fwd: {mpix_f} Mpix/s; fwd+bwd recompute: {mpix_r} Mpix/s")

    # roofline of the dominant kernel (per launch = per step); the committed PMC
    # traffic summary covers the default workload only
    comp = {"composite_fwd": FWD_OPS_PER_BLEND, "composite_bwd": BWD_OPS_PER_BLEND}
    traffic_wl = None if paper else "surface300k_4x800"
    prof = load_profile(traffic_wl)
    if dom in comp:
        ops = comp[dom] * blends / K
        t_launch = stage_ms[dom] / K / 1e3
        achieved = ops / t_launch / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_LANE_OPS / 1e12, 2),
                "unit": "Tlane-op/s", "frac": round(achieved * 1e12 / PEAK_LANE_OPS, 4),
                "traffic": load_traffic(dom, traffic_wl),
                "per_unit": f"{comp[dom]} lane-ops per blended (pixel, splat)",
                "units_per_launch": blends / K, "launch_ms": round(t_launch * 1e3, 4)}
    elif dom == "emit":
        # 4 B written per (tile, splat) pair; per depth-sorted item 32 B read
        # (its index 4, tile rectangle 8, exponent record 20)
        ops = (4.0 * pairs + EMIT_BYTES_PER_ITEM * items) / K
        t_launch = stage_ms[dom] / K / 1e3
        achieved = ops / t_launch / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": round(achieved * 1e9 / PEAK_HBM, 4), "traffic": load_traffic("tile_emit", traffic_wl),
                "per_unit": f"4 B per (tile, splat) pair + {EMIT_BYTES_PER_ITEM} B per item",
                "units_per_launch": {"pairs": pairs / K, "items": items / K}, "launch_ms": round(t_launch * 1e3, 4)}
    else:
        ops = None
        roof = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": None, "traffic": load_traffic(dom, traffic_wl)}
    # the same work over the committed rocprofv3 average duration of the kernel
    # (taken on the current kernel sources), beside the live HIP-event one
    pk = (prof or {}).get({"emit": "tile_emit"}.get(dom, dom))
    if ops is not None and pk:
        scale = 1e12 if roof["unit"] == "Tlane-op/s" else 1e9
        a = ops / (pk["avg_us"] * 1e-6) / scale
        roof["rocprof"] = {"launch_ms": round(pk["avg_us"] / 1e3, 4), "achieved": round(a, 3),
                           "frac": round(a / roof["peak"], 4), "valu_issue_pct": pk.get("valu_issue_pct"),
                           "salu_per_wave": pk.get("salu_per_wave")}

    # the loss kernel alone (Eq. 8, one launch for the step's views): HBM-bound,
    # 36 algorithmic bytes per pixel (render and target read, gradient written)
    tgt = targets[0]
    imgs = [torch.rand((S, S, 3), device=dev) for _ in range(V)]
    tl = [tgt[v] for v in range(V)]
    for _ in range(3):
        dpr.loss_l2_tv(imgs, tl, lam, grads=grads, workspace=loss_ws)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    nl = 50
    for _ in range(nl):
        dpr.loss_l2_tv(imgs, tl, lam, grads=grads, workspace=loss_ws)
    e1.record()
    torch.cuda.synchronize()
    t_loss = e0.elapsed_time(e1) / nl / 1e3
    loss_gbs = 36.0 * pix_step / t_loss / 1e9
    loss_kernel = {"bound": "hbm", "achieved": round(loss_gbs, 1), "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                   "frac": round(loss_gbs * 1e9 / PEAK_HBM, 4), "launch_ms": round(t_loss * 1e3, 4),
                   "per_unit": "36 B per pixel (render and target read, gradient written)",
                   "units_per_launch": pix_step, "lambda": lam}
    log(f"loss kernel: {t_loss * 1e3:.4f} ms for {V} x {S}x{S}, {loss_gbs:.0f} GB/s")
    del imgs

    if args.copy_calibration_mib > 0:
        copy_calibration(torch, dev, args.copy_calibration_mib)

    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle
        # the CPU baseline is the oracle on step 0 (all views, forward +
        # backward); the same results are step 0's parity check
        dt, renders, g = oracle_step(scene_np, step_views[0], weights0, ms, kn, cores)
        used = min(cores, oracle.max_threads())    # read before the one-thread run resets it
        p0 = parity_report(gpu0, renders, g, masks0)
        # the same work on one thread, for the first view only (a quarter of the step)
        dt1, _, _ = oracle_step(scene_np, step_views[0][:1], weights[:1], ms, kn, 1)
        cpu = {"value": pix_step / dt / 1e6, "unit": "Mpix/s", "cores": used, "kind": "oracle",
               "sample": f"step 0 of the trajectory: {V} views x {S}x{S}, forward + backward, FP64, {dt:.1f} s",
               "one_thread": {"value": S * S / dt1 / 1e6, "unit": "Mpix/s",
                              "sample": f"view 0 of step 0, forward + backward, FP64, {dt1:.1f} s"}}
        log(f"cpu baseline: {cpu}")
        _, renders, g = oracle_step(final_np, step_views[k_last], weights_last, ms, kn, cores)
        pl = parity_report(gpu_last, renders, g, masks_last)
        parity = {"step_0": p0, f"step_{k_last + 1}": pl, "pass": bool(p0["pass"] and pl["pass"]),
                  "what": f"all {V} views in full, image and T (max-abs <= {IMG_TOL}); gradients of xyz, SH and "
                          f"opacity in both backward modes (per element <= {GRAD_RTOL} max(|g*|, 1e-2 |g*|inf), "
                          f"rel-L2 <= {GRAD_L2}) of the linear loss sum(w I), w ~ N(0, 1) seeded; "
                          f"step {k_last + 1} is the cloud after {k_last + 1} Adam steps, on that step's views"
                          + ("; under the 15-splat cap, the pixels whose 15th splat rests on a predicate within "
                             "1e-4 of alpha_min (the oracle's near ties, near_tie_pixels) are left out: weight 0 on "
                             "both sides" if paper else "")}
        log(f"parity: step 0 {p0}; step {k_last + 1} {pl}")
        if not parity["pass"]:
            log("PARITY FAILED: the throughput figures of this run do not count")

    serving = None
    if args.serve_seconds > 0:
        del targets
        torch.cuda.empty_cache()
        serving = bench_serving(args.serve_seconds, args.serve_rate)
        if args.overload_rate > 0:
            serving["overload"] = bench_serving(args.overload_seconds, args.overload_rate)

    out = {
        "metric": METRIC if not paper else "Mpix/s fwd+bwd, paper-literal renderer (n = 15, normalised Eq. 5), "
                                           "L2 + 0.01 TV loss",
        "value": round(mpix_fb, 2), "unit": "Mpix/s", "n_gpus": 1, "steps": K,
        "warmup": W_, "ms_per_step": round(t_fb / K * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "300k points (30% on a 20-bump surface), SH degree 2, 4 views x 800x800 "
                               f"per step, training trajectory of {n_traj} Adam steps (xyz 8e-4, SH 3e-3, "
                               f"opacity logit 1e-2); steps {W_}..{W_ + K - 1} timed: forward + loss + backward "
                               "(stored T) on HIP events, the Adam update between steps outside; " +
                               ("n = 15 splats per pixel, normalised Eq. 5, L2 + 0.01 TV loss" if paper
                                else "L2 loss"),
                   "points": args.points, "views_per_step": V, "width": S, "height": S,
                   "trajectory_steps": n_traj, "persistent": bool(args.persistent)},
        "fwd_mpix_s": mpix_f, "fwd_bwd_mpix_s": round(mpix_fb, 2),
        "train_step": {"ms_per_step": round(t_train / K * 1e3, 4), "mpix_s": round(mpix_train, 2),
                       "what": "forward + loss + backward + Adam update, wall clock over the timed steps"},
        "fwd_bwd_recompute_mpix_s": mpix_r,
        "stage_ms_per_step": {s_: round(v, 4) for s_, v in breakdown.items()},
        "pairs_per_step": pairs / K, "blended_per_step": blends / K, "step_overheads": overheads,
        "parity": parity,
        "roofline": roof, "loss_kernel": loss_kernel, "cpu_baseline": cpu, "serving": serving,
    }
    print(json.dumps(out), flush=True)


HULL_OPS_PER_CANDIDATE = 90      # Philox4x32-10 and the box mapping, lane-ops
HULL_OPS_PER_TEST = 40           # one projection into a mask (two divisions) and the lookup, lane-ops


def bench_hull(args):
    """Visual-hull initialisation: 16 views of 800x800 of the 100k-point ball
    scene, masks where a render's transmittance is below 0.5 (untimed setup),
    rejection sampling of 2^24 candidates in [-1.2, 1.2]^3 per call; also the
    consistency predicate alone and the filter of the scene's own points."""
    import torch
    import workloads
    import paper_2205_14330_amd as dpr
    from paper_2205_14330_amd import hull
    scene_np, _, _, _ = workloads.ball100k_8x400()
    rng = workloads.seed_rng(7)
    cams = [workloads.random_sphere_camera(rng, 800, 800) for _ in range(16)]
    scene = dpr.SceneTensors.from_numpy(scene_np)
    plan = dpr.Plan([scene], [(0, c) for c in cams], dpr.RenderParams(bwd_mode="recompute"))
    plan.forward()
    masks = [(t < 0.5).to(torch.uint8).contiguous() for t in plan.trans]
    plan.free()
    lo, hi, n = [-1.2] * 3, [1.2] * 3, 1 << 24
    K, W = args.steps, args.warmup
    for k in range(W):
        hull.hull_sample(cams, masks, lo, hi, k, n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kept = 0
    for k in range(K):
        _, c = hull.hull_sample(cams, masks, lo, hi, W + k, n)
        kept += c
    torch.cuda.synchronize()
    t_call = (time.perf_counter() - t0) / K
    # the predicate alone on the candidates of one call, HIP events on the stream
    xyz = (torch.rand((n, 3), device="cuda", generator=torch.Generator(device="cuda").manual_seed(3)) * 2.4
           - 1.2).contiguous()
    for _ in range(W):
        hull.consistency(xyz, cams, masks)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(K):
        hull.consistency(xyz, cams, masks)
    e1.record()
    torch.cuda.synchronize()
    t_pred = e0.elapsed_time(e1) / K / 1e3
    # camera tests per candidate: item i is tested against camera c while it
    # is inside cameras 0 .. c-1 (survival fractions of camera prefixes)
    tests = 0.0
    for c in range(len(cams)):
        tests += 1.0 if c == 0 else float(hull.consistency(xyz, cams[:c], masks[:c]).float().mean())
    ops = n * (HULL_OPS_PER_CANDIDATE + HULL_OPS_PER_TEST * tests)
    achieved = ops / t_pred / 1e12
    # the filter of the scene's own points
    for _ in range(W):
        hull.consistency_filter(scene, cams, masks)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        out = hull.consistency_filter(scene, cams, masks)
    torch.cuda.synchronize()
    t_filt = (time.perf_counter() - t0) / K
    log(f"hull: sample {n} candidates {t_call * 1e3:.3f} ms/call ({n / t_call / 1e9:.2f} G/s, kept {kept / K:.0f}); "
        f"predicate {t_pred * 1e3:.3f} ms ({tests:.2f} tests per candidate); filter {scene.n} points "
        f"{t_filt * 1e3:.3f} ms, kept {out.n}")
    print(json.dumps({
        "metric": "visual-hull rejection sampling, candidates per second (16 masks of 800x800)",
        "value": round(n / t_call / 1e9, 3), "unit": "Gcandidates/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(t_call * 1e3, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "2^24 Philox candidates in [-1.2, 1.2]^3, 16 views of 800x800 of a 100k-point ball "
                               "scene, masks = rendered transmittance < 0.5", "candidates": n, "cameras": 16},
        "kept_per_call": kept / K, "camera_tests_per_candidate": round(tests, 3),
        "predicate_ms": round(t_pred * 1e3, 4), "filter_ms": round(t_filt * 1e3, 4), "filter_points": scene.n,
        "roofline": {"kernel": "hull_flags (+ upload, scan)", "bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(PEAK_LANE_OPS / 1e12, 2), "unit": "Tlane-op/s",
                     "frac": round(achieved * 1e12 / PEAK_LANE_OPS, 4), "traffic": None,
                     "per_unit": f"{HULL_OPS_PER_CANDIDATE} lane-ops per candidate + {HULL_OPS_PER_TEST} per camera "
                                 "test", "units_per_launch": n},
    }), flush=True)


NN_OPS_PER_PAIR = 10             # d2 (3 sub, 3 mul, 2 add) and the compare-select, lane-ops


def bench_warmstart(args):
    """Video warm start at the paper's frame size (45k points per frame, its
    Table 6 middle row): consecutive frames of the dynamic workload, the second
    jittered as the initial cloud; Chamfer distance of Eq. (9) with its
    gradient, top-k SH transfer, Adam step, and a 100-step warm start."""
    import torch
    import workloads
    from paper_2205_14330_amd import chamfer as cf
    n = 45000
    scenes, _, _ = workloads.dynamic30x200k_1024x768(frames=2, n=n)
    rng = workloads.seed_rng(8)
    s1 = torch.from_numpy(scenes[0].xyz).cuda()
    s2 = torch.from_numpy((scenes[1].xyz + 0.01 * rng.standard_normal(scenes[1].xyz.shape)).astype(np.float32)).cuda()
    sh1 = torch.from_numpy(scenes[0].sh).cuda()
    K, W = args.steps, args.warmup
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(W):
            fn()
        e0.record()
        for _ in range(K):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / K / 1e3

    t_cd = timed(lambda: cf.chamfer(s1, s2))
    t_topk = timed(lambda: cf.topk_sh(s1, sh1, s2, 4))
    p, g = s2.clone(), torch.randn_like(s2)
    m, v = torch.zeros_like(s2), torch.zeros_like(s2)
    t_adam = timed(lambda: cf.adam_step(p, g, m, v, 1, 1e-3))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pw, _ = cf.warm_start(s1, sh1, s2, steps=100, lr=1e-3, K=4)
    torch.cuda.synchronize()
    t_ws = time.perf_counter() - t0
    cd0 = float(cf.chamfer(s1, s2)["cd"].cpu()[0])
    cd1 = float(cf.chamfer(s1, pw)["cd"].cpu()[0])
    pairs = 2.0 * n * n
    achieved = pairs * NN_OPS_PER_PAIR / t_cd / 1e12
    log(f"warm start: chamfer fwd+bwd {t_cd * 1e3:.3f} ms ({pairs / t_cd / 1e9:.1f} G pairs/s), top-4 SH "
        f"{t_topk * 1e3:.3f} ms, adam {t_adam * 1e3:.4f} ms, 100-step warm start {t_ws * 1e3:.1f} ms "
        f"(CD {cd0:.3e} -> {cd1:.3e})")
    print(json.dumps({
        "metric": "Chamfer distance fwd+bwd (Eq. 9) between two 45k-point frames, pair distances per second",
        "value": round(pairs / t_cd / 1e9, 2), "unit": "Gpairs/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(t_cd * 1e3, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "frames 0 and 1 of the 30-frame sinusoidal workload at 45k points, frame 1 "
                               "jittered by N(0, 0.01^2)", "points": n},
        "topk_sh_ms": round(t_topk * 1e3, 4), "adam_ms": round(t_adam * 1e3, 4),
        "warm_start_100_steps_ms": round(t_ws * 1e3, 2), "cd_before": cd0, "cd_after": cd1,
        "roofline": {"kernel": "dpr_chamfer call (k_nn in both directions and its reductions)", "bound": "alu",
                     "achieved": round(achieved, 3),
                     "peak": round(PEAK_LANE_OPS / 1e12, 2), "unit": "Tlane-op/s",
                     "frac": round(achieved * 1e12 / PEAK_LANE_OPS, 4), "traffic": None,
                     "per_unit": f"{NN_OPS_PER_PAIR} lane-ops per pair distance", "units_per_launch": pairs},
    }), flush=True)


HYBRID_N, HYBRID_K, HYBRID_EPS = 128, 8, 0.01     # voxel grid, neighbours, spread threshold


def bench_hybrid(args):
    """Hybrid coarse-to-fine update (Sec. 3.3, Alg. 1) of the 300k-point
    training cloud: voxel reduction on a 128^3 grid, removal of points whose
    8-neighbour distance spread exceeds 0.01, one generated point per kept
    point.  Timed per call (each call waits once per stage for a count); also
    the voxel reduction and the neighbour search alone.  Parity: the points of
    the corner box x, y < -0.5, z < 0 (about 6.5k, at the cloud's density) bit
    for bit against the oracle, and the full cloud's voxel count against the
    oracle's voxel keys."""
    import torch
    import workloads
    import oracle
    import paper_2205_14330_amd as dpr
    from paper_2205_14330_amd import hybrid as hy
    scene_np, _, _ = workloads.surface300k_4x800(steps=1)
    scene = dpr.SceneTensors.from_numpy(scene_np)
    N, Kn, eps = HYBRID_N, HYBRID_K, HYBRID_EPS
    K, W = args.steps, args.warmup
    for _ in range(W):
        hy.hybrid_update(scene, N, Kn, eps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        out, counts = hy.hybrid_update(scene, N, Kn, eps)
    torch.cuda.synchronize()
    t_call = (time.perf_counter() - t0) / K
    for _ in range(W):
        hy.voxel_reduce(scene, N)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        red = hy.voxel_reduce(scene, N)
    torch.cuda.synchronize()
    t_red = (time.perf_counter() - t0) / K
    rxyz = red.xyz.contiguous()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(W):
        hy.knn(rxyz, Kn)
    e0.record()
    for _ in range(K):
        hy.knn(rxyz, Kn)
    e1.record()
    torch.cuda.synchronize()
    t_knn = e0.elapsed_time(e1) / K / 1e3
    # parity: the full cloud's voxels, and a subset bit for bit
    n_vox = len(np.unique(oracle.voxel_keys(scene_np.xyz, N)))
    x = scene_np.xyz
    sub = np.flatnonzero((x[:, 0] < -0.5) & (x[:, 1] < -0.5) & (x[:, 2] < 0.0))
    c = oracle.Cloud(scene_np.xyz[sub], scene_np.sh[sub], scene_np.opacity[sub], scene_np.radius[sub])
    got, gcounts = hy.hybrid_update(dpr.SceneTensors.from_numpy(c), N, Kn, eps)
    t0 = time.perf_counter()
    ref_red, ref_keep, ref = oracle.hybrid_update(c, N, Kn, eps)
    t_cpu = time.perf_counter() - t0
    mism = 0
    for g, r in zip((got.xyz, got.sh, got.opacity, got.radius), (ref.xyz, ref.sh, ref.opacity, ref.radius)):
        g = g.cpu().numpy()
        r32 = np.asarray(r).astype(np.float32)
        mism += int(g.size) if g.shape != r32.shape else int((g != r32).sum())
    ok = mism == 0 and counts["voxels"] == n_vox and gcounts["voxels"] == ref_red.n
    n = scene.n
    k3 = scene_np.sh.shape[1] * 3
    bytes_pt = 4 * (3 + k3 + 2)            # one point's parameters
    algo = n * bytes_pt + counts["points"] * bytes_pt
    achieved = algo / t_call
    log(f"hybrid update: {n} points -> {counts['voxels']} voxels, {counts['kept']} kept, {counts['points']} out; "
        f"{t_call * 1e3:.3f} ms/call ({n / t_call / 1e6:.1f} Mpoints/s); voxel reduce {t_red * 1e3:.3f} ms, "
        f"knn {t_knn * 1e3:.3f} ms; parity {'pass' if ok else 'FAIL'} ({mism} mismatches); "
        f"oracle {len(sub)} pts {t_cpu:.2f} s")
    print(json.dumps({
        "metric": "hybrid coarse-to-fine update (Alg. 1) of the 300k-point training cloud, input points per second",
        "value": round(n / t_call / 1e6, 3), "unit": "Mpoints/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(t_call * 1e3, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (f64 sums)", "data": "synthetic",
        "config": {"workload": f"300k-point surface cloud, SH degree 2; voxel grid {N}^3, K = {Kn}, eps = {eps}",
                   "points": n, "N": N, "K": Kn, "eps": eps},
        "counts": counts, "voxel_reduce_ms": round(t_red * 1e3, 4), "knn_ms": round(t_knn * 1e3, 4),
        "parity": {"pass": bool(ok), "subset_points": int(len(sub)), "mismatched_values": mism,
                   "full_voxels": counts["voxels"], "oracle_full_voxels": n_vox,
                   "what": "the corner-box subset: every output value bit for bit against the oracle; "
                           "full cloud: voxel count against the oracle's voxel keys"},
        "roofline": {"kernel": "dpr_hybrid_update call", "bound": "hbm", "achieved": round(achieved / 1e9, 2),
                     "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": round(achieved / PEAK_HBM, 5),
                     "traffic": None,
                     "per_unit": f"{bytes_pt} B read per input point + {bytes_pt} B written per output point "
                                 "(the parameters once each way)", "units_per_launch": n},
        "cpu_baseline": {"value": round(len(sub) / t_cpu / 1e6, 5), "unit": "Mpoints/s",
                         "cores": 1, "kind": "oracle",
                         "sample": f"the {len(sub)}-point corner-box subset (brute-force neighbours)"},
    }), flush=True)


def bench_dynamic(args):
    """30 frames x 200k points, one 1024x768 view per frame, all frames in one
    plan: forward + backward per step."""
    import torch
    import workloads
    import paper_2205_14330_amd as dpr
    scenes_np, cams, trng = workloads.dynamic30x200k_1024x768()
    scenes = [dpr.SceneTensors.from_numpy(s) for s in scenes_np]
    F = len(cams)
    views = [(t, cams[t]) for t in range(F)]
    gen = torch.Generator(device="cuda").manual_seed(4)
    targets = [torch.rand((c.height, c.width, 3), device="cuda", generator=gen) for c in cams]
    out = {}
    wss = [dpr.Workspace(), dpr.Workspace()]
    for persistent in (False, True):
        def step(k, params):
            plan = dpr.Plan(scenes, views, params, workspace=wss[k % 2])
            plan.forward()
            plan.backward([(2.0 * (plan.images[t] - targets[t])).contiguous() for t in range(F)], None)
            return plan
        params = dpr.RenderParams(timing=True, persistent=persistent)
        st = {k: 0.0 for k in dpr.STAGES}

        def collect(p):
            for k, v in p.stage_times().items():
                st[k] += max(v, 0.0) / args.steps
            p.free()

        prev = None
        for k in range(args.warmup):
            plan = step(k, params)
            if prev is not None:
                prev.free()
            prev = plan
        torch.cuda.synchronize()
        if prev is not None:
            prev.free()
        t0 = time.perf_counter()
        prev = None
        for k in range(args.steps):
            plan = step(k, params)
            if prev is not None:
                collect(prev)       # the new plan's host sync has passed the previous plan's work
            prev = plan
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        collect(prev)
        px = sum(c.pixels for c in cams)
        out["persistent" if persistent else "grid"] = {
            "ms_per_step": round(dt * 1e3, 3), "mpix_s": round(px / dt / 1e6, 1),
            "stage_ms": {k: round(v, 3) for k, v in st.items() if v > 0}}
        log(f"dynamic persistent={persistent}: {dt * 1e3:.2f} ms/step")
    best = min(out.values(), key=lambda d: d["ms_per_step"])
    print(json.dumps({"metric": "Mpix/s fwd+bwd, 30 frames x 200k points, 1024x768, one launch per stage",
                      "value": best["mpix_s"], "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "ms_per_step": best["ms_per_step"], "higher_is_better": True,
                      "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "30 frames x 200k points (sinusoidal motion), SH degree 2, "
                                             "one 1024x768 orbit view per frame, forward + backward"},
                      "modes": out}), flush=True)


def bench_serving(seconds: float, rate: float) -> dict:
    """16 resident scenes, Poisson requests of mixed resolution: continuous
    batching on 2 streams vs one view per launch on one stream, same trace."""
    import torch
    import workloads
    import paper_2205_14330_amd as dpr
    from paper_2205_14330_amd.serving import Request, RendererExecutor, Server, latency_stats
    scenes = [dpr.SceneTensors.from_numpy(s) for s in workloads.serving_scenes()]
    trace = workloads.serving_trace(n_scenes=len(scenes), rate=rate, duration=seconds)
    budget = 16 << 30
    res = {"trace": {"seconds": seconds, "rate_per_s": rate, "requests": len(trace),
                     "offered_mpix_s": round(sum(r.camera.pixels for r in trace) / seconds / 1e6, 1),
                     "points": [s.n for s in scenes]}, "hbm_budget_bytes": budget}
    # warm up both paths
    for slots, mv in ((2, 32), (1, 1)):
        srv = Server(RendererExecutor(scenes, n_slots=slots), hbm_budget=budget, max_views=mv)
        srv.run_trace(trace[:20], lambda i, tr: Request(i, tr.scene, tr.camera, 0.0))
    torch.cuda.synchronize()
    for name, slots, mv in (("continuous_batching", 2, 32), ("one_view_per_launch", 1, 1)):
        log(f"serving {name}: {len(trace)} requests over {seconds:.0f} s at {rate:.0f} req/s")
        srv = Server(RendererExecutor(scenes, n_slots=slots), hbm_budget=budget, max_views=mv)
        t0 = time.perf_counter()
        done = srv.run_trace(trace, lambda i, tr: Request(i, tr.scene, tr.camera, 0.0))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = latency_stats(done, wall)
        st["mean_batch"] = round(float(np.mean(srv.batches)), 2)
        st["max_batch"] = int(max(srv.batches))
        b = np.asarray(srv.batches)
        st["batch_views"] = {"p50": float(np.percentile(b, 50)), "p90": float(np.percentile(b, 90)),
                             "p99": float(np.percentile(b, 99)), "launches": int(b.size),
                             "share_of_requests_in_batches_of_2_or_more": round(float(b[b >= 2].sum() / b.sum()), 3)}
        st["peak_hbm_bytes"] = int(srv.peak_in_use)
        res[name] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
        log(f"serving {name}: p50 {st['p50_ms']:.2f} ms, p99 {st['p99_ms']:.2f} ms, "
            f"{st['served_mpix_s']:.1f} Mpix/s, mean batch {st['mean_batch']}")
    return res


if __name__ == "__main__":
    main()
