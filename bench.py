"""Throughput of the splat renderer on one MI355X.

Default workload: 300k points (30% on a bumpy surface), SH degree 2, four
800x800 views per step, FP32.  One step = the whole hot path over one batch:
projection + SH colour, depth sort, tile binning, compositing (forward), then
the L2-loss gradient and the compositing + per-point backward.  Inputs (scene,
cameras, target images) are resident in HBM before timing starts.

Prints ONE JSON line:  metric/value = forward+backward Mpix/s (stored-T mode),
plus forward-only and recompute-T rates, the roofline of the dominant kernel
(HIP events on the library's stream around that kernel only, in the timed
loop; algorithmic work from the per-pixel blended-splat counts of the same
steps), a per-stage breakdown from a short loop with every stage timed, and
the FP64 CPU oracle timed on one step's views.
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC summary
    profiles/traffic_<workload>.json, if it was taken on the current kernel
    sources; else None."""
    from paper_2205_14330_amd.profiling import kernel_source_hash
    if workload is None:
        return None
    p = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return None
    e = d.get("kernels", {}).get(kernel)
    if not e or d.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(scene, cams, targets_fn, max_splats=0, kernel_norm=0, lam=0.0):
    """FP64 oracle on one full step (all views, forward, Eq. 8 loss, backward)."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    op = oracle.Params(max_splats=max_splats, kernel_norm=kernel_norm)
    t0 = time.perf_counter()
    pix = 0
    for v, cam in enumerate(cams):
        r = oracle.render(scene, cam, op, threads=cores)
        _, gI = oracle.loss_l2_tv(r.image, targets_fn(v), lam)
        oracle.backward(scene, [cam], [gI], None, params=op, threads=cores)
        pix += cam.pixels
    dt = time.perf_counter() - t0
    used = min(cores, oracle.max_threads())    # read before the one-thread run resets it
    # the same work on one thread, for the first view only (a quarter of the step)
    t1 = time.perf_counter()
    r = oracle.render(scene, cams[0], op, threads=1)
    _, gI = oracle.loss_l2_tv(r.image, targets_fn(0), lam)
    oracle.backward(scene, [cams[0]], [gI], None, params=op, threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": pix / dt / 1e6, "unit": "Mpix/s", "cores": used, "kind": "oracle",
            "sample": f"one full step: {len(cams)} views x {cams[0].width}x{cams[0].height}, fwd+bwd, "
                      f"FP64, {dt:.1f} s",
            "one_thread": {"value": cams[0].pixels / dt1 / 1e6, "unit": "Mpix/s",
                           "sample": f"view 0 of the step, fwd+bwd, FP64, {dt1:.1f} s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--points", type=int, default=300_000)
    ap.add_argument("--size", type=int, default=800)
    ap.add_argument("--views", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--persistent", action="store_true")
    ap.add_argument("--main-only", action="store_true",
                    help="time only the forward + backward metric (skip the forward-only and recompute legs)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after timing, run one device copy of this many MiB (reference for HBM counters)")
    ap.add_argument("--workload", choices=["train", "paper", "dynamic", "serve", "hull", "warmstart"],
                    default="train",
                    help="train: the default step; paper: the same step with the paper-literal renderer "
                         "(n = 15 splats per pixel, normalised Eq. 5) and the L2 + 0.01 TV loss")
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="length of the serving trace (train: short leg in the same JSON line; 0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
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
    if args.workload == "serve":
        out = {"metric": "served p50/p99 latency and Mpix/s (16 resident scenes, Poisson requests)",
               "n_gpus": 1, "dtype": "f32", "data": "synthetic"}
        out.update(bench_serving(args.serve_seconds if args.serve_seconds > 0 else 60.0, args.serve_rate))
        print(json.dumps(out), flush=True)
        return
    V, S = args.views, args.size
    scene_np, cams, gt_np = workloads.surface300k_4x800(n=args.points, size=S, views_per_step=V, steps=100)
    scene = dpr.SceneTensors.from_numpy(scene_np, dev)
    gt = dpr.SceneTensors.from_numpy(gt_np, dev)
    nsteps = args.warmup + args.steps
    step_views = [cams[(k % 100) * V:(k % 100) * V + V] for k in range(nsteps)]

    # targets: renders of the ground-truth scene from each step's views (untimed)
    targets = []
    for k in range(min(nsteps, 100)):
        p = dpr.Plan([gt], [(0, c) for c in step_views[k]], dpr.RenderParams(bwd_mode="recompute"))
        p.forward()
        targets.append(torch.stack(p.images).clone())
        p.free()
    torch.cuda.synchronize()
    log(f"setup done: {args.points} points, {V} x {S}x{S}, {nsteps} steps")

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

    def step(k, params, backward=True):
        plan = dpr.Plan([scene], [(0, c) for c in step_views[k]], params, workspace=wss[k % 2])
        plan.forward()
        if backward:
            tgt = targets[k % len(targets)]
            dpr.loss_l2_tv(plan.images, [tgt[v] for v in range(V)], lam, grads=grads, workspace=loss_ws)
            plan.backward(grads, None)
        return plan

    def timed(params, backward, steps, warmup, collect=None, reset=None):
        """Times `steps` steps after `warmup`.  At most two plans are alive, on
        the two workspaces; a plan is inspected and freed once the next plan's
        host sync has passed its work.  The warmup runs the same loop, inspection
        included (its first calls load torch's kernels), then `reset` clears
        what the inspection accumulated."""
        prev = None
        for k in range(warmup):
            plan = step(k, params, backward)
            if prev is not None:
                if collect:
                    collect(prev)
                prev.free()
            prev = plan
        if prev is not None:
            if collect:
                collect(prev)
            prev.free()
        torch.cuda.synchronize()
        if reset:
            reset()
        n_alloc = torch.cuda.memory_stats().get("num_device_alloc", 0)
        host = []
        t0 = time.perf_counter()
        prev = None
        for k in range(steps):
            ts = time.perf_counter()
            plan = step(warmup + k, params, backward)
            if prev is not None:
                if collect:
                    collect(prev)
                prev.free()
            prev = plan
            host.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        n_alloc = torch.cuda.memory_stats().get("num_device_alloc", 0) - n_alloc
        log(f"  timed loop: {steps} steps, host ms/step median {1e3 * float(np.median(host)):.2f} "
            f"max {1e3 * max(host):.2f} (step {int(np.argmax(host))}), device allocations {n_alloc}")
        if collect:
            collect(prev)
        prev.free()
        return dt

    pix_step = V * S * S
    base = dict(persistent=args.persistent, **variant)
    stage_ms = {s: 0.0 for s in dpr.STAGES}
    blend_acc = torch.zeros((), dtype=torch.int64, device=dev)
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
        blend_acc.zero_()
        pair_acc[0] = 0
        item_acc[0] = 0

    # stage breakdown: every stage timed.  Each timed stage records two HIP
    # events on the stream, which stretch the step, so this loop is short and
    # only names the dominant kernel and splits the step into stages.
    KB = min(args.steps, 10)
    timed(dpr.RenderParams(timing=True, **base), True, KB, args.warmup, collect, reset)
    breakdown = {s_: v / KB for s_, v in stage_ms.items()}
    dom = max(breakdown, key=lambda s_: breakdown[s_])
    log("stage ms/step (every stage timed): " + ", ".join(f"{s_}={v:.3f}" for s_, v in breakdown.items()))

    # main metric: forward + backward (stored T), HIP events around the dominant
    # kernel only (its live launch duration for the roofline)
    t_fb = timed(dpr.RenderParams(timing=True, timing_stages=(dom,), **base), True, args.steps,
                 args.warmup, collect, reset)
    pairs = pair_acc[0]
    items = item_acc[0]
    K = args.steps
    # blended (pixel, splat) pairs of the timed steps, from the forward's
    # per-pixel counters in a pass of their own over the same views (the
    # forward is bitwise deterministic, so the counts are those of the timed
    # launches; counting inside the timed loop would add a reduction per step)
    overheads = None
    for k in range(args.warmup, args.warmup + K):
        p = dpr.Plan([scene], [(0, c) for c in step_views[k]], dpr.RenderParams(stats=True, **base),
                     workspace=wss[k % 2])
        p.forward()
        inf = p.info()
        nu = p.ws[inf.stats_off: inf.stats_off + 4 * inf.pixels].view(torch.int32)
        blend_acc.add_(nu.sum())
        if k == args.warmup + K - 1:
            # the overheads of the last step: blended splats per pixel n(u), tile list lengths
            rng = p.plan_ws[inf.range_off: inf.range_off + 4 * (inf.tiles + 1)].view(torch.int32).long()
            lens = (rng[1:] - rng[:-1]).float()
            nuf = nu.float()
            overheads = {"pairs": int(inf.pairs), "n_u_mean": round(float(nuf.mean()), 1),
                         "n_u_p99": float(torch.quantile(nuf[:: max(1, nuf.numel() // 1000000)], 0.99)),
                         "n_u_max": int(nu.max()), "list_len_mean": round(float(lens.mean()), 1),
                         "list_len_max": int(lens.max())}
        p.free()
    blends = int(blend_acc.item())
    mpix_fb = pix_step * K / t_fb / 1e6
    log(f"fwd+bwd: {t_fb / K * 1e3:.3f} ms/step, {mpix_fb:.1f} Mpix/s; {dom} {stage_ms[dom] / K:.3f} ms/launch")

    mpix_f = mpix_r = None
    if not args.main_only:
        t_f = timed(dpr.RenderParams(**base), False, K, args.warmup)
        mpix_f = round(pix_step * K / t_f / 1e6, 2)
        t_r = timed(dpr.RenderParams(bwd_mode="recompute", **base), True, K, args.warmup)
        mpix_r = round(pix_step * K / t_r / 1e6, 2)
        log(f"fwd: {mpix_f} Mpix/s; fwd+bwd recompute: {mpix_r} Mpix/s")

    # roofline of the dominant kernel (per launch = per step); the committed PMC
    # traffic summary covers the default workload only
    comp = {"composite_fwd": FWD_OPS_PER_BLEND, "composite_bwd": BWD_OPS_PER_BLEND}
    traffic_wl = None if paper else "surface300k_4x800"
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
        nbytes = (4.0 * pairs + EMIT_BYTES_PER_ITEM * items) / K
        t_launch = stage_ms[dom] / K / 1e3
        achieved = nbytes / t_launch / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": round(achieved * 1e9 / PEAK_HBM, 4), "traffic": load_traffic("tile_emit", traffic_wl),
                "per_unit": f"4 B per (tile, splat) pair + {EMIT_BYTES_PER_ITEM} B per item",
                "units_per_launch": {"pairs": pairs / K, "items": items / K}, "launch_ms": round(t_launch * 1e3, 4)}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": None, "traffic": load_traffic(dom, traffic_wl)}

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
        src = torch.empty(args.copy_calibration_mib * (1 << 20) // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration_mib} MiB read + written")
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        t_np = targets[0].cpu().numpy().astype(np.float64)
        cpu = cpu_baseline(scene_np, step_views[0], lambda v: t_np[v], 15 if paper else 0, int(paper), lam)
        log(f"cpu baseline: {cpu}")

    serving = None
    if args.serve_seconds > 0:
        del targets
        torch.cuda.empty_cache()
        serving = bench_serving(args.serve_seconds, args.serve_rate)

    out = {
        "metric": METRIC if not paper else "Mpix/s fwd+bwd, paper-literal renderer (n = 15, normalised Eq. 5), "
                                           "L2 + 0.01 TV loss",
        "value": round(mpix_fb, 2), "unit": "Mpix/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(t_fb / K * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "300k points (30% on a 20-bump surface), SH degree 2, 4 views x 800x800 "
                               "per step, forward + backward (stored T), " +
                               ("n = 15 splats per pixel, normalised Eq. 5, L2 + 0.01 TV loss" if paper
                                else "L2 loss"),
                   "points": args.points, "views_per_step": V, "width": S, "height": S,
                   "persistent": bool(args.persistent)},
        "fwd_mpix_s": mpix_f, "fwd_bwd_mpix_s": round(mpix_fb, 2),
        "fwd_bwd_recompute_mpix_s": mpix_r,
        "stage_ms_per_step": {s_: round(v, 4) for s_, v in breakdown.items()},
        "pairs_per_step": pairs / K, "blended_per_step": blends / K, "step_overheads": overheads,
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
        srv = Server(RendererExecutor(scenes, n_slots=slots), hbm_budget=budget, max_views=mv)
        t0 = time.perf_counter()
        done = srv.run_trace(trace, lambda i, tr: Request(i, tr.scene, tr.camera, 0.0))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = latency_stats(done, wall)
        st["mean_batch"] = round(float(np.mean(srv.batches)), 2)
        st["max_batch"] = int(max(srv.batches))
        st["peak_hbm_bytes"] = int(srv.peak_in_use)
        res[name] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
        log(f"serving {name}: p50 {st['p50_ms']:.2f} ms, p99 {st['p99_ms']:.2f} ms, "
            f"{st['served_mpix_s']:.1f} Mpix/s, mean batch {st['mean_batch']}")
    return res


if __name__ == "__main__":
    main()
