"""Benchmark of the MI355X shell fill (Guidefill, arXiv 1611.05319).

A step is one complete fill (every shell, tracked front, out of place) of the
1920x1080 RGB binary32 synthetic frame with eps = 3, mu = 50 (six silhouette
bands 5-20 px wide, spline / structure-tensor guide).  Inputs are resident on
the device before the timed region.  The JSON line reports Mpix filled per
second, the fill call's algorithmic HBM bytes against the 8 TB/s peak, the
FP64 CPU oracle on the host cores, and the side comparisons named by the
metric: tracked vs untracked, one batched launch of 64 fp16 frames vs 64
single-frame launches, forward vs forward + backward on 16 x 512 x 512, and
the 3840x2160 deep front (eps = 5, about 100 shells).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --profile          (fill steps only, for rocprofv3 runs)
    python bench.py --profile-batched  (64-frame batch fill steps only)
    python bench.py --profile-grad     (16 x 512^2 forward + backward steps only)
    python bench.py --profile-deep     (3840x2160 deep-front fill steps only)
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synthetic as syn  # noqa: E402

HBM_PEAK_GBS = 8000.0
# what the fill computes in: binary32 storage; FP64 ghost geometry, weights
# and weighted sums; FP32 bilinear interpolation of each ghost value
DTYPE = "f64+f32 (binary32 storage; FP64 geometry, weights and sums; FP32 bilinear values)"
METRIC = "Mpix filled/s + HBM GB/s fraction @1080p eps=3; batched vs plain; fwd+bwd ms"


def algorithmic_bytes(B, H, W, C, elem, n_hole, inplace=False):
    """Bytes the fill must move: image in and out, labels in, shell map out,
    guide on hole pixels (8 B each)."""
    px = B * H * W
    if inplace:
        return px * (1 + 4) + n_hole * (8 + 2 * C * elem)
    return px * (C * elem + 1 + C * elem + 4) + n_hole * 8


# the headers that hold the device code of the fill and adjoint kernels
FILL_KERNEL_SOURCES = ("device_common.h", "fill_core.h", "global_engine.h", "tile_engine.h")


def kernel_source_digest():
    """SHA-256 over the fill and adjoint kernels' device sources (in the order
    above): a recorded HBM traffic figure is valid only for the kernel code it
    was measured on (the launch shape is recorded beside it)."""
    import hashlib

    d = os.path.join(ROOT, "paper_1611_05319_amd", "csrc")
    h = hashlib.sha256()
    for name in FILL_KERNEL_SOURCES:
        h.update(name.encode())
        with open(os.path.join(d, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def launch_key(p, H, W, C):
    """Canonical text of the launch shape the library resolves for these
    parameters (automatic fields filled in), as recorded beside a counter
    summary."""
    import paper_1611_05319_amd as gf

    if p.engine == gf.ENGINE_TILED:
        tw, th, S, _, _, G = gf.tile_geometry(H, W, C, params=p)
        return (f"engine=0 tile={tw}x{th} pass_shells={S} group={G} "
                f"tile_threads={p.tile_threads or 768} blocks_per_cu={p.blocks_per_cu}")
    return f"engine=1 group={p.group} blocks_per_cu={p.blocks_per_cu}"


def recorded_traffic(params, H, W, C, summary="traffic_c2_1080p.md"):
    """HBM bytes per launch of a kernel from its committed counter summary
    under profiles/ (FETCH_SIZE + WRITE_SIZE scaled by a plain copy), or None
    when it is missing, was taken on other kernel sources or another launch
    shape."""
    path = os.path.join(ROOT, "profiles", summary)
    try:
        with open(path) as f:
            rec = dict(line.split(":", 1) for line in f.read().splitlines()
                       if line.startswith(("source_sha256:", "launch:", "traffic_bytes_per_launch:")))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256", "").strip() != kernel_source_digest():
        return None
    if rec.get("launch", "").strip() != launch_key(params, H, W, C):
        return None
    try:
        return int(float(rec["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def cpu_baseline(w, budget_s=10.0):
    """The FP64 oracle, as it stands, on the host cores, on repeated fills of
    the same frame until ~budget_s of CPU time."""
    import oracle

    threads = min(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), os.cpu_count() or 1)
    img, lab, g = w.image[0], w.label[0], w.guide[0]
    r = oracle.fill(img, lab, g, eps=w.eps, mu=w.mu, threads=threads)  # warm (build, page-in)
    n = r.n_filled
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.fill(img, lab, g, eps=w.eps, mu=w.mu, threads=threads)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 1000:
            break
    return {"value": round(n * reps / el / 1e6, 4), "unit": "Mpix filled/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{reps} complete FP64 fills of the 1920x1080 frame ({n} hole px each), "
                      f"{el:.1f} s"}


def launch_fields(p):
    """The autotuned launch shape (engine 0: tiled, 1: global front)."""
    return {"engine": "tiled" if p.engine == 0 else "front", "group": p.group,
            "blocks_per_cu": p.blocks_per_cu, "tile": [p.tile_w, p.tile_h],
            "pass_shells": p.pass_shells}


def time_steps(fn, steps, warmup, torch):
    """Warm up, then time exactly `steps` calls back to back: wall clock
    between two device synchronisations, and one pair of HIP events on the
    current stream around the same calls (their time per call: the average
    launch duration plus the dispatch gap between launches, ~1 us; an event
    pair around every call would add ~8 us per call to the region)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / steps
    return wall_ms, a.elapsed_time(b) / steps


def deep_front(w3, torch, gf, autotune, dev, args):
    """The 4K deep-front fill (about 100 shells): Mpix filled/s, us per shell
    and the algorithmic-byte roofline of the autotuned launch."""
    B, H, W, C = w3.image.shape
    i3 = torch.from_numpy(w3.image).to(dev)
    l3 = torch.from_numpy(w3.label).to(dev)
    g3 = torch.from_numpy(w3.guide).to(dev)
    p3 = autotune.tune(i3, l3, g3, gf.Params(eps=w3.eps, mu=w3.mu), reps=3)
    plan = gf.FillPlan(i3, l3, g3, p3)
    plan.run()
    torch.cuda.synchronize()
    st = gf.stats_fields(plan.stats)
    steps = max(5, args.steps // 4)
    wall, ev = time_steps(plan.run, steps, 2, torch)
    nbytes = algorithmic_bytes(B, H, W, C, 4, st["hole"])
    achieved = nbytes / (ev * 1e-3) / 1e9
    return {"workload": "3840x2160 RGB binary32, 200-px wiggly band + 20 discs, eps=5, mu=100",
            "hole_px": st["hole"], "filled_px": st["filled"], "shells": st["K"],
            "launch": launch_fields(p3), "ms_per_step": round(wall, 4),
            "mpix_filled_per_s": round(st["filled"] / (wall * 1e-3) / 1e6, 2),
            "us_per_shell": round(ev * 1e3 / max(st["K"], 1), 3),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                         "algorithmic_bytes": nbytes, "event_ms_per_launch": round(ev, 5)}}


def guidance_extras(w2, torch, gf, dev, args):
    """The two guide constructions on the 1080p frame: the spline guide
    field (Sec. 3.2) from six random Bezier splines sampled every 2 px, and
    the coherence-transport comparison fill (guide re-estimated from the
    modified structure tensor before every shell, lattice ball)."""
    B, H, W, C = w2.image.shape
    lab = torch.from_numpy(w2.label).to(dev)
    rng = np.random.default_rng(12)
    seg, off = syn.pack_segments([syn.spline_segments(rng, H, W, n_splines=6, spacing=2.0)])
    seg_d = torch.from_numpy(seg).to(dev)
    off_d = torch.from_numpy(off).to(dev)
    g_out = torch.empty((B, H, W, 2), dtype=torch.float32, device=dev)

    def run_guide():
        gf.guide_field(lab, seg_d, off_d, out=g_out, check_offsets=False)

    n_hole = int((w2.label == 1).sum())
    wall_g, ev_g = time_steps(run_guide, max(5, args.steps // 5), 2, torch)
    img = torch.from_numpy(w2.image).to(dev)
    out = torch.empty_like(img)
    ws = gf.Workspace()
    pc = gf.Params(eps=w2.eps, mu=w2.mu, ghost=False)
    r = gf.fill_coherence(img, lab, pc, out=out, workspace=ws)
    st = gf.stats_fields(r.stats)

    def run_ct():
        gf.fill_coherence(img, lab, pc, out=out, workspace=ws, want_guide=False)

    wall_c, _ = time_steps(run_ct, max(3, args.steps // 10), 1, torch)
    return {
        "guide_field": {"workload": "1920x1080 silhouette holes, 6 random Bezier splines as "
                                    f"{seg.shape[0]} segments, eta=3, cutoff 9 px",
                        "ms": round(ev_g, 4), "hole_px": n_hole, "segments": int(seg.shape[0]),
                        "gpairs_per_s": round(n_hole * seg.shape[0] / (ev_g * 1e-3) / 1e9, 2)},
        "coherence": {"workload": "1920x1080 RGB binary32, 6 silhouette bands, guide from the "
                                  "modified structure tensor (sigma=2, rho=4, Lambda=1e-5) before "
                                  "every shell, lattice ball, eps=3, mu=50",
                      "ms_per_fill": round(wall_c, 4), "shells": st["K"], "filled_px": st["filled"],
                      "us_per_shell": round(wall_c * 1e3 / max(st["K"], 1), 2),
                      "mpix_filled_per_s": round(st["filled"] / (wall_c * 1e-3) / 1e6, 2)},
    }


def studies(torch, gf, dev, args):
    """The paper's synthetic studies on the device: signal degradation of the
    73-degree band at its four resolutions (L^1 / L^2 error over the hole and
    at the cross-sections y = 0.25 and 0, observed rates), and a camera-pan
    video batch (16 frames 1920x1080 binary16, one launch)."""
    res = []
    for W in (200, 400, 4000, 8000):
        prob = syn.degradation_problem(W)
        i = torch.from_numpy(prob.image[None]).to(dev)
        l = torch.from_numpy(prob.label[None]).to(dev)
        g = torch.from_numpy(prob.guide[None]).to(dev)
        plan = gf.FillPlan(i, l, g, gf.Params(eps=3.0, mu=50.0))
        plan.run()
        torch.cuda.synchronize()
        st = gf.stats_fields(plan.stats)
        wall, _ = time_steps(plan.run, 3, 1, torch)
        u = plan.out[0, ..., 0].double().cpu().numpy()
        e = np.abs(u - prob.exact)
        hole = prob.label == 1
        row = {"px": f"{W}x{W // 2}", "ms": round(wall, 3), "shells": st["K"],
               "L1": float(prob.h * prob.h * e[hole].sum()),
               "L2": float(np.sqrt(prob.h * prob.h * (e[hole] ** 2).sum()))}
        for yc in (0.25, 0.0):
            j = int(np.argmin(np.abs(prob.y - yc)))
            sel = hole[j]
            row[f"L1_y{yc}"] = float(prob.h * e[j, sel].sum())
        res.append(row)
        del i, l, g, plan
    for p in ("L1", "L2"):
        a, b = res[0], res[-1]
        w0, w1 = 200, 8000
        for r in res:
            r[p] = round(r[p], 6)
        res_rate = np.log(a[p] / b[p]) / np.log(w1 / w0)
        res[-1][f"rate_{p}_200_to_8000"] = round(float(res_rate), 3)
    wl, _ = syn.pan_video(seed=6, B=16, H=1080, W=1920, step=(3, 1))
    i = torch.from_numpy(wl.image).to(dev)
    l = torch.from_numpy(wl.label).to(dev)
    g = torch.from_numpy(wl.guide).to(dev)
    plan = gf.FillPlan(i, l, g, gf.Params(eps=wl.eps, mu=wl.mu, engine=gf.ENGINE_FRONT))
    plan.run()
    torch.cuda.synchronize()
    st = gf.stats_fields(plan.stats)
    wall, _ = time_steps(plan.run, 5, 1, torch)
    return {"degradation": {"workload": "band |y - tan(73 deg) x| <= 0.1 on [-1,1]x[-0.5,0.5], "
                                        "hole (-0.8,0.8)x(-0.3,0.3), eps=3, mu=50, guide along "
                                        "the band", "resolutions": res},
            "pan_video": {"workload": "16 x 1920x1080 RGB binary16 camera pan (3, 1) px per frame "
                                      "over one scene, 6 silhouette bands, eps=3, mu=50, one launch",
                          "hole_px": st["hole"], "shells": st["K"], "ms": round(wall, 4),
                          "mpix_filled_per_s": round(st["filled"] / (wall * 1e-3) / 1e6, 2)}}


def profile_guide(args):
    """Only the spline guide field of the 1080p frame (for rocprofv3)."""
    import torch

    import paper_1611_05319_amd as gf

    w2 = syn.config2()
    dev = torch.device("cuda:0")
    B, H, W, C = w2.image.shape
    lab = torch.from_numpy(w2.label).to(dev)
    rng = np.random.default_rng(12)
    seg, off = syn.pack_segments([syn.spline_segments(rng, H, W, n_splines=6, spacing=2.0)])
    seg_d = torch.from_numpy(seg).to(dev)
    off_d = torch.from_numpy(off).to(dev)
    g_out = torch.empty((B, H, W, 2), dtype=torch.float32, device=dev)

    def run_guide():
        gf.guide_field(lab, seg_d, off_d, out=g_out, check_offsets=False)

    wall, ev = time_steps(run_guide, args.steps, args.warmup, torch)
    print(json.dumps({"profile": "guide", "steps": args.steps, "event_ms": ev,
                      "segments": int(seg.shape[0])}), flush=True)


def profile_coherence(args):
    """Only the comparison fill of the 1080p frame (for rocprofv3)."""
    import torch

    import paper_1611_05319_amd as gf

    w2 = syn.config2()
    dev = torch.device("cuda:0")
    img = torch.from_numpy(w2.image).to(dev)
    lab = torch.from_numpy(w2.label).to(dev)
    out = torch.empty_like(img)
    ws = gf.Workspace()
    pc = gf.Params(eps=w2.eps, mu=w2.mu, ghost=False)

    def run_ct():
        gf.fill_coherence(img, lab, pc, out=out, workspace=ws, want_guide=False)

    wall, _ = time_steps(run_ct, args.steps, args.warmup, torch)
    print(json.dumps({"profile": "coherence", "steps": args.steps, "ms_per_fill": wall}), flush=True)


def profile_deep(args):
    """The 4K deep-front fill alone, one launch per step, autotuned launch."""
    w3 = syn.config3()
    import torch

    import paper_1611_05319_amd as gf
    from paper_1611_05319_amd import autotune

    dev = torch.device("cuda:0")
    print(json.dumps({"profile": "deep", **deep_front(w3, torch, gf, autotune, dev, args)}), flush=True)


def profile_batched(args):
    """The 64-frame binary16 batch alone, one launch per step, with the launch
    shape the autotuner picks (as in the full run's batched leg)."""
    w4 = syn.config4()
    import torch

    import paper_1611_05319_amd as gf
    from paper_1611_05319_amd import autotune

    dev = torch.device("cuda:0")
    i4 = torch.from_numpy(w4.image).to(dev)
    l4 = torch.from_numpy(w4.label).to(dev)
    g4 = torch.from_numpy(w4.guide).to(dev)
    p4 = autotune.tune(i4, l4, g4, gf.Params(eps=w4.eps, mu=w4.mu), reps=3)
    plan = gf.FillPlan(i4, l4, g4, p4)
    plan.run()
    torch.cuda.synchronize()
    st = gf.stats_fields(plan.stats)
    wall, ev = time_steps(plan.run, args.steps, args.warmup, torch)
    print(json.dumps({"profile": "batched", "steps": args.steps, "fill_event_ms": ev, "wall_ms": wall,
                      "launch": launch_fields(p4), "K": st["K"], "filled": st["filled"]}), flush=True)


def profile_grad(args):
    """Forward (recording the fill order) then backward on the 16-frame
    512 x 512 workload, one launch each per step, as in the full run."""
    w5, _ = syn.config5()
    import torch

    import paper_1611_05319_amd as gf

    dev = torch.device("cuda:0")
    i5 = torch.from_numpy(w5.image).to(dev)
    l5 = torch.from_numpy(w5.label).to(dev)
    g5 = torch.from_numpy(w5.guide).to(dev)
    from paper_1611_05319_amd import autotune

    p5 = autotune.tune(i5, l5, g5, gf.Params(eps=w5.eps, mu=w5.mu), reps=3)
    plan_f = gf.FillPlan(i5, l5, g5, p5)
    plan_f.run()
    torch.cuda.synchronize()
    K5 = int(plan_f.stats[0].item())
    gi = torch.empty_like(i5)
    gg = torch.empty(i5.shape[:3] + (2,), dtype=torch.float32, device=dev)
    bw = gf.BackwardPlan(plan_f, torch.randn_like(i5), gi, gg)

    def fwd_bwd():
        plan_f.run()
        bw.run()

    wall_f, ev_f = time_steps(plan_f.run, args.steps, args.warmup, torch)
    wall_fb, ev_fb = time_steps(fwd_bwd, args.steps, args.warmup, torch)
    print(json.dumps({"profile": "grad", "steps": args.steps, "fwd_ms": wall_f, "fwd_bwd_ms": wall_fb,
                      "fwd_event_ms": ev_f, "fwd_bwd_event_ms": ev_fb, "K": K5,
                      "launch": launch_fields(p5)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--profile", action="store_true", help="fill steps only (for rocprofv3)")
    ap.add_argument("--profile-batched", action="store_true",
                    help="64-frame batch fill steps only (for rocprofv3)")
    ap.add_argument("--profile-grad", action="store_true",
                    help="16 x 512^2 forward + backward steps only (for rocprofv3)")
    ap.add_argument("--profile-guide", action="store_true",
                    help="the spline guide field only (for rocprofv3)")
    ap.add_argument("--profile-coherence", action="store_true",
                    help="the coherence-transport comparison fill only (for rocprofv3)")
    ap.add_argument("--profile-deep", action="store_true",
                    help="3840x2160 deep-front fill steps only (for rocprofv3)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--copy-mb", type=int, default=512, help="plain copy size in --profile mode")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the benchmark runs on one GPU only (frames shard with no exchange; "
              "see the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.profile_batched:
        profile_batched(args)
        return
    if args.profile_grad:
        profile_grad(args)
        return
    if args.profile_guide:
        profile_guide(args)
        return
    if args.profile_coherence:
        profile_coherence(args)
        return
    if args.profile_deep:
        profile_deep(args)
        return

    # ---- inputs (generated before the device is touched) ---------------------
    w2 = syn.config2()
    extras = not (args.no_extras or args.profile)
    if extras:
        w3 = syn.config3()
        w4 = syn.config4()
        w5, theta5 = syn.config5()
    base = None
    if not (args.no_cpu_baseline or args.profile):
        base = cpu_baseline(w2)

    import torch

    import paper_1611_05319_amd as gf

    dev = torch.device("cuda:0")
    B, H, W, C = w2.image.shape
    img = torch.from_numpy(w2.image).to(dev)
    lab = torch.from_numpy(w2.label).to(dev)
    gd = torch.from_numpy(w2.guide).to(dev)
    from paper_1611_05319_amd import autotune

    params = autotune.tune(img, lab, gd, gf.Params(eps=w2.eps, mu=w2.mu))
    plan = gf.FillPlan(img, lab, gd, params)
    plan.run()
    torch.cuda.synchronize()
    st = gf.stats_fields(plan.stats)
    n_filled = st["filled"]

    if args.profile:
        # a plain copy of known size, for scaling the HBM counters
        nb = args.copy_mb << 20
        src = torch.empty(nb // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        wall, ev_mean = time_steps(plan.run, args.steps, args.warmup, torch)
        print(json.dumps({"profile": True, "steps": args.steps, "fill_event_ms": ev_mean,
                          "copy_bytes": nb, "K": st["K"], "filled": n_filled}), flush=True)
        return

    wall, ev_mean = time_steps(plan.run, args.steps, args.warmup, torch)
    mpix = n_filled / (wall * 1e-3) / 1e6
    nbytes = algorithmic_bytes(B, H, W, C, 4, st["hole"])
    achieved = nbytes / (ev_mean * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": round(mpix, 3),
        "unit": "Mpix filled/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE,
        "data": "synthetic",
        "config": {"workload": "plain fill 1920x1080 RGB, binary32 storage, 6 silhouette bands "
                               "5-20 px, spline/structure-tensor guide, eps=3, mu=50, onion "
                               "order, ghost pixels, tracked front, out of place",
                   "global_batch": 1, "hole_px": st["hole"], "filled_px": n_filled,
                   "shells": st["K"], "max_front": st["max_front"], "parallelism": "none",
                   "launch": launch_fields(params)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": recorded_traffic(params, H, W, C),
                     "algorithmic_bytes": nbytes, "event_ms_per_launch": round(ev_mean, 5),
                     "us_per_shell": round(ev_mean * 1e3 / max(st["K"], 1), 3)},
        "cpu_baseline": base,
    }

    if extras:
        # tracked vs untracked (one lane per pixel per shell)
        plan_u = gf.FillPlan(img, lab, gd, gf.Params(eps=w2.eps, mu=w2.mu, tracking=False))
        wall_u, ev_u = time_steps(plan_u.run, args.steps, args.warmup, torch)
        out["untracked"] = {"ms_per_step": round(wall_u, 5), "event_ms": round(ev_u, 5),
                            "value": round(n_filled / (wall_u * 1e-3) / 1e6, 3),
                            "tracked_speedup": round(wall_u / wall, 3)}
        # batched: 64 frames fp16, one launch vs 64 single-frame launches
        i4 = torch.from_numpy(w4.image).to(dev)
        l4 = torch.from_numpy(w4.label).to(dev)
        g4 = torch.from_numpy(w4.guide).to(dev)
        p4 = autotune.tune(i4, l4, g4, gf.Params(eps=w4.eps, mu=w4.mu), reps=3)
        plan_b = gf.FillPlan(i4, l4, g4, p4)
        # the plain form: one launch per frame, each with the library's default shape
        p1 = gf.Params(eps=w4.eps, mu=w4.mu)
        plans_1 = [gf.FillPlan(i4[f:f + 1], l4[f:f + 1], g4[f:f + 1], p1) for f in range(i4.shape[0])]
        plan_b.run()
        torch.cuda.synchronize()
        st4 = gf.stats_fields(plan_b.stats)

        def run_singles():
            for pl in plans_1:
                pl.run()

        steps4 = max(3, args.steps // 10)
        wall_b, ev_b = time_steps(plan_b.run, steps4, 2, torch)
        wall_s, ev_s = time_steps(run_singles, steps4, 1, torch)
        nb4 = algorithmic_bytes(*i4.shape, 2, st4["hole"])
        out["batched"] = {"workload": "64 x 1920x1080 RGB fp16 storage, lognormal hole fraction "
                                      "(median 2%), eps=3, mu=50",
                          "hole_px": st4["hole"], "max_frame_shells": max(st4["frame_K"]),
                          "launch": launch_fields(p4),
                          "batched_ms": round(wall_b, 4), "plain_64_launches_ms": round(wall_s, 4),
                          "batched_speedup": round(wall_s / wall_b, 3),
                          "mpix_filled_per_s": round(st4["filled"] / (wall_b * 1e-3) / 1e6, 2),
                          "hbm_gbs": round(nb4 / (ev_b * 1e-3) / 1e9, 1),
                          "hbm_frac": round(nb4 / (ev_b * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "algorithmic_bytes": nb4,
                          "traffic": recorded_traffic(p4, *i4.shape[1:],
                                                      summary="traffic_c4_batched.md")}
        del i4, l4, g4, plan_b, plans_1
        # deep front: 3840x2160, one 200-px band plus 20 discs, eps = 5, mu = 100
        out["deep_front"] = deep_front(w3, torch, gf, autotune, dev, args)
        out.update(guidance_extras(w2, torch, gf, dev, args))
        out["studies"] = studies(torch, gf, dev, args)
        # forward vs forward + backward (reverse-shell adjoint)
        i5 = torch.from_numpy(w5.image).to(dev)
        l5 = torch.from_numpy(w5.label).to(dev)
        g5 = torch.from_numpy(w5.guide).to(dev)
        p5 = autotune.tune(i5, l5, g5, gf.Params(eps=w5.eps, mu=w5.mu), reps=3)
        plan_f = gf.FillPlan(i5, l5, g5, p5)
        plan_f.run()
        torch.cuda.synchronize()
        K5 = int(plan_f.stats[0].item())
        grad = torch.randn_like(i5)
        gi = torch.empty_like(i5)
        gg = torch.empty(i5.shape[:3] + (2,), dtype=torch.float32, device=dev)
        bw = gf.BackwardPlan(plan_f, grad, gi, gg)

        def fwd_bwd():
            plan_f.run()
            bw.run()

        steps5 = max(5, args.steps // 5)
        wall_f, _ = time_steps(plan_f.run, steps5, 2, torch)
        wall_fb, _ = time_steps(fwd_bwd, steps5, 2, torch)
        out["fwd_bwd"] = {"workload": "16 x 512x512 RGB fp32, band masks 6-16 px, smooth angle "
                                      "field, eps=3, mu=50",
                          "launch": launch_fields(p5),
                          "fwd_ms": round(wall_f, 4), "fwd_bwd_ms": round(wall_fb, 4),
                          "ratio": round(wall_fb / wall_f, 3), "shells": K5,
                          "bwd_traffic": recorded_traffic(p5, *i5.shape[1:],
                                                          summary="traffic_c5_grad.md")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
