"""Benchmark of the batched-window hot path on one MI355X.

Workload: 500k surfel Gaussians on 50 random planes, 8 keyframes at 1280x1024
on a smooth trajectory (0.3 m / 5 degrees apart), L1 photometric loss against
a target rendered from a copy with means jittered by N(0, 0.02 m).  One step
is one pass of the whole path over the window — projection, depth sort, tile
binning, tile sort, one fused forward/loss/backward launch over every
(camera, tile) item, the projection adjoint to means, scales, quaternions,
opacities, colours and the 8 camera poses — replayed as one HIP graph.
Inputs are resident in HBM before the timed region.

Prints one JSON line; besides the metric it carries
  fwd_ms_per_frame  forward only (gsl_window_render: project + bin_sort + render_fwd as one graph) per frame
  per_frame         the same window as 8 sequential single-camera eager steps
  roofline          the fused render kernel (dominant), ALU-bound: algorithmic
                    FLOPs from the pair counts / its duration (HIP events on
                    its stream) against the FP32 vector peak
  cpu_baseline      the FP64 oracle, forward + backward, on a pixel sample
  pose_jacobian     the IESKF measurement model (per-pixel twist Jacobians and
                    normal equations) on 32 perturbed poses of a 640x512 view
  window_update     the incremental sliding-window update (hash classification
                    of a LiDAR frame's voxels, in-place compaction) at 500k
  sh3_window        the same window step with SH degree 3 colour
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# settings the paper states (Sec. III-B, III-D): 10 optimisation iterations per
# frame, outdoor root voxels of 0.5 m, and the window sizes the sweep spans
OPT_ITERS = 10
ROOT_VOXEL_M = 0.5
SWEEP_N = (20_000, 100_000, 500_000, 2_000_000)
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (256 CU x 4 SIMD x 16 lanes x 2 FMA x 2 packed x 2.4 GHz)
# FLOPs per (pixel, Gaussian) pair, counted from the per-pair formulas of the
# compositing and its adjoint (add/mul/min/exp = 1, fma = 2):
F_EVAL = 13        # alpha of one pair (forward walk, and again in the backward walk)
F_CONTRIB = 52     # a contributor: 9 in the forward, 43 in the backward
F_JVP_CONTRIB = 145  # a contributor in the forward-mode pose walk: 9 colour + 136 for the 6 twist tangents
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_render_traffic.txt")
RENDER_SRC = os.path.join(ROOT, "paper_2501_08672_amd", "csrc", "render.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--tile", type=int, default=0, help="0 = autotune")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-pixels", type=int, default=4096,
                    help="oracle sample: pixels per camera (the default is about 20 s of host time, which keeps "
                         "the default run within minutes; full frames of this window would take hours)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-per-frame", action="store_true")
    ap.add_argument("--no-jac", action="store_true", help="skip the pose-Jacobian measurement")
    ap.add_argument("--no-window-update", action="store_true", help="skip the window-update measurement")
    ap.add_argument("--no-sh", action="store_true", help="skip the SH-colour window measurement")
    ap.add_argument("--no-optimize", action="store_true", help="skip the 10-iteration optimisation loop")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the 1k forward, 100k forward+backward and 2M uneven-batch measurements")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark line: window step time vs N in {20k, 100k, 500k, 2M} at "
                         "640x512 and 1280x1024 (8 keyframes), one JSON line per point")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration runs)")
    return ap.parse_args()


def source_digest():
    return hashlib.sha1(open(RENDER_SRC, "rb").read()).hexdigest()[:16]


def read_traffic():
    """HBM bytes per fused launch from the committed counter summary, or None
    when it is missing or was taken on a different render.hip."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for ln in open(TRAFFIC_FILE):
        if ":" in ln and not ln.startswith("#"):
            k, v = ln.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        if kv.get("render_hip_sha1") != source_digest():
            return None
        f = float(kv["copy_bytes"]) / (float(kv["copy_fetch_kib"]) * 1024)
        w = float(kv["copy_bytes"]) / (float(kv["copy_write_kib"]) * 1024)
        return float(kv["fused_fetch_kib"]) * 1024 * f + float(kv["fused_write_kib"]) * 1024 * w
    except (KeyError, ValueError, ZeroDivisionError):
        return None


COUNTER_FILE = os.path.join(ROOT, "profiles", "fused_render_counters.txt")
# L2 atomic requests the MI355X can retire per second, derived (no published
# figure): one request per L2 channel per clock, 16 channels in each of the 8
# XCDs at 2.4 GHz
L2_ATOMIC_PEAK_PER_S = 8 * 16 * 2.4e9


def read_counter(name):
    """One per-dispatch counter of the fused kernel from the committed SQ/TCC
    summary, or None when it is missing or was taken on a different render.hip."""
    if not os.path.exists(COUNTER_FILE):
        return None
    kv = {}
    for ln in open(COUNTER_FILE):
        if ":" in ln and not ln.startswith("#"):
            k, v = ln.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        return float(kv[name]) if kv.get("render_hip_sha1") == source_digest() else None
    except (KeyError, ValueError):
        return None


def read_atomics():
    """(L2 atomic requests, atomic wave instructions) per fused launch from
    the committed SQ/TCC counter summary, or None when it is missing or was
    taken on a different render.hip."""
    if not os.path.exists(COUNTER_FILE):
        return None
    kv = {}
    for ln in open(COUNTER_FILE):
        if ":" in ln and not ln.startswith("#"):
            k, v = ln.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        if kv.get("render_hip_sha1") != source_digest():
            return None
        return float(kv["TCC_ATOMIC"]), float(kv["TA_FLAT_ATOMIC_WAVEFRONTS"])
    except (KeyError, ValueError):
        return None


def copy_peak_gbs(torch, mib=1024, reps=10):
    """HBM bandwidth a plain device copy reaches on this GPU: bytes read plus
    written per second (HIP events around `reps` copies of `mib` MiB)."""
    src = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * (mib << 20) * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def cpu_baseline(sc, cams, per_cam, seed=0):
    """The FP64 oracle, as it stands, on `per_cam` seeded pixels of every camera."""
    from oracle import oracle as O
    O.build(force=False)
    rng = np.random.default_rng(seed)
    pix, vs = [], []
    for cam in cams:
        p = np.stack([rng.integers(0, cam.width, per_cam), rng.integers(0, cam.height, per_cam)], 1)
        pix.append(p.astype(np.int32))
        vs.append(rng.normal(size=(per_cam, 3)))
    o = O.Opts()
    t0 = time.perf_counter()
    for cam, p in zip(cams, pix):
        O.render(sc, cam, o, pixels=p)
    t1 = time.perf_counter()
    O.render_bwd(sc, cams, vs, o, pixels=pix)
    t2 = time.perf_counter()
    n = per_cam * len(cams)
    cpu = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                cpu = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(n / (t2 - t0) / 1e6, 6), "unit": "Mpixels/s", "cores": O.num_threads(),
            "cpu_model": cpu, "kind": "oracle",
            "sample": f"{per_cam} seeded pixels per camera x {len(cams)} cameras of the same window; forward "
                      f"{t1 - t0:.2f} s + backward (random cotangent on those pixels) {t2 - t1:.2f} s; each call "
                      f"projects and depth-orders all {sc.n} Gaussians"}


def pose_jacobian_bench(ctx, ops, S, torch, reps=5, tiles=(8, 16, 32)):
    """The IESKF measurement model on a batch of 32 perturbed poses of one
    view (200k surfels on 20 planes, 640x512): project + bin_sort +
    gsl_pose_jacobian (per-pixel twist Jacobians and the per-camera normal
    equations against the image at the true pose).  Every tile size is timed
    and the fastest reported (its per-tile times beside it)."""
    sc, true_cam, cams, _ = S.config4()
    g = ops.Gaussians.from_scene(sc)
    c1 = ops.CameraSet([true_cam])
    cs = ops.CameraSet(cams)
    P = cs.P_total
    per_tile, best = {}, None
    for tile in tiles:
        o = ops.opts(tile)
        p1 = ops.project(ctx, g, c1, o)
        b1 = ops.bin_sort(ctx, c1, g.N, o, p1)
        img, _, _ = ops.render_fwd(ctx, c1, g.N, o, p1, b1)
        target = img.repeat(cs.C).contiguous()
        proj = ops.project(ctx, g, cs, o)
        bins = ops.bin_sort(ctx, cs, g.N, o, proj)
        ops.pose_jacobian(ctx, g, cs, o, proj, bins, target=target)
        torch.cuda.synchronize()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        t_all, t_jac = [], []
        for _ in range(reps):
            e0.record()
            ops.project(ctx, g, cs, o, out=proj)
            ops.bin_sort(ctx, cs, g.N, o, proj, capacity=bins.capacity, bins=bins, grow=False)
            e1.record()
            pj = ops.pose_jacobian(ctx, g, cs, o, proj, bins, target=target)
            e2.record()
            torch.cuda.synchronize()
            t_all.append(e0.elapsed_time(e2))
            t_jac.append(e1.elapsed_time(e2))
        ms, jac_ms = float(np.median(t_all)), float(np.median(t_jac))
        per_tile[tile] = round(ms, 4)
        if best is None or ms < best[1]:
            ev_f, n_contrib, _ = ops.render_stats(ctx, cs, g.N, o, proj, bins)
            rms = float(np.sqrt(pj.zz.sum().item() / (3 * P)))
            best = (tile, ms, jac_ms, ev_f, n_contrib, bins.K, rms)
        del proj, bins, pj, target
    tile, ms, jac_ms, ev_f, n_contrib, K, rms = best
    flops = F_EVAL * ev_f + F_JVP_CONTRIB * n_contrib
    ach = flops / (jac_ms * 1e-3) / 1e12
    return {"workload": "IESKF photometric model: 200k surfels on 20 planes, 32 perturbed poses of a 640x512 view "
                        "(0.05 m, 1 deg), per-pixel twist Jacobians + per-camera normal equations",
            "ms_per_batch": round(ms, 4), "mpix_s": round(P / (ms * 1e-3) / 1e6, 2),
            "jacobian_ms": round(jac_ms, 4), "tile": tile, "ms_per_batch_by_tile": per_tile, "instances_K": K,
            "alu": {"achieved": round(ach, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(ach / FP32_VECTOR_PEAK_TFLOPS, 4),
                    "pairs": {"evaluated": ev_f, "contributors": n_contrib}},
            "residual_rms": round(rms, 5)}


def optimize_bench(ctx, ops, torch, g, win):
    """The optimisation loop of one keyframe: 10 iterations of window step +
    Adam recorded as one graph (it moves the Gaussians, so it runs after the
    window-step measurements)."""
    st = ops.AdamState.from_gaussians(ctx, g)
    ops.adam_activate(ctx, st, g)
    hp = ops.adam_hparams()
    win.optimize(st, hp, iters=OPT_ITERS)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        losses = win.optimize(st, hp, iters=OPT_ITERS)
    torch.cuda.synchronize()
    t_opt = (time.perf_counter() - t1) / reps
    assert win.status() == 0, "instance capacity exceeded during the optimisation loop"
    return {"iters": OPT_ITERS, "ms": round(t_opt * 1e3, 4), "ms_per_iter": round(t_opt * 1e3 / OPT_ITERS, 4),
            "last_losses": [round(float(x), 6) for x in losses[[0, -1]].cpu().tolist()],
            "how": "gsl_window_optimize: 10 x (window step + Adam step over the 500k raw parameters), one graph"}


def _target_image(ops, ctx, cs, tgt_sc, tile=16):
    gt = ops.Gaussians.from_scene(tgt_sc)
    o = ops.opts(tile)
    pt = ops.project(ctx, gt, cs, o)
    bt = ops.bin_sort(ctx, cs, gt.N, o, pt)
    target, _, _ = ops.render_fwd(ctx, cs, gt.N, o, pt, bt)
    return target


def _timed_steps(torch, win, steps):
    """Median of HIP-event times around `steps` graph replays of the window step (ms)."""
    for _ in range(3):
        win.step(True)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
    for k in range(steps):
        evs[2 * k].record()
        win.step(True)
        evs[2 * k + 1].record()
    torch.cuda.synchronize()
    assert win.status() == 0, "instance capacity exceeded"
    return float(np.median([evs[2 * k].elapsed_time(evs[2 * k + 1]) for k in range(steps)]))


def workloads_bench(ctx, ops, S, torch, steps, with_oracle):
    """The other workloads of the metric, beside the headline window:
    the 1k / 128x96 plain forward render (ms per frame: gsl_window_render
    replayed as a graph, and the eager three calls; tile 16), the 100k /
    640x512 forward + backward
    (L1, tuned window step replayed as a graph, Mpixels/s) and the 2M /
    16-camera uneven batch (tuned tile, chunk and variant, graph, Mpixels/s);
    with the oracle's full-frame times for the first two."""
    from oracle import oracle as O
    out = {}
    # 1k Gaussians, one 128x96 camera: plain forward
    sc1 = S.config1()
    cs1 = ops.CameraSet(sc1.cams)
    g1 = ops.Gaussians.from_scene(sc1)
    o1 = ops.opts(16)
    proj = ops.project(ctx, g1, cs1, o1)
    bins = ops.bin_sort(ctx, cs1, g1.N, o1, proj)
    # the instance capacity both timed paths use: the window render's own
    # sizing (K with 25 % headroom + 4096), which at this size keeps the
    # tile sort in one workgroup
    cap1 = int(bins.K * 1.25) + 4096
    bins = ops.bin_sort(ctx, cs1, g1.N, o1, proj, capacity=cap1)
    ops.render_fwd(ctx, cs1, g1.N, o1, proj, bins)
    torch.cuda.synchronize()
    times = []
    for _ in range(max(20, steps)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ops.project(ctx, g1, cs1, o1, out=proj)
        ops.bin_sort(ctx, cs1, g1.N, o1, proj, capacity=bins.capacity, bins=bins, grow=False)
        ops.render_fwd(ctx, cs1, g1.N, o1, proj, bins)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    # the same render as one recorded unit (gsl_window_render), replayed
    r1 = ops.WindowRender(ctx, g1, cs1, o1, capacity=cap1)
    for _ in range(20):
        r1(use_graph=True)
    torch.cuda.synchronize()
    # back-to-back frames (throughput), then each frame on its own (latency)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(100):
        r1(use_graph=True)
    e1.record()
    torch.cuda.synchronize()
    b2b = e0.elapsed_time(e1) / 100
    gtimes = []
    for _ in range(max(20, steps)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        r1(use_graph=True)
        e1.record()
        torch.cuda.synchronize()
        gtimes.append(e0.elapsed_time(e1))
    assert r1.status() == 0
    c1 = {"workload": "plain forward render: 1,000 Gaussians, one 128x96 camera, tile 16",
          "fwd_ms_per_frame": round(float(np.median(gtimes)), 4), "instances_K": bins.K,
          "how": "gsl_window_render replayed as a HIP graph (camera upload + projection + binning + "
                 "compositing), HIP events around each frame, median",
          "fwd_ms_per_frame_back_to_back": round(b2b, 4),
          "fwd_ms_per_frame_eager": round(float(np.median(times)), 4),
          "eager_how": "gsl_project + gsl_bin_sort + gsl_render_fwd, eager launches, HIP events, median"}
    del r1
    if with_oracle:
        O.build(force=False)
        t0 = time.perf_counter()
        O.render_image(sc1, sc1.cams[0], O.Opts())
        c1["oracle_fwd_ms_per_frame"] = round((time.perf_counter() - t0) * 1e3, 2)
    out["config1"] = c1
    del proj, bins
    # 100k Gaussians, one 640x512 camera: forward + backward, L1
    sc2, tgt2 = S.config2()
    cs2 = ops.CameraSet(sc2.cams)
    target = _target_image(ops, ctx, cs2, tgt2)
    win = ops.Window(ctx, ops.Gaussians.from_scene(sc2), cs2, ops.opts(16), target, loss="l1")
    tile, _ = win.tune()
    ms = _timed_steps(torch, win, steps)
    c2 = {"workload": "forward + backward: 100k Gaussians, one 640x512 camera, L1 against a jittered copy",
          "tile": tile, "ms_per_step": round(ms, 4), "mpix_s": round(cs2.P_total / (ms * 1e-3) / 1e6, 2),
          "instances_K": win.bins.K, "how": "tuned window step replayed as a graph, HIP events, median"}
    del win
    if with_oracle:
        cam = sc2.cams[0]
        rng = np.random.default_rng(7)
        t0 = time.perf_counter()
        O.render_image(sc2, cam, O.Opts())
        t1 = time.perf_counter()
        O.render_bwd(sc2, [cam], [rng.normal(size=(3, cam.height, cam.width))], O.Opts())
        t2 = time.perf_counter()
        c2["oracle"] = {"fwd_s": round(t1 - t0, 2), "bwd_s": round(t2 - t1, 2),
                        "mpix_s": round(cs2.P_total / (t2 - t0) / 1e6, 6), "cores": O.num_threads(),
                        "how": "full frame, forward then the adjoint of a random cotangent image"}
    out["config2"] = c2
    # 2M Gaussians, 16 cameras of mixed resolution
    sc5, tgt5 = S.config5()
    cs5 = ops.CameraSet(sc5.cams)
    target = _target_image(ops, ctx, cs5, tgt5)
    win = ops.Window(ctx, ops.Gaussians.from_scene(sc5), cs5, ops.opts(16), target, loss="l1")
    tile, times5 = win.tune()
    ms = _timed_steps(torch, win, steps)
    out["config5"] = {"workload": "uneven batch: 2M surfel Gaussians on 200 planes, 16 cameras from 320x256 to "
                                  "1920x1080, each seeing 50k-600k Gaussians, L1",
                      "pixels": cs5.P_total, "ms_per_step": round(ms, 4),
                      "mpix_s": round(cs5.P_total / (ms * 1e-3) / 1e6, 2), "instances_K": win.bins.K,
                      "autotune": tune_table(ops, times5, tile),
                      "how": "tuned tile, LDS chunk depth and variant; window step replayed as a graph, HIP "
                             "events, median"}
    del win
    torch.cuda.empty_cache()
    return out


def sh_window_bench(ctx, ops, S, torch, sc, cs, target, tile, steps=10):
    """The bench window with view-dependent colour: the same 500k surfels and
    8 keyframes with SH degree 3 (15 coefficients per channel, N(0, 0.15/l)),
    one window step (projection with the SH colour, binning, fused render,
    projection adjoint + SH adjoint) replayed as a graph, against the same
    target."""
    sc3 = S.with_sh(sc, 3, 33)
    g = ops.Gaussians.from_scene(sc3)
    win = ops.Window(ctx, g, cs, ops.opts(tile), target, loss="l1")
    for _ in range(3):
        win.step(True)
    torch.cuda.synchronize()
    assert win.status() == 0
    t0 = time.perf_counter()
    for _ in range(steps):
        win.step(True)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    st_ms = np.array([win.profiled_step() for _ in range(3)]).mean(0)
    res = {"workload": "the bench window with SH degree 3 colour (500k surfels, 8 keyframes 1280x1024, L1)",
           "sh_degree": 3, "ms_per_step": round(t * 1e3, 4), "mpix_s": round(cs.P_total / t / 1e6, 2),
           "stage_ms": {"project": round(float(st_ms[0]), 4), "bin_sort": round(float(st_ms[1]), 4),
                        "fused_render": round(float(st_ms[2]), 4), "adjoint": round(float(st_ms[3]), 4)}}
    del win, g
    return res


def window_update_bench(ctx, ops, S, torch, frames=8):
    """The incremental window update (Sec. II-C) on a synthetic LiDAR stream:
    a 500k-Gaussian window (42 rows: raw parameters and Adam moments) at a
    capacity of 2^20, 100k points per frame, root voxels of 0.5 m, the sensor
    moving 1 m per frame.  Per frame: gsl_window_classify, the host read of
    (D, A), the appended Gaussians (as many per ADD voxel as the window holds
    per voxel on average) copied from pinned host memory to the device,
    gsl_window_compact, and the evicted Gaussians copied back to pinned host
    memory (gsl_window_transfer both ways)."""
    n, P, cap, vs, R = 500_000, 100_000, 1 << 20, ROOT_VOXEL_M, 42
    pts_np, means = S.lidar_stream(71, frames + 1, P, n)
    pts = [torch.from_numpy(p).cuda() for p in pts_np]
    sw = ops.SlidingWindow(ctx, cap, vs)
    sw.keys[:n] = ops.voxel_keys(ctx, torch.from_numpy(means).cuda(), vs)
    gen = torch.Generator(device="cuda").manual_seed(5)
    sw.block.normal_(generator=gen)
    sw.n = n
    per_voxel = max(1, round(n / int(torch.unique(sw.keys[:n]).numel())))
    # host-side map stand-in: pinned rows of the Gaussians to append, and pinned room for the evicted ones
    pool_h = torch.randn(R, cap // 4, generator=torch.Generator().manual_seed(6)).pin_memory()
    keys_in_h = torch.empty(cap // 4, dtype=torch.int64).pin_memory()
    keys_out_h = torch.empty(cap, dtype=torch.int64).pin_memory()
    rows_out_h = torch.empty(R, cap, dtype=torch.float32).pin_memory()
    add_k = torch.empty(cap // 4, dtype=torch.int64, device="cuda")
    add_r = torch.empty(R, cap // 4, dtype=torch.float32, device="cuda")
    ws = ops.window_workspace(ctx, cap, P)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    rows = []
    for f in range(frames + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record()
        counts, addv = ops.window_classify(ctx, pts[f], vs, sw.keys, sw.n, ws)
        ev[1].record()
        D, A = (int(x) for x in counts.cpu())
        Ag = A * per_voxel
        keys_in_h[:Ag].copy_(addv[:A].cpu().repeat_interleave(per_voxel))
        ev[2].record()
        ops.window_transfer(ctx, ops.A.GSL_H2D, keys_in_h, pool_h, add_k, add_r, Ag)
        ev[3].record()
        ek, er, status = ops.window_compact(ctx, sw.keys, sw.block, sw.n, D, add_k[:Ag],
                                            add_r[:, :Ag].contiguous(), ws)
        ev[4].record()
        ops.window_transfer(ctx, ops.A.GSL_D2H, ek, er, keys_out_h, rows_out_h, D)
        ev[5].record()
        torch.cuda.synchronize()
        t_frame = time.perf_counter() - t0
        assert int(status.item()) == 0
        n_before = sw.n
        sw.n = sw.n - D + Ag
        if f == 0:
            continue  # warm-up frame
        rows.append((n_before, D, A, Ag, ev[0].elapsed_time(ev[1]), ev[3].elapsed_time(ev[4]),
                     ev[2].elapsed_time(ev[3]), ev[4].elapsed_time(ev[5]), t_frame * 1e3))
    a = np.array(rows, dtype=np.float64)
    n_m, D_m, Av_m, Ag_m, cls_ms, cmp_ms, h2d_ms, d2h_ms, frame_ms = (float(x) for x in a.mean(0))
    rec = 8 + 4 * R
    cls_bytes = 12 * P + 8 * n_m + 8 * Av_m
    cmp_bytes = 2 * D_m * rec + 2 * D_m * rec + 2 * Ag_m * rec  # evict, move (<= D), append
    return {"workload": "sliding-window update: 500k Gaussians x 42 rows (raw + Adam moments), capacity 2^20, "
                        "100k LiDAR points per frame, 0.5 m root voxels, sensor moving 1 m per frame",
            "frames": frames, "window": round(n_m), "deleted": round(D_m), "add_voxels": round(Av_m),
            "appended": round(Ag_m), "classify_ms": round(cls_ms, 4), "compact_ms": round(cmp_ms, 4),
            "h2d_ms": round(h2d_ms, 4), "d2h_ms": round(d2h_ms, 4), "frame_ms": round(frame_ms, 4),
            "hbm": {"classify_bytes": int(cls_bytes), "compact_bytes_max": int(cmp_bytes),
                    "classify_gbs": round(cls_bytes / (cls_ms * 1e-3) / 1e9, 1),
                    "compact_gbs": round(cmp_bytes / (cmp_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS},
            "pcie": {"h2d_bytes": int(Ag_m * rec), "d2h_bytes": int(D_m * rec),
                     "h2d_gbs": round(Ag_m * rec / (h2d_ms * 1e-3) / 1e9, 1),
                     "d2h_gbs": round(D_m * rec / (d2h_ms * 1e-3) / 1e9, 1)},
            "how": "HIP events around each call; frame_ms is the host's clock over the frame, with the read of "
                   "(D, A) and the pinned staging both ways (the per-frame synchronisation the host-side global map "
                   "needs)"}


def sweep(args):
    import torch

    import scenegen as S
    from paper_2501_08672_amd import ops

    ctx = ops.Context(0)
    for (W, H) in ((640, 512), (1280, 1024)):
        for n in SWEEP_N:
            sc, tgt_sc = S.config3(per_plane=n // 50, width=W, height=H, f=0.78125 * W)
            cs = ops.CameraSet(sc.cams)
            g, gt = ops.Gaussians.from_scene(sc), ops.Gaussians.from_scene(tgt_sc)
            o = ops.opts(16)
            pt = ops.project(ctx, gt, cs, o)
            bt = ops.bin_sort(ctx, cs, gt.N, o, pt)
            target, _, _ = ops.render_fwd(ctx, cs, gt.N, o, pt, bt)
            del pt, bt, gt
            win = ops.Window(ctx, g, cs, o, target, loss="l1")
            tile, _ = win.tune()
            for _ in range(3):
                win.step(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                win.step(True)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / args.steps
            st_ms = np.array([win.profiled_step() for _ in range(3)]).mean(0)
            print(json.dumps({"gaussians": n, "frames": cs.C, "width": W, "height": H, "tile": tile,
                              "instances_K": win.bins.K, "instances_per_pixel": round(win.bins.K / cs.P_total, 2),
                              "ms_per_step": round(t * 1e3, 4), "mpix_s": round(cs.P_total / t / 1e6, 2),
                              "stage_ms_eager": {"project": round(float(st_ms[0]), 4),
                                                 "bin_sort": round(float(st_ms[1]), 4),
                                                 "fused_render": round(float(st_ms[2]), 4),
                                                 "adjoint": round(float(st_ms[3]), 4)}}), flush=True)
            del win, g, target
            torch.cuda.empty_cache()
    # the uneven batch: 2M surfels, 16 cameras from 320x256 to 1920x1080
    sc, tgt_sc = S.config5()
    cs = ops.CameraSet(sc.cams)
    g, gt = ops.Gaussians.from_scene(sc), ops.Gaussians.from_scene(tgt_sc)
    o = ops.opts(16)
    pt = ops.project(ctx, gt, cs, o)
    bt = ops.bin_sort(ctx, cs, gt.N, o, pt)
    target, _, _ = ops.render_fwd(ctx, cs, gt.N, o, pt, bt)
    del pt, bt, gt
    win = ops.Window(ctx, g, cs, o, target, loss="l1")
    tile, _ = win.tune()
    for _ in range(3):
        win.step(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        win.step(True)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    print(json.dumps({"gaussians": sc.n, "frames": cs.C, "sizes": "uneven, 320x256 ... 1920x1080",
                      "pixels": cs.P_total, "tile": tile, "instances_K": win.bins.K,
                      "ms_per_step": round(t * 1e3, 4), "mpix_s": round(cs.P_total / t / 1e6, 2)}), flush=True)
    ctx.close()


def tune_table(ops, times, tile):
    """The autotuner's grid of eager step times, tile -> LDS chunk depth ->
    the five fused-kernel variants, and the configuration it chose (the
    fastest at the chosen tile)."""
    grid, k = {}, 0
    for t in ops.TUNE_TILES:
        grid[str(t)] = {}
        for ch in ops.TUNE_CHUNKS:
            grid[str(t)][str(ch)] = [round(x, 3) for x in times[k:k + ops.TUNE_VARIANTS]]
            k += ops.TUNE_VARIANTS
    best = min(((ms, int(ch), v) for ch, row in grid[str(tile)].items() for v, ms in enumerate(row)))
    return {"grid_ms": grid, "chosen": {"tile": tile, "chunk": best[1], "variant": best[2], "ms": best[0]}}


def main():
    args = parse()
    if args.sweep:
        sweep(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (no multi-GPU path is built)"}))
        sys.exit(2)
    import torch

    import scenegen as S
    from paper_2501_08672_amd import ops

    if args.copy_calib_mib:
        nb = args.copy_calib_mib << 20
        src = torch.empty(nb, dtype=torch.uint8, device="cuda").random_(0, 255)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nb} bytes x 3")
        del src, dst

    t0 = time.time()
    sc, tgt_sc = S.config3()
    log(f"scene generated in {time.time() - t0:.1f}s: N={sc.n}, cams={len(sc.cams)}, digest {sc.digest()}")
    ctx = ops.Context(0)
    cs = ops.CameraSet(sc.cams)
    g = ops.Gaussians.from_scene(sc)
    gt = ops.Gaussians.from_scene(tgt_sc)
    o = ops.opts(16)
    pt = ops.project(ctx, gt, cs, o)
    bt = ops.bin_sort(ctx, cs, gt.N, o, pt)
    target, _, _ = ops.render_fwd(ctx, cs, gt.N, o, pt, bt)
    del pt, bt, gt
    torch.cuda.synchronize()

    win = ops.Window(ctx, g, cs, o, target, loss="l1")
    tune_times = None
    if args.tile == 0:
        tile, tune_times = win.tune()
        log(f"autotune: {json.dumps(tune_table(ops, tune_times, tile)['chosen'])}")
    else:
        win.opts = ops._opts_copy(o, tile=args.tile)
        win._alloc(None)
    tile = int(win.opts.tile)
    use_graph = not args.no_graph
    for _ in range(args.warmup):
        win.step(use_graph)
    torch.cuda.synchronize()
    assert win.status() == 0, "instance capacity exceeded"
    K = win.bins.K
    t_start = time.perf_counter()
    for _ in range(args.steps):
        win.step(use_graph)
    torch.cuda.synchronize()
    t_win = (time.perf_counter() - t_start) / args.steps
    P = cs.P_total
    mpix = P / t_win / 1e6
    log(f"window step {t_win * 1e3:.3f} ms, {mpix:.1f} Mpix/s, K={K}, loss={float(win.d_loss.item()):.6f}")
    # per-step distribution (HIP events around each replay, outside the timed region above)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps)]
    for k in range(args.steps):
        evs[2 * k].record()
        win.step(use_graph)
        evs[2 * k + 1].record()
    torch.cuda.synchronize()
    per_step = np.array([evs[2 * k].elapsed_time(evs[2 * k + 1]) for k in range(args.steps)])
    step_pct = {"p10": round(float(np.percentile(per_step, 10)), 4), "p50": round(float(np.median(per_step)), 4),
                "p90": round(float(np.percentile(per_step, 90)), 4)}
    log(f"per-step ms p10/p50/p90: {step_pct}")

    # stage times: HIP events on the launch stream between the stages of eager
    # steps (the fused kernel's duration for the roofline: in the kernel trace
    # these dispatches take what the events show), and of replays of the
    # step's profiling graph, whose event nodes add their own time.  Reading
    # the events waits for the GPU, and after such an idle gap the clock takes
    # some ten steps to come back: every profiled step is queued behind ten
    # plain replays, so it runs at the clock of the timed region.
    def behind_replays(graph=False):
        for _ in range(10):
            win.step(use_graph)
        return win.profiled_step(graph=graph)

    st_ms = np.array([behind_replays() for _ in range(5)]).mean(0)
    log("eager stage ms (project, bin_sort, fused render, adjoint, total): " + " ".join(f"{x:.3f}" for x in st_ms))
    st_graph = None
    if use_graph:
        try:
            win.profiled_step(graph=True)  # capture
            st_graph = np.array([behind_replays(graph=True) for _ in range(10)]).mean(0)
            log("graph stage ms (project, bin_sort, fused render, adjoint, total): "
                + " ".join(f"{x:.3f}" for x in st_graph))
        except Exception as e:
            log(f"graph stage events unavailable: {e}")
    fused_ms = float(st_ms[2])

    # pair counts of the compositing on the window's bins -> algorithmic FLOPs
    ev_f, n_contrib, ev_b = ops.render_stats(ctx, cs, g.N, win.opts, win.proj, win.bins)
    flops = F_EVAL * (ev_f + ev_b) + F_CONTRIB * n_contrib
    achieved = flops / (fused_ms * 1e-3) / 1e12
    visible = [int((win.proj.tiles_touched[c] > 0).sum().item()) for c in range(cs.C)]
    log(f"pairs: fwd {ev_f}, contributors {n_contrib}, bwd {ev_b}; visible per camera {visible}")

    # algorithmic bytes of the fused kernel: instance list, splat records and
    # 2D-gradient records of the visible Gaussians, target read, image write
    fused_bytes = 4 * K + 72 * sum(visible) + 8 * cs.tiles(tile) + 24 * P
    # whole-step algorithmic bytes (every logical array read/written once per stage)
    N, C_ = g.N, cs.C
    step_bytes = N * 144 + C_ * N * 60 + sum(visible) * 144 + K * 48 + cs.tiles(tile) * 16 + P * 32

    # forward only: the window's render as one recorded unit (gsl_window_render,
    # camera upload + projection + binning + compositing) replayed as a graph,
    # and the same kernels as eager gsl_project + gsl_bin_sort + gsl_render_fwd
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rw = ops.WindowRender(ctx, g, cs, win.opts, capacity=win.bins.capacity)
    for it in range(20):  # the first ten bring the clock back after the last synchronisation
        if it == 10:
            ev0.record()
        rw(use_graph=True)
    ev1.record()
    torch.cuda.synchronize()
    assert rw.status() == 0
    fwd_ms = ev0.elapsed_time(ev1) / 10
    del rw
    proj = ops.Proj(cs.C, g.N, ctx.device)
    bins = ops.Bins(win.bins.capacity, cs.tiles(tile), ctx.device)
    for it in range(13):
        if it == 3:
            ev0.record()
        ops.project(ctx, g, cs, win.opts, out=proj)
        ops.bin_sort(ctx, cs, g.N, win.opts, proj, capacity=bins.capacity, bins=bins, grow=False)
        ops.render_fwd(ctx, cs, g.N, win.opts, proj, bins)
    ev1.record()
    torch.cuda.synchronize()
    fwd_ms_eager = ev0.elapsed_time(ev1) / 10
    del proj, bins
    log(f"forward only {fwd_ms:.3f} ms per window, {fwd_ms / cs.C:.3f} ms/frame (graph); "
        f"{fwd_ms_eager:.3f} ms per window eager")

    per_frame = None
    if not args.no_per_frame:
        frames = []
        for c in range(cs.C):
            c1 = ops.CameraSet([sc.cams[c]])
            tc = cs.unpack(target)[c].reshape(-1).contiguous()
            frames.append(ops.Window(ctx, g, c1, win.opts, tc, loss="l1"))
        for w1 in frames:
            w1.step(False)
        torch.cuda.synchronize()
        reps = max(2, args.steps // 4)
        t1 = time.perf_counter()
        for _ in range(reps):
            for w1 in frames:
                w1.step(False)
        torch.cuda.synchronize()
        t_pf = (time.perf_counter() - t1) / reps
        per_frame = {"ms_per_window": round(t_pf * 1e3, 4), "mpix_s": round(P / t_pf / 1e6, 2),
                     "how": "8 sequential single-camera eager window steps, same tile and kernels"}
        log(f"per-frame plain launches {t_pf * 1e3:.3f} ms per window ({P / t_pf / 1e6:.1f} Mpix/s)")
        del frames

    copy_gbs = copy_peak_gbs(torch)
    log(f"device copy: {copy_gbs:.0f} GB/s (read + write)")

    optimize = None
    if not args.no_optimize:
        optimize = optimize_bench(ctx, ops, torch, g, win)
        log(f"optimise 10 iterations: {optimize}")

    sh3 = None
    if not args.no_sh:
        sh3 = sh_window_bench(ctx, ops, S, torch, sc, cs, target, tile)
        log(f"SH degree 3 window: {sh3}")

    win_upd = None
    if not args.no_window_update:
        win_upd = window_update_bench(ctx, ops, S, torch)
        log(f"window update: {win_upd}")

    workloads = None
    if not args.no_workloads:
        workloads = workloads_bench(ctx, ops, S, torch, 20, not args.no_cpu)
        log(f"workloads: {workloads}")

    pose_jac = None
    if not args.no_jac:
        pose_jac = pose_jacobian_bench(ctx, ops, S, torch)
        log(f"pose Jacobian batch: {pose_jac}")

    traffic = read_traffic()
    atomics = read_atomics()
    # the VALU issue ceilings the compositing kernel's instruction mix meets
    valu_ceiling = {m: round(ops.valu_probe(ctx, m), 3) for m in ops.VALU_PROBE_MODES}
    valu_insts = read_counter("SQ_INSTS_VALU")
    log(f"VALU issue ceilings (wave64 instructions per CU per 2.4-GHz cycle): {valu_ceiling}")
    result = {
        "metric": "fwd+bwd Mpixels/s at 500k Gaussians, 8-frame window; fwd ms/frame",
        "value": round(mpix, 2),
        "unit": "Mpixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_win * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched window: 500k surfel Gaussians on 50 planes, 8 keyframes 1280x1024, "
                               "L1 loss, fwd+bwd to all Gaussian parameters and the 8 poses",
                   "gaussians": sc.n, "frames": cs.C, "width": 1280, "height": 1024, "tile": tile,
                   "instances_K": K, "hip_graph": use_graph},
        "step_ms_events": step_pct,
        "fwd_ms_per_frame": round(fwd_ms / cs.C, 4),
        "fwd_how": "the window's forward render (camera upload, projection, binning, compositing of all 8 "
                   "keyframes) as gsl_window_render replayed as a HIP graph, 10 back-to-back replays after 10 untimed ÷ 8 frames",
        "fwd_ms_per_frame_eager": round(fwd_ms_eager / cs.C, 4),
        "per_frame": per_frame,
        "stage_ms": {"project": round(float(st_ms[0]), 4), "bin_sort": round(float(st_ms[1]), 4),
                     "fused_render": round(float(st_ms[2]), 4), "adjoint": round(float(st_ms[3]), 4),
                     "timing": "eager steps"},
        "stage_ms_graph": None if st_graph is None else {
            "project": round(float(st_graph[0]), 4), "bin_sort": round(float(st_graph[1]), 4),
            "fused_render": round(float(st_graph[2]), 4), "adjoint": round(float(st_graph[3]), 4),
            "total": round(float(st_graph[4]), 4),
            "timing": "replays of the profiling graph; its event nodes add their own time"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                     "traffic": None if traffic is None else int(traffic),
                     "kernel": "k_render_fused", "kernel_ms": round(fused_ms, 4),
                     "algorithmic_flops": int(flops),
                     "pairs": {"fwd_evaluated": ev_f, "contributors": n_contrib, "bwd_evaluated": ev_b,
                               "fwd_per_pixel": round(ev_f / P, 2), "contributors_per_pixel": round(n_contrib / P, 2)},
                     "atomics": None if atomics is None else {
                         "l2_requests_per_launch": int(atomics[0]), "wave_instructions_per_launch": int(atomics[1]),
                         "l2_requests_per_s": round(atomics[0] / (fused_ms * 1e-3), 0),
                         "peak_per_s": L2_ATOMIC_PEAK_PER_S,
                         "frac": round(atomics[0] / (fused_ms * 1e-3) / L2_ATOMIC_PEAK_PER_S, 4),
                         "source": "TCC_ATOMIC and TA_FLAT_ATOMIC_WAVEFRONTS per dispatch from the committed "
                                   "counter summary of the same render.hip; peak derived: one request per L2 "
                                   "channel per clock, 8 XCDs x 16 channels x 2.4 GHz"},
                     "valu_issue": {"insts_per_cu_cycle": round(valu_insts / (fused_ms * 1e-3 * 2.4e9 * 256), 3)
                                    if valu_insts else None,
                                    "ceiling_per_kind": valu_ceiling,
                                    "source": "kernel's SQ_INSTS_VALU from the committed counter summary of the "
                                              "same render.hip over its duration here; ceilings from gsl_valu_probe "
                                              "(independent chains, eight waves per SIMD)"},
                     "hbm_view": {"algorithmic_bytes": int(fused_bytes),
                                  "gbs": round(fused_bytes / (fused_ms * 1e-3) / 1e9, 1),
                                  "frac": round(fused_bytes / (fused_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}},
        "window_hbm": {"algorithmic_bytes": int(step_bytes),
                       "frac": round(step_bytes / t_win / 1e9 / HBM_PEAK_GBS, 4),
                       "copy_peak_gbs": round(copy_gbs, 1),
                       "frac_of_copy_peak": round(step_bytes / t_win / 1e9 / copy_gbs, 4)},
    }
    if workloads is not None:
        result["workloads"] = workloads
    if optimize is not None:
        result["optimize"] = optimize
    if pose_jac is not None:
        result["pose_jacobian"] = pose_jac
    if win_upd is not None:
        result["window_update"] = win_upd
    if sh3 is not None:
        result["sh3_window"] = sh3
    if tune_times is not None:
        result["autotune"] = tune_table(ops, tune_times, tile)
    if not args.no_cpu:
        log("oracle baseline on a pixel sample ...")
        result["cpu_baseline"] = cpu_baseline(sc, sc.cams, args.cpu_pixels)
        log(f"oracle: {result['cpu_baseline']}")
    print(json.dumps(result), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
