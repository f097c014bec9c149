#!/usr/bin/env python3
"""Benchmark of the batched ray-cast renderer on one MI355X.

Default (headline) workload: 4096 environments, each with one rotating LiDAR
of 64 channels x 512 azimuths in a 60-tree forest (4802 triangles per
environment), 134,217,728 rays per step.  One step = one pass of the rendering
hot path over every environment with every object treated as moving: sensor
and instance poses uploaded, every instance re-transformed, every
environment's BVH refitted, every ray generated, traversed and written
(range + segmentation) in the batched form (one persistent launch, per-XCD
device work queues, autotuned launch shape).  The reset path (a full SAH
rebuild of every BVH, done at randomisation) is timed beside it, alone and as
a step that rebuilds instead of refitting.

Prints ONE JSON line: Mrays/s (whole job), env-steps/s, the render kernel's
roofline position, the same step in the flat form (one launch, no queue), on
the two-level form (per-mesh BVHs in the mesh frame under a per-environment
instance BVH) and on the plain per-environment path, the served form at its
stated size (10^4 requests of 1-512 environments arriving at 2000 req/s,
p50/p99 latency and throughput, with the plain server on the same arrivals for
a prefix), the camera-room workload (1024 envs, 480x270) and the uneven moving
batch (2048 envs, one captured HIP graph per step) as further legs, and the
CPU oracle timed on this host on a bounded sample.  --cfg 4 times the
per-step HIP graph of the uneven moving-obstacle batch alone, --cfg 5 the
serving run alone.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s & env-steps/s (4096-env cam+LiDAR) vs plain; served p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# Vector issue capacity of MI355X: 256 CUs x 2.4 GHz, one wave64 VALU
# instruction per CU per clock (4 SIMDs x 16 lanes; the 157.3 TFLOP/s FP32
# vector peak counts packed FMAs: 256 x 2.4e9 x 64 lanes x 2 flop x 2).
VALU_PEAK_GINST = 256 * 2.4


def roofline(kernel, cfg, rays, ms_launch, b_alg):
    """Position of the render kernel: it is bound by vector instruction issue
    (the counters show HBM far from busy), so `achieved` is its wave64 VALU
    instructions per launch (SQ_INSTS_VALU from the committed counter record,
    used only while the kernel source matches it) over the launch time
    measured here; HBM traffic (FETCH_SIZE + WRITE_SIZE) gives the HBM
    fraction beside it, and the canonical traversal's bytes per ray are the
    bytes the L1/L2/Infinity-cache hierarchy serves (no HBM fraction)."""
    rec = traffic_record(kernel, cfg)
    t = ms_launch * 1e-3
    out = {"bound": "alu", "achieved": None, "peak": VALU_PEAK_GINST, "unit": "Ginst/s (wave64 VALU issue)",
           "frac": None, "traffic": None, "kernel": kernel, "units_per_launch": rays, "launch_ms": ms_launch,
           "peak_model": "256 CUs x 2.4 GHz x one wave64 VALU instruction per CU-clock",
           "counters": None if rec is None else f"profiles/traffic_{kernel}_cfg{cfg}.json",
           "cache_bytes_per_ray": b_alg, "cache_GBs": b_alg * rays / t / 1e9,
           "cache_model": "canonical full-sweep SAH BVH2 traversal: 32 B/box test + 40 B/tri test + 8 B out, "
                          "served by L1/L2/Infinity cache"}
    if rec is not None:
        valu = rec["issue"]["valu_insts_per_launch"]
        out["achieved"] = valu / t / 1e9
        out["frac"] = out["achieved"] / VALU_PEAK_GINST
        out["valu_insts_per_ray"] = valu / rays
        out["lane_utilisation"] = rec["issue"]["valu_lane_utilisation"]
        out["traffic"] = rec["bytes_per_launch"]
        out["hbm"] = {"achieved_GBs": rec["bytes_per_launch"] / t / 1e9, "peak_GBs": HBM_PEAK_GBS,
                      "frac": rec["bytes_per_launch"] / t / 1e9 / HBM_PEAK_GBS,
                      "write_bytes": rec["write_size_kib_per_dispatch"] * 1024 * rec["write_factor"]}
        out["l2_hit_rate"] = rec.get("l2_hit_rate")
    return out


WORKLOADS = {
    1: "1 env, 64x48 pinhole camera, ground + 8 boxes (98 tris)",
    2: "1024 envs x 480x270 pinhole camera, room + 40 random box/cylinder/sphere obstacles (~5.3k tris/env)",
    3: "4096 envs x 64ch x 512az rotating LiDAR (360 x 90 deg, 0.5-30 m), 60-tree forest (4802 tris/env)",
    4: "2048 envs, 5-200 boxes (30% moving, refit every step), mixed 480x270 / 240x135 cameras and 32x512 "
       "LiDAR, 100 steps as one HIP graph each",
    5: "requests of 1-512 envs (uneven box scenes, one sensor type each), Poisson arrivals, resident BVHs",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def traffic_record(kernel, cfg):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_cfg{cfg}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for src in rec.get("sources", []):
        with open(os.path.join(ROOT, src), "rb") as g:
            h.update(g.read())
    if h.hexdigest() != rec.get("sources_sha256"):
        return None
    return rec


def calibration_copy(nbytes=1 << 28):
    """A plain device copy of known size: the profiler's FETCH_SIZE / WRITE_SIZE
    for it give the scale factor from counter units to bytes."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def cpu_baseline(cfg, seconds):
    """The oracle on a bounded sample of the same workload, all host cores."""
    from oracle import oracle as O
    from paper_2503_01471_amd import scenes as S
    cores = len(os.sched_getaffinity(0))
    n_env = 1
    sc = S.make(cfg, env_ids=[0]) if cfg != 1 else S.make_cfg1()
    O.render(sc, nthreads=cores)  # warm: library load, first-touch allocations
    t0 = time.perf_counter()
    O.render(sc, nthreads=cores)
    dt = time.perf_counter() - t0
    if cfg != 1:
        n_env = max(1, min(512, int(seconds / max(dt, 1e-3))))
        sc = S.make(cfg, env_ids=list(range(n_env)))
        t0 = time.perf_counter()
        O.render(sc, nthreads=cores)
        dt = time.perf_counter() - t0
    rays = sc.total_rays()
    # the same oracle on one thread, over the first 8192 rays of the first environment
    import numpy as np
    one = S.make(cfg, env_ids=[0]) if cfg != 1 else S.make_cfg1()
    n1 = min(8192, one.total_rays())
    t0 = time.perf_counter()
    O.render(one, nthreads=1, sensor_inst=np.zeros(n1, np.int64), ray_idx=np.arange(n1, dtype=np.int64))
    dt1 = time.perf_counter() - t0
    return {"value": rays / dt / 1e6, "unit": "Mrays/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_env} env(s) of cfg{cfg}, all {rays} rays, brute-force FP64, {dt:.1f} s",
            "env_steps_per_s": n_env / dt, "cpu": cpu_model(),
            "single_thread": {"Mrays_s": n1 / dt1 / 1e6, "sample": f"{n1} rays of 1 env of cfg{cfg}, {dt1:.2f} s"}}


def per_step(fn, k):
    """Each of k calls of fn timed by its own pair of HIP events (recorded on
    the current stream, read after one synchronisation at the end): the
    distribution of the step time."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(k)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = sorted(a.elapsed_time(b) for a, b in ev)
    pick = lambda q: t[min(len(t) - 1, int(round(q * (len(t) - 1))))]
    return {"steps": k, "median": pick(0.5), "p90": pick(0.9), "min": t[0], "max": t[-1]}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def timed(fn, k):
    import torch
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(k):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / k


# --------------------------------------------------------------------------
# render-step workloads (cfg 1-3)
# --------------------------------------------------------------------------
def bench_step(args):
    import torch
    from paper_2503_01471_amd import rc, scenes
    from paper_2503_01471_amd.renderer import Renderer

    mode = {"plain": rc.RC_RENDER_PLAIN, "flat": rc.RC_RENDER_FLAT, "batched": rc.RC_RENDER_BATCHED}[args.mode]
    log(f"generating cfg{args.cfg}")
    scene = scenes.make(args.cfg)
    scene.inst_dynamic[:] = 1  # every object may move: re-transform and refit all of them each step
    # cameras become stereo pairs (second camera 9.5 cm to the right) for the stereo-shadow measurement;
    # the rendering of every other output is unaffected
    import dataclasses
    stereo = any(d.kind == scenes.PINHOLE for d in scene.sensors)
    scene.sensors = [dataclasses.replace(d, stereo=(0.0, -0.095, 0.0)) if d.kind == scenes.PINHOLE else d
                     for d in scene.sensors]
    n_envs = scene.n_envs
    log(f"loading {n_envs} envs, {int(scene.env_tri_counts().sum())} tris, {scene.total_rays()} rays")
    R = Renderer(scene, build=True)
    out = R.alloc(depth=True, seg=True)
    rays = R.total_rays
    ctx = R.ctx
    tuning = rc.rc_autotune(ctx, args.tune_cache) if (mode == rc.RC_RENDER_BATCHED and not args.no_autotune) else None
    log(f"tuning {tuning}")

    def render(m=mode):
        rc.rc_render(ctx, out["depth"], out["seg"], None, None, m, None, rays)

    def step():
        rc.rc_set_sensor_poses(ctx, R.sensor_T)
        rc.rc_set_instance_poses(ctx, R.inst_T)
        rc.rc_refit(ctx)
        render()

    def rebuild_step():
        rc.rc_set_sensor_poses(ctx, R.sensor_T)
        rc.rc_set_instance_poses(ctx, R.inst_T)
        rc.rc_build(ctx)
        render()

    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    ms = timed(step, args.steps)
    ms_render = timed(render, args.steps)
    ms_refit = timed(lambda: rc.rc_refit(ctx), args.steps)
    dist = per_step(step, args.steps)
    log(f"per step: median {dist['median']:.3f} ms, p90 {dist['p90']:.3f} ms")
    widths = None
    if tuning is not None:
        # the same launch shape with the other node width (binary nodes / four-wide records)
        alt = list(tuning)
        alt[3] = 6 - alt[3]
        rc.rc_tuning_set(ctx, *alt)
        ms_alt_render = timed(render, args.steps)
        ms_alt_step = timed(step, args.steps)
        rc.rc_tuning_set(ctx, *tuning)
        widths = {"chosen": tuning[3], "other": alt[3], "other_render_ms": ms_alt_render,
                  "other_step_ms": ms_alt_step, "render_speedup_chosen_vs_other": ms_alt_render / ms_render}
        log(f"node width {alt[3]}: render {ms_alt_render:.3f} ms, step {ms_alt_step:.3f} ms")
    # --quick (profiling runs): only the step and the render above
    ms_build = ms_rebuild_step = ms_build_lbvh = ms_render_lbvh = ms_rebuild_step_lbvh = float("nan")
    further = flat = None
    if not args.quick:
        ms_build = timed(lambda: rc.rc_build(ctx), max(2, args.steps // 2))
        ms_rebuild_step = timed(rebuild_step, max(2, args.steps // 2))
        log(f"step {ms:.3f} ms: render {ms_render:.3f} ms, transform+refit {ms_refit:.3f} ms; reset: build "
            f"{ms_build:.3f} ms, step with rebuild {ms_rebuild_step:.3f} ms")
        # the linear BVH builder (faster build, slower trees); the SAH trees are restored afterwards

        def rebuild_step_lbvh():
            rc.rc_set_sensor_poses(ctx, R.sensor_T)
            rc.rc_set_instance_poses(ctx, R.inst_T)
            rc.rc_build(ctx, rc.RC_BUILD_LBVH)
            render()

        ms_build_lbvh = timed(lambda: rc.rc_build(ctx, rc.RC_BUILD_LBVH), max(2, args.steps // 2))
        ms_render_lbvh = timed(render, args.steps)
        ms_rebuild_step_lbvh = timed(rebuild_step_lbvh, max(2, args.steps // 2))
        rc.rc_build(ctx)
        torch.cuda.synchronize()
        log(f"lbvh: build {ms_build_lbvh:.3f} ms, render {ms_render_lbvh:.3f} ms, step with rebuild "
            f"{ms_rebuild_step_lbvh:.3f} ms")
        # further data types from the same hits (Sec. III-D): normal, barycentrics, sensor-frame point and
        # vertex ids derived by a second pass from the winner ids; stereo shadows by segment tests
        xo = R.alloc(depth=True, seg=True, tri=True, normal=True, bary=True, point=True, vert=True, shadow=stereo)

        def render_tri():
            rc.rc_render(ctx, xo["depth"], xo["seg"], xo["tri"], None, mode, None, rays)

        def render_all():
            rc.rc_render(ctx, xo["depth"], xo["seg"], xo["tri"], None, mode, None, rays, normal=xo["normal"],
                         bary=xo["bary"], point=xo["point"], vert=xo["vert"])

        def render_shadow():
            rc.rc_render(ctx, xo["depth"], xo["seg"], xo["tri"], None, mode, None, rays, shadow=xo["shadow"])

        n_x = max(2, args.steps // 2)
        ms_tri = timed(render_tri, n_x)
        ms_all = timed(render_all, n_x)
        further = {"render_with_tri_ms": ms_tri, "render_with_all_further_outputs_ms": ms_all,
                   "further_outputs_pass_ms": ms_all - ms_tri,
                   "outputs": "depth, seg, tri, normal[3], bary[2], sensor-frame point[3], vertex ids[3]"}
        if stereo:
            ms_sh = timed(render_shadow, n_x)
            torch.cuda.synchronize()
            hits = int((xo["tri"] >= 0).sum())
            further.update({"render_with_stereo_shadow_ms": ms_sh, "stereo_shadow_pass_ms": ms_sh - ms_tri,
                            "stereo_baseline_m": 0.095, "shadowed_fraction_of_hits":
                            float(xo["shadow"].sum()) / max(hits, 1)})
        log(f"further outputs: {further}")
        del xo
        # FLAT: one launch over every tile, no queue (the one-launch baseline of the batched form)
        def flat_step():
            rc.rc_set_sensor_poses(ctx, R.sensor_T)
            rc.rc_set_instance_poses(ctx, R.inst_T)
            rc.rc_refit(ctx)
            render(rc.RC_RENDER_FLAT)
        ms_flat = timed(flat_step, args.steps)
        ms_flat_render = timed(lambda: render(rc.RC_RENDER_FLAT), args.steps)
        flat = {"ms_per_step": ms_flat, "Mrays_s": rays / ms_flat / 1e3, "ms_render": ms_flat_render,
                "render_Mrays_s": rays / ms_flat_render / 1e3, "speedup_batched_vs_flat": ms_flat / ms,
                "render_speedup_batched_vs_flat": ms_flat_render / ms_render}
        log(f"flat step {ms_flat:.3f} ms, flat render {ms_flat_render:.3f} ms")
        two_level = bench_two_level(args, R, render, step, mode, ms, ms_render)
    else:
        two_level = bench_two_level(args, R, render, step, mode, ms, ms_render) if args.two_level else None
    plain = None
    if not args.no_plain and not args.quick:
        def plain_step():
            rc.rc_set_sensor_poses(ctx, R.sensor_T)
            rc.rc_set_instance_poses(ctx, R.inst_T)
            rc.rc_refit(ctx)
            render(rc.RC_RENDER_PLAIN)
        ms_plain = timed(plain_step, max(2, args.steps // 4))
        ms_plain_render = timed(lambda: render(rc.RC_RENDER_PLAIN), max(2, args.steps // 4))
        plain = {"ms_per_step": ms_plain, "Mrays_s": rays / ms_plain / 1e3, "ms_render": ms_plain_render,
                 "render_Mrays_s": rays / ms_plain_render / 1e3, "speedup_batched_vs_plain": ms_plain / ms,
                 "render_speedup_batched_vs_plain": ms_plain_render / ms_render}
        log(f"plain step {ms_plain:.3f} ms, plain render {ms_plain_render:.3f} ms")
    stats = R.stats()
    from bytemodel import bytemodel
    b_ray = bytemodel.load()[f"cfg{args.cfg}"]["bytes_per_ray"]
    # the batched mode's autotuned launch form: the persistent queue, or one launch without it (tiles per pop 0)
    kernel = "k_render_batched" if mode == rc.RC_RENDER_BATCHED and (tuning is None or tuning[1] > 0) \
        else "k_render_flat"
    if args.calib:
        calibration_copy()
    result = {
        "metric": METRIC,
        "value": rays / ms / 1e3,
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"cfg{args.cfg}: {WORKLOADS[args.cfg]}", "envs": n_envs, "rays_per_step": rays,
                   "mode": args.mode, "outputs": "depth+seg", "tuning": tuning,
                   "step": "sensor + instance poses, transform of every instance, refit of every env's BVH, "
                           "batched render"},
        "env_steps_per_s": n_envs / (ms * 1e-3),
        "per_step_ms": dist,
        "render_ms": ms_render,
        "render_Mrays_s": rays / ms_render / 1e3,
        "transform_refit_ms": ms_refit,
        "reset": None if args.quick else {"sah_build_ms": ms_build, "step_with_rebuild_ms": ms_rebuild_step,
                  "step_with_rebuild_Mrays_s": rays / ms_rebuild_step / 1e3,
                  "env_steps_per_s": n_envs / (ms_rebuild_step * 1e-3),
                  "lbvh": {"build_ms": ms_build_lbvh, "render_ms_on_lbvh_trees": ms_render_lbvh,
                           "step_with_rebuild_ms": ms_rebuild_step_lbvh,
                           "step_with_rebuild_Mrays_s": rays / ms_rebuild_step_lbvh / 1e3,
                           "env_steps_per_s": n_envs / (ms_rebuild_step_lbvh * 1e-3)}},
        "flat": flat,
        "two_level": two_level,
        "plain": plain,
        "further_outputs": further,
        "traversal": {"box_tests_per_ray": stats[0] / rays, "tri_tests_per_ray": stats[1] / rays,
                      "fp64_evals_per_ray": stats[2] / rays},
        "node_width": widths,
        "roofline": roofline(kernel, args.cfg, rays, ms_render, b_ray),
        "cpu_baseline": None,
    }
    R.close()
    del out
    torch.cuda.synchronize()
    return result


def bench_two_level(args, R, render, step, mode, ms_step, ms_render):
    """The same step on the two-level form (one BVH per mesh in its own frame,
    per environment a BVH over instance boxes; rays enter each instance's
    frame): build time, step (inverse poses and instance boxes, refit of the
    instance BVH, render), render alone and the library memory the form adds.
    The single-level SAH trees are rebuilt afterwards."""
    import torch
    from paper_2503_01471_amd import rc
    ctx = R.ctx
    torch.cuda.synchronize()
    used0 = rc.rc_memory_used(ctx)
    rc.rc_build(ctx, rc.RC_BUILD_TWO_LEVEL)
    torch.cuda.synchronize()
    added = rc.rc_memory_used(ctx) - used0
    ms_build = timed(lambda: rc.rc_build(ctx, rc.RC_BUILD_TWO_LEVEL), max(2, args.steps // 2))
    tuning = rc.rc_autotune(ctx, args.tune_cache) if (mode == rc.RC_RENDER_BATCHED and not args.no_autotune) else None
    for _ in range(args.warmup):
        step()
    ms = timed(step, args.steps)
    ms_r = timed(render, args.steps)
    ms_refit = timed(lambda: rc.rc_refit(ctx), args.steps)
    stats = R.stats()
    rays = R.total_rays
    rc.rc_build(ctx)
    if tuning is not None:
        rc.rc_autotune(ctx, args.tune_cache)
    torch.cuda.synchronize()
    out = {"build_ms": ms_build, "ms_per_step": ms, "Mrays_s": rays / ms / 1e3, "render_ms": ms_r,
           "render_Mrays_s": rays / ms_r / 1e3, "inst_prep_refit_ms": ms_refit, "tuning": tuning,
           "step_vs_single_level": ms_step / ms, "render_vs_single_level": ms_render / ms_r,
           "added_library_bytes": added,
           "single_level_library_bytes": used0,
           "traversal": {"box_tests_per_ray": stats[0] / rays, "tri_tests_per_ray": stats[1] / rays,
                         "fp64_evals_per_ray": stats[2] / rays}}
    log(f"two-level: build {ms_build:.3f} ms, step {ms:.3f} ms, render {ms_r:.3f} ms, refit {ms_refit:.3f} ms, "
        f"+{added / 2**20:.1f} MiB")
    out["two_level_only"] = bench_two_level_only(args, R, rays)
    return out


def bench_two_level_only(args, R, rays):
    """The same scene loaded with RC_SCENE_TWO_LEVEL_ONLY in a context of its
    own (no per-triangle arrays of the single-level form): library memory,
    step and render (autotuned as the first context)."""
    import torch
    from paper_2503_01471_amd import rc
    from paper_2503_01471_amd.renderer import Renderer
    B = Renderer(R.scene, scene_flags=rc.RC_SCENE_TWO_LEVEL_ONLY)
    torch.cuda.synchronize()
    used = rc.rc_memory_used(B.ctx)
    out_b = B.alloc(depth=True, seg=True)
    ctx = B.ctx
    tuning = rc.rc_autotune(ctx, args.tune_cache) if not args.no_autotune else None

    def render():
        rc.rc_render(ctx, out_b["depth"], out_b["seg"], None, None, rc.RC_RENDER_BATCHED, None, rays)

    def step():
        rc.rc_set_sensor_poses(ctx, B.sensor_T)
        rc.rc_set_instance_poses(ctx, B.inst_T)
        rc.rc_refit(ctx)
        render()

    for _ in range(args.warmup):
        step()
    ms = timed(step, args.steps)
    ms_r = timed(render, args.steps)
    B.close()
    log(f"two-level only: library {used / 2**20:.1f} MiB, step {ms:.3f} ms, render {ms_r:.3f} ms")
    return {"library_bytes": used, "ms_per_step": ms, "render_ms": ms_r, "tuning": tuning,
            "Mrays_s": rays / ms / 1e3}


# --------------------------------------------------------------------------
# cfg 4: uneven batch, moving obstacles, one HIP graph per step
# --------------------------------------------------------------------------
def bench_graph(args):
    import torch
    from paper_2503_01471_amd import rc, scenes
    from paper_2503_01471_amd.renderer import Renderer

    log("generating cfg4")
    scene = scenes.make(4)
    R = Renderer(scene, build=True)
    rays, ctx = R.total_rays, R.ctx
    tuning = rc.rc_autotune(ctx, args.tune_cache) if not args.no_autotune else None
    out = R.alloc(depth=True, seg=True)
    g = rc.rc_step_graph_create(ctx, R.inst_vel, float(scene.dt), depth=out["depth"], seg=out["seg"],
                                total_rays=rays)
    n_steps = 100
    rc.rc_graph_set_step(g, 0)
    for _ in range(10):
        rc.rc_graph_launch(g)
    rc.rc_graph_set_step(g, 0)
    ms = timed(lambda: rc.rc_graph_launch(g), n_steps)
    rc.rc_graph_set_step(g, 0)
    dist = per_step(lambda: rc.rc_graph_launch(g), n_steps)
    log(f"graph step {ms:.3f} ms (per step: median {dist['median']:.3f} ms, p90 {dist['p90']:.3f} ms)")

    step = [0]

    def plain_step():
        R.move(step[0])
        R.refit()
        rc.rc_render(ctx, out["depth"], out["seg"], None, None, rc.RC_RENDER_PLAIN, None, rays)
        step[0] += 1

    ms_plain = timed(plain_step, 5)
    log(f"plain step {ms_plain:.3f} ms")
    rc.rc_graph_destroy(g)
    # the same graph on the two-level form (instance boxes refitted, no triangle transformed per step)
    used0 = rc.rc_memory_used(ctx)
    rc.rc_build(ctx, rc.RC_BUILD_TWO_LEVEL)
    torch.cuda.synchronize()
    added = rc.rc_memory_used(ctx) - used0
    tuning2 = rc.rc_autotune(ctx, args.tune_cache) if not args.no_autotune else None
    g2 = rc.rc_step_graph_create(ctx, R.inst_vel, float(scene.dt), depth=out["depth"], seg=out["seg"],
                                 total_rays=rays)
    rc.rc_graph_set_step(g2, 0)
    for _ in range(10):
        rc.rc_graph_launch(g2)
    rc.rc_graph_set_step(g2, 0)
    ms2 = timed(lambda: rc.rc_graph_launch(g2), n_steps)
    rc.rc_graph_destroy(g2)
    log(f"two-level graph step {ms2:.3f} ms")
    R.close()
    return {"metric": METRIC, "value": rays / ms / 1e3, "unit": "Mrays/s", "n_gpus": 1, "steps": n_steps,
            "warmup": 10, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"cfg4: {WORKLOADS[4]}", "envs": scene.n_envs, "rays_per_step": rays,
                       "tuning": tuning, "step": "move + transform + refit + batched render in the autotuned launch form (graph)"},
            "env_steps_per_s": scene.n_envs / (ms * 1e-3),
            "per_step_ms": dist,
            "plain": {"ms_per_step": ms_plain, "Mrays_s": rays / ms_plain / 1e3, "speedup_graph_vs_plain":
                      ms_plain / ms},
            "two_level": {"ms_per_step": ms2, "Mrays_s": rays / ms2 / 1e3, "tuning": tuning2,
                          "step_vs_single_level": ms / ms2, "added_library_bytes": added,
                          "single_level_library_bytes": used0}}


# --------------------------------------------------------------------------
# cfg 5: serving
# --------------------------------------------------------------------------
def make_requests(n_envs_pool, n_sensors, n_req, rate, seed):
    import numpy as np
    rng = np.random.default_rng(np.random.SeedSequence([seed, 5]))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
    reqs = []
    for _ in range(n_req):
        k = int(rng.integers(1, 513))
        envs = rng.choice(n_envs_pool, k, replace=False).astype(np.int32)
        reqs.append((envs, int(rng.integers(0, n_sensors))))
    return arrivals, reqs


def serve_run(R, reqs, arrivals, mode, budget, n_streams, lib_outputs):
    """Submit requests at their arrival times.  Every request gets its own
    output buffers (library outputs carved from the server's slab at
    admission); the client releases each one as soon as it has completed,
    checking its completions in submission order between arrivals."""
    from collections import deque

    import numpy as np
    from paper_2503_01471_amd import rc
    srv = rc.rc_server_create(R.ctx, mode, n_streams, budget)
    lat, pending = [], deque()
    rays = 0

    def reap(block):
        while pending:
            t = pending[0]
            if block:
                lat.append(rc.rc_server_wait(srv, t))
            else:
                done, l = rc.rc_server_poll(srv, t)
                if not done:
                    return
                lat.append(l)
            rc.rc_server_release(srv, t)
            pending.popleft()
    try:
        # the slab of library outputs is allocated by the first such request: not timed
        rc.rc_server_release(srv, _wait(rc, srv, rc.rc_server_submit(srv, reqs[0][0][:1], reqs[0][1],
                                                                    lib_outputs=lib_outputs)))
        t0 = time.perf_counter()
        for i, (envs, sid) in enumerate(reqs):
            while time.perf_counter() - t0 < arrivals[i]:
                reap(False)
                time.sleep(0)  # yield the GIL: the server's worker may call back into Python
            pending.append(rc.rc_server_submit(srv, envs, sid, lib_outputs=lib_outputs))
            rays += len(envs) * R.scene.sensors[sid].n_rays
        reap(True)
        t_end = time.perf_counter()
    finally:
        rc.rc_server_destroy(srv)
    lat = np.array(lat)
    return {"requests": len(reqs), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "Mrays_s": rays / (t_end - t0) / 1e6, "req_s": len(reqs) / (t_end - t0),
            "offered_req_s": len(reqs) / arrivals[-1], "wall_s": t_end - t0}


def _wait(rc, srv, t):
    rc.rc_server_wait(srv, t)
    return t


def bench_serve(args):
    """cfg5: the stated run (10^4 requests, Poisson arrivals at 2000 req/s) on
    the batched server, the plain per-environment server on the same arrivals
    for a prefix, a saturated burst, and a sweep below saturation where
    latency is not backlog."""
    import torch
    from paper_2503_01471_amd import rc, scenes
    from paper_2503_01471_amd.renderer import Renderer

    log("generating the resident pool (cfg4 scenes at step 0)")
    scene = scenes.make(4)
    R = Renderer(scene, build=True)
    if not args.no_autotune:
        rc.rc_autotune(R.ctx, args.tune_cache)
    torch.cuda.synchronize()
    budget, K = 0, 4  # 0: half of the device memory free when the server starts
    outs = rc.RC_OUT_DEPTH | rc.RC_OUT_SEG
    free, total = torch.cuda.mem_get_info()
    res = {"workload": f"cfg5: {WORKLOADS[5]}", "budget": "half of the free device memory at server start",
           "free_bytes_at_start": free, "streams": K, "outputs": "depth+seg, library-allocated per request"}
    # the stated arrival process: 10^4 requests at 2000 req/s, batched
    arr, reqs = make_requests(scene.n_envs, len(scene.sensors), args.requests, 2000.0, 0)
    log(f"stated run: {args.requests} requests at 2000 req/s")
    res["stated_2000_req_s"] = st = serve_run(R, reqs, arr, rc.RC_SERVE_BATCHED, budget, K, outs)
    log(f"stated: p50 {st['p50_ms']:.1f} ms p99 {st['p99_ms']:.1f} ms, {st['Mrays_s']:.0f} Mrays/s, "
        f"{st['req_s']:.0f} req/s")
    m = min(len(reqs), args.plain_requests)
    res["plain_same_arrivals"] = p = serve_run(R, reqs[:m], arr[:m], rc.RC_SERVE_PLAIN, budget, 1, outs)
    log(f"plain, first {m}: p50 {p['p50_ms']:.1f} ms p99 {p['p99_ms']:.1f} ms, {p['Mrays_s']:.0f} Mrays/s")
    # saturated throughput: a burst of requests all arriving at t = 0
    arr, reqs = make_requests(scene.n_envs, len(scene.sensors), 1000, 1e9, 1)
    sat = serve_run(R, reqs, arr, rc.RC_SERVE_BATCHED, budget, K, outs)
    mean_rays = sum(len(e) * scene.sensors[s].n_rays for e, s in reqs) / len(reqs)
    sat_req_s = sat["Mrays_s"] * 1e6 / mean_rays
    res.update({"saturated_Mrays_s": sat["Mrays_s"], "saturated_req_s": sat_req_s})
    log(f"saturated {sat['Mrays_s']:.0f} Mrays/s ({sat_req_s:.0f} req/s)")
    # below saturation, where latency is meaningful; plain server on the same arrivals
    sweep = []
    for frac in (0.25, 0.5, 0.75):
        rate = frac * sat_req_s
        n = max(40, int(rate * 3.0))
        arr, reqs = make_requests(scene.n_envs, len(scene.sensors), n, rate, 2)
        b = serve_run(R, reqs, arr, rc.RC_SERVE_BATCHED, budget, K, outs)
        m = min(n, 60)
        p = serve_run(R, reqs[:m], arr[:m], rc.RC_SERVE_PLAIN, budget, 1, outs)
        sweep.append({"load_frac": frac, "rate_req_s": rate, "batched": b, "plain_same_arrivals_first_n": p})
        log(f"load {frac}: batched p50 {b['p50_ms']:.1f} p99 {b['p99_ms']:.1f} ms; plain p50 {p['p50_ms']:.1f} "
            f"p99 {p['p99_ms']:.1f} ms")
    res["sweep"] = sweep
    R.close()
    torch.cuda.synchronize()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cfg", type=int, default=3, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--mode", default="batched", choices=["plain", "flat", "batched"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--requests", type=int, default=10000, help="cfg5 requests at the stated arrival rate")
    ap.add_argument("--plain-requests", type=int, default=150,
                    help="prefix of the same arrivals served by the plain per-environment server")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-other", action="store_true", help="cfg3 run: skip the cfg2 and cfg4 legs")
    ap.add_argument("--two-level", action="store_true", help="with --quick: time the two-level form as well")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (reused choices skip the timing)")
    ap.add_argument("--calib", action="store_true", help="also run a 256 MiB copy kernel (counter calibration)")
    ap.add_argument("--quick", action="store_true",
                    help="time the step and the render only (for profiler runs): no reset, linear-BVH, further "
                         "outputs, flat or plain legs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): environments shard across GPUs "
              "with no exchange, so N GPUs run N independent copies of the one-GPU job.", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench needs a HIP device"
    if args.cfg == 4:
        result = bench_graph(args)
    elif args.cfg == 5:
        result = {"metric": METRIC, "n_gpus": 1, "data": "synthetic", "served": bench_serve(args)}
    else:
        result = bench_step(args)
        if not args.no_serve and args.cfg == 3:
            log("served (cfg5)")
            result["served"] = bench_serve(args)
        if not args.no_other and args.cfg == 3:
            # the camera room and the uneven moving batch, same run: refit step in the three forms (cfg2)
            # and the captured 100-step graph (cfg4)
            import copy
            a2 = copy.copy(args)
            a2.cfg = 2
            log("cfg2")
            r2 = bench_step(a2)
            log("cfg4")
            r4 = bench_graph(args)
            result["other_workloads"] = {
                "cfg2": {k: r2[k] for k in ("value", "unit", "ms_per_step", "config", "env_steps_per_s", "render_ms",
                                            "render_Mrays_s", "transform_refit_ms", "per_step_ms", "flat", "two_level", "plain",
                                            "traversal", "node_width", "further_outputs")},
                "cfg4": {k: r4[k] for k in ("value", "unit", "ms_per_step", "config", "env_steps_per_s", "per_step_ms", "plain",
                                            "two_level")}}
    if not args.no_cpu and args.cfg in (1, 2, 3, 4):
        log("cpu baseline")
        result["cpu_baseline"] = cpu_baseline(args.cfg, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
