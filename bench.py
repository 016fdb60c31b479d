#!/usr/bin/env python3
"""Benchmark of the MeshSplats hot path on one MI355X.

Workload (the batched-render configuration): 500,000 flat Gaussians (means
U[-1,1]^3, two scales log-U[0.01, 0.1], third 0, uniform rotations, opacity
sigmoid(N(0,1)), colours from degree-3 SH with coefficients N(0, 0.1^2)),
converted to K = 16 fans at sigma = 2 (8,000,000 triangles; the faces are laid
out along the Morton curve of the Gaussian means, msp_spatial_order, unless
--input-order), rendered from
eight 1920x1080 views on a ring of radius 3, forward and backward with a fixed
upstream gradient dL/dimage = 1e-3 N(0, 1) (seed 3).

One step = SH colour for all views + setup/bin/sort/composite of all views +
adjoint over the fragment lists the forward stored (recomputed for 8x8 blocks
whose lists exceed --list-rows) + SH adjoint, i.e. one msp_render and one
msp_render_backward. Conversion runs once before timing. Inputs are resident
in HBM before the timed region starts.

Prints one JSON line on stdout; a per-stage breakdown goes to stderr.
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

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3           # packed FP32 (two lanes per instruction)
FP32_VECTOR_UNPACKED_TFLOPS = 78.6        # what this build can reach: it never emits packed FP32

# HBM bytes per launch (read, written) of the two heaviest kernels at the
# autotuned configuration (tile 32x16, ordering buffer 16), from rocprofv3
# --pmc FETCH_SIZE and --pmc WRITE_SIZE runs scaled by the same counters over a
# 1 GiB device copy (profiles/batched_render_8x1080p_tile32x16_kbuf16.md).
# They describe the kernel sources they were measured on: with any other
# source (hash below) or configuration the traffic is reported as null.
MEASURED_TRAFFIC = {
    "sources_sha256": "711b1a14895eb95cf7c3adcd26e98d276e4a29ff3c8edf1996cafae3087c5e68",
    "tile": [32, 16], "kbuf": 16,
    "composite": (18012911872, 9168792608),
    "bwd_grads": (9148881536, 9270458464),
}


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("paper_2502_07754_amd/csrc/raster.hip", "paper_2502_07754_amd/csrc/common.h"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


_CPU = {}


def _cpu_prepare(n: int, views: int):
    """Oracle inputs of the batched-render workload (view 0), kept in module state for forked workers."""
    import numpy as np

    from oracle import convert as oc
    from oracle import render as orr
    from oracle import sh as osh
    from paper_2502_07754_amd import scenes

    g, cams, p = scenes.config3(n=n, views=views)
    f = oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, p["K"], p["sigma"], sh=g.sh)
    f = {k: (v.astype(np.float32).astype(np.float64) if v.dtype == np.float64 else v) for k, v in f.items()}
    cam = cams[0]
    col, _ = osh.face_colours(f["sh"], f["pos"], f["idx"], cam)
    _CPU.update(f=f, cam=cam, col=col, geom=orr.face_geometry(f["pos"], f["idx"], cam),
                dimg=scenes.upstream_grad(1, cam.height, cam.width, 3, 1e-3))


def _cpu_worker(args):
    """Forward + backward of seeded pixels of the central half of view 0 until the deadline."""
    import numpy as np

    from oracle import render as orr
    from oracle import sh as osh
    wid, deadline = args
    f, cam, col, geom, dimg = (_CPU[k] for k in ("f", "cam", "col", "geom", "dimg"))
    rng = np.random.default_rng(7 + wid)
    done = 0
    while time.time() < deadline and done < 64:
        i = int(rng.integers(cam.width // 4, 3 * cam.width // 4))
        j = int(rng.integers(cam.height // 4, 3 * cam.height // 4))
        fr = orr.pixel_fragments(f, cam, i, j, geom)
        a, _, c = orr.fragment_attributes(f, fr, col)
        orr.composite(a, c, (0.0, 0.0, 0.0))
        r = orr.pixel_backward(f, cam, i, j, dimg[0, :, j, i], fr, view_col=col, geom=geom)
        osh.face_colours_backward(f["sh"][:, r["fid"]], f["pos"], f["idx"][:, r["fid"]], cam, r["dcol"].T)
        done += 1
    return done


def cpu_baseline_child(n: int, views: int, seconds: float, procs: int) -> dict:
    """Runs in a process of its own that never touches the GPU: the float64
    oracle (brute force over every face per pixel) on seeded pixels of view 0
    of the same workload, forward and backward, one forked worker per core."""
    import multiprocessing as mp
    _cpu_prepare(n, views)
    t0 = time.time()
    deadline = t0 + seconds
    with mp.get_context("fork").Pool(procs) as pool:
        counts = pool.map(_cpu_worker, [(w, deadline) for w in range(procs)])
    el = time.time() - t0
    done = int(sum(counts))
    return dict(value=done / el / 1e6, unit="Mpix/s", cores=procs, kind="oracle",
                sample=f"{done} pixels of view 0 (central half), forward + backward, brute force over all "
                       f"{_CPU['f']['idx'].shape[1]} faces per pixel, float64, {procs} processes, {el:.1f} s")


def cpu_baseline(n: int, views: int, seconds: float) -> dict:
    """The oracle leg, started as a child process (the GPU process only waits for its JSON line)."""
    import subprocess
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", "--n", str(n), "--views", str(views),
           "--cpu-seconds", str(seconds), "--cpu-procs", str(procs)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=seconds + 600)
    if r.returncode != 0:
        raise RuntimeError(f"cpu baseline failed: {r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])


def copy_bandwidth(gib: float, reps: int):
    """A plain copy kernel of known size: its HBM counters calibrate the
    FETCH_SIZE / WRITE_SIZE readings, its rate is the achievable copy bandwidth."""
    import torch
    n = int(gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 2 * 4 * n
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "ms_per_copy": ms,
                      "GB_per_s": nbytes / (ms * 1e-3) / 1e9}), flush=True)


def bench_rays(args):
    """Secondary rays through the faces of the batched-render scene: one step is
    a transmittance query over R shadow segments (to a point light) and a
    closest-hit query over R incoherent rays, both against one hierarchy."""
    import numpy as np
    import torch

    import paper_2502_07754_amd as msp
    from paper_2502_07754_amd import scenes

    dev = torch.device("cuda:0")
    g, _, p = scenes.config3(n=args.n, views=1, width=64, height=64)
    gg = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in
          dict(mean=g.mean, scale=g.scale, quat=g.quat, opacity=g.opacity, rgb=g.rgb).items()}
    faces = msp.convert(gg, p["K"], p["sigma"])
    R = args.rays
    shadow = [torch.from_numpy(a).to(dev) for a in scenes.shadow_rays(R, 0)]
    scatter = [torch.from_numpy(a).to(dev) for a in scenes.scatter_rays(R, 1)]
    ev = lambda: torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    b0, b1 = ev(), ev()
    b0.record()
    bvh = msp.Bvh(faces)
    b1.record()
    torch.cuda.synchronize()
    build_ms = b0.elapsed_time(b1)
    log(f"hierarchy over {faces['idx'].shape[1]} faces built in {build_ms:.2f} ms")

    def step(times=None):
        # rays are traced in the Morton order of their origins (computed inside the step)
        e = [ev() for _ in range(3)]
        e[0].record()
        T = bvh.transmittance(*shadow, t_eps=1e-6, order=msp.point_order(shadow[0]))
        e[1].record()
        hit = bvh.closest(*scatter, alpha_min=0.0, order=msp.point_order(scatter[0]))
        e[2].record()
        if times is not None:
            times.append(e)
        return T, hit

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st0 = bvh.status()
    times = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(times)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    st1 = bvh.status()
    ms_T = sum(e[0].elapsed_time(e[1]) for e in times) / args.steps
    ms_C = sum(e[1].elapsed_time(e[2]) for e in times) / args.steps
    T, hit = step()
    torch.cuda.synchronize()
    occl = float((T < 1).float().mean())
    hits = float((hit[1] >= 0).float().mean())
    visits = (st1["node_visits"] - st0["node_visits"]) / args.steps
    leaf = (st1["leaf_tests"] - st0["leaf_tests"]) / args.steps
    log(f"transmittance {ms_T:.3f} ms, closest {ms_C:.3f} ms per query; occluded {occl:.3f}, hit {hits:.3f}; "
        f"per ray {visits / (2 * R):.1f} node visits, {leaf / (2 * R):.1f} leaf tests")
    # algorithmic bytes of the dominant query: 64-byte node and leaf records per visit, ray in/out
    dom, dom_ms = ("trace_closest", ms_C) if ms_C >= ms_T else ("trace_transmittance", ms_T)
    nbytes = 64.0 * (visits + leaf) / 2 + R * (32 + (16 if dom == "trace_closest" else 4))
    roof = dict(bound="hbm", achieved=nbytes / (dom_ms * 1e-3) / 1e9, peak=HBM_PEAK_GBS, unit="GB/s", traffic=None)
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = dom
    roof["ms_per_launch"] = dom_ms
    roof["timing"] = "hip events on the query stream over the timed steps"
    out = {
        "metric": "Mrays/s (shadow transmittance + closest hit) through the converted soup",
        "value": 2 * R / dt / 1e6, "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.n} flat Gaussians, one fan of K={p['K']}, {faces['idx'].shape[1]} faces; "
                               f"{R} shadow segments to a point light and {R} isotropic rays per step",
                   "rays_per_query": R, "ray_order": "morton of the origins", "build_ms": build_ms, "transmittance_ms": ms_T, "closest_ms": ms_C,
                   "occluded_fraction": occl, "hit_fraction": hits,
                   "node_visits_per_ray": visits / (2 * R), "leaf_tests_per_ray": leaf / (2 * R)},
        "roofline": roof,
    }
    print(json.dumps(out), flush=True)


def stage_roofline(stages: dict, steps: int, st: dict, F: int, views: int) -> dict:
    """Per timed stage: duration per launch and its algorithmic work against the
    roofline that bounds it. Work per unit (flop or bytes the method needs, not
    what the kernel happens to move):
      composite   8 flop per (face, pixel of its footprint) coverage test + 60 per composited fragment
      bwd_grads   120 flop per fragment (adjoint recurrence, barycentrics, ray/triangle Jacobian)
      bwd_lists   as composite (the forward's ordering recomputed)
      setup       12 B indices + 36 B corners + 48 B record per (view, face)
      emit        8 B per tile entry + 16 B footprint per (view, face)
      sort        16 B per tile entry (read + write)
      sh_eval     192 B coefficients + 36 B corners per face + 16 B colour per (view, face)
      sh_bwd      192 B coefficients in + 192 B out + 36 B corners per face + 16 B per (view, face)
    The arithmetic stages are priced against the FP32 vector peak (packed), with
    the unpacked peak this build can reach beside it."""
    frags, entries, fp = st["fragments"], st["entries"], st["footprint_pixels"]
    work = {
        "composite": ("alu", 8.0 * fp + 60.0 * frags),
        "bwd_lists": ("alu", 8.0 * fp + 60.0 * frags),
        "bwd_grads": ("alu", 120.0 * frags),
        "setup": ("hbm", 96.0 * F * views),
        "emit": ("hbm", 8.0 * entries + 16.0 * F * views),
        "sort": ("hbm", 16.0 * entries),
        "sh_eval": ("hbm", (192.0 + 36.0 + 16.0 * views) * F),
        "sh_bwd": ("hbm", (384.0 + 36.0 + 16.0 * views) * F),
    }
    out = {}
    for name, (ms_sum, calls) in stages.items():
        if not calls or name not in work:
            continue
        ms = ms_sum / calls
        bound, amount = work[name]
        per_launch = amount  # every launch of a stage covers the whole step (all views)
        if bound == "alu":
            ach = per_launch / (ms * 1e-3) / 1e12
            d = dict(bound="alu", achieved=ach, peak=FP32_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                     frac=ach / FP32_VECTOR_PEAK_TFLOPS, peak_unpacked=FP32_VECTOR_UNPACKED_TFLOPS,
                     frac_unpacked=ach / FP32_VECTOR_UNPACKED_TFLOPS, flop_per_launch=per_launch)
        else:
            ach = per_launch / (ms * 1e-3) / 1e9
            d = dict(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                     bytes_per_launch=per_launch)
        d["ms"] = ms
        d["calls"] = calls // max(1, steps)
        out[name] = d
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=500_000, help="Gaussians")
    ap.add_argument("--views", type=int, default=8)
    ap.add_argument("--tile", type=int, default=0, help="tile width (and height unless --tile-h); 0: autotuned")
    ap.add_argument("--tile-h", type=int, default=0, help="tile height (default: --tile)")
    ap.add_argument("--kbuf", type=int, default=0, help="0: autotuned")
    ap.add_argument("--no-graph", action="store_true", help="eager calls instead of the captured step")
    ap.add_argument("--list-rows", type=int, default=128,
                    help="fragment-list rows per pixel the forward stores for the backward (0: recompute)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--scene", choices=("flat", "3d", "prior", "rays"), default="flat",
                    help="flat: the batched-render scene; 3d: the same count of 3D Gaussians, scales "
                         "log-U[0.005, 0.05] on all three axes; prior: mesh-prior mode, secondary triangles "
                         "on an icosphere geometry mesh (positions from their logits and the logits' "
                         "adjoint inside every step); rays: secondary rays through the batched-render "
                         "scene's faces (hierarchy build, shadow transmittance and closest hit)")
    ap.add_argument("--rays", type=int, default=4 * 1920 * 1080,
                    help="rays per query for --scene rays (shadow segments and as many incoherent rays)")
    ap.add_argument("--prior-level", type=int, default=7, help="icosphere subdivision level (20 4^level faces)")
    ap.add_argument("--prior-n", type=int, default=2, help="secondary triangles per mesh face: n^2")
    ap.add_argument("--fan3", action="store_true",
                    help="convert with three fans per Gaussian (3D-Gaussian conversion) instead of one")
    ap.add_argument("--rgb", action="store_true",
                    help="per-vertex RGB colours instead of degree-3 SH (the colour mode of fine-tuning)")
    ap.add_argument("--deterministic", action="store_true",
                    help="fixed-point gradient sums (identical bits on every run) instead of float atomics")
    ap.add_argument("--input-order", action="store_true",
                    help="convert the Gaussians in their drawn order instead of the spatial (Morton) order")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="only time a plain device-to-device copy of this many GiB (bandwidth and "
                         "HBM-counter calibration) and exit")
    ap.add_argument("--cpu-baseline-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-procs", type=int, default=1, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_baseline_child:
        print(json.dumps(cpu_baseline_child(args.n, args.views, args.cpu_seconds, args.cpu_procs)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_gib > 0:
        copy_bandwidth(args.copy_gib, max(1, args.steps))
        return

    if args.scene == "rays":
        bench_rays(args)
        return

    import paper_2502_07754_amd as msp
    from paper_2502_07754_amd import _lib, scenes

    W, H = 1920, 1080
    g, cams, p = scenes.config3(n=args.n, views=args.views, width=W, height=H)
    K, sigma = p["K"], p["sigma"]
    if args.scene == "3d":
        g = scenes.gaussians(args.n, 0, 0.005, 0.05, flat=False, sh=True)
    dev = torch.device("cuda:0")
    gg = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in
          dict(mean=g.mean, scale=g.scale, quat=g.quat, opacity=g.opacity, rgb=g.rgb, sh=g.sh).items()}
    ctx = _lib.Context.get(0)
    ctx.timing(True)
    mesh = None
    prep_ms = {}
    if args.scene == "prior":
        m = scenes.icosphere(args.prior_level, 0)
        mesh = {k: torch.from_numpy(v).to(dev) for k, v in dict(pos=m.pos, idx=m.idx, rgb=m.rgb).items()}
        faces, logits = msp.prior_init(mesh, args.prior_n, shrink=0.05, opacity0=0.5)
        dlogits = torch.empty_like(logits)
        cm = msp.MSP_COLOR_RGB
    else:
        # the same scene with its faces laid out along the Morton curve of the Gaussian means
        torch.cuda.synchronize()
        t_c = time.perf_counter()
        order = None if args.input_order else msp.spatial_order(gg)
        torch.cuda.synchronize()
        t_o = time.perf_counter()
        if args.rgb:
            gg.pop("sh", None)
        faces = msp.convert(gg, K, sigma, mode=msp.MSP_FAN_3D if args.fan3 else msp.MSP_FAN_FLAT, order=order)
        torch.cuda.synchronize()
        prep_ms = dict(spatial_order_ms=(t_o - t_c) * 1e3, convert_ms=(time.perf_counter() - t_o) * 1e3)
        cm = msp.MSP_COLOR_RGB if args.rgb else msp.MSP_COLOR_SH3
    dimg = torch.from_numpy(scenes.upstream_grad(args.views, H, W, 3, 1e-3)).to(dev)
    th = args.tile_h or args.tile
    det = 1 if args.deterministic else 0
    opts = msp.RenderOptions(tile_w=args.tile, tile_h=th, kbuf=args.kbuf, t_eps=1e-6, color_mode=cm,
                             list_rows=args.list_rows, deterministic=det)
    if args.tile == 0 or args.kbuf == 0:
        t0 = time.perf_counter()
        tuned = msp.autotune(faces, cams, opts, dimg)
        log(f"autotuned tile {tuned.tile_w}x{tuned.tile_h}, kbuf {tuned.kbuf} in {time.perf_counter() - t0:.1f} s")
        opts = msp.RenderOptions(tile_w=args.tile or tuned.tile_w, tile_h=th or tuned.tile_h,
                                 kbuf=args.kbuf or tuned.kbuf, t_eps=1e-6, color_mode=cm, list_rows=args.list_rows,
                                 deterministic=det)
    state = msp.RenderState(ctx)
    if args.no_graph:
        def step():
            img, _ = msp.render(faces, cams, opts, state=state)
            grads = msp.render_backward(state, faces, dimg)
            return img, grads
    else:
        gstep = msp.GraphStep(faces, cams, opts)
        gstep.dimg.copy_(dimg)
        state = gstep.state

        def step():
            return gstep()

    if mesh is not None:
        render_step = step

        def step():
            msp.prior_vertices(mesh, args.prior_n, logits, out=faces["pos"])
            img, grads = render_step()
            msp.prior_backward(mesh, args.prior_n, logits, grads["dpos"], out=dlogits)
            return img, grads

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.read_timing()  # discard warm-up stage times
    log(f"warm-up done ({args.warmup} steps)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = ctx.read_timing()  # graph replays carry their own event-record nodes
    timing_src = "hip events over the timed steps"
    if not any(c for _, c in stages.values()):
        # no stage events came back from the replays: time one eager step instead
        img, st_ = msp.render(faces, cams, opts)
        msp.render_backward(st_, faces, dimg)
        torch.cuda.synchronize()
        stages = ctx.read_timing()
        stages = {k: (v[0] * args.steps, v[1] * args.steps) for k, v in stages.items()}
        timing_src = "hip events of one eager step after the timed steps"
    if not args.no_graph:
        log(f"graph: {gstep.info()}")
    st = state.stats()
    dt = (t1 - t0) / args.steps
    pix = args.views * W * H
    value = pix / dt / 1e6
    for name, (ms, calls) in sorted(stages.items(), key=lambda kv: -kv[1][0]):
        if calls:
            log(f"  {name:10s} {ms / calls:9.3f} ms/launch x {calls // args.steps}/step")
    log(f"stats: {st}")

    # dominant kernel and its algorithmic work
    frags, entries = st["fragments"], st["entries"]
    per_kernel = stage_roofline(stages, args.steps, st, int(faces["idx"].shape[1]), args.views)
    dom = max(per_kernel, key=lambda k: per_kernel[k]["ms"] * per_kernel[k]["calls"])
    roof = {k: v for k, v in per_kernel[dom].items() if k not in ("ms", "calls")}
    roof["traffic"] = None
    mt = MEASURED_TRAFFIC
    if (dom in mt and args.scene == "flat" and not args.fan3 and not args.input_order and not args.rgb
            and not args.deterministic and kernel_sources_sha256() == mt["sources_sha256"]
            and [opts.tile_w, opts.tile_h] == mt["tile"] and opts.kbuf == mt["kbuf"] and args.n == 500_000
            and args.views == 8):
        roof["traffic"] = float(sum(mt[dom]))
    roof["kernel"] = dom
    roof["ms_per_launch"] = per_kernel[dom]["ms"]
    roof["timing"] = timing_src
    # every stage against its own roofline, and the step's time-weighted fraction
    tot = sum(v["ms"] * v["calls"] for v in per_kernel.values())
    roof["path_frac"] = sum(v["ms"] * v["calls"] * v["frac"] for v in per_kernel.values()) / tot if tot else None
    roof["per_kernel"] = per_kernel
    for name, v in sorted(per_kernel.items(), key=lambda kv: -kv[1]["ms"] * kv[1]["calls"]):
        log(f"  roofline {name:10s} {v['ms']:8.3f} ms  {v['achieved']:10.2f} {v['unit']:8s} frac {v['frac']:.4f}")
    log(f"  time-weighted path fraction {roof['path_frac']:.4f}")

    if mesh is not None:
        workload = (f"mesh prior: icosphere level {args.prior_level} ({mesh['idx'].shape[1]} faces), "
                    f"{args.prior_n ** 2} secondary triangles per face, RGB, {args.views} views {W}x{H}, "
                    f"secondary positions + fwd + bwd + logit adjoint")
    else:
        workload = (f"{args.n} {'flat' if args.scene == 'flat' else '3D'} Gaussians, "
                    f"{'three fans' if args.fan3 else 'one fan'} of K={K}, sigma={sigma}, "
                    f"{'RGB' if args.rgb else 'SH degree 3'}, "
                    f"{args.views} views {W}x{H}, fwd+bwd")
    out = {
        "metric": "Mpix/s fwd+bwd at 1080p, 500k Gaussians K=16; fine-tune s to target MSE",
        "value": value, "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload, "views": args.views, "width": W, "height": H,
                   "faces": int(faces["idx"].shape[1]), "tile": [opts.tile_w, opts.tile_h], "kbuf": opts.kbuf,
                   "hip_graph": not args.no_graph, "stored_lists_rows": args.list_rows,
                   "deterministic_sums": bool(args.deterministic),
                   "face_order": "input" if (args.input_order or mesh is not None) else "morton",
                   "entries_per_step": entries, "fragments_per_step": frags,
                   "fragments_per_s": frags / dt, "entries_per_s": entries / dt, **prep_ms},
        "roofline": roof,
    }
    if not args.no_cpu_baseline and args.scene == "flat" and not args.fan3 and not args.rgb:
        log("timing the oracle on a sample ...")
        out["cpu_baseline"] = cpu_baseline(args.n, args.views, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
