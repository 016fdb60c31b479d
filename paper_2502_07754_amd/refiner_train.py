"""Refiner training and evaluation (the learned part; not in the paper).

Pairs come from the method's own optimisation: for each seeded scene the plain
fans are fine-tuned (pruning off, so every fine-tuned fan still lines up with
its Gaussian) against target views, and per-Gaussian least-squares targets
y* are fitted to the fine-tuned fans (msp_refiner_targets). The MLP is trained
full-batch with Adam on its float32 masters by the library's own MFMA forward
and backward kernels. Evaluation compares, on held-out scenes, the image error
of refiner-initialised fans with plain conversion (no fine-tuning), and the
wall-clock time fine-tuning needs from each start to reach the same error.

Targets: the scene (for the end-to-end comparison, a seeded perturbed copy of
it: scenes.perturbed) is converted with the multi-ring conversion (a smoother
stand-in for a Gaussian than the fan) and rendered by msp_render. Pairs come
from the unperturbed scene: a perturbation adds per-Gaussian changes that no
function of the Gaussian's own parameters predicts, and the mean of those
changes is no image-space improvement (applied to every fan it raises the
image error), whereas against the Gaussians' own ring rendering the fine-tuned
change is the systematic fan-versus-Gaussian difference the refiner can learn.

    python -m paper_2502_07754_amd.refiner_train --help
"""
from __future__ import annotations

import argparse
import json
import math
import time

from . import (MSP_LOSS_MSE, Refiner, RenderOptions, RenderState, adam_step, autotune, convert, convert_rings, loss,
               refiner_apply, refiner_apply_backward, refiner_features, refiner_loss, refiner_targets,
               refiner_weights, render, render_backward, scenes, spatial_order)
from . import _lib
from .finetune import FineTuneConfig, FineTuner

HIDDEN = 256


def views(res: int):
    """16 views: two rings of 8 at elevations +30 and -30 degrees, radius 3."""
    return scenes.ring_cameras(8, res, res, 3.0, 30.0) + scenes.ring_cameras(8, res, res, 3.0, -30.0)


def to_gpu(g: scenes.Gaussians):
    import numpy as np
    import torch
    return {k: (None if v is None else torch.from_numpy(np.ascontiguousarray(v)).cuda())
            for k, v in dict(mean=g.mean, scale=g.scale, quat=g.quat, opacity=g.opacity, rgb=g.rgb, sh=None).items()}


def target_images(g: scenes.Gaussians, cams, seed: int, ring_k=16, rings=3, perturb=True, views_per_call=16):
    """Target views: the multi-ring conversion of the (perturbed) scene, rendered
    a few views per call (the ring soup of a large scene is big)."""
    import torch
    tg = scenes.perturbed(g, seed) if perturb else g
    tf = convert_rings(to_gpu(tg), ring_k, rings, 3.0)
    out = []
    for v0 in range(0, len(cams), views_per_call):
        img, st = render(tf, cams[v0:v0 + views_per_call], RenderOptions())
        out.append(img[:, :3].clone())
        del img, st
    del tf
    return torch.cat(out).contiguous()


def make_pairs(seeds, n=12_500, K=8, sigma=2.0, steps=500, res=256, lr_color=1e-2, log=print, ref_len=0.1,
               perturb=False, deterministic=0):
    """(features, targets, loss weights) of every Gaussian of the seeded scenes."""
    import torch
    xs, ys, ws = [], [], []
    for s in seeds:
        g = scenes.gaussians(n, s, 0.01, 0.1, flat=True)
        cams = views(res)
        tgt = target_images(g, cams, s + 1, perturb=perturb)
        gg = to_gpu(g)
        faces = convert(gg, K, sigma)
        ft = FineTuner(faces, cams, tgt, FineTuneConfig(lr_color=lr_color, prune_every=0),
                       RenderOptions(deterministic=deterministic))
        l0 = None
        for i in range(steps):
            L = ft.step()
            if i == 0:
                l0 = float(L.item())
        xs.append(refiner_features(gg, K))
        ys.append(refiner_targets(gg, K, sigma, ft.faces))
        ws.append(refiner_weights(gg, K, sigma, ref_len))
        log(f"pairs: scene {s}: fine-tune loss {l0:.5f} -> {float(L.item()):.5f}")
    return torch.cat(xs), torch.cat(ys), torch.cat(ws)


def init_params(n_out, seed=0):
    """He-initialised hidden layers, zero last layer (the untrained refiner is the plain conversion)."""
    import torch
    gen = torch.Generator(device="cuda").manual_seed(seed)
    p = dict(W1=torch.randn((HIDDEN, 15), generator=gen, device="cuda") * math.sqrt(2 / 15),
             b1=torch.zeros(HIDDEN, device="cuda"),
             W2=torch.randn((HIDDEN, HIDDEN), generator=gen, device="cuda") * math.sqrt(2 / HIDDEN),
             b2=torch.zeros(HIDDEN, device="cuda"),
             W3=torch.zeros((n_out, HIDDEN), device="cuda"), b3=torch.zeros(n_out, device="cuda"))
    return {k: v.contiguous() for k, v in p.items()}


def train(x, ys, w=None, steps=400, lr=1e-3, seed=0, log=print):
    """Full-batch Adam on the float32 masters; forward/backward on the MFMA kernels.
    w: per-output loss weights (refiner_weights), so that offsets count by the
    world-space displacement they cause and colour/opacity by the fan's area."""
    import torch
    n_out = ys.shape[1]
    R = Refiner(n_out)
    p = init_params(n_out, seed)
    m = {k: torch.zeros_like(v) for k, v in p.items()}
    v = {k: torch.zeros_like(t) for k, t in p.items()}
    R.set_weights(p)
    hist = []
    for t in range(1, steps + 1):
        y = R.forward(x)
        L, dy = refiner_loss(R, y, ys, w)
        g = R.backward(x, dy)
        adam_step([dict(param=p[k], grad=g[k], m=m[k], v=v[k], lr=lr) for k in p], t)
        R.set_weights(p)
        if t == 1 or t % 50 == 0 or t == steps:
            hist.append((t, float(L.item())))
            log(f"train: step {t} loss {hist[-1][1]:.6f}")
    return R, p, hist


def scene_data(seeds, n=12_500, K=8, res=256, perturb=False):
    """Per training scene: Gaussians on the GPU, cameras, target images, refiner features."""
    out = []
    for s in seeds:
        g = scenes.gaussians(n, s, 0.01, 0.1, flat=True)
        cams = views(res)
        tgt = target_images(g, cams, s + 1, perturb=perturb)
        gg = to_gpu(g)
        out.append((gg, cams, tgt, refiner_features(gg, K)))
    return out


def train_image(data, K=8, sigma=2.0, steps=1000, lr=1e-3, seed=0, log=print, deterministic=0):
    """Trains the refiner on the fine-tuning objective itself: each step renders
    the refined fans of one training scene, takes the image MSE against its
    targets, and brings dL/dimage back through msp_render_backward, the adjoint
    of msp_refiner_apply and the MFMA backward to the weights (Adam on the
    float32 masters). The data are the method's own: the plain conversion's
    inputs and the targets its fine-tuning fits."""
    import torch
    n_out = 3 * K + 4
    R = Refiner(n_out)
    p = init_params(n_out, seed)
    m = {k: torch.zeros_like(v) for k, v in p.items()}
    v = {k: torch.zeros_like(t) for k, t in p.items()}
    R.set_weights(p)
    state = RenderState(_lib.Context.get(torch.cuda.current_device()))
    opts = RenderOptions(deterministic=deterministic)
    hist = []
    for t in range(1, steps + 1):
        gg, cams, tgt, x = data[(t - 1) % len(data)]
        y = R.forward(x)
        faces = refiner_apply(gg, K, sigma, y)
        img, st = render(faces, cams, opts, state=state)
        L, dimg = loss(img, tgt, MSP_LOSS_MSE)
        gr = render_backward(st, faces, dimg, need=("dpos", "dopacity", "drgb"))
        dy = refiner_apply_backward(gg, K, sigma, y, gr)
        gw = R.backward(x, dy)
        adam_step([dict(param=p[k], grad=gw[k], m=m[k], v=v[k], lr=lr) for k in p], t)
        R.set_weights(p)
        if t == 1 or t % 100 == 0 or t == steps:
            hist.append((t, float(L.item())))
            log(f"train (image): step {t} scene MSE {hist[-1][1]:.6f}")
    return R, p, hist


def image_mse(faces, cams, tgt) -> float:
    img, _ = render(faces, cams, RenderOptions())
    L, _ = loss(img, tgt, MSP_LOSS_MSE, want_grad=False)
    return float(L.item())


def evaluate(R, seeds, n=12_500, K=8, sigma=2.0, res=256, perturb=False):
    """Image MSE against the targets of plain and refiner-initialised fans (no fine-tuning)."""
    out = []
    for s in seeds:
        g = scenes.gaussians(n, s, 0.01, 0.1, flat=True)
        cams = views(res)
        tgt = target_images(g, cams, s + 1, perturb=perturb)
        gg = to_gpu(g)
        plain = image_mse(convert(gg, K, sigma), cams, tgt)
        y = R.forward(refiner_features(gg, K))
        refined = image_mse(refiner_apply(gg, K, sigma, y), cams, tgt)
        out.append(dict(seed=s, plain=plain, refined=refined))
    return out


def time_to_mse(g: scenes.Gaussians, cams, tgt, K=8, sigma=2.0, steps=1000, R=None, target=None, lr_color=1e-2,
                prune_every=10, opts=None, log=None):
    """Wall-clock seconds of conversion (+ refiner inference) + fine-tuning until the
    image MSE (of the render a step starts from, mean over all views) reaches
    `target`, or `steps` steps when target is None. The fine-tuning loss is the
    FineTuner's (the paper's Eq. loss by default); the stopping measure is the
    MSE. Every step synchronises once (the MSE is read back) in both modes.
    Also returned: seconds per step, and at every prune the face and vertex
    counts after it and the fragments the last render composited."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gg = to_gpu(g)
    if R is None:
        faces = convert(gg, K, sigma)
    else:
        faces = refiner_apply(gg, K, sigma, R.forward(refiner_features(gg, K)))
    ft = FineTuner(faces, cams, tgt, FineTuneConfig(lr_color=lr_color, prune_every=prune_every), opts,
                   track_mse=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter() - t0
    curve, prunes = [], []
    reached = None
    n_done = 0
    for i in range(steps):
        ft.step()
        n_done = i + 1
        lv = float(ft.last_mse.item())  # the MSE of the render this step started from
        if i % 10 == 0 or i == steps - 1:
            curve.append((i, lv, time.perf_counter() - t0))
        if prune_every and (i + 1) % prune_every == 0:
            st = ft.state.stats()
            prunes.append(dict(step=i + 1, faces=int(ft.faces["idx"].shape[1]), verts=int(ft.faces["pos"].shape[1]),
                               fragments=int(st["fragments"]), mse=lv, seconds=time.perf_counter() - t0))
        if log is not None and i % 50 == 0:
            log(f"  step {i}: MSE {lv:.6f} at {time.perf_counter() - t0:.1f} s, faces {int(ft.faces['idx'].shape[1])}")
        if target is not None and lv <= target:
            reached = i
            break
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    return dict(seconds=secs, setup_seconds=t_start, steps=(reached if reached is not None else steps),
                steps_run=n_done, seconds_per_step=(secs - t_start) / max(1, n_done),
                reached=reached is not None or target is None, final_mse=lv,
                curve=curve, prunes=prunes)


def save_params(p: dict, path: str):
    import numpy as np
    np.savez(path, **{k: v.detach().cpu().numpy() for k, v in p.items()})


def load_refiner(path: str, K=8):
    import numpy as np
    import torch
    d = np.load(path)
    p = {k: torch.from_numpy(d[k]).cuda().contiguous() for k in d.files}
    R = Refiner(3 * K + 4)
    R.set_weights(p)
    return R, p


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--train-seeds", type=int, default=20)
    ap.add_argument("--n", type=int, default=12_500)
    ap.add_argument("--pair-steps", type=int, default=500)
    ap.add_argument("--res", type=int, default=256)
    ap.add_argument("--train-steps", type=int, default=1000)
    ap.add_argument("--unweighted", action="store_true", help="plain MSE on the outputs instead of refiner_weights")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--image-steps", type=int, default=1000, help="steps of training on the fine-tuning objective")
    ap.add_argument("--image-lr", type=float, default=1e-3)
    ap.add_argument("--skip-pairs", action="store_true", help="train only on the objective; no pair comparison")
    ap.add_argument("--load-weights", default="", help="refiner weights (.npz) instead of training")
    ap.add_argument("--save-weights", default="")
    ap.add_argument("--infer-n", type=int, default=1_000_000)
    ap.add_argument("--infer-only", action="store_true",
                    help="time the inference forward of a randomly initialised refiner (no training)")
    ap.add_argument("--train-n", type=int, default=0,
                    help="samples of a timed training step (backward, and forward + backward + Adam); 0: skip")
    ap.add_argument("--ft-n", type=int, default=0, help="Gaussians of the time-to-MSE run (0: skip)")
    ap.add_argument("--ft-views", type=int, default=16)
    ap.add_argument("--ft-res", type=int, nargs=2, default=(1920, 1080))
    ap.add_argument("--ft-steps", type=int, default=1000)
    ap.add_argument("--ft-mode", choices=("both", "plain", "refined"), default="both")
    ap.add_argument("--ft-target", type=float, default=0.0, help="target MSE of a refined-only run")
    ap.add_argument("--ft-list-rows", type=int, default=0,
                    help="fragment-list rows per pixel the forward stores for the backward (0: recompute)")
    ap.add_argument("--ft-seed", type=int, default=0, help="scene seed of the time-to-MSE run (targets: seed + 1)")
    ap.add_argument("--ft-tile", type=int, nargs=2, default=(0, 0), help="tile w h (0 0: autotuned once)")
    ap.add_argument("--ft-kbuf", type=int, default=0, help="ordering-buffer depth (0: autotuned)")
    ap.add_argument("--ft-order", choices=("morton", "input"), default="morton",
                    help="storage order of the Gaussians for both runs (morton: along the Morton curve of the means)")
    ap.add_argument("--deterministic", action="store_true",
                    help="fixed-point gradient sums in the renders of training and fine-tuning (repeatable runs)")
    ap.add_argument("--skip-eval", action="store_true", help="no held-out evaluation after training")
    args = ap.parse_args()
    import statistics as st

    import torch

    def log(*a):
        print(*a, flush=True)

    res = {}
    if args.infer_only:
        p = init_params(3 * 8 + 4, seed=0)
        gen = torch.Generator(device="cuda").manual_seed(1)
        p["W3"] = (torch.randn(p["W3"].shape, generator=gen, device="cuda") * math.sqrt(2 / HIDDEN)).contiguous()
        R = Refiner(3 * 8 + 4)
        R.set_weights(p)
        args.ft_n = 0
    elif args.load_weights:
        R, p = load_refiner(args.load_weights)
    else:
        if not args.skip_pairs:
            t = time.perf_counter()
            x, ys, w = make_pairs(range(1000, 1000 + args.train_seeds), n=args.n, steps=args.pair_steps, res=args.res,
                                  log=log, deterministic=1 if args.deterministic else 0)
            res["pairs"] = dict(samples=int(x.shape[0]), faces=int(x.shape[0]) * 8, seconds=time.perf_counter() - t)
            t = time.perf_counter()
            Rs, _, hist = train(x, ys, None if args.unweighted else w, steps=args.train_steps, lr=args.lr, log=log)
            torch.cuda.synchronize()
            res["train_on_pairs"] = dict(seconds=time.perf_counter() - t, loss=hist)
            del x, ys, w
        t = time.perf_counter()
        data = scene_data(range(1000, 1000 + args.train_seeds), n=args.n, res=args.res)
        R, p, hist = train_image(data, steps=args.image_steps, lr=args.image_lr, log=log,
                                 deterministic=1 if args.deterministic else 0)
        torch.cuda.synchronize()
        res["train_on_objective"] = dict(seconds=time.perf_counter() - t, loss=hist)
        del data
        nets = [("objective", R)] + ([] if args.skip_pairs else [("pairs", Rs)])
        for key, pert in (() if args.skip_eval else (("heldout", False), ("heldout_perturbed_targets", True))):
            for name, net in nets:
                ev = evaluate(net, range(2000, 2005), n=args.n, res=args.res, perturb=pert)
                gain = [e["plain"] / e["refined"] for e in ev]
                k2 = f"{key}_{name}"
                res[k2] = dict(per_seed=ev, plain_mean=st.mean(e["plain"] for e in ev),
                               refined_mean=st.mean(e["refined"] for e in ev), ratio_mean=st.mean(gain),
                               ratio_sd=st.pstdev(gain))
                log(f"{k2}: plain {res[k2]['plain_mean']:.6f} refined {res[k2]['refined_mean']:.6f} "
                    f"(plain/refined {res[k2]['ratio_mean']:.3f} +- {res[k2]['ratio_sd']:.3f})")
        if args.save_weights:
            save_params(p, args.save_weights)
    if args.infer_n:
        # inference throughput (MFMA forward)
        g = scenes.gaussians(args.infer_n, 7, 0.01, 0.1, flat=True)
        xi = refiner_features(to_gpu(g), 8)
        R.forward(xi)
        torch.cuda.synchronize()
        t = time.perf_counter()
        reps = 10
        for _ in range(reps):
            R.forward(xi)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / reps
        flop = 2.0 * (16 * 256 + 256 * 256 + 256 * 32) * args.infer_n   # padded operands as executed
        res["inference"] = dict(n=args.infer_n, ms=dt * 1e3, tflops=flop / dt / 1e12,
                                frac_of_bf16_peak=flop / dt / 2.5e15)
        log(json.dumps(res["inference"]))
        del xi
    if args.train_n:
        # one training step on random output gradients: the MFMA backward (forward recomputed,
        # dH2, dH1, split-K weight gradients), then the whole step with Adam and the repack
        g = scenes.gaussians(args.train_n, 8, 0.01, 0.1, flat=True)
        xt = refiner_features(to_gpu(g), 8)
        gen = torch.Generator(device="cuda").manual_seed(2)
        dy = torch.randn((args.train_n, R.n_out), generator=gen, device="cuda")
        m = {k: torch.zeros_like(v) for k, v in p.items()}
        v = {k: torch.zeros_like(t) for k, t in p.items()}
        R.backward(xt, dy)
        torch.cuda.synchronize()
        reps = 10
        t = time.perf_counter()
        for _ in range(reps):
            R.backward(xt, dy)
        torch.cuda.synchronize()
        dtb = (time.perf_counter() - t) / reps
        t = time.perf_counter()
        for s in range(1, reps + 1):
            R.forward(xt)
            gr = R.backward(xt, dy)
            adam_step([dict(param=p[k], grad=gr[k], m=m[k], v=v[k], lr=1e-6) for k in p], s)
            R.set_weights(p)
        torch.cuda.synchronize()
        dts = (time.perf_counter() - t) / reps
        flop = 3 * 2.0 * (16 * 256 + 256 * 256 + 256 * 32) * args.train_n
        res["training"] = dict(n=args.train_n, backward_ms=dtb * 1e3, backward_tflops=flop / dtb / 1e12,
                               backward_frac_of_bf16_peak=flop / dtb / 2.5e15, step_ms=dts * 1e3)
        log(json.dumps(res["training"]))
        del xt, dy
    if args.ft_n:
        g = scenes.gaussians(args.ft_n, args.ft_seed, 0.01, 0.1, flat=True)
        cams = scenes.ring_cameras(args.ft_views, args.ft_res[0], args.ft_res[1])
        t = time.perf_counter()
        tgt = target_images(g, cams, args.ft_seed + 1, views_per_call=2)
        torch.cuda.synchronize()
        log(f"targets: {args.ft_views} views {args.ft_res[0]}x{args.ft_res[1]} in {time.perf_counter() - t:.1f} s")
        if args.ft_order == "morton":
            # scene preparation before both runs: neighbouring Gaussians (and so the faces
            # of a binning workgroup) stored together; the targets above are unchanged
            g = scenes.permuted(g, spatial_order(dict(mean=torch.from_numpy(g.mean).cuda())).cpu().numpy())
        # the same render options for both runs: fragment lists recomputed by the backward (the
        # workload's setting; --ft-list-rows > 0 stores them instead), the tile size and
        # ordering-buffer depth given or autotuned once on this scene and view set
        det = 1 if args.deterministic else 0
        if args.ft_tile[0] and args.ft_kbuf:
            opts = RenderOptions(tile_w=args.ft_tile[0], tile_h=args.ft_tile[1], kbuf=args.ft_kbuf,
                                 list_rows=args.ft_list_rows, deterministic=det)
        else:
            f0 = convert(to_gpu(g), 8, 2.0)
            d0 = torch.zeros((args.ft_views, 4, args.ft_res[1], args.ft_res[0]), dtype=torch.float32, device="cuda")
            opts = autotune(f0, cams, RenderOptions(list_rows=args.ft_list_rows), d0)
            opts = RenderOptions(tile_w=opts.tile_w, tile_h=opts.tile_h, kbuf=opts.kbuf, list_rows=args.ft_list_rows,
                                 deterministic=det)
            del f0, d0
        log(f"render options: tile {opts.tile_w}x{opts.tile_h}, ordering buffer {opts.kbuf}, "
            f"stored list rows {opts.list_rows} (0: recomputed), deterministic {det}")
        out = dict(n=args.ft_n, seed=args.ft_seed, views=args.ft_views, res=list(args.ft_res), steps=args.ft_steps,
                   order=args.ft_order,
                   tile=[opts.tile_w, opts.tile_h], kbuf=opts.kbuf, list_rows=opts.list_rows, deterministic=det,
                   loss="0.6 L1 + 0.4 (1 - SSIM)", stop="image MSE of the render a step starts from")
        target = args.ft_target or None
        if args.ft_mode in ("both", "plain"):
            plain = time_to_mse(g, cams, tgt, steps=args.ft_steps, opts=opts, log=log)
            log(f"plain: {plain['seconds']:.1f} s, final MSE {plain['final_mse']:.6f}, "
                f"{plain['seconds_per_step']:.4f} s/step")
            out["plain"] = plain
            target = plain["final_mse"]
        if args.ft_mode in ("both", "refined"):
            refined = time_to_mse(g, cams, tgt, steps=args.ft_steps, R=R, target=target, opts=opts, log=log)
            log(f"refined: {refined['seconds']:.1f} s to MSE {target} ({refined['steps']} steps, "
                f"{refined['seconds_per_step']:.4f} s/step)")
            out["refined"] = refined
            out["target_mse"] = target
        res["time_to_mse"] = out
    print(json.dumps(res))


if __name__ == "__main__":
    main()
