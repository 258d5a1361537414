"""Benchmark of the ray-traced Gaussian renderer on one MI355X.

A step is one pass of the whole hot path over one workload: BVH rebuild
(preprocess, Morton codes, radix sort, leaf boxes, PLOC clustering), forward render,
an L1 loss against a fixed target image, and the adjoint render producing
gradients for all five parameter groups. Inputs are resident in HBM before the
timed region. The default workload is the scene-scale one (1M Gaussians, one
1920x1080 view); --workload 3 (8 views) also times one launch per view against
the batched launch, --workload 5 runs the mesh path (reflection and shadow
rays), --workload 6 the three-bounce path with glass and a mirror.

The launch shape (hit-buffer size, grid form, packet tile) is autotuned on the
workload before timing unless --no-autotune; the timed steps replay a HIP
graph of the step unless --no-graph (the eager step is timed as well).

Prints one JSON line. `value` is forward+backward throughput in Mrays/s
(primary rays).
"""

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s fwd and fwd+bwd at 1M Gaussians, % HBM roofline, vs oracle error"

# Algorithmic FP32 work of the render kernels per unit of the library's work
# counters (an FMA is 2, min/max/compare/rcp/sqrt/exp are 1):
FLOPS_CHILD = 22.0      # child-box slab test whose box the lane's ray overlaps
FLOPS_LEAF = 90.0       # ray / ellipsoid test of a live lane at a visited leaf
FLOPS_COMPOSITE = 110.0  # composited hit (alpha recomputed + Eq. 3 step)
FLOPS_ADJOINT = 265.0    # adjoint of a composited hit (dL/dalpha + App. A.6)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=4, choices=(1, 2, 3, 4, 5, 6))
    ap.add_argument("--kbuf", type=int, default=0, help="fixed hit-buffer size (implies --no-autotune)")
    ap.add_argument("--persistent", action="store_true", help="persistent grid (implies --no-autotune)")
    ap.add_argument("--tile-width", type=int, default=0, help="packet tile width (implies --no-autotune)")
    ap.add_argument("--hit-list", type=int, default=512,
                    help="stored hit-list capacity per ray (0 = the adjoint re-traverses the BVH)")
    ap.add_argument("--paper-gradient", action="store_true",
                    help="the paper's backward variant (second threshold eps2 = --eps2); needs --hit-list >= 512")
    ap.add_argument("--eps2", type=float, default=1e-4)
    ap.add_argument("--loss", choices=("l1", "paper"), default="l1",
                    help="l1: mean L1 (gradient by torch); paper: (1 - 0.2) L2 + 0.2 D-SSIM per view (rs_loss)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rays", type=int, default=8000)
    ap.add_argument("--parity-rays", type=int, default=256)
    ap.add_argument("--profile", action="store_true",
                    help="one warm-up and one step, then a 256 MiB device copy that calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters; prints no JSON line")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the renderer shards over rays, but this build runs and reports "
              "a single MI355X only (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from synthetic import workload
    from synthetic.cameras import concat_rays
    from synthetic.scenes import jittered_target
    from paper_2501_19196_amd import renderer as R

    t0 = time.time()
    w = workload(args.workload)
    sc = w["scene"]
    o, d, views = concat_rays(w["cams"])
    views = [tuple(int(x) for x in v) for v in views]
    mesh_np = w.get("mesh")
    log(f"workload {w['name']}: {sc.n} Gaussians, {o.shape[0]} rays, {len(views)} views"
        f"{', mesh %d triangles' % mesh_np.n_tris if mesh_np is not None else ''} (setup {time.time() - t0:.1f}s)")

    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    g = R.Gaussians(*(t(a) for a in sc.arrays()))
    rays = R.Rays(t(o), t(d), views=views)
    fixed = args.kbuf or args.persistent or args.tile_width
    base = R.Params(kbuf=args.kbuf, flags=(2 if args.persistent else 0) | (16 if args.paper_gradient else 0),
                    tile_width=args.tile_width, hit_list=args.hit_list,
                    eps2=args.eps2)
    nr = o.shape[0]
    n = sc.n

    shading = None
    dm = mbvh = None
    if mesh_np is not None:
        dm = R.Mesh(t(mesh_np.verts), t(mesh_np.tris), t(mesh_np.mirror))
        mbvh = R.build_mesh_bvh(dm)
        L = w["light"]
        shading = R.Shading(light=(float(L[0]), float(L[1]), float(L[2])), max_bounces=int(w.get("bounces", 1)))
    frame = R.mesh_frame(nr, base, shading=shading) if mesh_np is not None else None

    def render(bvh, gs, p, out, state=None):
        if mesh_np is not None:
            R.render_mesh_fwd(bvh, mbvh, gs, dm, shading, rays, p, out=out, frame=frame)
        else:
            R.render_fwd(bvh, gs, rays, p, out=out, state=state)

    def adjoint(bvh, p, grad, state):
        if mesh_np is not None:
            R.render_mesh_bwd(bvh, mbvh, g, dm, shading, rays, p, grad, frame, grads=grads)
        else:
            R.render_bwd(bvh, g, rays, p, grad, state, grads=grads)

    # fixed target: the scene rendered with means jittered by N(0, 0.01)
    tsc = w.get("target") or jittered_target(sc, seed=2, sigma=0.01)
    tg = R.Gaussians(*(t(a) for a in tsc.arrays()))
    target = torch.empty((nr, 3), dtype=torch.float32, device=dev)
    render(R.build_bvh(tg, base), tg, base, target)
    del tg

    ws = torch.empty(R.workspace_bytes(n), dtype=torch.uint8, device=dev)
    out = torch.empty((nr, 3), dtype=torch.float32, device=dev)
    state = R.new_state(nr, base, dev)  # colour + T, and the stored hit lists
    grads = (torch.empty_like(g.mean), torch.empty_like(g.scale), torch.empty_like(g.quat),
             torch.empty_like(g.opacity), torch.empty_like(g.rgb))
    ev = lambda: torch.cuda.Event(enable_timing=True)

    # ---- launch shape: autotuned on this workload (plain render form)
    pf = pb = base
    tune = None
    if not fixed and not args.no_autotune and not args.profile:
        bvh = R.build_bvh(g, base, workspace=ws)
        R.render_fwd(bvh, g, rays, base, out=out, state=state)
        gr = torch.sign(out - target) * (1.0 / (3.0 * nr))
        t1 = time.time()
        pf, pb, rows = R.autotune(bvh, g, rays, base, grad_rgb=gr, reps=2)
        if mesh_np is not None:
            # the mesh forward traces the secondary ray sets in the same launch, and
            # those favour other shapes than the primaries the library timed: time
            # every shape on the launch the step makes
            best = None
            for shape in dict.fromkeys((r["kbuf"], r["persistent"], r["tile_width"]) for r in rows):
                p = dataclasses.replace(base, kbuf=shape[0], tile_width=shape[2],
                                        flags=(base.flags & ~2) | (2 if shape[1] else 0))
                render(bvh, g, p, out)
                ms = []
                for _ in range(3):
                    e0, e1 = ev(), ev()
                    e0.record()
                    render(bvh, g, p, out)
                    e1.record()
                    e1.synchronize()
                    ms.append(e0.elapsed_time(e1))
                if best is None or min(ms) < best[0]:
                    best = (min(ms), p)
            pf = best[1]
        tune = dict(fwd=dict(kbuf=pf.kbuf, persistent=bool(pf.flags & 2), tile_width=pf.tile_width),
                    bwd=dict(kbuf=pb.kbuf, persistent=bool(pb.flags & 2), tile_width=pb.tile_width),
                    candidates=len(rows), seconds=round(time.time() - t1, 2))
        log("autotune", tune)

    kt = {"build": [], "fwd": [], "bwd": []}
    lws = [R.loss_workspace(vw, vh, dev) for _, vw, vh in views] if args.loss == "paper" else None
    lval = torch.empty(max(len(views), 1), dtype=torch.float32, device=dev)
    lgrad = torch.empty((nr, 3), dtype=torch.float32, device=dev)

    def loss_grad():
        if args.loss == "l1":
            return torch.sign(out - target) * (1.0 / (3.0 * nr))  # d/dout of mean L1
        for k, (off, vw, vh) in enumerate(views):  # the paper's loss, one launch set per view
            sl = slice(off, off + vw * vh)
            R.image_loss(out[sl], target[sl], vw, vh, 0.2, ws=lws[k], out=lval[k:k + 1], grad_out=lgrad[sl])
        return lgrad

    def step(record=False):
        e = [ev() for _ in range(5)] if record else None
        if record:
            e[0].record()
        bvh = R.build_bvh(g, base, workspace=ws)
        if record:
            e[1].record()
        render(bvh, g, pf, out, state)
        if record:
            e[2].record()
        grad = loss_grad()
        if record:
            e[3].record()
        adjoint(bvh, pb, grad, state)
        if record:
            e[4].record()
        return e

    def fwd_step():
        bvh = R.build_bvh(g, base, workspace=ws)
        render(bvh, g, pf, out, None)

    if args.profile:
        step()
        torch.cuda.synchronize()
        step()
        torch.cuda.synchronize()
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = src.clone()  # reads and writes exactly 256 MiB
        torch.cuda.synchronize()
        del src, dst
        log("profile step done")
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    status = R.read_status(R.build_bvh(g, base, workspace=ws))

    def timed(fn, steps):
        s0, s1 = ev(), ev()
        torch.cuda.synchronize()
        s0.record()
        res = [fn() for _ in range(steps)]
        s1.record()
        torch.cuda.synchronize()
        return s0.elapsed_time(s1) / steps, res

    # eager steps, with per-phase events
    ms_eager, recs = timed(lambda: step(True), args.steps)
    for e in recs:
        kt["build"].append(e[0].elapsed_time(e[1]))
        kt["fwd"].append(e[1].elapsed_time(e[2]))
        kt["bwd"].append(e[3].elapsed_time(e[4]))
    ms_fwd_eager, _ = timed(fwd_step, args.steps)

    # HIP-graph replays of the same steps
    ms_graph = ms_fwd_graph = None
    if not args.no_graph:
        graphs = []
        for fn in (step, fwd_step):
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                fn()
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            gph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gph):
                fn()
            torch.cuda.synchronize()
            gph.replay()
            torch.cuda.synchronize()
            graphs.append(gph)
        ms_graph, _ = timed(graphs[0].replay, args.steps)
        ms_fwd_graph, _ = timed(graphs[1].replay, args.steps)
        step()  # leave eager results (out, grads) of the current parameters
        torch.cuda.synchronize()
    ms_step = ms_graph if ms_graph is not None else ms_eager
    ms_fwd = ms_fwd_graph if ms_fwd_graph is not None else ms_fwd_eager

    med = {k: float(np.median(v)) for k, v in kt.items()}
    mrays_fb = nr / (ms_step * 1e-3) / 1e6
    mrays_f = nr / (ms_fwd * 1e-3) / 1e6
    mrays_render = nr / (med["fwd"] * 1e-3) / 1e6

    # ---- batched multi-view launch vs one launch per view (forward and adjoint render only)
    batching = None
    if len(views) > 1 and mesh_np is None:
        bvh = R.build_bvh(g, base, workspace=ws)
        gr = torch.sign(out - target) * (1.0 / (3.0 * nr))
        # per-view slices of the ray state need the plain layout: this comparison recomputes
        pf, pb = dataclasses.replace(pf, hit_list=0), dataclasses.replace(pb, hit_list=0)
        state = torch.empty((nr, 4), dtype=torch.float32, device=dev)
        per_rays = [R.Rays(rays.origin[off:off + vw * vh], rays.direction[off:off + vw * vh],
                           views=[(0, vw, vh)]) for off, vw, vh in views]

        def per_view_fwd():
            for (off, vw, vh), rr in zip(views, per_rays):
                R.render_fwd(bvh, g, rr, pf, out=out[off:off + vw * vh], state=state[off:off + vw * vh])

        def per_view_bwd():
            for (off, vw, vh), rr in zip(views, per_rays):
                R.render_bwd(bvh, g, rr, pb, gr[off:off + vw * vh], state[off:off + vw * vh], grads=grads)

        per_view_fwd()
        ms_pv_f, _ = timed(per_view_fwd, args.steps)
        ms_pv_b, _ = timed(per_view_bwd, args.steps)
        ms_b_f, _ = timed(lambda: R.render_fwd(bvh, g, rays, pf, out=out, state=state), args.steps)
        ms_b_b, _ = timed(lambda: R.render_bwd(bvh, g, rays, pb, gr, state, grads=grads), args.steps)
        batching = dict(batched_fwd_ms=round(ms_b_f, 4), per_view_fwd_ms=round(ms_pv_f, 4),
                        batched_bwd_ms=round(ms_b_b, 4), per_view_bwd_ms=round(ms_pv_b, 4),
                        note="per-view: one render launch per view (bwd: per view, accumulating gradients "
                             "only within its own launch)")
        pf, pb = dataclasses.replace(pf, hit_list=base.hit_list), dataclasses.replace(pb, hit_list=base.hit_list)
        state = R.new_state(nr, base, dev)
        step()
        torch.cuda.synchronize()

    # ---- algorithmic FLOPs from the library's work counters (one untimed forward + adjoint)
    qf = R.Params(**{**pf.__dict__, "flags": pf.flags | 8})
    qb = R.Params(**{**pb.__dict__, "flags": pb.flags | 8})
    bvh_c = R.build_bvh(g, qf, workspace=ws)
    render(bvh_c, g, qf, out, state)
    cf = R.read_counters(bvh_c)
    adjoint(bvh_c, qb, torch.sign(out - target) * (1.0 / (3.0 * nr)), state)
    cb = {k: R.read_counters(bvh_c)[k] - cf[k] for k in cf}
    fwd_flops = FLOPS_CHILD * cf["lane_child_overlaps"] + FLOPS_LEAF * cf["lane_leaf_tests"] + \
        FLOPS_COMPOSITE * cf["lane_composited"]
    # the adjoint replays composited hits from the stored lists (r10) or by re-traversal
    bwd_flops = FLOPS_CHILD * cb["lane_child_overlaps"] + FLOPS_LEAF * cb["lane_leaf_tests"] + \
        (FLOPS_COMPOSITE + FLOPS_ADJOINT) * (cb["lane_composited"] + cb["r10"])
    dom = "bwd" if med["bwd"] >= med["fwd"] else "fwd"
    dom_flops = bwd_flops if dom == "bwd" else fwd_flops
    achieved = dom_flops / (med[dom] * 1e-3) / 1e12

    # HBM traffic per launch from committed rocprofv3 FETCH_SIZE / WRITE_SIZE passes, used
    # only when they were taken on the current render and BVH sources, this workload and,
    # for the forward, this launch shape
    traffic = None
    try:
        import hashlib
        rec = json.load(open(os.path.join(ROOT, "profiles", "render_traffic.json")))
        src = b"".join(open(os.path.join(ROOT, "paper_2501_19196_amd", "csrc", f), "rb").read()
                       for f in rec["sources"])
        lf = dict(kbuf=pf.kbuf or 24, persistent=bool(pf.flags & 2), tile_width=pf.tile_width or 8)
        if rec.get("kernel_sources_sha256") == hashlib.sha256(src).hexdigest() and rec.get("workload") == w["name"] \
                and (dom == "bwd" or rec.get("launch_fwd") == lf):
            traffic = rec[f"render_{dom}_bytes"]
    except (OSError, KeyError, ValueError):
        traffic = None

    # ---- parity on a seeded sample of pixels against the FP64 oracle, and the oracle's own rate
    err = None
    cpu = None
    try:
        from oracle import oracle as O
        f32 = lambda x: float(np.float32(x))
        op = O.Params(Q=f32(base.Q), eps1=f32(base.eps1), max_hits=base.max_hits)
        rng = np.random.default_rng(123)
        out_h = out.cpu().numpy()
        if mesh_np is not None:
            from oracle import mesh as OM
            osh = OM.Shading(light=tuple(float(np.float32(x)) for x in shading.light),
                             intensity=f32(shading.intensity), albedo=f32(shading.albedo),
                             mirror_reflectance=f32(shading.mirror_reflectance),
                             mirror_diffuse=f32(shading.mirror_diffuse), offset=f32(shading.offset),
                             max_bounces=shading.max_bounces, ior=f32(shading.ior))
            ofwd = lambda s: OM.mesh_forward(sc, mesh_np, osh, o[s], d[s], op)
        if args.parity_rays > 0:
            sel = np.sort(rng.choice(nr, args.parity_rays, replace=False))
            if mesh_np is not None:
                ref = ofwd(sel)["rgb"]
                e_abs = np.abs(out_h[sel] - ref).max(axis=1)
                err = dict(max_abs_rgb=float(e_abs.max()), within_1e4=int((e_abs <= 1e-4).sum()),
                           sampled=int(args.parity_rays),
                           note="mesh path: plain comparison (the full protocol runs in the GPU tests)")
            else:
                ref, _, _ = O.render_fwd(sc, o[sel], d[sel], op)
                res = O.compare_with_alternatives(out_h[sel], ref, sc, o[sel], d[sel], op, tol=1e-4)
                err = dict(max_abs_rgb=res["max_err"], within_1e4=res["within"], resolved=res["resolved"],
                           unresolved=len(res["unresolved"]), sampled=int(args.parity_rays))
        if not args.no_cpu_baseline:
            sel = np.sort(rng.choice(nr, args.cpu_rays, replace=False))
            gsel = (np.sign(out_h[sel] - target.cpu().numpy()[sel]) / (3.0 * nr)).astype(np.float64)
            c0 = time.time()
            if mesh_np is not None:
                f = ofwd(sel)
                c1 = time.time()
                OM.mesh_backward(sc, mesh_np, osh, o[sel], d[sel], gsel, op, fwd=f)
            else:
                O.render_fwd(sc, o[sel], d[sel], op)
                c1 = time.time()
                O.render_bwd(sc, o[sel], d[sel], gsel, op)
            c2 = time.time()
            cores = O.lib().orc_max_threads()
            cpu = dict(value=args.cpu_rays / (c2 - c0) / 1e6, unit="Mrays/s", cores=int(cores), kind="oracle",
                       sample=f"{args.cpu_rays} seeded pixels of the same views, forward + adjoint, brute force "
                              f"over all {n} Gaussians (fwd {c1 - c0:.1f}s, bwd {c2 - c1:.1f}s)",
                       fwd_value=args.cpu_rays / (c1 - c0) / 1e6)
    except Exception as e:  # the oracle is optional on the GPU machine
        log(f"oracle leg skipped: {e}")

    line = {
        "metric": METRIC,
        "value": round(mrays_fb, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["name"], "gaussians": n, "rays": nr, "views": len(views),
                   "mesh_triangles": mesh_np.n_tris if mesh_np is not None else 0,
                   "mesh_bounces": shading.max_bounces if shading is not None else 0,
                   "step": "bvh+fwd+L1+bwd", "graph": ms_graph is not None, "hit_list": base.hit_list,
                   "gradient": f"paper (eps2 {args.eps2:g})" if args.paper_gradient else "exact",
                   "loss": "mean L1" if args.loss == "l1" else "0.8 L2 + 0.2 D-SSIM (11x11, sigma 1.5)",
                   "launch_fwd": dict(kbuf=pf.kbuf or 24, persistent=bool(pf.flags & 2),
                                      tile_width=pf.tile_width or 8),
                   "launch_bwd": dict(kbuf=pb.kbuf or 24, persistent=bool(pb.flags & 2),
                                      tile_width=pb.tile_width or 8)},
        "fwd_mrays_s": round(mrays_f, 3),
        "render_only_fwd_mrays_s": round(mrays_render, 3),
        "ms_fwd_step": round(ms_fwd, 4),
        "eager_ms_per_step": round(ms_eager, 4),
        "eager_ms_fwd_step": round(ms_fwd_eager, 4),
        "kernel_ms_median": {k: round(v, 4) for k, v in med.items()},
        "roofline": {"bound": "alu", "kernel": f"render_{dom}", "achieved": round(achieved, 3), "peak": 157.3,
                     "unit": "TFLOP/s", "frac": round(achieved / 157.3, 4), "traffic": traffic,
                     "algorithmic_flops": float(dom_flops)},
        "work_per_ray": {k: round(v / nr, 2) for k, v in cf.items() if v},
        "work_per_ray_bwd": {("list_packets" if k == "r9" else "list_composited" if k == "r10" else
                              "list_grad_groups" if k == "r11" else k): round(v / nr, 3) for k, v in cb.items() if v},
        "autotune": tune,
        "batching": batching,
        "device_status": status,
        "parity": err,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
