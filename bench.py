"""Benchmark: training iterations/s of the splatting operator on one MI355X.

Workload (mobile-budget training loop): 300k Gaussians seeded by PCA seeding
from a 300k-point noisy cloud of the synthetic spheres-and-planes scene,
1920x1440 ring cameras, targets rendered from a 500k-Gaussian ground truth,
loss 0.8 L1 + 0.2 (1 - SSIM), Adam, FP32.  One step = project -> bin/sort ->
composite with replay trace -> loss -> replay backward -> projection
backward -> Adam, on one training camera (cycling a seeded shuffle).

Prints one JSON line.  `--gpus N` with N > 1 is refused: the framework runs on
one GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "fwd+bwd iters/s, 300k Gaussians @1920x1440; PSNR@500 it learned vs plain init"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--backward", choices=["cached", "recompute"], default="cached")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the other backward variant")
    ap.add_argument("--gaussians", type=int, default=300_000)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1440)
    ap.add_argument("--views", type=int, default=0, help="training views to render targets for (0: all 52)")
    ap.add_argument("--no-psnr", action="store_true", help="skip the 500-step PSNR runs")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched multi-view step (1M Gaussians, 8 views, SH 3, tuned)")
    ap.add_argument("--batched-gaussians", type=int, default=1_000_000)
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched multi-view step, untuned 16x16 tiles / batch 256, 6 replays "
                         "(for rocprofv3)")
    ap.add_argument("--no-ba", action="store_true", help="skip the bundle-adjustment measurement")
    ap.add_argument("--ba-only", action="store_true", help="only the bundle-adjustment measurement")
    ap.add_argument("--no-mvs", action="store_true", help="skip the multi-view stereo measurement")
    ap.add_argument("--mvs-only", action="store_true", help="only the multi-view stereo measurement")
    ap.add_argument("--no-capture", action="store_true", help="skip the captures-to-model run")
    ap.add_argument("--capture-only", action="store_true", help="only the captures-to-model run")
    ap.add_argument("--no-cfg2", action="store_true",
                    help="skip the 100k / SH 3 / 1024x768 cached-vs-recompute comparison")
    ap.add_argument("--profile", action="store_true",
                    help="for rocprofv3: the headline training step only (its timed steps and the per-stage "
                         "pass), then one 1 GiB stream copy")
    ap.add_argument("--work-log", default=None,
                    help="write the pair count, trace entries and pixels of every compositing launch of the "
                         "training step here (JSON; synchronises after each launch)")
    ap.add_argument("--no-atomic", action="store_true", help="skip the float-atomic reference")
    ap.add_argument("--cpu-worker", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.profile:
        args.no_compare = args.no_cpu_baseline = args.no_psnr = args.no_batched = args.no_cfg2 = True
        args.no_ba = args.no_mvs = args.no_capture = args.no_atomic = True
    return args


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_times(trainer, steps, order, cams, targets):
    """Per-stage times (HIP events recorded on the compute stream) and the
    work (pair count P, trace entries E, pixels) of each of `steps` steps:
    (mean ms per stage, per-step records {P, E, pixels, view, ms: {stage}})."""
    import torch
    acc, recs = {}, []
    for k in range(steps):
        trainer.events = []
        cid = order[k % len(order)]
        trainer.rast.log_tag = int(cid)
        trainer.step(cams[cid], targets[cid])
        torch.cuda.synchronize()
        evs = trainer.events
        ms = {b: ea.elapsed_time(eb) for (a, ea), (b, eb) in zip(evs[:-1], evs[1:])}
        for b, v in ms.items():
            acc.setdefault(b, []).append(v)
        w = trainer.rast.work()
        w.update(view=int(cid), ms=ms)
        recs.append(w)
    trainer.events = None
    return {k: float(np.mean(v)) for k, v in acc.items()}, recs


def run_variant(wl, cached, steps, warmup, order, full_clear=False, work_log=None, trace_words=None):
    """The training step timed over `steps` steps after `warmup` (cycling the
    training views), then its per-stage times and work over min(20, steps)
    more steps.  full_clear=True zeroes the whole replay trace (entries and
    masks) inside every step before its forward: the ablation against the
    counter reset the step otherwise relies on.  trace_words picks the
    replay-trace entry layout (3: C_in only, the default; 4: C_in and alpha)."""
    import torch
    from paper_2601_17354_amd.train import Trainer
    tr = Trainer(wl["params0"].clone(), 0, wl["width"], wl["height"], cached=cached, lam=0.2,
                 extent=4.5, trace_words=trace_words)
    targets = wl["targets"]
    if work_log is not None:
        tr.rast.work_log = work_log
    # size buffers on every training view (synchronises), then warm up
    tr.rast.log_phase = "prepare"
    for cid in order:
        tr.rast.log_tag = int(cid)
        tr.prepare(wl["cams"][cid])
    tr.rast.reserve(2.0)
    full = [tr.rast.trace["entry"], tr.rast.trace["mask"]] if (full_clear and cached) else []

    def one(k):
        cid = order[k % len(order)]
        tr.rast.log_tag = int(cid)
        for t in full:
            t.zero_()
        tr.step(wl["cams"][cid], targets[cid])
        return cid

    tr.rast.log_phase = "warmup"
    for k in range(warmup):
        one(k)
    torch.cuda.synchronize()
    tr.rast.flags.zero_()
    tr.rast.log_phase = "timed"
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    last = None
    for k in range(steps):
        last = one(warmup + k)
        evs[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = evs[0].elapsed_time(evs[-1]) / steps
    per_step = np.array([a.elapsed_time(b) for a, b in zip(evs[:-1], evs[1:])])
    flags = tr.rast.read_flags()
    if flags:
        raise RuntimeError(f"buffer overflow during the timed region (flags={flags})")
    out = dict(ms=ms, wall_s=wall, trainer=tr, last_cam=wl["cams"][last],
               pct={f"p{q}": float(np.percentile(per_step, q)) for q in (10, 50, 90)})
    if full_clear:
        out["cleared_bytes"] = sum(t.numel() * t.element_size() for t in full)
        return out
    out["entry_bytes"] = 4 * tr.rast.trace_words if cached else 0
    tr.rast.log_phase = "stages"
    per, recs = kernel_times(tr, min(20, steps), order, wl["cams"], targets)
    tr.rast.log_phase = None
    r = tr.rast
    out.update(kernels=per, work=recs,
               stats=dict(pairs=int(np.mean([w["P"] for w in recs])), entries=int(np.mean([w["E"] for w in recs])),
                          visible=int((r.radius > 0).sum().item()), pixels=r.W * r.H, n=tr.n,
                          trace_gb=r.trace_bytes() / 1e9, capacity=r.capacity, loss=float(tr.loss.item()),
                          work_steps=len(recs)))
    return out


def variants_ab(params, wl, order, views=20, reps=5):
    """The backward variants on one model state, interleaved: in each of
    `reps` rounds, for each of the first `views` training views, one step
    without the Adam update (project .. project_bwd) of every variant in
    turn, so that drifting clocks or state affect all of them alike.  The
    variants: the replay trace with 12-byte entries (C_in; alpha recomputed
    in the backward), with 16-byte entries (C_in and alpha), and the
    recompute-T backward without a trace.  Returns per variant the median
    and mean time of each stage and the trace size."""
    import torch
    from paper_2601_17354_amd.train import Trainer
    kinds = {"cached_12B_entries": dict(cached=True, trace_words=3),
             "cached_16B_entries": dict(cached=True, trace_words=4),
             "recompute": dict(cached=False)}
    trs = {}
    for name, kw in kinds.items():
        tr = Trainer(params.detach().clone(), 0, wl["width"], wl["height"], lam=0.2, extent=4.5, **kw)
        for cid in order[:views]:
            tr.prepare(wl["cams"][cid])
        tr.rast.reserve(2.0)
        tr.rast.flags.zero_()
        trs[name] = tr
    acc = {name: {} for name in kinds}
    for _ in range(reps):
        for cid in order[:views]:
            for name, tr in trs.items():
                tr.events = []
                tr.step(wl["cams"][cid], wl["targets"][cid], adam=False)
                torch.cuda.synchronize()
                evs = tr.events
                for (_, ea), (b, eb) in zip(evs[:-1], evs[1:]):
                    acc[name].setdefault(b, []).append(ea.elapsed_time(eb))
    out = {"views": views, "rounds": reps, "state": "parameters after the timed steps; no Adam update"}
    for name, tr in trs.items():
        if tr.rast.read_flags():
            raise RuntimeError(f"buffer overflow in variant {name}")
        med = {k: float(np.median(v)) for k, v in acc[name].items()}
        out[name] = {"median_ms": med, "mean_ms": {k: float(np.mean(v)) for k, v in acc[name].items()},
                     "sum_of_medians_ms": float(sum(med.values())), "trace_gb": tr.rast.trace_bytes() / 1e9}
        tr.events = None
    del trs
    torch.cuda.empty_cache()
    return out


def graph_runs(wl, order, steps, warmup, views=20):
    """The cached training step recorded as HIP graphs through the library's
    graph calls (one graph per training view, the camera being a kernel
    argument; Adam's step counter on the device) and replayed cycling the
    views, against the same steps enqueued one call at a time, both from the
    same state."""
    import torch
    from paper_2601_17354_amd import binding as B
    from paper_2601_17354_amd.train import Trainer
    ids = order[:views]
    cams, targets = wl["cams"], wl["targets"]
    tr = Trainer(wl["params0"].clone(), 0, wl["width"], wl["height"], cached=True, lam=0.2, extent=4.5,
                 device_step_counter=True)
    for cid in ids:
        tr.prepare(cams[cid])
    tr.rast.reserve(2.0)
    for k in range(warmup):
        cid = ids[k % len(ids)]
        tr.step(cams[cid], targets[cid])
    torch.cuda.synchronize()
    tr.rast.flags.zero_()
    state = (tr.params, tr.m, tr.v, tr.adam_state)
    snap = [t.clone() for t in state]

    def timed(run):
        for dst, src in zip(state, snap):
            dst.copy_(src)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for k in range(steps):
            run(k)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    # the eager steps first: after a capture, event-timed eager steps have
    # read slower than their kernels
    ms_eager = timed(lambda k: tr.step(cams[ids[k % len(ids)]], targets[ids[k % len(ids)]]))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graphs = []
    with torch.cuda.stream(side):
        for cid in ids:
            B.pgs_graph_begin(side)
            try:
                tr.step(cams[cid], targets[cid])
            finally:
                graphs.append(B.pgs_graph_end(side))
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    ms_graph = timed(lambda k: B.pgs_graph_launch(graphs[k % len(graphs)]))
    flags = tr.rast.read_flags()
    for g in graphs:
        B.pgs_graph_destroy(g)
    del tr
    torch.cuda.empty_cache()
    if flags:
        raise RuntimeError(f"buffer overflow during the graph timing (flags={flags})")
    return {"views": len(ids), "steps": steps, "ms_per_step_graph": ms_graph, "ms_per_step_eager": ms_eager,
            "state": f"after {warmup} eager steps, both from the same parameters and Adam state"}


def trace_clear_ablation(tr, reps=5):
    """The replay-cache ablation: clearing the whole trace (entries and
    masks) before each iteration against the counter reset this design uses
    (the bump counter; the step counters and per-pixel counts are rewritten
    by every forward)."""
    import torch
    trace = tr.rast.trace
    full = [trace["entry"], trace["mask"]]
    nbytes = sum(t.numel() * t.element_size() for t in full)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    ms_full = timed(lambda: [t.zero_() for t in full])
    ms_reset = timed(lambda: trace["used"].zero_())
    return {"full_clear_ms": ms_full, "full_clear_bytes": nbytes, "counter_reset_ms": ms_reset,
            "counter_reset_bytes": trace["used"].numel() * trace["used"].element_size()}


def cfg2_runs(steps=50, warmup=5):
    """100k Gaussians with SH degree 3 on the scene (logit ~ N(0, 0.5^2),
    higher SH ~ N(0, 0.05^2)), ring camera 0 at 1024x768, L1 to the
    ground-truth render of that view; the cached and the recompute backward
    compared on step time, trace size and peak device memory."""
    import torch
    import synth
    from paper_2601_17354_amd.train import Trainer
    from paper_2601_17354_amd.workloads import render_targets
    W, H = 1024, 768
    scene = synth.spheres_planes_scene(0)
    cam = synth.ring_cameras(60, W, H)[0]
    gt = torch.as_tensor(synth.surface_gaussians(scene, 500_000, seed=1000, sh_degree=0, opacity=0.95),
                         device="cuda")
    target = render_targets(gt, 0, [cam], W, H)[0]
    del gt
    P = torch.as_tensor(synth.surface_gaussians(scene, 100_000, seed=300, sh_degree=3, logit_sigma=0.5),
                        device="cuda")
    out = {"workload": "100k Gaussians, SH 3, one 1024x768 view, L1 to the ground-truth render"}
    for cached in (True, False):
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats()
        tr = Trainer(P.clone(), 3, W, H, cached=cached, lam=0.0, extent=4.5)
        tr.prepare(cam)
        tr.rast.reserve(1.5)
        for _ in range(warmup):
            tr.step(cam, target)
        torch.cuda.synchronize()
        tr.rast.flags.zero_()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            tr.step(cam, target)
        b.record()
        torch.cuda.synchronize()
        if tr.rast.read_flags():
            raise RuntimeError("config-2 run overflowed its buffers")
        out["cached" if cached else "recompute"] = {
            "ms_per_step": a.elapsed_time(b) / steps, "trace_gb": tr.rast.trace_bytes() / 1e9,
            "peak_device_gb": torch.cuda.max_memory_allocated() / 1e9,
            "pairs": int(tr.rast.num_pairs.item()),
            "entries": int(tr.rast.trace["count"].sum().item()) if cached else 0}
        del tr
    return out


def ba_runs(n_cams=60, n_points=100_000, iters=15, cpu_points=3_000):
    """Bundle adjustment of synthetic tracks (ring cameras, scene points,
    0.5 px noise, 1% outliers, perturbed poses and points): per-kernel time of
    one Levenberg-Marquardt iteration (step = linearise + reduced camera
    system + solve + back-substitution, apply, cost) with HIP events, a full
    run's convergence against the truth, and the oracle's step (sparse
    normal equations + sparse direct solve) on a smaller problem."""
    import torch
    import synth
    from paper_2601_17354_amd import ba
    tr = synth.ba_tracks(6, n_cams=n_cams, n_points=n_points)
    pb = ba.BAProblem.from_tracks(tr)
    st = ba.state(tr["R0"], tr["c0"], tr["P0"])
    dpose = torch.empty((pb.n_cams, 6), dtype=torch.float64, device="cuda")
    dpoint = torch.empty((pb.n_points, 3), dtype=torch.float64, device="cuda")
    out = tuple(torch.empty_like(t) for t in st)
    cst = torch.empty(1, dtype=torch.float64, device="cuda")
    for _ in range(2):
        ba.step(pb, st, 1e-3, dpose, dpoint)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    t = {"step": 0.0, "apply": 0.0, "cost": 0.0}
    for _ in range(iters):
        ev[0].record()
        ba.step(pb, st, 1e-3, dpose, dpoint)
        ev[1].record()
        ba.apply(pb, st, dpose, dpoint, out)
        ev[2].record()
        ba.cost(pb, out, cst)
        ev[3].record()
        torch.cuda.synchronize()
        t["step"] += ev[0].elapsed_time(ev[1]) / iters
        t["apply"] += ev[1].elapsed_time(ev[2]) / iters
        t["cost"] += ev[2].elapsed_time(ev[3]) / iters
    final, hist, acc = ba.lm(pb, st, lam=1e-3, iters=20)
    R, c, P = (x.cpu().numpy() for x in final)
    R = R.reshape(-1, 3, 3)
    rot_err = np.degrees(np.arccos(np.clip((np.einsum("cij,cij->c", R, tr["R_true"]) - 1) / 2, -1, 1)))
    res = {"workload": f"{pb.n_cams} ring cameras, {pb.n_points} points, {pb.n_obs} observations "
                       "(0.5 px noise, 1% outliers), Huber delta 2 px",
           "ms_per_iteration": sum(t.values()), "ms": t, "iterations": len(hist) - 1,
           "accepted": int(sum(acc)), "cost_first": hist[0], "cost_last": hist[-1],
           "median_rotation_error_deg": float(np.median(rot_err)),
           "median_centre_error": float(np.median(np.linalg.norm(c - tr["c_true"], axis=1))),
           "median_point_error": float(np.median(np.linalg.norm(P - tr["P_true"], axis=1)))}
    # geometric refinement: one re-triangulation + filter pass and one
    # compaction at the converged state, then the refinement loop
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    tr_ms = {"refine": 0.0, "compact": 0.0}
    for _ in range(5):
        ev[0].record()
        Pr, kp, ko = ba.refine(pb, final)
        ev[1].record()
        ba.compact(pb, kp, ko, Pr)
        ev[2].record()
        torch.cuda.synchronize()
        tr_ms["refine"] += ev[0].elapsed_time(ev[1]) / 5
        tr_ms["compact"] += ev[1].elapsed_time(ev[2]) / 5
    res["refinement_ms"] = tr_ms
    t0 = time.perf_counter()
    pb2, st2, loop = ba.refine_loop(pb, st, rounds=3, lm_iters=5)
    torch.cuda.synchronize()
    R2 = st2[0].cpu().numpy().reshape(-1, 3, 3)
    rot2 = np.degrees(np.arccos(np.clip((np.einsum("cij,cij->c", R2, tr["R_true"]) - 1) / 2, -1, 1)))
    res["refinement_loop"] = {"rounds": loop, "wall_s": time.perf_counter() - t0,
                              "median_rotation_error_deg": float(np.median(rot2)),
                              "median_centre_error": float(np.median(np.linalg.norm(
                                  st2[1].cpu().numpy() - tr["c_true"], axis=1)))}
    # the oracle's step on a smaller problem: sparse normal equations + direct solve
    import time as _t
    import scipy.sparse as sps
    import scipy.sparse.linalg as spl
    from oracle import ba as oba
    trs = synth.ba_tracks(6, n_cams=n_cams, n_points=cpu_points)
    t0 = _t.perf_counter()
    H, b = oba.normal_equations_sparse(trs, trs["R0"], trs["c0"], trs["P0"], 2.0)
    free = np.r_[oba.free_pose_params(n_cams, trs["gauge_axis"]), 6 * n_cams + np.arange(trs["P0"].size)]
    A = H[free][:, free]
    A = (A + 1e-3 * sps.diags(A.diagonal())).tocsc()
    spl.spsolve(A, b[free])
    res["cpu_oracle_step_s"] = _t.perf_counter() - t0
    res["cpu_oracle_problem"] = f"{n_cams} cameras, {trs['P0'].shape[0]} points, 1 thread"
    return res


def mvs_runs(width=960, height=720, n_targets=8, iters=5):
    """Single-reference MVS on ray-cast views of the seeded scene (60 ring
    cameras at width x height, 128 planes, 100k scene points standing in for
    the refined sparse cloud): per-stage time with HIP events (Census of all
    60 views, depth ranges, reference choice, then cost volume, SGM and
    fusion for n_targets target views), the depth maps' accuracy against the
    exact ray-cast depth, and the oracle's per-view chain on a smaller view
    scaled by pixels x planes."""
    import torch
    import synth
    from paper_2601_17354_amd import mvs
    scene = synth.spheres_planes_scene(0)
    cams = synth.ring_cameras(60, width, height)
    pr = mvs.MVSParams()
    m = mvs.MVS(cams, width, height, pr, max_targets=n_targets)
    pts = torch.as_tensor(synth.sample_surface(scene, 100_000, 1)[0], device="cuda")
    ref = torch.empty(60, dtype=torch.int32, device="cuda")
    mvs.pgs_mvs_select_ref(m.cams_dev, 60, pr, ref)
    refs = ref.cpu().numpy()
    targets = [int(round(i * 60 / n_targets)) % 60 for i in range(n_targets)]
    need = sorted(set(targets) | {int(refs[t]) for t in targets})
    g_sub, d_sub = synth.textured_views(scene, [cams[i] for i in need], seed=5)
    grey = np.zeros((60, height, width), np.uint8)
    grey[need] = g_sub
    gt = {v: d_sub[i] for i, v in enumerate(need)}
    grey_d = torch.as_tensor(grey, device="cuda")
    tg = torch.as_tensor(np.int32(targets), device="cuda")
    cap = n_targets * width * height
    cloud = torch.empty((3, cap), dtype=torch.float32, device="cuda")
    from paper_2601_17354_amd import _lib
    rng_ws = torch.empty(_lib.load().pgs_mvs_range_workspace(60, pts.shape[0]), dtype=torch.uint8, device="cuda")
    stages = ["census", "range", "reference", "cost", "sgm", "fuse"]

    def run(ev=None):
        def mark(i):
            if ev is not None:
                ev[i].record()
        mark(0)
        mvs.pgs_mvs_census(grey_d, m.census)
        mark(1)
        mvs.pgs_mvs_depth_range(m.cams_dev, 60, width, height, pts, m.range, rng_ws)
        mark(2)
        mvs.pgs_mvs_select_ref(m.cams_dev, 60, pr, m.ref)
        mark(3)
        mvs.pgs_mvs_cost(m.cams_dev, width, height, m.census, tg, m.ref, m.range, pr, m.cost[:n_targets])
        mark(4)
        mvs.pgs_mvs_sgm(m.cost[:n_targets], tg, m.range, pr, m.depth[:n_targets], m.conf[:n_targets],
                        workspace=m.sgm_ws)
        mark(5)
        m.fuse(tg, cloud)
        mark(6)

    for _ in range(2):
        run()
    torch.cuda.synchronize()
    t = {k: 0.0 for k in stages}
    for _ in range(iters):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
        run(ev)
        torch.cuda.synchronize()
        for i, k in enumerate(stages):
            t[k] += ev[i].elapsed_time(ev[i + 1]) / iters
    depth = m.depth[:n_targets].cpu().numpy()
    kept, rel = [], []
    for i, v in enumerate(targets):
        ok = (depth[i] > 0) & (gt[v] > 0)
        kept.append(float((depth[i] > 0).mean()))
        rel.append(np.abs(depth[i][ok] - gt[v][ok]) / gt[v][ok])
    rel = np.concatenate(rel)
    npix, D = width * height, pr.n_planes
    cost_bytes = n_targets * (npix * D + 16 * npix)
    sgm_bytes = n_targets * (16 * npix * D + 8 * npix)
    per_view = (t["cost"] + t["sgm"] + t["fuse"]) / n_targets + (t["census"] + t["range"] + t["reference"]) / 60
    res = {"workload": f"60 ring views {width}x{height} (ray-cast, textured), {D} planes, Census 7x7, SGM 4 paths "
                       f"P1={pr.p1} P2={pr.p2}, {n_targets} target views, 100k sparse points",
           "ms_per_target_view": per_view, "views_per_s": 1e3 / per_view, "ms": t,
           "cost_GBps": cost_bytes / (t["cost"] * 1e-3) / 1e9, "sgm_GBps": sgm_bytes / (t["sgm"] * 1e-3) / 1e9,
           "algorithmic_bytes": {"cost": cost_bytes, "sgm": sgm_bytes},
           "references": {str(v): int(refs[v]) for v in targets},
           "kept_fraction": float(np.mean(kept)), "median_rel_depth_error": float(np.median(rel)),
           "within_1pct": float((rel < 0.01).mean()), "fused_points": int(m.count.item())}
    # the oracle's chain (Census, cost volume, SGM, winner) on a 320x240 view
    import time as _t
    from oracle import mvs as omvs
    cs = synth.ring_cameras(60, 320, 240)
    gs, _ = synth.textured_views(scene, [cs[0], cs[1]], seed=5)
    lo, hi = omvs.depth_range(cs[0], pts.cpu().numpy())
    t0 = _t.perf_counter()
    omvs.depth_map(gs[0], gs[1], cs[0], cs[1], lo, hi, D, pr.p1, pr.p2)
    dt = _t.perf_counter() - t0
    res["cpu_oracle_s_per_view"] = dt * npix / (320 * 240)
    res["cpu_oracle_sample"] = f"one 320x240 view, {D} planes ({dt:.1f} s), scaled by pixels to {width}x{height}"
    return res


def capture_runs(width=640, height=480, n_views=24, iters=500, stride=12):
    """Captures to a trained model: ray-cast greyscale views of the seeded
    scene -> MVS depth maps of every view and their fused, thinned cloud ->
    PCA seeding -> training against the captures (every 6th view held out),
    with the time of each stage and the held-out PSNR."""
    import torch
    import synth
    from paper_2601_17354_amd import mvs, train as tr_
    scene = synth.spheres_planes_scene(0)
    cams = synth.ring_cameras(n_views, width, height)
    grey_np, _ = synth.textured_views(scene, cams, seed=5)
    grey = torch.as_tensor(grey_np, device="cuda")
    sparse = torch.as_tensor(synth.sample_surface(scene, 20000, 1)[0], device="cuda")
    m = mvs.MVS(cams, width, height, mvs.MVSParams(), max_targets=n_views)
    targets = torch.arange(n_views, dtype=torch.int32, device="cuda")
    cap = n_views * width * height // stride + 1
    P = torch.empty((3, cap), dtype=torch.float32, device="cuda")
    C = torch.empty_like(P)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for rep in range(2):                      # the first pass warms up
        ev[0].record()
        m.prepare(grey, sparse)
        m.depth_maps(targets)
        cnt = m.fuse(targets, P, grey=grey, colours=C, stride=stride)
        ev[1].record()
    kept = int(cnt.item())
    n = (kept + stride - 1) // stride
    P, C = P[:, :n].contiguous(), C[:, :n].contiguous()
    ev[2].record()
    params = tr_.seed_pca(P, C)
    ev[3].record()
    torch.cuda.synchronize()
    t_mvs, t_seed = ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3])
    del m
    tgt = {i: (grey[i].float() / 255.0).expand(3, height, width).contiguous() for i in range(n_views)}
    test_ids = [i for i in range(n_views) if i % 6 == 0]
    order = [i for i in range(n_views) if i % 6 != 0]
    trainer = tr_.Trainer(params, 0, width, height)
    trainer.prepare(cams[order[0]])
    t0 = time.perf_counter()
    hist = tr_.train(trainer, cams, tgt, order, iters, eval_ids=test_ids, eval_at=(0, 100, iters))
    torch.cuda.synchronize()
    return {"workload": f"{n_views} ray-cast ring views {width}x{height}: MVS (128 planes) of every view, "
                        f"cloud thinned 1/{stride}, PCA seed, {iters} training steps, every 6th view held out",
            "mvs_ms_all_views": t_mvs, "kept_pixels": kept, "cloud_points": n, "seed_ms": t_seed,
            "train_s_incl_eval": time.perf_counter() - t0,
            "psnr_held_out": {str(k): v for k, v in hist.items()}}


def render_fps(wl, params, order, frames=50):
    """Render-only frames per second at the workload's resolution (projection,
    bin/sort, compositing without the trace) on the trained parameters: the
    deployment path that follows training."""
    import torch
    from paper_2601_17354_amd.raster import Rasterizer
    r = Rasterizer(params.shape[1], 0, wl["width"], wl["height"], cached=False)
    for cid in order[:8]:
        r.forward_checked(params, wl["cams"][cid])
    r.reserve(1.5)
    for k in range(5):
        r.forward(params, wl["cams"][order[k % len(order)]])
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for k in range(frames):
        r.forward(params, wl["cams"][order[k % len(order)]])
    b.record()
    torch.cuda.synchronize()
    if r.read_flags():
        raise RuntimeError("render-only pass overflowed")
    return 1000.0 * frames / a.elapsed_time(b)


ROOT = os.path.dirname(os.path.abspath(__file__))


def psnr_runs(wl, order, iters=500, at=(0, 100, 500)):
    """Held-out PSNR after `iters` training steps (the same step as timed
    above, cached backward) from each initialisation: the plain seed, the
    learned seed (committed network weights, plain-seed fall back), the
    control that adds the network's mean output to every point as one
    constant offset, and an isotropic seed (r_normal = 1) for context."""
    import torch
    from paper_2601_17354_amd.seed_mlp import load_weights, seed_constant_offset, seed_learned
    from paper_2601_17354_amd.train import Trainer, seed_pca, train
    inits = {"plain_pca": wl["params0"]}
    pts, col = wl["cloud"]
    inits["learned"], nfb = seed_learned(pts, col, load_weights())
    log(f"learned seed: {nfb} of {pts.shape[1]} points fell back to the plain seed")
    inits["constant_offset"], _, ybar = seed_constant_offset(pts, col, load_weights())
    log(f"control: the network's mean output {ybar} as one offset for every point")
    inits["isotropic"] = seed_pca(pts, col, r_normal=1.0)
    out = {}
    for name, p0 in inits.items():
        tr = Trainer(p0.clone(), 0, wl["width"], wl["height"], cached=True, lam=0.2, extent=4.5)
        hist = train(tr, wl["cams"], wl["targets"], order, iters, eval_ids=wl["test_ids"], eval_at=at)
        out[name] = {str(k): round(v, 3) for k, v in hist.items()}
        del tr
        torch.cuda.empty_cache()
    return out


def batched_runs(n, steps=20, warmup=3, tuned=None, compare=True):
    """The batched multi-view step: 8 views of uneven resolution (9.73M
    pixels), n Gaussians at SH degree 3, tuned tile shape and LDS batch,
    captured as a graph; beside it the same eight views stepped one view at
    a time with the single-view kernels (eager), for the batching gain."""
    import torch
    from paper_2601_17354_amd import binding as B
    from paper_2601_17354_amd.autotune import tune
    from paper_2601_17354_amd.batch import BatchedStep, time_steps
    from paper_2601_17354_amd.raster import Rasterizer
    from paper_2601_17354_amd.train import BETA1, BETA2, EPS, learning_rates
    from paper_2601_17354_amd.workloads import batched_workload
    wl = batched_workload(n=n)
    cams, targets, sh = wl["cams"], wl["targets"], wl["sh_degree"]
    log(f"batched workload ready: {n} Gaussians, {len(cams)} views")
    if tuned is None:
        tuned = tune(wl["params0"], sh, cams, targets, cached=True, use_cache=False, log=log, extent=4.5)
        log(f"tuned: tile {tuned['tile']} batch {tuned['batch']} ({tuned['seconds']} s)")
    st = BatchedStep(wl["params0"].clone(), sh, cams, targets, tile=tuple(tuned["tile"]), batch=tuned["batch"],
                     extent=4.5)
    st.prepare()
    st._alloc_pairs(int(st.capacity * 1.25), int(st.entry_capacity * 1.25))
    # per-stage times from eager steps before any graph is captured (after a
    # capture the stage events of eager steps have read up to twice the
    # kernel-trace durations of the persistent launches)
    kern, roofs = batched_kernel_times(st)
    # eager steps and graph replays from the same optimiser state, so that
    # both time the same work (training changes the pair and entry counts);
    # the eager steps are timed before the capture for the same reason as
    # the stage times above
    snap = st.snapshot()
    ms_eager = time_steps(st.step, steps, warmup)
    st.restore(snap)
    st.capture()
    st.restore(snap)
    ms_graph = time_steps(st.replay, steps, warmup)
    assert st.read_flags() == 0, "batched step overflowed during timing"
    stats = st.stats()
    del st
    torch.cuda.empty_cache()
    if not compare:
        return {"tile": tuned["tile"], "batch": tuned["batch"], "ms_per_step_graph": ms_graph,
                "ms_per_step_eager": ms_eager, "stats": stats, "kernels_ms": kern, "roofline": roofs}
    # one view at a time, single-view kernels, one Adam step per eight views
    params = wl["params0"].clone()
    grads, m, v = torch.zeros_like(params), torch.zeros_like(params), torch.zeros_like(params)
    lr = learning_rates(sh, 4.5)
    rasts = [Rasterizer(n, sh, c["width"], c["height"], cached=True) for c in cams]
    dls = [torch.empty_like(t) for t in targets]
    loss = torch.zeros(1, device=params.device)
    ws = torch.empty(max(B.pgs_loss_workspace(c["width"], c["height"]) for c in cams), dtype=torch.uint8,
                     device=params.device)
    for r, c in zip(rasts, cams):
        r.forward_checked(params, c)
        r.reserve(1.25)
    count = [0]

    def per_view_step():
        grads.zero_()
        for r, c, t, dl in zip(rasts, cams, targets, dls):
            r.forward(params, c)
            B.pgs_loss_l1_dssim(r.image, t, c["width"], c["height"], 0.2, loss, dl, ws)
            r.backward(params, c, dl, grads)
        count[0] += 1
        B.pgs_adam_step(params, grads, m, v, params.shape[0], n, lr, count[0], BETA1, BETA2, EPS)

    ms_views = time_steps(per_view_step, max(5, steps // 4), 2)
    flags = sum(r.read_flags() for r in rasts)
    del rasts
    torch.cuda.empty_cache()
    return {"workload": f"{n} Gaussians, SH 3, 8 views of uneven size (640x480 .. 1920x1440, "
                        f"{sum(c['width'] * c['height'] for c in cams)} pixels), cached backward, Adam",
            "tile": tuned["tile"], "batch": tuned["batch"], "ms_per_step_graph": ms_graph,
            "ms_per_step_eager": ms_eager, "iters_per_s": 1000.0 / ms_graph,
            "views_per_s": len(cams) * 1000.0 / ms_graph, "ms_per_step_one_view_at_a_time": ms_views,
            "one_view_at_a_time_flags": flags, "stats": stats, "kernels_ms": kern, "roofline": roofs,
            "tuning": tuned["table"]}


def batched_kernel_times(st, steps=5):
    """Per-stage times of eager batched steps (HIP events on the compute
    stream) and the persistent compositing launches' rooflines over those
    steps (scope-table bytes of all views' pixels, pairs and trace entries)."""
    import torch
    from paper_2601_17354_amd.profiling import design_bytes, sec8d_bytes
    acc, recs = {}, []
    for _ in range(steps):
        st.events = []
        st.step()
        torch.cuda.synchronize()
        evs = st.events
        ms = {b: ea.elapsed_time(eb) for (a, ea), (b, eb) in zip(evs[:-1], evs[1:])}
        for b, v in ms.items():
            acc.setdefault(b, []).append(v)
        E = int(st.trace["used"].item()) if st.trace is not None else 0
        recs.append(dict(P=min(int(st.num_pairs.item()), st.capacity), E=E, pixels=st.npx, ms=ms))
    st.events = None
    roofs = {}
    for k in ("render_fwd", "render_bwd"):
        t = sum(r["ms"][k] for r in recs)
        b8 = sum(sec8d_bytes(k, st.cached, r["P"], r["E"], r["pixels"]) for r in recs)
        bd = sum(design_bytes(k, st.cached, r["P"], r["E"], r["pixels"], waves=st.tw * st.th // 64) for r in recs)
        ach = b8 / (t * 1e-3) / 1e9
        roofs[k + "_views"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": ach / HBM_PEAK_GBS, "avg_ms": t / len(recs),
                               "algorithmic_bytes": b8 / len(recs), "pairs": recs[-1]["P"],
                               "entries": recs[-1]["E"], "pixels": st.npx,
                               "frac_design": bd / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return {k: float(np.mean(v)) for k, v in acc.items()}, roofs


def mlp_runs(rows=200_000, batch=16384, reps=20):
    """The seeding network on its own: inference over `rows` feature rows
    and one training step (forward, seed loss, backward, Adam) on a batch,
    timed with HIP events; matrix-core throughput against the bf16 dense
    peak (products only: 2 x 12,800 multiply-adds per row forward, twice
    that more backward, where the first layer's input gradient is skipped)."""
    import torch
    from paper_2601_17354_amd import binding as B
    from paper_2601_17354_amd.seed_mlp import SeedNetTrainer, load_weights
    dev = torch.device("cuda")
    g = torch.Generator(device=dev).manual_seed(0)
    w = load_weights()
    x = torch.randn((rows, 64), generator=g, device=dev)
    y = torch.empty((rows, 8), device=dev)
    for _ in range(3):
        B.pgs_mlp_forward(w, x, rows, y)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        B.pgs_mlp_forward(w, x, rows, y)
    b.record()
    torch.cuda.synchronize()
    ms_inf = a.elapsed_time(b) / reps
    base = torch.zeros((batch, 16), device=dev)
    base[:, 0] = base[:, 4] = base[:, 8] = 1.0
    base[:, 9:12] = -3.0
    base[:, 12] = 1.0
    tgt = torch.zeros((batch, 8), device=dev)
    tr = SeedNetTrainer(w, max_rows=batch)
    xb = x[:batch].contiguous()
    for _ in range(3):
        tr.step(xb, base, tgt)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        tr.step(xb, base, tgt)
    b.record()
    torch.cuda.synchronize()
    ms_step = a.elapsed_time(b) / reps
    fwd_flop = 2.0 * (3 * 64 * 64 + 64 * 8)
    return {"inference_rows": rows, "inference_ms": ms_inf, "inference_rows_per_s": rows / (ms_inf * 1e-3),
            "inference_tflops": rows * fwd_flop / (ms_inf * 1e-3) / 1e12,
            "train_batch": batch, "train_step_ms": ms_step,
            "train_tflops": batch * fwd_flop * 3 / (ms_step * 1e-3) / 1e12, "bf16_dense_peak_tflops": 2500.0}


def achievable_bandwidth(nbytes=1 << 30, reps=10):
    """GB/s of the library's plain streaming copy (reads and writes nbytes)."""
    import torch
    from paper_2601_17354_amd import binding as B
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    B.pgs_stream_copy(src, dst, nbytes)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        B.pgs_stream_copy(src, dst, nbytes)
    b.record()
    torch.cuda.synchronize()
    return 2.0 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9


def traffic_sources():
    """Files whose change invalidates the render kernels' counters: the
    kernels and the rasterizer that chooses their launch order."""
    pkg = os.path.join(ROOT, "paper_2601_17354_amd")
    return ",".join(os.path.join(pkg, f) for f in ("csrc/render.hip", "csrc/render_tile.hpp", "raster.py"))


def roofline(kernel, recs, cached, achievable, backward, entry_bytes=12):
    """Roofline entry of one compositing kernel over exactly the steps whose
    work was recorded: algorithmic bytes (the scope-table model; the design
    model beside it) summed over those steps, divided by the summed event
    times of the same launches, against the 8 TB/s HBM peak and the measured
    stream-copy rate; HBM traffic from the rocprofv3 counters in profiles/
    (with the algorithmic bytes of the very launches they were taken on)
    when they describe the current kernel source."""
    from paper_2601_17354_amd.profiling import (design_bytes, read_issue_fraction, read_summary, read_traffic,
                                                sec8d_bytes)
    t_ms = sum(r["ms"][kernel] for r in recs)
    b8 = sum(sec8d_bytes(kernel, cached, r["P"], r["E"], r["pixels"]) for r in recs)
    bd = sum(design_bytes(kernel, cached, r["P"], r["E"], r["pixels"], entry_bytes=entry_bytes) for r in recs)
    achieved = b8 / (t_ms * 1e-3) / 1e9
    achieved_d = bd / (t_ms * 1e-3) / 1e9
    summary = os.path.join(ROOT, "profiles", f"{kernel}_{backward}_300k_1920x1440_pmc.txt")
    traffic = read_traffic(summary, traffic_sources())
    traffic_work = None
    if traffic is not None:
        kv = read_summary(summary)
        if "algorithmic_bytes_per_launch" in kv:
            traffic_work = dict(algorithmic_bytes=float(kv["algorithmic_bytes_per_launch"].split()[0]),
                                pairs=float(kv["pairs_per_launch"]), entries=float(kv["entries_per_launch"]),
                                views=kv.get("work_log", ""))
    issue = read_issue_fraction(os.path.join(ROOT, "profiles", f"{kernel}_{backward}_300k_1920x1440_counters.txt"),
                                traffic_sources())
    n = len(recs)
    return {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_launches": traffic_work,
            "algorithmic_bytes": b8 / n, "avg_ms": t_ms / n, "launches": n,
            "pairs": sum(r["P"] for r in recs) / n, "entries": sum(r["E"] for r in recs) / n,
            "views": sorted({r["view"] for r in recs}),
            "achievable": achievable, "frac_of_achievable": achieved / achievable,
            "algorithmic_bytes_design": bd / n, "achieved_design": achieved_d, "trace_entry_bytes": entry_bytes,
            "frac_design": achieved_d / HBM_PEAK_GBS,
            # vector-issue share of the kernel's GPU-active time from its
            # instruction counters (VALU wave instructions / 614.4e9 per s)
            "valu_issue_fraction": issue}


def bin_sort_roofline(recs, n):
    """Roofline entry of the binning stage (depth sort, scan, emit, pair sort,
    ranges and the tile order) over the recorded steps: scope-table bytes
    (12 B per Gaussian for the scan; per pair 12 B emitted, 6 x 24 B for a
    46-bit key sort, 8 B for the ranges) and the bytes of this design (depth
    sort of the Gaussians: 4 passes x 24 B plus 12 B of keys and 8 B of
    scan per Gaussian; per pair 12 B emitted, 2 x 24 B for the tile-bit
    sort, 8 B for the ranges) over the stage's event time."""
    t_ms = sum(r["ms"]["bin_sort"] for r in recs)
    b8 = sum(12 * n + 164 * r["P"] for r in recs)
    bd = sum(124 * n + 68 * r["P"] for r in recs)
    k = len(recs)
    return {"kernel": "bin_sort", "bound": "hbm", "achieved": b8 / (t_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": b8 / (t_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "avg_ms": t_ms / k,
            "algorithmic_bytes": b8 / k, "algorithmic_bytes_design": bd / k,
            "frac_design": bd / (t_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "launches_per_step": 28,
            "note": "latency-bound: 28 dependent launches, most of them a few microseconds long"}


def atomic_runs(tr, reps=5):
    """Float-atomic throughput of the render backward's gradient scatter:
    the backward's own targets (the sorted pair values of the last view, each
    Gaussian once per tile it touches) against distinct records (no
    contention) and all adds on 64 records (heavy contention), nine adds per
    target as the backward issues them; beside it the atomic rate the cached
    backward itself sustains (nine adds per pair)."""
    import torch
    from paper_2601_17354_amd import binding as B
    r = tr.rast
    P = min(int(r.num_pairs.item()), r.capacity)
    n = tr.n
    dev = r.values.device
    records = torch.zeros((max(n, P), 16), dtype=torch.float32, device=dev)
    cases = {"backward_targets": (r.values[:P].contiguous(), n),
             "distinct_records": (torch.arange(P, dtype=torch.int32, device=dev), P),
             "64_hot_records": (torch.arange(P, dtype=torch.int32, device=dev) % 64, 64)}
    out = {"adds_per_target": 9, "targets": P}
    for name, (tg, nrec) in cases.items():
        B.pgs_atomic_scatter(records, nrec, tg, P)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            B.pgs_atomic_scatter(records, nrec, tg, P)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        out[name] = {"ms": ms, "gatomics_per_s": 9 * P / (ms * 1e-3) / 1e9}
    del records
    return out


# -- the CPU oracle baseline ------------------------------------------------
#
# Runs in a child process of its own (`bench.py --cpu-worker DIR`), which
# never touches the GPU, so it can fork a pool of workers over tiles.  The
# parent writes the state the GPU step trains (the parameters after the
# timed steps and the camera of the last timed step) into DIR.

_CPU = {}


def _cpu_tiles(tiles):
    """Oracle compositing forward + backward of a list of tiles (run in a pool
    worker); returns the touched Gaussians' 2D gradients (ids, values)."""
    from oracle import render
    st = _CPU
    grad = np.zeros((9, st["proj"]["n"]))
    for k in range(0, len(tiles), 8):
        fwd = render.render_forward(st["proj"], st["bins"], st["cam"], 16, 16, (0.0, 0.0, 0.0),
                                    tiles=tiles[k:k + 8])
        g2d, _ = render.render_backward(st["proj"], st["bins"], fwd, st["dl"], "cached")
        grad += g2d
    ids = np.nonzero(np.any(grad != 0.0, axis=0))[0]
    return ids, grad[:, ids]


def _split_by_pairs(tiles, lens, parts):
    """Tiles dealt to `parts` lists of about equal pair counts (longest first)."""
    order = sorted(tiles, key=lambda t: -int(lens[t]))
    out, load = [[] for _ in range(parts)], np.zeros(parts)
    for t in order:
        k = int(np.argmin(load))
        out[k].append(int(t))
        load[k] += lens[t]
    return [o for o in out if o]


def _cpu_iteration(P, cam, loss, workers, pair_share=1.0, seed=0):
    """One oracle fwd+bwd iteration (projection, binning and sort, compositing
    forward + backward over tiles in a pool, the loss and its gradient, the
    projection VJP).  With pair_share < 1 the compositing runs on seeded
    random tiles holding about that share of the pairs and its wall time is
    scaled by the share they hold.  Returns the stage times in seconds."""
    import multiprocessing as mp

    import torch
    from oracle import binning, loss as oloss, projection
    W, H = int(cam["width"]), int(cam["height"])
    rng = np.random.default_rng(seed)
    t = {}
    t0 = time.perf_counter()
    proj = projection.project(P, cam)
    t["projection"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    bins = binning.bin_and_sort(proj)
    t["binning_sort"] = time.perf_counter() - t0
    lens = bins["ranges"][:, 1] - bins["ranges"][:, 0]
    busy = [int(x) for x in np.nonzero(lens > 0)[0]]
    if pair_share < 1.0:
        perm = rng.permutation(busy)
        cum = np.cumsum(lens[perm])
        k = int(np.searchsorted(cum, pair_share * lens.sum())) + 1
        sample = [int(x) for x in perm[:k]]
    else:
        sample = busy
    share = float(lens[sample].sum() / max(1, lens.sum()))
    dl = rng.normal(size=(3, H, W))
    _CPU.update(proj=proj, bins=bins, cam=cam, dl=dl)
    with mp.get_context("fork").Pool(workers) as pool:
        t0 = time.perf_counter()
        parts = pool.map(_cpu_tiles, _split_by_pairs(sample, lens, workers * 4))
        t["compositing_fwd_bwd"] = (time.perf_counter() - t0) / share
    g2d = np.zeros((9, proj["n"]))
    for ids, vals in parts:
        g2d[:, ids] += vals
    img = rng.uniform(size=(3, H, W))
    t0 = time.perf_counter()
    if loss == "l1":
        oloss.l1(img, img * 0.5)
    else:
        oloss.l1_dssim(img, img * 0.5)
    t["loss"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    projection.project_vjp(P, cam, g2d, proj["visible"])
    t["projection_vjp"] = time.perf_counter() - t0
    _CPU.clear()
    return dict(seconds=sum(t.values()), stages=t, pairs=int(bins["num_pairs"]), tiles_run=len(sample),
                tiles=len(lens), pair_share=share, threads=torch.get_num_threads())


def cpu_worker_main(d):
    """The --cpu-worker leg: config 1 and config 2 iterations in full and the
    benchmark iteration on the state in directory d on a bounded tile
    sample; writes d/result.json."""
    import torch
    import synth
    workers = max(1, min(len(os.sched_getaffinity(0)), 16))
    torch.set_num_threads(workers)
    out = {"workers": workers, "cpu_model": _cpu_model()}
    P1, cam1, _ = synth.cfg1_inputs(0)
    out["cfg1"] = _cpu_iteration(P1, cam1, "l1", workers)
    scene = synth.spheres_planes_scene(0)
    P2 = synth.surface_gaussians(scene, 100_000, seed=300, sh_degree=3, logit_sigma=0.5)
    out["cfg2"] = _cpu_iteration(P2, synth.ring_cameras(60, 1024, 768)[0], "l1", workers)
    P3 = np.load(os.path.join(d, "params.npy"))
    cam3 = json.load(open(os.path.join(d, "cam.json")))
    cam3["viewmat"] = np.asarray(cam3["viewmat"], np.float32)
    out["cfg3"] = _cpu_iteration(P3, cam3, "l1_dssim", workers,
                                 pair_share=float(json.load(open(os.path.join(d, "share.json")))))
    json.dump(out, open(os.path.join(d, "result.json"), "w"))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(trainer, cam, pair_share=0.1):
    """The FP64 oracle timed on the host cores on the GPU step's own state:
    the parameters after the timed steps and the camera of the last timed
    step (compositing on seeded tiles holding pair_share of the pairs,
    scaled), with config 1 and config 2 iterations in full beside it."""
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        np.save(os.path.join(d, "params.npy"), trainer.params.detach().cpu().numpy())
        json.dump({k: np.asarray(v).tolist() for k, v in cam.items()}, open(os.path.join(d, "cam.json"), "w"))
        json.dump(pair_share, open(os.path.join(d, "share.json"), "w"))
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-worker", d],
                           capture_output=True, text=True, timeout=900)
        if r.returncode != 0:
            raise RuntimeError(f"cpu worker failed:\n{r.stderr[-2000:]}")
        res = json.load(open(os.path.join(d, "result.json")))
    c3 = res["cfg3"]
    return dict(value=1.0 / c3["seconds"], unit="iters/s", cores=res["workers"], kind="oracle",
                cpu_model=res["cpu_model"],
                sample=(f"FP64 oracle on the benchmark step's state (trained parameters, last timed camera): "
                        f"projection, binning and sort of all {c3['pairs']} pairs, compositing fwd+bwd on "
                        f"{c3['tiles_run']} seeded tiles holding {100 * c3['pair_share']:.1f}% of the pairs "
                        f"({res['workers']} worker processes over tiles; wall time scaled by that share), "
                        f"L1 + D-SSIM loss and its gradient, projection VJP"),
                stages_s=c3["stages"], cfg1_fwd_bwd_s=res["cfg1"]["seconds"],
                cfg2_fwd_bwd_s=res["cfg2"]["seconds"],
                cfg1=res["cfg1"], cfg2=res["cfg2"])


def main():
    args = parse()
    if args.cpu_worker:
        cpu_worker_main(args.cpu_worker)        # child process: no GPU
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this framework runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(3)
    if args.ba_only:
        print(json.dumps({"bundle_adjustment": ba_runs()}))
        return
    if args.mvs_only:
        print(json.dumps({"multi_view_stereo": mvs_runs()}))
        return
    if args.capture_only:
        print(json.dumps({"captures_to_model": capture_runs()}))
        return
    if args.batched_only:
        r = batched_runs(args.batched_gaussians, steps=6, warmup=2, tuned={"tile": [16, 16], "batch": 256,
                                                                           "table": []}, compare=False)
        print(json.dumps({"batched_views": r}))
        return
    from paper_2601_17354_amd.workloads import training_workload
    torch.manual_seed(0)
    rng = np.random.default_rng(0)
    t = time.perf_counter()
    n_cams = 60
    train_ids = [i for i in range(n_cams) if i % 8 != 0]
    order = [int(i) for i in rng.permutation(train_ids)]
    if args.views:
        order = order[:args.views]
        args.no_psnr = True
    test_ids = [i for i in range(n_cams) if i % 8 == 0]
    wl = training_workload(n_train=args.gaussians, width=args.width, height=args.height,
                           target_cams=sorted(order) + ([] if args.no_psnr else test_ids))
    log(f"workload ready in {time.perf_counter() - t:.1f} s")
    cached = args.backward == "cached"
    work_log = [] if args.work_log else None
    res = run_variant(wl, cached, args.steps, args.warmup, order, work_log=work_log)
    log(f"{args.backward}: {res['ms']:.3f} ms/step, kernels {res['kernels']}, stats {res['stats']}")
    if work_log is not None:
        res["trainer"].rast.work_log = None
        json.dump(work_log, open(args.work_log, "w"))
    tr = res["trainer"]
    cpu_state = None if args.no_cpu_baseline else (tr, res["last_cam"])
    fps = None if args.profile else render_fps(wl, tr.params, order)
    if fps is not None:
        log(f"render-only: {fps:.1f} frames/s")
    atomic = None if args.no_atomic else atomic_runs(tr)
    if atomic:
        log(f"float-atomic reference: {atomic}")
    ablation = trace_clear_ablation(tr) if cached and not args.profile else None
    if ablation:
        log(f"trace clear vs counter reset: {ablation}")
    ab = None
    graph = None
    if not args.profile:
        ab = variants_ab(tr.params, wl, order)
        for name in ("cached_12B_entries", "cached_16B_entries", "recompute"):
            log(f"same state, {name}: {ab[name]['sum_of_medians_ms']:.3f} ms, {ab[name]['median_ms']}")
    if cached and not args.profile:
        graph = graph_runs(wl, order, args.steps, args.warmup)
        log(f"step as HIP graphs: {graph['ms_per_step_graph']:.3f} ms, eager {graph['ms_per_step_eager']:.3f} ms")
    if cpu_state is not None:
        # keep what the CPU oracle will run on; free the trainer's buffers
        cpu_state = (SimpleState(tr.params.detach().cpu()), res["last_cam"])
    del res["trainer"], tr
    torch.cuda.empty_cache()
    if cached and not args.profile:
        full = run_variant(wl, cached, args.steps, args.warmup, order, full_clear=True)
        del full["trainer"]
        torch.cuda.empty_cache()
        ablation["step_full_clear_ms"] = full["ms"]
        ablation["step_counter_reset_ms"] = res["ms"]
        ablation["step_full_clear_extra_bytes"] = full["cleared_bytes"]
        log(f"step with the whole trace cleared: {full['ms']:.3f} ms against {res['ms']:.3f} ms")
    other = None
    if not args.no_compare:
        other = run_variant(wl, not cached, args.steps, args.warmup, order)
        log(f"other: {other['ms']:.3f} ms/step, kernels {other['kernels']}")
        del other["trainer"]
        torch.cuda.empty_cache()
    kern = res["kernels"]
    st = res["stats"]
    achievable = achievable_bandwidth()
    log(f"stream copy: {achievable:.0f} GB/s")
    roofs = {k: roofline(k, res["work"], cached, achievable, args.backward, res["entry_bytes"])
             for k in ("render_fwd", "render_bwd")}
    dom = max(roofs, key=lambda k: roofs[k]["avg_ms"])
    if atomic:
        P = roofs["render_bwd"]["pairs"]
        rate = 9 * P / (roofs["render_bwd"]["avg_ms"] * 1e-3) / 1e9
        atomic["render_bwd_gatomics_per_s"] = rate
        atomic["render_bwd_frac_of_backward_targets_rate"] = rate / atomic["backward_targets"]["gatomics_per_s"]
    out = {
        "metric": METRIC,
        "value": 1000.0 / res["ms"],
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms"],
        "ms_per_step_percentiles": res["pct"],
        "ms_fwd_bwd": res["ms"] - res["kernels"].get("adam", 0.0),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mobile-budget training step: 300k PCA-seeded Gaussians, 1920x1440 "
                               "ring camera, 0.8 L1 + 0.2 D-SSIM, Adam, SH degree 0",
                   "gaussians": st["n"], "resolution": f"{args.width}x{args.height}", "tile": "16x16",
                   "backward": args.backward, "step_includes": "project, bin_sort, render_fwd, loss, "
                   "render_bwd, project_bwd, adam"},
        "roofline": roofs[dom],
        "roofline_render_bwd": roofs["render_bwd"],
        "roofline_bin_sort": bin_sort_roofline(res["work"], st["n"]),
        "achievable_hbm_gbs": achievable,
        "kernels_ms": kern,
        "work": st,
    }
    out["render_only_fps"] = fps
    if atomic:
        out["atomic_reference"] = atomic
    if ablation:
        out["ablation_trace_clear"] = ablation
    if ab is not None:
        out["backward_variants_same_state"] = ab
    if graph is not None:
        out["graph_vs_eager"] = graph
    if other is not None:
        out["other_backward"] = {"backward": "recompute" if cached else "cached",
                                 "ms_per_step": other["ms"], "iters_per_s": 1000.0 / other["ms"],
                                 "ms_per_step_percentiles": other["pct"],
                                 "kernels_ms": other["kernels"], "trace_gb": other["stats"]["trace_gb"],
                                 "roofline_render_bwd": roofline("render_bwd", other["work"], not cached,
                                                                 achievable, "recompute" if cached else "cached")}
    if not args.no_psnr:
        log("held-out PSNR after 500 training steps per initialisation")
        out["psnr_held_out"] = psnr_runs(wl, order)
        log(f"psnr {out['psnr_held_out']}")
        del wl
        torch.cuda.empty_cache()
        from paper_2601_17354_amd.seed_mlp import load_weights
        from paper_2601_17354_amd.workloads import compare_inits
        log("learned vs plain seeding on three fresh scenes (200k points, 1024x768, GT opacity 0.95 / 0.75 / 0.55)")
        out["seeding_fresh_scenes"] = compare_inits(load_weights(), log=log, gt_opacity=(0.95, 0.75, 0.55))
    if not args.no_batched:
        log("batched multi-view step")
        out["batched_views"] = batched_runs(args.batched_gaussians)
        b = out["batched_views"]
        log(f"batched: {b['ms_per_step_graph']:.2f} ms/step graph, {b['ms_per_step_eager']:.2f} eager, "
            f"{b['ms_per_step_one_view_at_a_time']:.2f} one view at a time")
    if not args.no_cfg2:
        log("config 2: 100k Gaussians, SH 3, 1024x768, cached vs recompute backward")
        out["cfg2_backward_variants"] = cfg2_runs()
        log(f"config 2: {out['cfg2_backward_variants']}")
    if not args.no_ba:
        log("bundle adjustment: 60 cameras, 100k points")
        out["bundle_adjustment"] = ba_runs()
        log(f"bundle adjustment: {out['bundle_adjustment']}")
    if not args.no_mvs:
        log("multi-view stereo: 60 views 960x720, 128 planes, 8 targets")
        out["multi_view_stereo"] = mvs_runs()
        log(f"multi-view stereo: {out['multi_view_stereo']}")
    if not args.no_capture:
        log("captures to model: 24 views 640x480, MVS, seed, 500 steps")
        out["captures_to_model"] = capture_runs()
        log(f"captures to model: {out['captures_to_model']}")
    log("seeding network alone")
    out["seed_network"] = mlp_runs()
    log(f"seed network: {out['seed_network']}")
    if cpu_state is not None:
        log("timing the CPU oracle on the benchmark state (bounded tile sample, worker pool)")
        out["cpu_baseline"] = cpu_baseline(*cpu_state)
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out))


class SimpleState:
    """The parameters the CPU oracle runs on (a host copy of the trainer's)."""

    def __init__(self, params):
        self.params = params


if __name__ == "__main__":
    main()
