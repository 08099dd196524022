#!/usr/bin/env python3
"""Per-frame benchmark of the voxel ray tracing hot path on one MI355X.

One step is one frame of the 5.5M-segment tractography-shaped line set at
1920x1080: voxelization (pass 1 + occupancy pyramid), the opaque pass (cull
with one blocking voxel, lists, opaque trace) and the transparent pass (cull
with the alpha-layer limit, lists, sorted compositing at alpha = 0.2).  Inputs
are resident in HBM before the timed region.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "per-frame AS build ms + Mrays/s at 1080p, 5M segs; batched/FP16 vs plain"
TUNE_CACHE = os.path.join(ROOT, "paper_2510_09081_amd", "tune_cache.json")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_bundles_5m_plain.md")


def source_digest():
    """sha256 over the library sources and build flags: HBM counters taken for another digest are stale."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2510_09081_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    with open(os.path.join(ROOT, "paper_2510_09081_amd", "build.py"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, shapes):
    """HBM bytes per launch of `kernel` from the committed PMC summary (FETCH_SIZE + WRITE_SIZE, each scaled by
    the copy-kernel calibration), or None when the summary is missing or was taken for other sources or launch
    shapes."""
    import re
    try:
        with open(PMC_SUMMARY) as f:
            m = re.search(r"<!-- pmc (\{.*\}) -->", f.read())
    except OSError:
        return None
    if not m:
        return None
    d = json.loads(m.group(1))
    k = d.get("kernels", {}).get(kernel)
    if k is None or d.get("source_sha256") != source_digest() or d.get("shapes") != shapes:
        return None
    return {"bytes_per_launch": int(k["fetch_bytes"] + k["write_bytes"]), "fetch_bytes": int(k["fetch_bytes"]),
            "write_bytes": int(k["write_bytes"])}


def calibrate_copy():
    """A plain device copy of known size (for scaling the FETCH_SIZE / WRITE_SIZE counters)."""
    import torch
    n = 64 << 20
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 4 * n, "copies": 3}))
HBM_PEAK_GBS = 8000.0
VREC_BYTES = 32  # quantized position, flags, clip normal per vertex


def kernel_bytes(name, n):
    """Algorithmic HBM bytes of one launch (each distinct item moved once),
    averaged over the frame's launches of that kernel (the list-building and
    trace kernels run once per pass)."""
    passes = ("opaque", "alpha")
    if name == "k_vox_count":   # vertex records once; each occupied word read + written once
        return VREC_BYTES * n["N_v"] + 8 * n["V_o"]
    if name == "k_scatter":     # vertex records; visibility byte of touched voxels; cursor RMW; id writes
        return float(np.mean([VREC_BYTES * n["N_v"] + n["V_o"] + 8 * n["V_v_" + p] + 4 * n["F_v_" + p]
                              for p in passes]))
    if name == "k_ingest":      # xyz + offsets in, records out
        return 12 * n["N_v"] + 4 * n["N_p"] + VREC_BYTES * n["N_v"]
    if name == "k_cull_walk":   # occupied-voxel list in, visibility byte out; per occupied brick its voxel
        # blocking bits and 2^3-cell mask (9 words), the brick and 16^3-cell bits and the 32^3- and
        # 64^3-cell flags once each
        return 5 * n["V_o"] + 72 * n["bricks"] + n["NB"] / 8 + n["NB"] / 64 + n["NB"] / 64 + n["NB"] / 512
    if name == "k_cull_brick":  # per occupied brick: words, visibility read + written, mips 1-3, brick total
        return (2048 + 1024 + 64 + 8 + 1 + 4) * n["bricks"]
    if name == "k_trace_march":  # every pixel: brick table once, miss outputs (RGBA + depth + id)
        return 24 * n["P"] + n["NB"]
    if name == "k_trace_shade":  # per pass: distinct voxel descriptors (8 B), list entries (4 B) and segments
        # (two 32-B vertex records) any ray touched, and the outputs of the rays that reached a list
        return float(np.mean([8 * n[p]["distinct_list_voxels"] + 4 * n[p]["distinct_list_entries"]
                              + 2 * VREC_BYTES * n[p]["distinct_segments"] + 24 * n[p]["rays_hit"]
                              for p in ("trace_opaque", "trace_alpha")]))
    return None


def bench_dynamic(torch, vrt, synth, warmup):
    """Dynamic pathlines: every frame re-advects the line set and rebuilds everything; the whole
    frame (voxelize, alpha cull, lists, transparent trace) is one captured HIP graph replayed per
    frame, against the same frames issued eagerly."""
    frames = synth.pathline_frames()
    traj, origin, vs, dims, radius = frames
    S, L, F = traj.shape[0], 100, 120
    traj_d = torch.from_numpy(traj.astype(np.float32)).cuda()
    ls0 = synth.pathline_frame(frames, 0)
    cam = synth.grid_camera(ls0, 1280, 720)
    P = cam.width * cam.height
    xyz = torch.from_numpy(ls0.xyz).cuda()
    off = torch.from_numpy(ls0.offsets).cuda()
    rgba = torch.empty(4 * P, device="cuda")
    depth = torch.empty(P, device="cuda")
    fid = torch.empty(P, dtype=torch.int32, device="cuda")
    eye = np.asarray(cam.eye, np.float32)
    cam_a = vrt.make_camera(cam.eye, cam.target, cam.up, cam.fovy_deg, cam.width, cam.height,
                            vrt.TRACE_TRANSPARENT, 0.3)
    ctx = vrt.Context(max_vertices=ls0.n_vertices, max_fragments=16 * ls0.n_segments, max_dim=max(dims),
                      max_pixels=P)
    view = (eye, vrt.CULL_ALPHA, 0.3, 1.0 / 256.0)
    graph = ctx.frame_graph(xyz, off, radius, origin, vs, dims, [(view, cam_a, rgba, depth, fid)])
    xv = xyz.view(S, L + 1, 3)

    def load(f):
        xv.copy_(traj_d[:, 2 * f:2 * f + L + 1])

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for f in range(warmup):
        load(f)
        graph.launch()
    torch.cuda.synchronize()
    ev0.record()
    for f in range(F):
        load(f)
        graph.launch()
    ev1.record()
    torch.cuda.synchronize()
    t_graph = ev0.elapsed_time(ev1) / F
    st = ctx.frame_status()
    ev0.record()
    for f in range(F):
        load(f)
        ctx.voxelize(xyz, off, radius, origin, vs, dims)
        ctx.cull(*view)
        ctx.trace(cam_a, rgba, depth, fid)
    ev1.record()
    torch.cuda.synchronize()
    t_eager = ev0.elapsed_time(ev1) / F
    if ctx.frame_status()["device_status"] != 0 or st["device_status"] != 0:
        raise SystemExit("device status error in the dynamic frames")
    graph.close()
    ctx.close()
    return {"workload": "pathlines_abc_2m: 20k seeds x 100 RK4 segments (2M segments/frame), 120 frames, "
                        "256^3, 1280x720, alpha 0.3, alpha culling",
            "frames": F, "graph_ms_per_frame": round(t_graph, 4), "eager_ms_per_frame": round(t_eager, 4),
            "graph_speedup": round(t_eager / t_graph, 4), "mrays_s_graph": round(P / (t_graph * 1e-3) / 1e6, 2),
            "fragments_last_frame": st["n_fragments"], "listed_last_frame": st["n_listed"]}


def bench_batched(torch, vrt, synth, steps, warmup):
    """64 uneven line sets (1k-1M segments, 64^3-256^3 grids, 512x512 each, opaque, culled):
    one persistent launch and one launch per phase against the plain calls set by set."""
    ws = synth.batch_sets()
    items, capsl = [], []
    for w in ws:
        ls, cam = w.lines, w.camera
        n = cam.width * cam.height
        items.append(dict(xyz=torch.from_numpy(ls.xyz).cuda(), offsets=torch.from_numpy(ls.offsets).cuda(),
                          radius=ls.radius, origin=ls.origin, voxel_size=ls.voxel_size, dims=ls.dims,
                          view=(np.asarray(cam.eye, np.float32), vrt.CULL_OPAQUE, 1.0, 1.0 / 256.0),
                          camera=vrt.make_camera(cam.eye, cam.target, cam.up, cam.fovy_deg, cam.width, cam.height),
                          rgba=torch.empty(4 * n, device="cuda"), depth=torch.empty(n, device="cuda"),
                          first_id=torch.empty(n, dtype=torch.int32, device="cuda")))
        capsl.append((ls.n_vertices, 16 * ls.n_segments, max(ls.dims), n))
    b = vrt.Batch(capsl)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    for label, mode in (("persistent", vrt.BATCH_PERSISTENT), ("staged", vrt.BATCH_STAGED),
                        ("sequential", vrt.BATCH_SEQUENTIAL)):
        for _ in range(warmup):
            b.run(items, mode)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(steps):
            b.run(items, mode)
        ev1.record()
        torch.cuda.synchronize()
        res[label] = ev0.elapsed_time(ev1) / steps
        res[label + "_ids"] = [it["first_id"].clone() for it in items]
    same = all(torch.equal(a, c) and torch.equal(s, c)
               for a, s, c in zip(res["persistent_ids"], res["staged_ids"], res["sequential_ids"]))
    bad = [i for i in range(len(ws)) if b.context(i).frame_status()["device_status"] != 0]
    b.close()
    if bad:
        raise SystemExit(f"device status error in batch sets {bad}")
    rays = sum(w.camera.width * w.camera.height for w in ws)
    return {"workload": "batch64: 64 sets, log-uniform 1k-1M segments, random-walk and bundle generators, "
                        "64^3-256^3 grids, 512x512 each, opaque with opaque culling",
            "sets": len(ws), "segments": int(sum(w.lines.n_segments for w in ws)), "rays": rays,
            "persistent_ms": round(res["persistent"], 4), "staged_ms": round(res["staged"], 4),
            "sequential_ms": round(res["sequential"], 4),
            "persistent_speedup": round(res["sequential"] / res["persistent"], 4),
            "staged_speedup": round(res["sequential"] / res["staged"], 4),
            "mrays_s_persistent": round(rays / (res["persistent"] * 1e-3) / 1e6, 2),
            "mrays_s_staged": round(rays / (res["staged"] * 1e-3) / 1e6, 2),
            "first_ids_identical": bool(same)}


def autotune_passes(ctx, passes, rgba, depth, fid, args, key):
    """Autotunes the launch shape of each pass's trace on its own culled structure (outside the timed region)."""
    res = {}
    for label, view, cm in passes:
        ctx.cull(*view)
        r = ctx.autotune(cm, rgba, depth, fid, reps=3, warmup=1, sweeps=2, cache_path=args.tune_cache, key=key)
        res[label] = {"best": r["best"], "best_ms": round(r["best_ms"], 4), "start_ms": round(r["start_ms"], 4),
                      "evaluated": r["evaluated"], "from_cache": r["from_cache"]}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bundles_5m")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-pixels", type=int, default=20000)
    ap.add_argument("--no-fp16", action="store_true")
    ap.add_argument("--no-dynamic", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="trace with the default launch shapes")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="autotuner cache file ('' to search every run); default: the shipped MI355X table")
    ap.add_argument("--calibrate-copy", action="store_true", help="only run a 256 MiB device copy three times")
    args = ap.parse_args()
    if args.tune_cache == "":
        args.tune_cache = None
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path has no multi-GPU leg)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2510_09081_amd import synth, vrt

    w = synth.workload(args.workload)
    ls, cam = w.lines, w.camera
    opq = next(p for p in w.passes if p.trace_mode == synth.MODE_OPAQUE)
    alp = next(p for p in w.passes if p.trace_mode == synth.MODE_TRANSPARENT)
    P = cam.width * cam.height
    dev = torch.device("cuda", 0)
    xyz = torch.from_numpy(ls.xyz).to(dev)
    off = torch.from_numpy(ls.offsets).to(dev)
    rgba = torch.empty(4 * P, device=dev)
    depth = torch.empty(P, device=dev)
    fid = torch.empty(P, dtype=torch.int32, device=dev)
    cam_o = vrt.make_camera(cam.eye, cam.target, cam.up, cam.fovy_deg, cam.width, cam.height, vrt.TRACE_OPAQUE)
    cam_a = vrt.make_camera(cam.eye, cam.target, cam.up, cam.fovy_deg, cam.width, cam.height,
                            vrt.TRACE_TRANSPARENT, alp.alpha, alp.tau)
    eye = np.asarray(cam.eye, np.float32)
    cap = 8 * ls.n_segments
    ctx = vrt.Context(max_vertices=ls.n_vertices, max_fragments=cap, max_dim=max(ls.dims), device=0)

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]

    def frame(stage_events=False):
        if stage_events:
            ev[0].record()
        ctx.voxelize(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims)
        if stage_events:
            ev[1].record()
        ctx.cull(eye, opq.cull_mode, opq.alpha, opq.tau)
        if stage_events:
            ev[2].record()
        ctx.trace(cam_o, rgba, depth, fid)
        if stage_events:
            ev[3].record()
        ctx.cull(eye, alp.cull_mode, alp.alpha, alp.tau)
        if stage_events:
            ev[4].record()
        ctx.trace(cam_a, rgba, depth, fid)
        if stage_events:
            ev[5].record()

    # counts for the algorithmic-byte model (outside the timed region)
    frame()
    st = ctx.frame_status()
    if st["device_status"] != 0:
        raise SystemExit(f"device status {st['device_status']} during the first frame")
    ctx.voxelize(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims)
    ctx.cull(eye, opq.cull_mode, opq.alpha, opq.tau)
    st_o = ctx.frame_status()
    v = ctx.query_as()
    nb = v.n_bricks
    bricks = vrt.copy_to_host(v.brick_list, nb * 4, np.int32, nb).astype(np.int64)
    top = int(bricks.max()) + 1
    words = vrt.copy_to_host(v.words, top * 512 * 4, np.uint32, top * 512).reshape(top, 512)[bricks]
    vis0 = vrt.copy_to_host(v.vis[0], top * 512, np.uint8, top * 512).reshape(top, 512)[bricks]
    V_o = int(((words & 0xFFFF) > 0).sum())
    V_v_o = int((vis0 > 0).sum())
    ctx.cull(eye, alp.cull_mode, alp.alpha, alp.tau)
    st_a = ctx.frame_status()
    vis0a = vrt.copy_to_host(v.vis[0], top * 512, np.uint8, top * 512).reshape(top, 512)[bricks]
    V_v_a = int((vis0a > 0).sum())
    NB = (ls.dims[0] // 8) * (ls.dims[1] // 8) * (ls.dims[2] // 8)
    tune_passes = [("opaque", (eye, opq.cull_mode, opq.alpha, opq.tau), cam_o),
                   ("transparent", (eye, alp.cull_mode, alp.alpha, alp.tau), cam_a)]
    tune = None if args.no_tune else autotune_passes(ctx, tune_passes, rgba, depth, fid, args, w.name)

    ctx_shapes = (ctx.get_tune(vrt.TRACE_OPAQUE), ctx.get_tune(vrt.TRACE_TRANSPARENT))
    for _ in range(args.warmup):
        frame()
    torch.cuda.synchronize()

    # timed region: K frames, stage events on the stream
    stage_ms = np.zeros(5)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record()
    for _ in range(args.steps):
        frame(stage_events=True)
        torch.cuda.synchronize()
        stage_ms += np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(5)])
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    frame_ms_sync = t_start.elapsed_time(t_end) / args.steps
    stage_ms /= args.steps

    # back-to-back frames (no host synchronization between frames)
    torch.cuda.synchronize()
    t_start.record()
    for _ in range(args.steps):
        frame()
    t_end.record()
    torch.cuda.synchronize()
    frame_ms = t_start.elapsed_time(t_end) / args.steps

    # per-kernel durations: the library brackets every launch with HIP events on its stream
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t_start.record()
    for _ in range(args.steps):
        frame()
    t_end.record()
    torch.cuda.synchronize()
    frame_ms_kev = t_start.elapsed_time(t_end) / args.steps
    kern = ctx.profile_read()
    ctx.profile_enable(False)
    st_end = ctx.frame_status()
    if st_end["device_status"] != 0:
        raise SystemExit(f"device status {st_end['device_status']} in the timed frames")

    # work counters of both traces (outside the timed region)
    ctx.voxelize(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims)
    ctx.cull(eye, opq.cull_mode, opq.alpha, opq.tau)
    ts_o = ctx.trace_stats(cam_o, rgba, depth, fid)
    ctx.cull(eye, alp.cull_mode, alp.alpha, alp.tau)
    ts_a = ctx.trace_stats(cam_a, rgba, depth, fid)

    counts = {"N_v": ls.n_vertices, "N_p": ls.n_polylines, "N_s": ls.n_segments, "F": st_o["n_fragments"],
              "F_v_opaque": st_o["n_listed"], "F_v_alpha": st_a["n_listed"], "bricks": nb, "V_o": V_o,
              "V_v_opaque": V_v_o, "V_v_alpha": V_v_a, "P": P, "NB": NB}
    per_kernel = {k: {"launches_per_frame": n / args.steps, "avg_ms": ms / n, "ms_per_frame": ms / args.steps}
                  for k, (n, ms) in sorted(kern.items(), key=lambda kv: -kv[1][1])}
    dom = next(iter(per_kernel))
    b = kernel_bytes(dom, dict(counts, trace_opaque=ts_o, trace_alpha=ts_a))
    roofline = None
    if b is not None:
        ach = b / (per_kernel[dom]["avg_ms"] * 1e-3) / 1e9
        shapes = {"opaque": ctx_shapes[0], "transparent": ctx_shapes[1]}
        tr = measured_traffic(dom, shapes)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None if tr is None else tr["bytes_per_launch"],
                    "traffic_detail": tr, "bytes_per_launch": int(b)}

    as_build_ms = stage_ms[0] + stage_ms[1]
    out = {
        "metric": METRIC,
        "value": round(2 * P / (frame_ms * 1e-3) / 1e6, 3),
        "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(frame_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "segments": ls.n_segments, "polylines": ls.n_polylines,
                   "grid": list(ls.dims), "radius_vox": 0.35, "image": [cam.width, cam.height],
                   "passes": ["opaque, cull opaque", f"transparent alpha={alp.alpha}, cull alpha"]},
        "as_build_ms": round(as_build_ms, 4),
        "trace_opaque_ms": round(stage_ms[2], 4),
        "trace_opaque_mrays_s": round(P / (stage_ms[2] * 1e-3) / 1e6, 2),
        "cull_alpha_ms": round(stage_ms[3], 4),
        "trace_alpha_ms": round(stage_ms[4], 4),
        "trace_alpha_mrays_s": round(P / (stage_ms[4] * 1e-3) / 1e6, 2),
        "stage_ms": {"voxelize": round(stage_ms[0], 4), "cull_opaque": round(stage_ms[1], 4),
                     "trace_opaque": round(stage_ms[2], 4), "cull_alpha": round(stage_ms[3], 4),
                     "trace_alpha": round(stage_ms[4], 4)},
        "frame_ms_host_sync_per_frame": round(frame_ms_sync, 4),
        "frame_ms_with_kernel_events": round(frame_ms_kev, 4),
        "kernels": {k: {kk: round(vv, 5) for kk, vv in d.items()} for k, d in per_kernel.items()},
        "counts": counts,
        "trace_work": {"opaque": ts_o, "alpha": ts_a},
        "roofline": roofline,
        "tune": tune,
        "wall_s_timed": round(wall, 3),
    }

    if not args.no_cpu_baseline:
        from oracle import oracle as O
        t0 = time.perf_counter()
        fo = O.build_frame(ls, eye, opq.cull_mode, opq.alpha, opq.tau)
        t_build_o = time.perf_counter() - t0
        t0 = time.perf_counter()
        fa = O.recull_frame(fo, ls, eye, alp.cull_mode, alp.alpha, alp.tau)
        t_build_a = time.perf_counter() - t0
        S = min(args.cpu_sample_pixels, P)
        pix = np.random.default_rng(0).choice(P, S, replace=False)
        t0 = time.perf_counter()
        O.trace(fo, ls, cam, pix, 0)
        t_tr_o = time.perf_counter() - t0
        t0 = time.perf_counter()
        O.trace(fa, ls, cam, pix, 1, alpha=alp.alpha, tau=alp.tau)
        t_tr_a = time.perf_counter() - t0
        t_frame = t_build_o + t_build_a + (t_tr_o + t_tr_a) * P / S
        out["cpu_baseline"] = {
            "value": round(2 * P / t_frame / 1e6, 5), "unit": "Mrays/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": (f"full oracle build of the frame (voxelize, mips, erosion, both culls, both list sets: "
                       f"{t_build_o + t_build_a:.1f} s) + both traces on {S} random pixels scaled to {P} "
                       f"({t_tr_o + t_tr_a:.2f} s)"),
            "frame_s": round(t_frame, 3), "stage_s": {k: round(v, 3) for k, v in {**fo.times, **{
                "cull_alpha": fa.times["cull"], "lists_alpha": fa.times["lists"]}}.items()},
        }
    ctx.close()

    # FP16 precision form: same frame, the tracer reads brick-relative binary16 records
    if not args.no_fp16:
        ctx16 = vrt.Context(max_vertices=ls.n_vertices, max_fragments=cap, max_dim=max(ls.dims), device=0,
                            form=vrt.FORM_FP16)
        rgba16 = torch.empty_like(rgba)
        depth16 = torch.empty_like(depth)
        fid16 = torch.empty_like(fid)
        plain_img = {}

        def frame16(stage_events=False):
            if stage_events:
                ev[0].record()
            ctx16.voxelize(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims)
            if stage_events:
                ev[1].record()
            ctx16.cull(eye, opq.cull_mode, opq.alpha, opq.tau)
            if stage_events:
                ev[2].record()
            ctx16.trace(cam_o, rgba16, depth16, fid16)
            if stage_events:
                ev[3].record()
            ctx16.cull(eye, alp.cull_mode, alp.alpha, alp.tau)
            if stage_events:
                ev[4].record()
            ctx16.trace(cam_a, rgba16, depth16, fid16)
            if stage_events:
                ev[5].record()

        ctx16.voxelize(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims)
        tune16 = None if args.no_tune else autotune_passes(ctx16, tune_passes, rgba16, depth16, fid16, args,
                                                           w.name)
        for _ in range(args.warmup):
            frame16()
        torch.cuda.synchronize()
        s16 = np.zeros(5)
        for _ in range(args.steps):
            frame16(stage_events=True)
            torch.cuda.synchronize()
            s16 += np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(5)])
        s16 /= args.steps
        t_start.record()
        for _ in range(args.steps):
            frame16()
        t_end.record()
        torch.cuda.synchronize()
        f16 = t_start.elapsed_time(t_end) / args.steps
        if ctx16.frame_status()["device_status"] != 0:
            raise SystemExit("device status error in the FP16 frames")
        # accuracy against the plain form on the full image (same rays)
        agree = {}
        for label, c_, cm in (("opaque", opq, cam_o), ("alpha", alp, cam_a)):
            ctx16.cull(eye, c_.cull_mode, c_.alpha, c_.tau)
            ctx16.trace(cm, rgba16, depth16, fid16)
            ref = vrt.Context(max_vertices=ls.n_vertices, max_fragments=cap, max_dim=max(ls.dims), device=0)
            ref.voxelize(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims)
            ref.cull(eye, c_.cull_mode, c_.alpha, c_.tau)
            ref.trace(cm, rgba, depth, fid)
            torch.cuda.synchronize()
            ref.close()
            d = (rgba16 - rgba).abs().view(-1, 4).amax(dim=1)
            agree[label] = {"first_id_equal": float((fid16 == fid).float().mean()),
                            "colour_diff_max": float(d.max()), "colour_diff_mean": float(d.mean()),
                            "pixels_diff_gt_1e-4": float((d > 1e-4).float().mean())}
        ctx16.close()
        out["fp16"] = {"ms_per_step": round(f16, 4), "speedup_vs_plain": round(frame_ms / f16, 4),
                       "value": round(2 * P / (f16 * 1e-3) / 1e6, 3),
                       "stage_ms": {k: round(v, 4) for k, v in zip(
                           ["voxelize", "cull_opaque", "trace_opaque", "cull_alpha", "trace_alpha"], s16)},
                       "trace_speedup_vs_plain": round((stage_ms[2] + stage_ms[4]) / (s16[2] + s16[4]), 4),
                       "agreement_with_plain": agree, "tune": tune16}
    if not args.no_dynamic:
        out["dynamic_pathlines"] = bench_dynamic(torch, vrt, synth, args.warmup)
    if not args.no_batched:
        out["batched"] = bench_batched(torch, vrt, synth, args.steps, args.warmup)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
