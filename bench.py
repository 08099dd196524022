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
SQ_SUMMARY = os.path.join(ROOT, "profiles", "sq_bundles_5m_plain.md")
# Vector-ALU issue peak of MI355X: 256 compute units x 4 SIMDs, each issuing one wave64 instruction per
# 4 cycles (64 lanes on 16-lane units) at 2.4 GHz = 614.4 G wave64 VALU instructions/s (39.3 T lane-ops/s).
VALU_ISSUE_PEAK_G = 256 * 4 * 2.4 / 4


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


def measured_valu(kernel, shapes):
    """Wave64 VALU instructions per launch of `kernel` from the committed SQ counter summary (SQ_INSTS_VALU,
    averaged over the kernel's dispatches), or None when the summary is missing or was taken for other sources
    or launch shapes."""
    import re
    try:
        with open(SQ_SUMMARY) as f:
            m = re.search(r"<!-- sq (\{.*\}) -->", f.read())
    except OSError:
        return None
    if not m:
        return None
    d = json.loads(m.group(1))
    k = d.get("kernels", {}).get(kernel)
    if k is None or d.get("source_sha256") != source_digest() or d.get("shapes") != shapes:
        return None
    return float(k["valu_per_launch"])


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
# Algorithmic record sizes (bytes each distinct item must move): a vertex record is its int32 position and
# binary32 clip normal (24 B; the 32-B layout pads it), a segment record its two vertex records (48 B), or in
# the FP16 form its binary16 endpoints and normals and a 32-bit brick id (28 B).
R_V = {"plain": 24, "fp16": 12}
R_S = {"plain": 48, "fp16": 28}


def kernel_bytes(name, n, form="plain"):
    """Algorithmic HBM bytes of one launch (each distinct item moved once),
    averaged over the frame's launches of that kernel (the list-building and
    trace kernels run once per pass)."""
    passes = ("opaque", "alpha")
    rv = R_V[form]
    if name == "k_ingest":      # xyz + offsets in, vertex records out
        return 12 * n["N_v"] + 4 * n["N_p"] + rv * n["N_v"]
    if name == "k_cull_walk":   # occupied-voxel list in, visibility byte out; per occupied brick its voxel
        # blocking bits and 2^3-cell mask (9 words), the brick and 16^3-cell bits and the 32^3- and
        # 64^3-cell flags once each
        return 5 * n["V_o"] + 72 * n["bricks"] + n["NB"] / 8 + n["NB"] / 64 + n["NB"] / 64 + n["NB"] / 512
    if name == "k_cull_brick":  # per occupied brick: words, visibility read + written, mips 1-3, brick total
        return (2048 + 1024 + 64 + 8 + 1 + 4) * n["bricks"]
    if name == "k_trace_march":  # every pixel: brick table once, miss outputs (RGBA + depth + id)
        return 24 * n["P"] + n["NB"]
    if name == "k_trace_shade":  # per pass: distinct voxel descriptors (8 B), list entries (4 B) and segment
        # records any ray touched, and the outputs of the rays that reached a list
        return float(np.mean([8 * n[p]["distinct_list_voxels"] + 4 * n[p]["distinct_list_entries"]
                              + R_S[form] * n[p]["distinct_segments"] + 24 * n[p]["rays_hit"]
                              for p in ("trace_opaque", "trace_alpha")]))
    return None


def frame_bytes(n, form="plain"):
    """Algorithmic bytes of one whole frame (voxelization, then cull + lists + trace per pass), term by term:
    every distinct item moved once by each pass that needs it."""
    rv, rs = R_V[form], R_S[form]
    passes = (("opaque", "trace_opaque"), ("alpha", "trace_alpha"))
    t = {
        "xyz_in": 12 * n["N_v"],
        "records_pass1": rv * n["N_v"],
        "words_rmw_pass1": 8 * n["V_o"],
        "occupancy_finalize_and_mips": 4 * n["V_o"] + 16 * n["V_o"] / 7,
        "erosion_and_visibility": sum(2 * n["V_o"] for _ in passes),
        "scan_and_offsets": sum(8 * n["V_o"] for _ in passes),
        "records_pass2": sum(rv * n["N_v"] for _ in passes),
        "cursor_rmw_pass2": sum(8 * n["V_v_" + p] for p, _ in passes),
        "ids_write_pass2": sum(4 * n["F_v_" + p] for p, _ in passes),
        "trace_outputs": sum(24 * n["P"] for _ in passes),
        "trace_voxel_descriptors": sum(8 * n[tp]["distinct_list_voxels"] for _, tp in passes),
        "trace_list_entries": sum(4 * n[tp]["distinct_list_entries"] for _, tp in passes),
        "trace_segment_records": sum(rs * n[tp]["distinct_segments"] for _, tp in passes),
    }
    return {k: int(v) for k, v in t.items()}


def valu_issue(valu_per_launch, avg_ms):
    """The kernel against the vector-ALU issue peak: counted VALU instructions per launch over the live average
    launch time (the shade kernel issues instructions more than it waits on memory)."""
    if valu_per_launch is None:
        return None
    ach = valu_per_launch / (avg_ms * 1e-3) / 1e9
    return {"valu_per_launch": int(valu_per_launch), "achieved": round(ach, 2), "peak": VALU_ISSUE_PEAK_G,
            "unit": "G wave64 VALU instructions/s", "frac": round(ach / VALU_ISSUE_PEAK_G, 4)}


def memory_ceilings(torch, vrt):
    """Measured streaming-copy bandwidth and device-atomic rates (random words, and 64 atomics per wave step
    inside one 2 KiB brick region) over a 512 MiB array."""
    out = {}
    big = torch.empty(2 << 30, dtype=torch.uint8, device="cuda")  # 1 GiB read + 1 GiB written per copy
    vrt.microbench(vrt.MB_COPY, big)  # warm-up
    ms = min(vrt.microbench(vrt.MB_COPY, big) for _ in range(5))
    out["copy"] = {"bytes": big.numel(), "ms": round(ms, 4), "GB_s": round(big.numel() / (ms * 1e-3) / 1e9, 1)}
    del big
    buf = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    ops = 1 << 28
    for label, kind in (("atomic_random", vrt.MB_ATOMIC_RANDOM), ("atomic_brick_local", vrt.MB_ATOMIC_BRICK)):
        vrt.microbench(kind, buf, 1 << 24)
        ms = min(vrt.microbench(kind, buf, ops) for _ in range(2))
        out[label] = {"ops": ops, "ms": round(ms, 4), "Gops_s": round(ops / (ms * 1e-3) / 1e9, 2)}
    del buf
    return out


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
    one persistent launch, one launch per phase, and the split form (one cooperative launch for the build, then one
    launch per view-dependent phase) against the plain calls set by set."""
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

    def timed(suffix):
        for label, mode in (("persistent", vrt.BATCH_PERSISTENT), ("staged", vrt.BATCH_STAGED),
                            ("split", vrt.BATCH_SPLIT), ("sequential", vrt.BATCH_SEQUENTIAL)):
            for _ in range(warmup):
                b.run(items, mode)
            torch.cuda.synchronize()
            ev0.record()
            for _ in range(steps):
                b.run(items, mode)
            ev1.record()
            torch.cuda.synchronize()
            res[label + suffix] = ev0.elapsed_time(ev1) / steps
            res[label + suffix + "_ids"] = [it["first_id"].clone() for it in items]

    timed("")
    # per-set launch shapes: the autotuner on each set's own structure (left by the last sequential run)
    groups = {}
    for i, it in enumerate(items):
        r = b.context(i).autotune(it["camera"], it["rgba"], it["depth"], it["first_id"], reps=2, warmup=1,
                                  sweeps=1)
        groups[r["best"]["shade_group"]] = groups.get(r["best"]["shade_group"], 0) + 1
    timed("_tuned")
    same = all(torch.equal(a, c) and torch.equal(s, c) and torch.equal(x, c) and torch.equal(a2, c)
               and torch.equal(s2, c) and torch.equal(x2, c)
               for a, s, x, c, a2, s2, x2 in zip(res["persistent_ids"], res["staged_ids"], res["split_ids"],
                                                 res["sequential_ids"], res["persistent_tuned_ids"],
                                                 res["staged_tuned_ids"], res["split_tuned_ids"]))
    bad = [i for i in range(len(ws)) if b.context(i).frame_status()["device_status"] != 0]
    b.close()
    if bad:
        raise SystemExit(f"device status error in batch sets {bad}")
    rays = sum(w.camera.width * w.camera.height for w in ws)
    return {"workload": "batch64: 64 sets, log-uniform 1k-1M segments, random-walk and bundle generators, "
                        "64^3-256^3 grids, 512x512 each, opaque with opaque culling",
            "sets": len(ws), "segments": int(sum(w.lines.n_segments for w in ws)), "rays": rays,
            "persistent_ms": round(res["persistent"], 4), "staged_ms": round(res["staged"], 4),
            "split_ms": round(res["split"], 4), "sequential_ms": round(res["sequential"], 4),
            "persistent_speedup": round(res["sequential"] / res["persistent"], 4),
            "staged_speedup": round(res["sequential"] / res["staged"], 4),
            "split_speedup": round(res["sequential"] / res["split"], 4),
            "tuned": {"persistent_ms": round(res["persistent_tuned"], 4), "staged_ms": round(res["staged_tuned"], 4),
                      "split_ms": round(res["split_tuned"], 4), "sequential_ms": round(res["sequential_tuned"], 4),
                      "persistent_speedup_vs_untuned_sequential": round(res["sequential"] / res["persistent_tuned"], 4),
                      "shade_groups_chosen": {str(k): v for k, v in sorted(groups.items())}},
            "mrays_s_persistent": round(rays / (res["persistent"] * 1e-3) / 1e6, 2),
            "mrays_s_staged": round(rays / (res["staged"] * 1e-3) / 1e6, 2),
            "mrays_s_split": round(rays / (res["split"] * 1e-3) / 1e6, 2),
            "first_ids_identical": bool(same)}


def cpu_baseline_leg(out, ctx, w, vrt, synth, torch, xyz, off, eye, opq, alp, args, img_plain, img_fp16):
    """The CPU oracle on the host cores: its time for the frame (the CPU baseline), and the accuracy of the
    GPU frame against it -- the plain form's structure bit for bit and both forms' images on every pixel --
    plus the precision-form comparison on the 10k-segment random-walk set (plain and FP16 against FP64)."""
    from oracle import oracle as O
    from tests import _gpu as G
    ls, cam = w.lines, w.camera
    P = cam.width * cam.height
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
    nt = O.num_threads()
    out["cpu_baseline"] = {
        "value": round(2 * P / t_frame / 1e6, 5), "unit": "Mrays/s", "cores": nt, "kind": "oracle",
        "sample": (f"full oracle build of the frame (voxelize, mips, erosion, both culls, both list sets: "
                   f"{t_build_o + t_build_a:.1f} s) + both traces on {S} random pixels scaled to {P} "
                   f"({t_tr_o + t_tr_a:.2f} s)"),
        "threads_per_stage": {"ingest": 1, "voxelize": 1, "mips": 1, "erode": 1, "cull": nt, "cull_mips": 1,
                              "lists": 1, "trace": nt},
        "frame_s": round(t_frame, 3), "stage_s": {k: round(v, 3) for k, v in {**fo.times, **{
            "cull_alpha": fa.times["cull"], "lists_alpha": fa.times["lists"]}}.items()},
    }
    # parity of the timed frame with the oracle frame just built (full image, both passes)
    par = {}
    for label, fr, pas, mode in (("opaque", fo, opq, 0), ("alpha", fa, alp, 1)):
        ctx.voxelize(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims)
        ctx.cull(eye, pas.cull_mode, pas.alpha, pas.tau)
        st = ctx.frame_status()
        rep = G.structure_report(fr, G.fetch_as(ctx), G.fetch_ids(ctx, fr.total), st)
        tr = O.trace(fr, ls, cam, np.arange(P), mode, alpha=pas.alpha, tau=pas.tau)
        rep["trace"] = G.trace_report(tr, *img_plain[label], ls.voxel_size, mode)
        if img_fp16 is not None:
            rep["trace_fp16"] = G.trace_report(tr, *img_fp16[label], ls.voxel_size, mode)
        par[label] = rep
    exact = all(v for p in par.values() for k, v in p.items() if not k.startswith("trace"))
    out["parity"] = {"workload": w.name, "structure_bit_exact": bool(exact),
                     "trace_within_tolerance": all(p["trace"]["pass"] for p in par.values()), "passes": par}
    # precision form on the 10k-segment random-walk set: plain and FP16 against the FP64 oracle
    pw = synth.workload("random_walk_10k")
    pls, pcam = pw.lines, pw.camera
    pP = pcam.width * pcam.height
    pxyz, poff = torch.from_numpy(pls.xyz).cuda(), torch.from_numpy(pls.offsets).cuda()
    prgba, pdepth = torch.empty(4 * pP, device="cuda"), torch.empty(pP, device="cuda")
    pfid = torch.empty(pP, dtype=torch.int32, device="cuda")
    prec = {}
    for mode, alpha in ((0, 1.0), (1, 0.3)):
        fr = O.build_frame(pls, pcam.eye, O.CULL_NONE)
        tr = O.trace(fr, pls, pcam, np.arange(pP), mode, alpha=alpha)
        for form, fname in ((vrt.FORM_PLAIN, "plain"), (vrt.FORM_FP16, "fp16")):
            c = vrt.Context(max_vertices=pls.n_vertices, max_fragments=4 * fr.total + 16, max_dim=max(pls.dims),
                            max_pixels=pP, form=form)
            c.voxelize(pxyz, poff, pls.radius, pls.origin, pls.voxel_size, pls.dims)
            c.cull(np.asarray(pcam.eye, np.float32), vrt.CULL_NONE)
            c.trace(vrt.make_camera(pcam.eye, pcam.target, pcam.up, pcam.fovy_deg, pcam.width, pcam.height, mode,
                                    alpha), prgba, pdepth, pfid)
            torch.cuda.synchronize()
            c.close()
            prec[f"{'opaque' if mode == 0 else 'alpha_0.3'}_{fname}"] = G.trace_report(
                tr, pfid.cpu().numpy().astype(np.int64), pdepth.cpu().numpy(), prgba.cpu().numpy().reshape(pP, 4),
                pls.voxel_size, mode)
    out["precision_random_walk_10k"] = prec


def bench_static(torch, vrt, ctx, w, xyz, off, eye, opq, alp, cam_o, cam_a, cap, steps, warmup, dynamic_ms):
    """Static line set: the structure of each pass is built once (and its lists sorted into canonical order);
    every frame only traces (the opaque and the transparent pass)."""
    ls, cam = w.lines, w.camera
    P = cam.width * cam.height
    ctx_a = vrt.Context(max_vertices=ls.n_vertices, max_fragments=cap, max_dim=max(ls.dims), device=0)
    rgba, depth = torch.empty(4 * P, device="cuda"), torch.empty(P, device="cuda")
    fid = torch.empty(P, dtype=torch.int32, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sort_ms = {}
    for c, pas, label in ((ctx, opq, "opaque"), (ctx_a, alp, "alpha")):
        c.voxelize(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims)
        c.cull(eye, pas.cull_mode, pas.alpha, pas.tau)
        torch.cuda.synchronize()
        ev0.record()
        c.sort_lists()
        ev1.record()
        torch.cuda.synchronize()
        sort_ms[label] = round(ev0.elapsed_time(ev1), 4)
    ctx_a.set_tune(vrt.TRACE_TRANSPARENT, **ctx.get_tune(vrt.TRACE_TRANSPARENT))

    def frame():
        ctx.trace(cam_o, rgba, depth, fid)
        ctx_a.trace(cam_a, rgba, depth, fid)

    for _ in range(warmup):
        frame()
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(steps):
        frame()
    ev1.record()
    torch.cuda.synchronize()
    t = ev0.elapsed_time(ev1) / steps
    bad = ctx.frame_status()["device_status"] or ctx_a.frame_status()["device_status"]
    ctx_a.close()
    if bad:
        raise SystemExit("device status error in the static frames")
    return {"frame_ms": round(t, 4), "mrays_s": round(2 * P / (t * 1e-3) / 1e6, 2),
            "speedup_vs_dynamic": round(dynamic_ms / t, 4), "sort_lists_ms": sort_ms,
            "note": "both passes traced per frame on structures built once (lists sorted by segment id)"}


def bench_alpha_sweep(torch, vrt, ctx, w, xyz, off, eye, steps):
    """Opacity sweep of the transparent pass: alpha culling (the blocking limit M follows alpha) against no
    culling at each opacity; cull + trace time, listed fragments and the image difference of the two."""
    ls, cam = w.lines, w.camera
    P = cam.width * cam.height
    out = []
    imgs = [torch.empty(4 * P, device="cuda") for _ in range(2)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ctx.voxelize(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims)
    for alpha in (0.05, 0.1, 0.2, 0.3, 0.5, 0.8, 1.0):
        cm = vrt.make_camera(cam.eye, cam.target, cam.up, cam.fovy_deg, cam.width, cam.height,
                             vrt.TRACE_TRANSPARENT, alpha)
        row = {"alpha": alpha}
        for k, (label, mode) in enumerate((("alpha_cull", vrt.CULL_ALPHA), ("no_cull", vrt.CULL_NONE))):
            cull_ms, trace_ms = [], []
            for _ in range(max(steps // 2, 3)):
                ev[0].record()
                ctx.cull(eye, mode, alpha)
                ev[1].record()
                ctx.trace(cm, imgs[k])
                ev[2].record()
                torch.cuda.synchronize()
                cull_ms.append(ev[0].elapsed_time(ev[1]))
                trace_ms.append(ev[1].elapsed_time(ev[2]))
            st = ctx.frame_status()
            if st["device_status"] != 0:
                raise SystemExit(f"device status error in the alpha sweep ({alpha}, {label})")
            row[label] = {"cull_ms": round(float(np.median(cull_ms)), 4),
                          "trace_ms": round(float(np.median(trace_ms)), 4), "listed": st["n_listed"],
                          "visible_voxels": st["n_visible"]}
        d = (imgs[0] - imgs[1]).abs().view(-1, 4).amax(dim=1)
        row["image_diff_max"] = float(d.max())
        row["image_diff_mean"] = float(d.mean())
        row["speedup_alpha_cull"] = round((row["no_cull"]["cull_ms"] + row["no_cull"]["trace_ms"]) /
                                          (row["alpha_cull"]["cull_ms"] + row["alpha_cull"]["trace_ms"]), 4)
        out.append(row)
    return out


def bench_voxelizers(torch, vrt, synth, ctx, w, steps):
    """The voxelizer comparison of Table 2 and the segment-length figure: voxelization (pass 1 and the
    occupancy pyramid) with the capsule voxelizer and the two comparison voxelizers (thin line, capsule
    AABB), over segment length (every n-th vertex kept) on the benchmark grid, and over grid resolution."""
    ls = w.lines
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    modes = (("capsule", vrt.VOX_CAPSULE), ("thin", vrt.VOX_THIN), ("aabb", vrt.VOX_AABB))

    def run(l, extra):
        xyz, off = torch.from_numpy(l.xyz).cuda(), torch.from_numpy(l.offsets).cuda()
        seg = l.xyz[1:] - l.xyz[:-1]
        valid = np.ones(l.n_vertices - 1, bool)
        valid[l.offsets[1:-1] - 1] = False
        mean_len = float(np.linalg.norm(seg[valid], axis=1).mean() / l.voxel_size)
        row = dict(extra, segments=l.n_segments, mean_segment_vox=round(mean_len, 3))
        for name, m in modes:
            ts = []
            for _ in range(max(steps // 2, 3)):
                ev0.record()
                ctx.voxelize(xyz, off, l.radius, l.origin, l.voxel_size, l.dims, voxelizer=m)
                ev1.record()
                torch.cuda.synchronize()
                ts.append(ev0.elapsed_time(ev1))
            st = ctx.frame_status()
            row[name] = {"ms": round(float(np.median(ts)), 4), "fragments": st["n_fragments"],
                         "fragments_per_segment": round(st["n_fragments"] / max(l.n_segments, 1), 3),
                         "status": st["device_status"]}
        return row

    out = {"segment_length": [run(synth.decimate(ls, n), {"every_nth_vertex": n}) for n in (1, 2, 4, 8, 16)],
           "grid": [run(synth.regrid(ls, G), {"grid": G}) for G in (128, 256, 512)],
           "radius_vox_at_512": 0.35}
    return out


def bench_shading(torch, vrt, ctx, w, xyz, off, eye, opq, alp, cam_o, cam_a, steps):
    """Voxel-space shading (Sec. 3.4, Table 6's shading stage): ambient occlusion (16 cones, 4 samples) and a
    directional shadow for the visible voxels of each pass, and the shaded trace."""
    ls, cam = w.lines, w.camera
    P = cam.width * cam.height
    rgba = torch.empty(4 * P, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    out = {"cones": 16, "samples": 4, "light_dir": [0.3, 0.5, 0.8], "ambient": 0.3}
    ctx.voxelize(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims)
    for label, pas, cm in (("opaque", opq, cam_o), ("alpha", alp, cam_a)):
        sh_ms, tr_ms = [], []
        for _ in range(max(steps // 2, 3)):
            ctx.cull(eye, pas.cull_mode, pas.alpha, pas.tau)
            ev[0].record()
            ctx.shade((0.3, 0.5, 0.8), 16, 4, 0.3)
            ev[1].record()
            ctx.trace(cm, rgba)
            ev[2].record()
            torch.cuda.synchronize()
            sh_ms.append(ev[0].elapsed_time(ev[1]))
            tr_ms.append(ev[1].elapsed_time(ev[2]))
        st = ctx.frame_status()
        if st["device_status"] != 0:
            raise SystemExit("device status error in the shading leg")
        out[label] = {"shade_ms": round(float(np.median(sh_ms)), 4),
                      "shaded_trace_ms": round(float(np.median(tr_ms)), 4), "visible_voxels": st["n_visible"]}
    return out


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
    ap.add_argument("--no-static", action="store_true")
    ap.add_argument("--no-alpha-sweep", action="store_true")
    ap.add_argument("--no-voxelizers", action="store_true")
    ap.add_argument("--no-shading", action="store_true")
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

    # back-to-back frames (no host synchronization between frames); an event between frames gives each
    # frame's time for the median and 90th percentile
    fev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t_start.record()
    fev[0].record()
    for k in range(args.steps):
        frame()
        fev[k + 1].record()
    t_end.record()
    torch.cuda.synchronize()
    frame_ms = t_start.elapsed_time(t_end) / args.steps
    per_frame = np.array([fev[k].elapsed_time(fev[k + 1]) for k in range(args.steps)])

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
    nctx = dict(counts, trace_opaque=ts_o, trace_alpha=ts_a)
    b = kernel_bytes(dom, nctx)
    fb = frame_bytes(nctx)
    b_alg = sum(fb.values())
    roofline = None
    if b is not None:
        ach = b / (per_kernel[dom]["avg_ms"] * 1e-3) / 1e9
        shapes = {"opaque": ctx_shapes[0], "transparent": ctx_shapes[1]}
        tr = measured_traffic(dom, shapes)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None if tr is None else tr["bytes_per_launch"],
                    "traffic_detail": tr, "bytes_per_launch": int(b),
                    "valu_issue": valu_issue(measured_valu(dom, shapes), per_kernel[dom]["avg_ms"]),
                    "kernel_avg_ms": round(per_kernel[dom]["avg_ms"], 5),
                    "frame_bytes": b_alg, "frame_bytes_terms": fb,
                    "frame_achieved": round(b_alg / (frame_ms * 1e-3) / 1e9, 2),
                    "frame_frac": round(b_alg / (frame_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)}
    ceilings = memory_ceilings(torch, vrt)
    if roofline is not None:
        roofline["copy_ceiling_GB_s"] = ceilings["copy"]["GB_s"]

    as_build_ms = stage_ms[0] + stage_ms[1]
    out = {
        "metric": METRIC,
        "value": round(2 * P / (frame_ms * 1e-3) / 1e6, 3),
        "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(frame_ms, 4),
        "frame_ms_median": round(float(np.median(per_frame)), 4),
        "frame_ms_p90": round(float(np.percentile(per_frame, 90)), 4),
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
        "memory_ceilings": dict(ceilings, per_fragment_atomics=(
            f"pass 1 and pass 2 with one device atomic per fragment (F + F_v = "
            f"{counts['F'] + counts['F_v_opaque'] + counts['F_v_alpha']}) would take at least "
            f"{(counts['F'] + counts['F_v_opaque'] + counts['F_v_alpha']) / (ceilings['atomic_brick_local']['Gops_s'] * 1e6):.3f}"
            f" ms at the brick-local rate")),
        "tune": tune,
        "wall_s_timed": round(wall, 3),
    }

    def images():
        torch.cuda.synchronize()
        return (fid.cpu().numpy().astype(np.int64), depth.cpu().numpy(), rgba.cpu().numpy().reshape(P, 4))

    # the plain frame's images of both passes, for the accuracy comparisons
    ctx.voxelize(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims)
    ctx.cull(eye, opq.cull_mode, opq.alpha, opq.tau)
    ctx.trace(cam_o, rgba, depth, fid)
    img_plain = {"opaque": images()}
    ctx.cull(eye, alp.cull_mode, alp.alpha, alp.tau)
    ctx.trace(cam_a, rgba, depth, fid)
    img_plain["alpha"] = images()

    # FP16 precision form: same frame, the tracer reads brick-relative binary16 records
    img_fp16 = None
    if not args.no_fp16:
        ctx16 = vrt.Context(max_vertices=ls.n_vertices, max_fragments=cap, max_dim=max(ls.dims), device=0,
                            form=vrt.FORM_FP16)

        def frame16(stage_events=False):
            if stage_events:
                ev[0].record()
            ctx16.voxelize(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims)
            if stage_events:
                ev[1].record()
            ctx16.cull(eye, opq.cull_mode, opq.alpha, opq.tau)
            if stage_events:
                ev[2].record()
            ctx16.trace(cam_o, rgba, depth, fid)
            if stage_events:
                ev[3].record()
            ctx16.cull(eye, alp.cull_mode, alp.alpha, alp.tau)
            if stage_events:
                ev[4].record()
            ctx16.trace(cam_a, rgba, depth, fid)
            if stage_events:
                ev[5].record()

        ctx16.voxelize(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims)
        tune16 = None if args.no_tune else autotune_passes(ctx16, tune_passes, rgba, depth, fid, args, w.name)
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
        ctx16.voxelize(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims)
        ctx16.cull(eye, opq.cull_mode, opq.alpha, opq.tau)
        ctx16.trace(cam_o, rgba, depth, fid)
        img_fp16 = {"opaque": images()}
        ctx16.cull(eye, alp.cull_mode, alp.alpha, alp.tau)
        ctx16.trace(cam_a, rgba, depth, fid)
        img_fp16["alpha"] = images()
        ctx16.close()
        agree = {}
        for label in ("opaque", "alpha"):
            (ia, _, ca), (ib, _, cb) = img_plain[label], img_fp16[label]
            d = np.abs(ca - cb).max(axis=1)
            agree[label] = {"first_id_equal": float((ia == ib).mean()), "colour_diff_max": float(d.max()),
                            "colour_diff_mean": float(d.mean()), "pixels_diff_gt_1e-4": float((d > 1e-4).mean())}
        out["fp16"] = {"ms_per_step": round(f16, 4), "speedup_vs_plain": round(frame_ms / f16, 4),
                       "value": round(2 * P / (f16 * 1e-3) / 1e6, 3),
                       "stage_ms": {k: round(v, 4) for k, v in zip(
                           ["voxelize", "cull_opaque", "trace_opaque", "cull_alpha", "trace_alpha"], s16)},
                       "trace_speedup_vs_plain": round((stage_ms[2] + stage_ms[4]) / (s16[2] + s16[4]), 4),
                       "agreement_with_plain": agree, "tune": tune16}

    if not args.no_static:
        out["static"] = bench_static(torch, vrt, ctx, w, xyz, off, eye, opq, alp, cam_o, cam_a, cap, args.steps,
                                     args.warmup, frame_ms)
    if not args.no_shading:
        out["shading"] = bench_shading(torch, vrt, ctx, w, xyz, off, eye, opq, alp, cam_o, cam_a, args.steps)
    if not args.no_voxelizers:
        out["voxelizers"] = bench_voxelizers(torch, vrt, synth, ctx, w, args.steps)
    if not args.no_alpha_sweep:
        out["alpha_sweep"] = bench_alpha_sweep(torch, vrt, ctx, w, xyz, off, eye, args.steps)
    if not args.no_cpu_baseline:
        cpu_baseline_leg(out, ctx, w, vrt, synth, torch, xyz, off, eye, opq, alp, args, img_plain, img_fp16)
    ctx.close()

    if not args.no_dynamic:
        out["dynamic_pathlines"] = bench_dynamic(torch, vrt, synth, args.warmup)
    if not args.no_batched:
        out["batched"] = bench_batched(torch, vrt, synth, args.steps, args.warmup)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
