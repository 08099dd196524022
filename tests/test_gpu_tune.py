"""Tracer launch shapes and the autotuner: every shape gives the same image,
bit for bit (opaque and transparent, plain and FP16 records); invalid shapes
are rejected without changing the context; the autotuner sets a valid shape,
stores it in its cache file and finds it there on the next call."""
import json

import numpy as np
import pytest

from paper_2510_09081_amd import synth, vrt

from . import _gpu as G

pytestmark = pytest.mark.gpu

SHAPES = [
    dict(march_threads=128, shade_group=8, shade_batch=2, lane_keys=4, shade_blocks=256),
    dict(march_threads=512, shade_group=32, shade_batch=4, lane_keys=8, shade_blocks=8192),
    dict(march_threads=256, shade_group=8, shade_batch=4, lane_keys=8, shade_blocks=1024),
    dict(march_threads=128, shade_group=32, shade_batch=2, lane_keys=4, shade_blocks=65535),
    dict(march_threads=256, shade_group=16, shade_batch=2, lane_keys=8, shade_blocks=300),
]


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU: the gpu tests need an MI355X")


def _passes(w):
    return [(p.cull_mode, vrt.TRACE_OPAQUE if p.trace_mode == synth.MODE_OPAQUE else vrt.TRACE_TRANSPARENT,
             p.alpha)
            for p in w.passes]


@pytest.mark.parametrize("form", [vrt.FORM_PLAIN, vrt.FORM_FP16])
def test_every_shape_gives_the_same_image(form):
    _need_gpu()
    w = synth.workload("bundles_small")
    ls, cam = w.lines, w.camera
    ctx = vrt.Context(max_vertices=ls.n_vertices, max_fragments=40 * ls.n_segments, max_dim=max(ls.dims),
                      form=form)
    try:
        dev = G.to_device(ls)
        for cull, mode, alpha in _passes(w):
            G.run_build(ctx, ls, cam.eye, cull, alpha, dev=dev)
            ref = G.run_trace(ctx, cam, mode, alpha)
            assert (ref[0] >= 0).sum() > 1000
            default = ctx.get_tune(mode)
            for shape in SHAPES:
                ctx.set_tune(mode, **shape)
                assert ctx.get_tune(mode) == shape
                got = G.run_trace(ctx, cam, mode, alpha)
                for a, b, what in zip(got, ref, ("ids", "depth", "rgba")):
                    assert np.array_equal(a, b), f"cull {cull} mode {mode} shape {shape}: {what} differ"
            ctx.set_tune(mode, **default)
    finally:
        ctx.close()


def test_invalid_shapes_are_rejected():
    _need_gpu()
    ctx = vrt.Context(max_vertices=64, max_fragments=1024, max_dim=16)
    try:
        before = ctx.get_tune(vrt.TRACE_OPAQUE)
        for bad in (dict(march_threads=64), dict(march_threads=1024), dict(shade_group=4), dict(shade_group=64),
                    dict(shade_batch=3), dict(lane_keys=16), dict(shade_blocks=255), dict(shade_blocks=65536)):
            with pytest.raises(vrt.VrtError) as e:
                ctx.set_tune(vrt.TRACE_OPAQUE, **bad)
            assert e.value.status == vrt.VRT_ERR_INVALID_ARG
            assert ctx.get_tune(vrt.TRACE_OPAQUE) == before
        with pytest.raises(vrt.VrtError):
            ctx.get_tune(7)
    finally:
        ctx.close()


def test_autotune_sets_a_shape_and_uses_its_cache(tmp_path):
    import torch
    _need_gpu()
    w = synth.workload("bundles_small")
    ls, cam = w.lines, w.camera
    n = cam.width * cam.height
    ctx = vrt.Context(max_vertices=ls.n_vertices, max_fragments=40 * ls.n_segments, max_dim=max(ls.dims))
    cache = tmp_path / "tune.json"
    try:
        G.run_build(ctx, ls, cam.eye, synth.CULL_ALPHA, 0.2)
        ref = G.run_trace(ctx, cam, vrt.TRACE_TRANSPARENT, 0.2)
        cs = G.camera_struct(cam, vrt.TRACE_TRANSPARENT, 0.2)
        rgba = torch.empty(4 * n, device="cuda")
        r1 = ctx.autotune(cs, rgba, reps=2, warmup=1, sweeps=1, cache_path=str(cache), key="bundles_small")
        assert not r1["from_cache"] and r1["evaluated"] == 11  # start + 2 + 2 + 1 + 1 + 4
        assert r1["best"] == ctx.get_tune(vrt.TRACE_TRANSPARENT)
        assert 0 < r1["best_ms"] <= r1["start_ms"] * 1.0001
        # the opaque shape is untouched
        assert ctx.get_tune(vrt.TRACE_OPAQUE) == dict(march_threads=256, shade_group=16, shade_batch=2, lane_keys=4,
                                                      shade_blocks=4096)
        got = G.run_trace(ctx, cam, vrt.TRACE_TRANSPARENT, 0.2)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
        entries = json.loads(cache.read_text())
        assert len(entries) == 1
        (key, val), = entries.items()
        assert key.endswith("|bundles_small") and "|transparent|" in key
        assert {k: val[k] for k in r1["best"]} == r1["best"]
        # a later call finds the entry without timing anything
        ctx.set_tune(vrt.TRACE_TRANSPARENT, march_threads=128, shade_group=8, shade_batch=2, lane_keys=4,
                     shade_blocks=256)
        r2 = ctx.autotune(cs, rgba, reps=2, warmup=1, sweeps=1, cache_path=str(cache), key="bundles_small")
        assert r2["from_cache"] and r2["evaluated"] == 0 and r2["best"] == r1["best"]
        assert ctx.get_tune(vrt.TRACE_TRANSPARENT) == r1["best"]
        # another key searches again and adds an entry
        r3 = ctx.autotune(cs, rgba, reps=1, warmup=0, sweeps=1, cache_path=str(cache), key="other")
        assert not r3["from_cache"]
        assert len(json.loads(cache.read_text())) == 2
        with pytest.raises(vrt.VrtError):
            ctx.autotune(cs, rgba, reps=0)
    finally:
        ctx.close()


def test_autotune_grid_times_fitting_grids():
    import torch
    _need_gpu()
    w = synth.workload("bundles_small")
    ls, cam = w.lines, w.camera
    n = cam.width * cam.height
    base = ls.dims[0]
    grids = [(ls.origin, ls.voxel_size * base / g, (g, g, g)) for g in (64, 128, 256)]
    eye = np.asarray(cam.eye, np.float32)
    xyz, off = G.to_device(ls)
    out = [(torch.empty(4 * n, device="cuda"), torch.empty(n, device="cuda"),
            torch.empty(n, dtype=torch.int32, device="cuda")) for _ in range(2)]
    passes = [((eye, vrt.CULL_OPAQUE, 1.0, 1 / 256), G.camera_struct(cam, vrt.TRACE_OPAQUE), *out[0]),
              ((eye, vrt.CULL_ALPHA, 0.2, 1 / 256), G.camera_struct(cam, vrt.TRACE_TRANSPARENT, 0.2), *out[1])]
    big = vrt.Context(max_vertices=ls.n_vertices, max_fragments=80 * ls.n_segments, max_dim=256)
    need, ids = [], []
    try:
        for origin, vs, dims in grids:
            big.voxelize(xyz, off, ls.radius, origin, vs, dims)
            req = 0
            for view, cm, r, d, f in passes:
                big.cull(*view)
                big.trace(cm, r, d, f)
                st = big.frame_status()
                assert st["device_status"] == 0
                req = max(req, st["n_listed"])
            need.append(req)
            ids.append(out[0][2].cpu().numpy().copy())
    finally:
        big.close()
    # the grid only narrows the search: the opaque first hits agree across grids up to rounding near ties
    hit = ids[1] >= 0
    assert hit.sum() > 1000
    for other in (ids[0], ids[2]):
        assert (other == ids[1]).mean() >= 0.999
    assert need[2] > max(need[0], need[1])  # the finest grid needs the most list entries
    ctx = vrt.Context(max_vertices=ls.n_vertices, max_fragments=max(need[0], need[1]), max_dim=256)
    try:
        best, ms = ctx.autotune_grid(xyz, off, ls.radius, grids, passes, reps=2, warmup=1)
        assert ms[2] == float("inf")  # does not fit the capacity
        assert all(0 < m < float("inf") for m in ms[:2])
        assert best in (0, 1) and ms[best] == min(ms)
        assert ctx.frame_status()["device_status"] == 0
        with pytest.raises(vrt.VrtError) as e:
            ctx.autotune_grid(xyz, off, ls.radius, [(ls.origin, ls.voxel_size, (12, 12, 12))], passes)
        assert e.value.status == vrt.VRT_ERR_INVALID_ARG
        with pytest.raises(vrt.VrtError) as e:
            ctx.autotune_grid(xyz, off, ls.radius, grids[2:], passes)
        assert e.value.status == vrt.VRT_ERR_CAPACITY
    finally:
        ctx.close()
