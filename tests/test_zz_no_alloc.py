"""The no-allocation frame (vrt_frame_noalloc, fixed per-device arena) gives
exactly the images of the per-stage calls (vrt_voxelize, vrt_cull,
vrt_trace on a context) for the same inputs, on two calls in a row (the
second with a smaller input), and rejects sizes beyond its limits before
enqueuing anything."""
import numpy as np
import pytest

from paper_2510_09081_amd import synth, vrt

from . import _gpu as G

pytestmark = pytest.mark.gpu


def _images(n):
    import torch
    return (torch.full((4 * n,), -7.0, device="cuda"), torch.full((n,), -7.0, device="cuda"),
            torch.full((n,), -7, dtype=torch.int32, device="cuda"))


def _reference(ls, cam, view, mode, alpha):
    """The per-stage calls on a context of the same capacities."""
    import torch
    ctx = vrt.Context(max_vertices=vrt.NOALLOC_MAX_VERTICES, max_fragments=vrt.NOALLOC_MAX_FRAGMENTS,
                      max_dim=vrt.NOALLOC_MAX_DIM, max_pixels=vrt.NOALLOC_MAX_PIXELS)
    try:
        xyz, off = G.to_device(ls)
        ctx.voxelize(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims)
        ctx.cull(*view)
        rgba, depth, fid = _images(cam.width * cam.height)
        ctx.trace(G.camera_struct(cam, mode, alpha), rgba, depth, fid)
        st = ctx.frame_status()
        torch.cuda.synchronize()
        return st, rgba.cpu().numpy(), depth.cpu().numpy(), fid.cpu().numpy()
    finally:
        ctx.close()


def _noalloc(ls, cam, view, mode, alpha):
    import torch
    xyz, off = G.to_device(ls)
    rgba, depth, fid = _images(cam.width * cam.height)
    st = vrt.frame_noalloc(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims, view,
                           G.camera_struct(cam, mode, alpha), rgba, depth, fid)
    torch.cuda.synchronize()
    return st, rgba.cpu().numpy(), depth.cpu().numpy(), fid.cpu().numpy()


CASES = [
    # (line set, image, cull, trace mode, alpha): the second is smaller in every respect
    (lambda: synth.random_walk_set(seed=0, n_poly=200, n_seg=50, G=64), (256, 256), vrt.CULL_OPAQUE, 0, 1.0),
    (lambda: synth.random_walk_set(seed=9, n_poly=40, n_seg=30, G=32), (97, 61), vrt.CULL_ALPHA, 1, 0.3),
]


def test_noalloc_frames_equal_the_per_stage_calls():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU: the gpu tests need an MI355X")
    for k, (make, (W, H), cull, mode, alpha) in enumerate(CASES):
        ls = make()
        cam = synth.grid_camera(ls, W, H)
        view = (np.asarray(cam.eye, np.float32), cull, alpha, 1.0 / 256.0)
        print(f"case {k}: {ls.n_segments} segments, {ls.dims}, {W}x{H}, cull {cull}, mode {mode}", flush=True)
        got = _noalloc(ls, cam, view, mode, alpha)
        ref = _reference(ls, cam, view, mode, alpha)
        assert got[0] == ref[0], (got[0], ref[0])
        assert got[0]["device_status"] == 0 and got[0]["n_listed"] > 0
        for a, b, what in zip(got[1:], ref[1:], ("rgba", "depth", "first_id")):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"case {k}: {what} differs"
        assert (got[3] >= 0).sum() > 100


def test_noalloc_rejects_sizes_beyond_its_limits():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU: the gpu tests need an MI355X")
    ls = synth.random_walk_set(seed=3, n_poly=10, n_seg=10, G=32)
    cam = synth.grid_camera(ls, 16, 16)
    view = (np.asarray(cam.eye, np.float32), vrt.CULL_NONE, 1.0, 1.0 / 256.0)
    xyz, off = G.to_device(ls)
    rgba, depth, fid = _images(16 * 16)
    with pytest.raises(vrt.VrtError) as e:  # grid beyond the largest dimension
        vrt.frame_noalloc(xyz, off, ls.radius, ls.origin, ls.voxel_size, (128, 32, 32), view,
                          G.camera_struct(cam, 0), rgba, depth, fid)
    assert e.value.status == vrt.VRT_ERR_CAPACITY
    big = synth.grid_camera(ls, 1024, 512)
    with pytest.raises(vrt.VrtError) as e:  # image beyond the largest pixel count
        vrt.frame_noalloc(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims, view,
                          G.camera_struct(big, 0), rgba, depth, fid)
    assert e.value.status == vrt.VRT_ERR_CAPACITY
    # a valid call afterwards works
    st = vrt.frame_noalloc(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims, view,
                           G.camera_struct(cam, 0), rgba, depth, fid)
    assert st["device_status"] == 0
