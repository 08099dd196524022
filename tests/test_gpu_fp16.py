"""FP16 precision form: brick-relative binary16 segment records in the tracer.

Voxel membership, lists and culling are unchanged (int32); the tracer reads
binary16 endpoints (exact here: offsets below 8 voxels on the 1/256 grid) and
16-bit fixed-point clip normals (absolute error below 2^-16), so results differ
from the plain form only where a hit point lies within ~1e-5 voxel of a clip
plane.  The
error against the binary64 oracle is reported and bounded.
"""
import numpy as np
import pytest

from paper_2510_09081_amd import synth, vrt

from . import _gpu as G
from .test_gpu_parity import certified

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctxs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU: the gpu tests need an MI355X")
    plain = vrt.Context(max_vertices=300_000, max_fragments=4_000_000, max_dim=128, form=vrt.FORM_PLAIN)
    half = vrt.Context(max_vertices=300_000, max_fragments=4_000_000, max_dim=128, form=vrt.FORM_FP16)
    yield plain, half
    plain.close()
    half.close()


def error_report(tr, gid, gdepth, grgba, ls):
    cert = certified(tr, 0)
    hit = tr.id >= 0
    match = (gid == tr.id)
    vs = float(ls.voxel_size)
    both = hit & (gid >= 0) & match
    derr = np.abs(gdepth[both].astype(np.float64) - tr.depth[both]) / vs
    cerr = np.abs(grgba.astype(np.float64) - tr.rgba)
    return {
        "id_match_all": float(match.mean()),
        "id_match_certified": float(match[cert].mean()),
        "depth_err_max_vox": float(derr.max(initial=0)), "depth_err_mean_vox": float(derr.mean() if derr.size else 0),
        "colour_err_max": float(cerr.max()), "colour_err_mean": float(cerr.mean()),
    }


@pytest.mark.parametrize("name", ["random_walk_10k", "bundles_small"])
@pytest.mark.parametrize("mode,cull,alpha", [(0, vrt.CULL_NONE, 1.0), (1, vrt.CULL_NONE, 0.3)])
def test_fp16_form_error_against_oracle(orc, ctxs, name, mode, cull, alpha):
    plain, half = ctxs
    w = synth.workload(name)
    ls, cam = w.lines, w.camera
    fr = orc.build_frame(ls, cam.eye, cull, alpha=alpha)
    tr = orc.trace(fr, ls, cam, np.arange(cam.width * cam.height), mode, alpha=alpha)
    out = {}
    for label, ctx in (("plain", plain), ("fp16", half)):
        G.run_build(ctx, ls, cam.eye, cull, alpha=alpha)
        assert ctx.frame_status()["device_status"] == 0
        out[label] = G.run_trace(ctx, cam, mode, alpha=alpha)
        out[label + "_err"] = error_report(tr, *out[label], ls)
    print(f"\n{name} mode={mode}: plain {out['plain_err']}\n{name} mode={mode}: fp16  {out['fp16_err']}")
    e = out["fp16_err"]
    # the FP16 form agrees with the oracle on every certified pixel (exact endpoints, normals within 2^-16) ...
    assert e["id_match_certified"] == 1.0
    assert e["colour_err_mean"] <= 1e-6
    # ... and with the plain form except where a hit lies within ~1e-5 voxel of
    # a clip plane (a flipped clip decision changes that pixel by one layer)
    same = out["plain"][0] == out["fp16"][0]
    assert same.mean() >= 0.9999
    d = np.abs(out["plain"][2] - out["fp16"][2]).max(axis=1)
    assert (d > 1e-4).mean() <= 2e-4
    assert d.mean() <= 1e-5


def test_fp16_form_reads_long_segments_from_plain_records(orc, ctxs):
    """Single-segment polylines of 40-60 voxels: 99% have a brick-relative offset of 8 voxels or more,
    which binary16 cannot hold on the 1/256 grid, and the FP16 form reads those from the plain vertex
    records.  Without clip planes (no interior vertices) both kinds of record give the same binary32
    endpoints, so the FP16 images equal the plain form's bit for bit (and match the oracle)."""
    plain, half = ctxs
    ls = synth.random_walk_set(seed=17, n_poly=200, n_seg=1, G=128, step_lo=40.0, step_hi=60.0)
    cam = synth.grid_camera(ls, 200, 150)
    for mode, cull, alpha in ((0, vrt.CULL_OPAQUE, 1.0), (1, vrt.CULL_NONE, 0.3)):
        out = []
        for ctx in (plain, half):
            G.run_build(ctx, ls, cam.eye, cull, alpha=alpha)
            assert ctx.frame_status()["device_status"] == 0
            out.append(G.run_trace(ctx, cam, mode, alpha=alpha))
        for a, b in zip(out[0], out[1]):
            assert np.array_equal(a, b)
        fr = orc.build_frame(ls, cam.eye, cull, alpha=alpha)
        tr = orc.trace(fr, ls, cam, np.arange(cam.width * cam.height), mode, alpha=alpha)
        cert = certified(tr, mode)
        assert (tr.id >= 0).sum() > 500
        assert not (cert & (out[1][0] != tr.id)).any()


def test_fp16_form_mixed_long_and_short(orc, ctxs):
    """Short segments (exact binary16 offsets) next to long ones (plain records): first hits agree with the
    oracle on the certified pixels."""
    plain, half = ctxs
    short = synth.random_walk_set(seed=18, n_poly=60, n_seg=40, G=128)
    long_ = synth.random_walk_set(seed=19, n_poly=30, n_seg=4, G=128, step_lo=20.0, step_hi=60.0)
    ls = synth.LineSet(xyz=np.concatenate([short.xyz, long_.xyz]),
                       offsets=np.concatenate([short.offsets, short.offsets[-1] + long_.offsets[1:]]).astype(np.int32),
                       radius=short.radius, origin=short.origin, voxel_size=short.voxel_size, dims=short.dims)
    cam = synth.grid_camera(ls, 240, 180)
    fr = orc.build_frame(ls, cam.eye, vrt.CULL_NONE)
    tr = orc.trace(fr, ls, cam, np.arange(cam.width * cam.height), 0)
    G.run_build(half, ls, cam.eye, vrt.CULL_NONE)
    gid, gdepth, grgba = G.run_trace(half, cam, 0)
    cert = certified(tr, 0)
    assert (tr.id >= 0).sum() > 1000
    assert ((gid == tr.id)[cert]).mean() == 1.0
    e = error_report(tr, gid, gdepth, grgba, ls)
    assert e["colour_err_mean"] <= 1e-6
