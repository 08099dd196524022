"""Batched form: many uneven line sets built and traced in one persistent
(cooperative) launch give exactly the results of the plain calls set by set,
and a set of the batch matches the oracle."""
import numpy as np
import pytest

from paper_2510_09081_amd import synth, vrt

from . import _gpu as G
from .test_gpu_parity import compare_structure, certified

pytestmark = pytest.mark.gpu


def small_batch(n=10, seed=7):
    rng = np.random.default_rng(seed)
    sets = []
    for k in range(n):
        G_ = int(rng.choice([32, 48, 64, 96, 128]))
        if k % 2 == 0:
            ls = synth.random_walk_set(seed=int(rng.integers(1 << 30)), n_poly=int(rng.integers(5, 80)),
                                       n_seg=int(rng.integers(5, 50)), G=G_)
        else:
            ls = synth.bundle_set(seed=int(rng.integers(1 << 30)), n_bundles=int(rng.integers(1, 3)),
                                  per_bundle=int(rng.integers(20, 300)), G=G_, len_lo=10, len_hi=60)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        c = np.array([0.5, 0.5, 0.5])
        up = (0.0, 1.0, 0.0) if abs(u[2]) > 0.99 else (0.0, 0.0, 1.0)
        W, H = int(rng.integers(40, 130)), int(rng.integers(30, 110))
        cam = synth.Camera(eye=c + 2.0 * u, target=c, up=np.array(up), fovy_deg=60.0, width=W, height=H)
        mode = k % 3 == 2  # some transparent passes
        cull = [vrt.CULL_OPAQUE, vrt.CULL_NONE, vrt.CULL_ALPHA][k % 3]
        sets.append((ls, cam, cull, 1 if mode else 0))
    return sets


def make_items(sets):
    import torch
    items = []
    for ls, cam, cull, mode in sets:
        n = cam.width * cam.height
        x, o = G.to_device(ls)
        alpha = 0.3 if (mode or cull == vrt.CULL_ALPHA) else 1.0
        items.append(dict(xyz=x, offsets=o, radius=ls.radius, origin=ls.origin, voxel_size=ls.voxel_size, dims=ls.dims,
                          view=(np.asarray(cam.eye, np.float32), cull, alpha, 1 / 256),
                          camera=G.camera_struct(cam, mode, alpha), rgba=torch.zeros(4 * n, device="cuda"),
                          depth=torch.zeros(n, device="cuda"), first_id=torch.zeros(n, dtype=torch.int32, device="cuda")))
    return items


def caps(sets):
    return [(ls.n_vertices, 30 * max(ls.n_segments, 1), max(ls.dims), cam.width * cam.height) for ls, cam, _, _ in sets]


def test_persistent_batch_equals_sequential(orc):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU: the gpu tests need an MI355X")
    sets = small_batch()
    pb, sb, tb, xb = vrt.Batch(caps(sets)), vrt.Batch(caps(sets)), vrt.Batch(caps(sets)), vrt.Batch(caps(sets))
    try:
        ip, isq, ist, isp = make_items(sets), make_items(sets), make_items(sets), make_items(sets)
        for rep in range(3):  # repeated launches reuse the arenas and the ticket counters
            pb.run(ip, vrt.BATCH_PERSISTENT)
            sb.run(isq, vrt.BATCH_SEQUENTIAL)
            tb.run(ist, vrt.BATCH_STAGED)
            xb.run(isp, vrt.BATCH_SPLIT)
            torch.cuda.synchronize()
            for i in range(len(sets)):
                sp, ss, s3 = pb.context(i).frame_status(), sb.context(i).frame_status(), tb.context(i).frame_status()
                s4 = xb.context(i).frame_status()
                assert sp["device_status"] == ss["device_status"] == s3["device_status"] == s4["device_status"] == 0
                assert (sp["n_fragments"], sp["n_listed"], sp["n_bricks"]) == \
                       (ss["n_fragments"], ss["n_listed"], ss["n_bricks"]) == \
                       (s3["n_fragments"], s3["n_listed"], s3["n_bricks"]) == \
                       (s4["n_fragments"], s4["n_listed"], s4["n_bricks"]), (rep, i)
                for key in ("rgba", "depth", "first_id"):
                    assert torch.equal(ip[i][key], isq[i][key]), (rep, i, key)
                    assert torch.equal(ist[i][key], isq[i][key]), (rep, i, key)
                    assert torch.equal(isp[i][key], isq[i][key]), (rep, i, key)
        # one set of the persistent batch against the oracle
        k = 4
        ls, cam, cull, mode = sets[k]
        alpha = 0.3 if (mode or cull == vrt.CULL_ALPHA) else 1.0
        fr = orc.build_frame(ls, cam.eye, cull, alpha=alpha)
        compare_structure(orc, fr, G.fetch_as(pb.context(k)), ids=G.fetch_ids(pb.context(k), fr.total))
        tr = orc.trace(fr, ls, cam, np.arange(cam.width * cam.height), mode, alpha=alpha)
        gid = ip[k]["first_id"].cpu().numpy()
        cert = certified(tr, mode)
        assert not (cert & (gid != tr.id)).any()
        assert (tr.id >= 0).sum() > 50
    finally:
        pb.close()
        sb.close()
        tb.close()
        xb.close()


def test_batch_uses_each_sets_shade_group(orc):
    """Sets whose contexts carry different tuned shade groups (8, 16, 32 lanes per ray): the persistent and
    staged and split launches still give the sequential calls' images exactly."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU: the gpu tests need an MI355X")
    sets = small_batch(n=6, seed=11)
    pb, sb, tb, xb = vrt.Batch(caps(sets)), vrt.Batch(caps(sets)), vrt.Batch(caps(sets)), vrt.Batch(caps(sets))
    try:
        for bb in (pb, sb, tb, xb):
            for i, (_, _, _, mode) in enumerate(sets):
                bb.context(i).set_tune(mode, shade_group=(8, 16, 32)[i % 3])
        ip, isq, ist, isp = make_items(sets), make_items(sets), make_items(sets), make_items(sets)
        pb.run(ip, vrt.BATCH_PERSISTENT)
        sb.run(isq, vrt.BATCH_SEQUENTIAL)
        tb.run(ist, vrt.BATCH_STAGED)
        xb.run(isp, vrt.BATCH_SPLIT)
        torch.cuda.synchronize()
        for i in range(len(sets)):
            for key in ("rgba", "depth", "first_id"):
                assert torch.equal(ip[i][key], isq[i][key]), (i, key)
                assert torch.equal(ist[i][key], isq[i][key]), (i, key)
                assert torch.equal(isp[i][key], isq[i][key]), (i, key)
    finally:
        pb.close()
        sb.close()
        tb.close()
        xb.close()
