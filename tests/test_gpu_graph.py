"""Per-frame HIP graph: a dynamic line set (ABC pathlines advanced every
frame) replayed from one captured graph gives exactly the eager results, on
every replay, with eager work on another context interleaved."""
import numpy as np
import pytest

from paper_2510_09081_amd import synth, vrt

from . import _gpu as G

pytestmark = pytest.mark.gpu


def test_graph_replay_equals_eager():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU: the gpu tests need an MI355X")
    frames = synth.pathline_frames(seed=2, n_seeds=1500, seg_per_line=40, n_frames=6, G=64)
    ls0 = synth.pathline_frame(frames, 0, seg_per_line=40)
    cam = synth.grid_camera(ls0, 160, 96)
    n = cam.width * cam.height
    cap = 40 * ls0.n_segments
    gctx = vrt.Context(max_vertices=ls0.n_vertices, max_fragments=cap, max_dim=64)
    ectx = vrt.Context(max_vertices=ls0.n_vertices, max_fragments=cap, max_dim=64)
    xyz = torch.from_numpy(ls0.xyz).cuda()
    off = torch.from_numpy(ls0.offsets).cuda()
    outs = [(torch.empty(4 * n, device="cuda"), torch.empty(n, device="cuda"),
             torch.empty(n, dtype=torch.int32, device="cuda")) for _ in range(2)]
    eye = np.asarray(cam.eye, np.float32)
    cam_o = G.camera_struct(cam, vrt.TRACE_OPAQUE)
    cam_a = G.camera_struct(cam, vrt.TRACE_TRANSPARENT, 0.3)
    passes = [((eye, vrt.CULL_OPAQUE, 1.0, 1 / 256), cam_o, *outs[0]),
              ((eye, vrt.CULL_ALPHA, 0.3, 1 / 256), cam_a, *outs[1])]
    graph = gctx.frame_graph(xyz, off, ls0.radius, ls0.origin, ls0.voxel_size, ls0.dims, passes)
    try:
        for f in range(6):
            ls = synth.pathline_frame(frames, f, seg_per_line=40)
            xyz.copy_(torch.from_numpy(ls.xyz))  # in place: the graph reads this address
            graph.launch()
            torch.cuda.synchronize()
            got = [[t.cpu().numpy().copy() for t in o] for o in outs]
            assert gctx.frame_status()["device_status"] == 0
            # eager reference on another context, interleaved with the replays
            exyz, eoff = G.to_device(ls)
            ectx.voxelize(exyz, eoff, ls.radius, ls.origin, ls.voxel_size, ls.dims)
            ref = []
            for (view, cm, *_), mode in zip(passes, (0, 1)):
                ectx.cull(*view)
                ref.append(G.run_trace(ectx, cam, mode, alpha=view[2]))
            for (gr, gd, gi), (ei, ed, er) in zip(got, ref):
                assert np.array_equal(gi, ei.astype(np.int32)), f"frame {f}: ids differ"
                assert np.array_equal(gd, ed), f"frame {f}: depth differs"
                assert np.array_equal(gr.reshape(-1, 4), er), f"frame {f}: colour differs"
            assert (got[0][2] >= 0).sum() > 200
    finally:
        graph.close()
        gctx.close()
        ectx.close()
