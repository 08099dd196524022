"""Drive every oracle entry point on small inputs, for the AddressSanitizer /
UndefinedBehaviorSanitizer build of the oracle (tests/test_sanitizers.py).

Usage: python sanitize_oracle_run.py <path of the sanitized liboracle.so>

The inputs cover the same shapes the parity tests use: random walks on a
non-cubic grid, segments leaving the grid on every side, zero-length and
zero-radius segments, a brick crowded past the 16-bit count, segments whose
box spans many bricks; all four membership modes, the three culling modes,
opaque and transparent traces with and without per-segment colours and
shading.  Prints "ok" when every call returned.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2510_09081_amd import synth  # noqa: E402


def _lines(polys, G, radius_vox, dims=None):
    vs = np.float32(1.0 / G)
    xyz = np.concatenate([np.asarray(p, np.float64).reshape(-1, 3) for p in polys]) * float(vs)
    off = np.concatenate([[0], np.cumsum([len(p) for p in polys])]).astype(np.int32)
    return synth.LineSet(xyz=xyz.astype(np.float32), offsets=off, radius=float(np.float32(radius_vox * vs)),
                         origin=np.zeros(3, np.float32), voxel_size=float(vs), dims=dims or (G, G, G))


def sets():
    rng = np.random.default_rng(3)
    yield "random_walk", synth.random_walk_set(seed=11, n_poly=40, n_seg=20, G=32)
    rw = synth.random_walk_set(seed=5, n_poly=20, n_seg=15, G=24)
    yield "non_cubic", synth.LineSet(**{**rw.__dict__, "dims": (24, 16, 40)})
    yield "outside_and_zero", _lines([[[-3, 8, 8], [20, 8.5, 7.5]], [[8, -4, 8], [8.3, 19, 9]],
                                      [[5.5, 5.5, 5.5], [5.5, 5.5, 5.5], [6.5, 5.5, 5.5]],
                                      [[15.9, 15.9, 15.9], [17, 17, 17]], [[2, 2, 2]]], 16, 0.5)
    yield "zero_radius", _lines([[[1.3, 2.7, 3.1], [14.2, 12.9, 6.6]]], 16, 0.0)
    yield "long", _lines([[[2.5, 3.1, 4.2], [60.3, 41.7, 55.9], [10.2, 58.8, 30.1]],
                          [[63.5, 0.5, 32.0], [0.5, 63.5, 32.0]]], 64, 0.7)
    crowd = [1.0 + np.cumsum(rng.uniform(-0.3, 0.3, (12, 3)), axis=0).clip(-0.5, 5.5) + rng.uniform(0, 1, 3)
             for _ in range(300)]
    yield "crowded_brick", _lines(crowd, 16, 0.3)


def main(lib_path):
    orc.LIB = lib_path  # the sanitized build, loaded instead of the plain one
    for name, ls in sets():
        cam = synth.grid_camera(ls, 48, 32)
        pix = np.arange(cam.width * cam.height)
        for mode in (orc.VOX_CAPSULE, 1, 2, 3):
            lit_kw = {"literal": True} if mode == 1 else {"mode": mode}
            fr = orc.build_frame(ls, cam.eye, orc.CULL_OPAQUE, **lit_kw)
            orc.recull_frame(fr, ls, cam.eye, orc.CULL_ALPHA, 0.3)
            orc.recull_frame(fr, ls, cam.eye, orc.CULL_NONE)
        fr = orc.build_frame(ls, cam.eye, orc.CULL_ALPHA, alpha=0.3)
        rgba = np.random.default_rng(1).uniform(0, 1, (len(ls.xyz), 4)).astype(np.float32)
        lit = None
        if len(fr.occ) >= 3:
            _, _, lit = orc.shade(fr.occ, fr.vis, n_cones=6, n_samples=2)
        for tmode in (0, 1):
            orc.trace(fr, ls, cam, pix, tmode, alpha=0.3)
            orc.trace(fr, ls, cam, pix[::7], tmode, alpha=0.3, seg_rgba=rgba, lit=lit)
        orc.trace(fr, ls, cam, pix[::5], 0, brute=True)
        print(name, fr.n_fragments, fr.total, flush=True)
    assert orc.lib()._name == lib_path, "the plain oracle was loaded"
    print("ok", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
