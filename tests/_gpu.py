"""Test helpers: run the HIP path on a workload and read its outputs back.

The library exports brick-major arrays (8^3 bricks, x fastest inside a
brick); these helpers gather the occupied bricks into dense x-fastest numpy
arrays, the layout the oracle uses.
"""
from __future__ import annotations

import numpy as np

from paper_2510_09081_amd import vrt

BRICK_SHAPES = {0: 8, 1: 4, 2: 2}


def to_device(ls):
    import torch
    xyz = torch.from_numpy(np.ascontiguousarray(ls.xyz, np.float32)).cuda()
    off = torch.from_numpy(np.ascontiguousarray(ls.offsets, np.int32)).cuda()
    return xyz, off


def run_build(ctx, ls, eye, cull_mode, alpha=1.0, tau=1.0 / 256.0, dev=None):
    import torch
    xyz, off = dev if dev is not None else to_device(ls)
    ctx.voxelize(xyz, off, ls.radius, ls.origin, ls.voxel_size, ls.dims)
    ctx.cull(np.asarray(eye, np.float32), cull_mode, alpha, tau)
    torch.cuda.synchronize()
    return xyz, off


def camera_struct(cam, mode, alpha=1.0, tau=1.0 / 256.0):
    return vrt.make_camera(cam.eye, cam.target, cam.up, cam.fovy_deg, cam.width, cam.height, mode, alpha, tau)


def run_trace(ctx, cam, mode, alpha=1.0, tau=1.0 / 256.0):
    import torch
    n = cam.width * cam.height
    rgba = torch.empty(n * 4, dtype=torch.float32, device="cuda")
    depth = torch.empty(n, dtype=torch.float32, device="cuda")
    fid = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx.trace(camera_struct(cam, mode, alpha, tau), rgba, depth, fid)
    torch.cuda.synchronize()
    return fid.cpu().numpy().astype(np.int64), depth.cpu().numpy(), rgba.cpu().numpy().reshape(n, 4)


def debug_rays(ctx, cam, pix):
    import torch
    p = torch.from_numpy(np.ascontiguousarray(pix, np.int64)).cuda()
    d = torch.empty(len(pix) * 3, dtype=torch.float32, device="cuda")
    ctx.debug_rays(camera_struct(cam, 0), p, d)
    torch.cuda.synchronize()
    return d.cpu().numpy().reshape(-1, 3)


def _dense_from_bricks(raw, bricks, dims, level, dtype):
    """raw: per-brick blocks (brick-major) at `level` (0, 1, 2) -> dense (Gz, Gy, Gx)."""
    e = BRICK_SHAPES[level]
    gx, gy, gz = (d >> level for d in dims)
    nbx, nby, nbz = dims[0] // 8, dims[1] // 8, dims[2] // 8
    out = np.zeros((nbz, nby, nbx, e, e, e), dtype)
    blocks = raw.reshape(-1, e, e, e)
    bz, rem = np.divmod(bricks, nbx * nby)
    by, bx = np.divmod(rem, nbx)
    out[bz, by, bx] = blocks[bricks]
    return out.transpose(0, 3, 1, 4, 2, 5).reshape(gz, gy, gx)


def fetch_as(ctx):
    """Reads the acceleration structure into dense arrays."""
    v = ctx.query_as()
    dims = tuple(v.dims)
    nb = v.n_bricks
    bricks = vrt.copy_to_host(v.brick_list, nb * 4, np.int32, nb).astype(np.int64)
    top = int(bricks.max()) + 1 if nb else 0
    nbx, nby, nbz = dims[0] // 8, dims[1] // 8, dims[2] // 8
    NB = nbx * nby * nbz

    def lvl(ptr, level, dtype):
        per = 512 >> (3 * level)
        raw = vrt.copy_to_host(ptr, top * per * np.dtype(dtype).itemsize, dtype, top * per)
        return _dense_from_bricks(raw, bricks, dims, level, dtype)

    out = {"dims": dims, "bricks": bricks, "n_levels": v.n_levels}
    out["words"] = lvl(v.words, 0, np.uint32)
    out["occ"] = [lvl(v.occ[0], 0, np.uint16), lvl(v.occ[1], 1, np.uint16), lvl(v.occ[2], 2, np.uint16)]
    out["occ"].append(vrt.copy_to_host(v.occ[3], NB * 2, np.uint16, NB).reshape(nbz, nby, nbx))
    out["blocking"] = lvl(v.blocking, 0, np.uint8)
    out["vis"] = [lvl(v.vis[0], 0, np.uint8), lvl(v.vis[1], 1, np.uint8), lvl(v.vis[2], 2, np.uint8)]
    out["vis"].append(vrt.copy_to_host(v.vis[3], NB, np.uint8, NB).reshape(nbz, nby, nbx))
    # levels >= 4, dense, back to back
    d = [nbx, nby, nbz]
    off_elems = 0
    hi_dims = []
    while d != [1, 1, 1]:
        d = [(x + 1) // 2 for x in d]
        hi_dims.append(tuple(d))
    tot = sum(a * b * c for a, b, c in hi_dims)
    occ_hi = vrt.copy_to_host(v.occ_hi, tot * 2, np.uint16, tot)
    vis_hi = vrt.copy_to_host(v.vis_hi, tot, np.uint8, tot)
    for (a, b, c) in hi_dims:
        n = a * b * c
        out["occ"].append(occ_hi[off_elems:off_elems + n].reshape(c, b, a))
        out["vis"].append(vis_hi[off_elems:off_elems + n].reshape(c, b, a))
        off_elems += n
    out["list_end"] = lvl(v.list_end, 0, np.uint32)
    return out


def fetch_ids(ctx, n):
    v = ctx.query_as()
    return vrt.copy_to_host(v.ids, n * 4, np.uint32, n)


def canonical_lists(words, vis, start, ids):
    """{dense voxel index: sorted id tuple} over visible voxels with a list."""
    cnt = (words & 0xFFFF).astype(np.int64)
    sel = np.flatnonzero((vis.ravel() > 0) & (cnt.ravel() > 0))
    s = start.ravel()[sel].astype(np.int64)
    c = cnt.ravel()[sel]
    return {int(v): tuple(sorted(ids[a:a + n].tolist())) for v, a, n in zip(sel, s, c)}
