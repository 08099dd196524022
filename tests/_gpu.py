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
    out["lit"] = lvl(v.lit, 0, np.float32)
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


def lists_equal(words, vis, start, ids, offsets_ref, ids_ref):
    """Canonical list comparison for large grids (vectorized): the visible
    voxels' list starts agree, their ranges tile the id array in brick-major
    order, and every voxel's list holds the same ids in both arrays."""
    cnt = (np.ascontiguousarray(words).ravel() & 0xFFFF).astype(np.int64)
    sel = np.flatnonzero((np.ascontiguousarray(vis).ravel() > 0) & (cnt > 0))
    c = cnt[sel]
    so = np.ascontiguousarray(offsets_ref).ravel()[sel].astype(np.int64)
    sg = np.ascontiguousarray(start).ravel()[sel].astype(np.int64)
    if not np.array_equal(sg, so):
        return False
    order = np.argsort(so, kind="stable")
    so, c = so[order], c[order]
    if len(c) and not np.array_equal(so, np.concatenate([[0], np.cumsum(c)[:-1]])):
        return False
    total = int(c.sum())
    if len(ids) < total or len(ids_ref) < total:
        return False
    label = np.repeat(np.arange(len(c), dtype=np.int64), c) << 32
    kg = np.sort(label | np.asarray(ids[:total], np.int64))
    ko = np.sort(label | np.asarray(ids_ref[:total], np.int64))
    return bool(np.array_equal(kg, ko))


# Certification of a traced pixel by the oracle: every decision that can change
# its result (hit/miss and clip-plane distances, hit-order gaps) has a margin
# above EPS_GEOM voxel, and the hit point lies farther than EPS_FACE0 +
# EPS_FACE_T * t voxel from any voxel face across which its listed status
# changes (binary32 boundary parameters have relative error 2^-24).
EPS_GEOM = 2e-5
EPS_FACE0 = 1e-5
EPS_FACE_T = 2.4e-7
MAX_UNCERTIFIED = 2e-3


def certified(tr):
    t = np.where(np.isfinite(tr.t), tr.t, 0.0)
    return (tr.m_geom > EPS_GEOM) & (tr.m_face > EPS_FACE0 + EPS_FACE_T * t)


def structure_report(fr, got, ids, st=None):
    """Bit-exact comparison of a fetched acceleration structure with the oracle frame, as booleans."""
    r = {"dims": got["dims"] == fr.dims}
    r["words"] = bool(np.array_equal(got["words"], fr.words))
    r["occupancy_levels"] = len(got["occ"]) == len(fr.occ) and all(
        np.array_equal(a, b) for a, b in zip(got["occ"], fr.occ))
    r["blocking"] = bool(np.array_equal(got["blocking"], fr.blocking))
    r["culling_levels"] = len(got["vis"]) == len(fr.vis_levels) and all(
        np.array_equal(a, b) for a, b in zip(got["vis"], fr.vis_levels))
    cnt = (fr.words & 0xFFFF).astype(np.int64)
    start = got["list_end"].astype(np.int64) - cnt * (fr.vis > 0)
    nbx, nby, nbz = fr.dims[0] // 8, fr.dims[1] // 8, fr.dims[2] // 8
    occ_b = np.zeros(nbx * nby * nbz, bool)
    occ_b[got["bricks"]] = True
    occupied = np.repeat(np.repeat(np.repeat(occ_b.reshape(nbz, nby, nbx), 8, 0), 8, 1), 8, 2)
    r["offsets"] = bool(np.array_equal(start[occupied], fr.offsets.astype(np.int64)[occupied]))
    r["lists"] = lists_equal(fr.words, fr.vis, start, ids, fr.offsets, fr.ids)
    if st is not None:
        r["totals"] = (st["n_fragments"] == fr.n_fragments and st["n_listed"] == fr.total
                       and st["n_occupied"] == int((cnt > 0).sum()) and st["n_visible"] == int((fr.vis > 0).sum()))
    return r


def trace_report(tr, gid, gdepth, grgba, voxel_size, mode):
    """Image against the oracle: certified fraction, id equality and errors on certified pixels (with the
    parity tolerances), and the plain error statistics over every pixel."""
    cert = certified(tr)
    hit = cert & (tr.id >= 0)
    dd = np.abs(gdepth[hit].astype(np.float64) - tr.depth[hit]) / float(voxel_size)
    derr_ok = bool((dd <= 1e-5 * tr.t[hit] + 1e-4).all())
    cerr = np.abs(grgba.astype(np.float64) - tr.rgba)
    cc = cerr[cert]
    ctol = 1e-6 if mode == 0 else 1e-4
    same = (gid == tr.id)
    both = (tr.id >= 0) & same
    d_all = np.abs(gdepth[both].astype(np.float64) - tr.depth[both]) / float(voxel_size)
    r = {
        "certified_frac": float(cert.mean()),
        "ids_equal_certified": bool(same[cert].all()),
        "depth_within_tol_certified": derr_ok and bool(np.isinf(gdepth[cert & (tr.id < 0)]).all()),
        "colour_within_tol_certified": bool(cc.max(initial=0) <= ctol and (mode == 0 or cc.mean() <= 1e-6)),
        "id_match_all": float(same.mean()),
        "id_match_certified": float(same[cert].mean()) if cert.any() else 1.0,
        "colour_err_max": float(cerr.max()), "colour_err_mean": float(cerr.mean()),
        "depth_err_max_vox": float(d_all.max(initial=0)), "depth_err_mean_vox": float(d_all.mean()) if d_all.size else 0.0,
        "hit_pixels": int((tr.id >= 0).sum()),
    }
    r["pass"] = (r["ids_equal_certified"] and r["depth_within_tol_certified"] and r["colour_within_tol_certified"]
                 and 1.0 - r["certified_frac"] <= MAX_UNCERTIFIED)
    return r

