"""Python driver for the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It loads ``liboracle.so`` built from ``vrt_oracle.c``
(plain C, gcc, ``-ffp-contract=off``) and returns numpy arrays in plain dense
x-fastest layout: a level of shape (Gz, Gy, Gx).

The oracle follows arXiv 2510.09081 Section 3: voxelization (3.1, Alg. 1-3),
culling (3.2), per-voxel fragment lists (3.3) and ray tracing (3.5).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import time
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vrt_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

ST_OK, ST_RANGE, ST_COUNT_OVERFLOW = 0, 2, 5
CULL_NONE, CULL_OPAQUE, CULL_ALPHA = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99 + OpenMP, no FMA contraction)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-Wall", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        i64, i32, f32, f64 = C.c_int64, C.c_int32, C.c_float, C.c_double
        L.orc_quantize.argtypes = [P, i64, P, f32, P]
        L.orc_radius_q.argtypes = [f32, f32]
        L.orc_radius_q.restype = i64
        L.orc_eye_q.argtypes = [P, P, f32, P]
        L.orc_vertex_attrs.argtypes = [P, P, i64, P, P, P]
        L.orc_segment_voxels.argtypes = [P, P, i64, P, P, i64, C.c_int]
        L.orc_segment_voxels.restype = i64
        L.orc_occupancy_q.argtypes = [P, P, P, P, C.c_int, C.c_int, f32, f32, i64, i64, i64]
        L.orc_pwaa_consts.argtypes = [i64, P, P]
        L.orc_voxelize.argtypes = [P, P, P, P, i64, i64, P, P, P, C.c_int]
        L.orc_occupancy_level0.argtypes = [P, i64, P]
        L.orc_mip_average.argtypes = [P, P, P]
        L.orc_mip_or.argtypes = [P, P, P]
        L.orc_erode_blocking.argtypes = [P, P, P]
        L.orc_culling_ray.argtypes = [i64, i64, i64, P, P, P, i64, P]
        L.orc_culling_ray.restype = i64
        L.orc_visibility.argtypes = [P, P, P, P, i64, P]
        L.orc_offsets.argtypes = [P, P, P, P]
        L.orc_offsets.restype = i64
        L.orc_fill_lists.argtypes = [P, P, i64, i64, P, P, P, P, C.c_int]
        L.orc_camera_consts.argtypes = [P, P, P, f32, i32, i32, P, P, P]
        L.orc_ray_dirs.argtypes = [P, P, P, i32, i32, P, i64, P]
        L.orc_trace.argtypes = [i32, i32, i32, P, P, P, P, i64, i64, P, P, P, P, P, P, i64, C.c_int,
                                f64, f64, P, P, C.c_int, P, P, P, P, P, P]
        L.orc_shade_dirs.argtypes = [i32, P]
        L.orc_shade_light.argtypes = [P, P]
        L.orc_shade.argtypes = [P, P, i32, P, i32, P, P, f64, P, P, P]
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ---------------------------------------------------------------------------
# stages


def cull_limit(mode: int, alpha: float = 1.0, tau: float = 1.0 / 256.0) -> int:
    """Blocking voxels that hide a voxel: 1 (opaque), the number of alpha
    layers after which transmittance is below tau (alpha), or -1 (no culling)."""
    if mode == CULL_NONE:
        return -1
    if mode == CULL_OPAQUE:
        return 1
    T, k = 1.0, 0
    while not (T < tau):
        T *= (1.0 - alpha)
        k += 1
    return max(k, 1)


@dataclass
class Ingest:
    q: np.ndarray         # int32 [nv, 3]
    nrm: np.ndarray       # float32 [nv, 3]
    interior: np.ndarray  # uint8 [nv]
    seg_valid: np.ndarray # uint8 [nv]
    rq: int
    status: int


def ingest(ls) -> Ingest:
    L = lib()
    xyz = np.ascontiguousarray(ls.xyz, dtype=np.float32)
    nv = xyz.shape[0]
    q = np.zeros((nv, 3), np.int32)
    origin = np.ascontiguousarray(ls.origin, dtype=np.float32)
    st = L.orc_quantize(_p(xyz), nv, _p(origin), C.c_float(ls.voxel_size), _p(q))
    nrm = np.zeros((nv, 3), np.float32)
    interior = np.zeros(nv, np.uint8)
    seg_valid = np.zeros(nv, np.uint8)
    off = _i32(ls.offsets)
    L.orc_vertex_attrs(_p(q), _p(off), len(off) - 1, _p(nrm), _p(interior), _p(seg_valid))
    rq = int(L.orc_radius_q(C.c_float(ls.radius), C.c_float(ls.voxel_size)))
    return Ingest(q, nrm, interior, seg_valid, rq, st)


def eye_q(eye, ls) -> np.ndarray:
    e = np.ascontiguousarray(eye, dtype=np.float32)
    out = np.zeros(3, np.int64)
    lib().orc_eye_q(_p(e), _p(np.ascontiguousarray(ls.origin, np.float32)), C.c_float(ls.voxel_size), _p(out))
    return out


# membership modes: the capsule voxelizer (Alg. 1 with the corrected Eq. (1)), the printed Alg. 1 + Eq. (1),
# and the two comparison voxelizers of Table 2 (thin line, capsule AABB)
VOX_CAPSULE, VOX_LITERAL, VOX_THIN, VOX_AABB = 0, 1, 2, 3


def _mode(literal, mode):
    return VOX_LITERAL if literal else int(mode)


def segment_voxels(A, B, rq, dims, literal=False, mode=VOX_CAPSULE) -> np.ndarray:
    """Voxel set S(s) of one segment as an (n, 3) int array of (x, y, z)."""
    A, B, G = _i32(A), _i32(B), _i32(dims)
    L = lib()
    m = _mode(literal, mode)
    n = L.orc_segment_voxels(_p(A), _p(B), int(rq), _p(G), None, 0, m)
    out = np.zeros((max(n, 1), 3), np.int32)
    L.orc_segment_voxels(_p(A), _p(B), int(rq), _p(G), _p(out), n, m)
    return out[:n]


def pwaa_consts(rq):
    rc, corr = C.c_float(), C.c_float()
    lib().orc_pwaa_consts(int(rq), C.byref(rc), C.byref(corr))
    return rc.value, corr.value


def occupancy_q(A, B, n0, n1, a_int, b_int, rq, v) -> int:
    rc, corr = pwaa_consts(rq)
    A, B = _i32(A), _i32(B)
    n0 = np.ascontiguousarray(n0, np.float32)
    n1 = np.ascontiguousarray(n1, np.float32)
    return int(lib().orc_occupancy_q(_p(A), _p(B), _p(n0), _p(n1), int(a_int), int(b_int), C.c_float(rc),
                                     C.c_float(corr), int(v[0]), int(v[1]), int(v[2])))


def voxelize(ing: Ingest, dims, literal=False, mode=VOX_CAPSULE):
    """Pass 1: packed words (count low 16 bits, occupancy sum high 16 bits)."""
    G = _i32(dims)
    gx, gy, gz = dims
    words = np.zeros((gz, gy, gx), np.uint32)
    nf = C.c_int64()
    st = lib().orc_voxelize(_p(ing.q), _p(ing.nrm), _p(ing.interior), _p(ing.seg_valid), ing.q.shape[0], ing.rq,
                            _p(G), _p(words), C.byref(nf), _mode(literal, mode))
    return words, st, nf.value


def occupancy_pyramid(words):
    """Levels of the occupancy pyramid (uint16, 1/256 units), level 0 first."""
    L = lib()
    o0 = np.zeros(words.shape, np.uint16)
    L.orc_occupancy_level0(_p(np.ascontiguousarray(words)), words.size, _p(o0))
    levels = [o0]
    while max(levels[-1].shape) > 1:
        src = levels[-1]
        ds = _i32(src.shape[::-1])
        dst = np.zeros(tuple((s + 1) // 2 for s in src.shape), np.uint16)
        L.orc_mip_average(_p(src), _p(ds), _p(dst))
        levels.append(dst)
    return levels


def erode_blocking(o0):
    b = np.zeros(o0.shape, np.uint8)
    lib().orc_erode_blocking(_p(np.ascontiguousarray(o0)), _p(_i32(o0.shape[::-1])), _p(b))
    return b


def visibility(words, blocking, eyeq, limit):
    vis = np.zeros(words.shape, np.uint8)
    lib().orc_visibility(_p(words), _p(blocking), _p(_i32(words.shape[::-1])),
                         _p(np.ascontiguousarray(eyeq, np.int64)), int(limit), _p(vis))
    return vis


def culling_ray(v, eyeq, blocking, limit):
    nvis = C.c_int64()
    n = lib().orc_culling_ray(int(v[0]), int(v[1]), int(v[2]), _p(np.ascontiguousarray(eyeq, np.int64)),
                              _p(_i32(blocking.shape[::-1])), _p(np.ascontiguousarray(blocking)), int(limit),
                              C.byref(nvis))
    return n, nvis.value


def visibility_pyramid(vis):
    L = lib()
    levels = [vis]
    while max(levels[-1].shape) > 1:
        src = levels[-1]
        dst = np.zeros(tuple((s + 1) // 2 for s in src.shape), np.uint8)
        L.orc_mip_or(_p(src), _p(_i32(src.shape[::-1])), _p(dst))
        levels.append(dst)
    return levels


def csr(ing: Ingest, words, vis, literal=False, mode=VOX_CAPSULE):
    """Offsets (dense index, brick-major exclusive prefix) and ascending id lists."""
    G = _i32(words.shape[::-1])
    offsets = np.zeros(words.shape, np.uint32)
    total = lib().orc_offsets(_p(words), _p(vis), _p(G), _p(offsets))
    ids = np.zeros(max(total, 1), np.uint32)
    lib().orc_fill_lists(_p(ing.q), _p(ing.seg_valid), ing.q.shape[0], ing.rq, _p(G), _p(vis), _p(offsets),
                         _p(ids), _mode(literal, mode))
    return offsets, ids[:total], total


def camera_consts(cam):
    F, R, U = (np.zeros(3, np.float32) for _ in range(3))
    lib().orc_camera_consts(_p(np.ascontiguousarray(cam.eye, np.float32)),
                            _p(np.ascontiguousarray(cam.target, np.float32)),
                            _p(np.ascontiguousarray(cam.up, np.float32)), C.c_float(cam.fovy_deg),
                            int(cam.width), int(cam.height), _p(F), _p(R), _p(U))
    return F, R, U


def ray_dirs(cam, pix):
    F, R, U = camera_consts(cam)
    pix = np.ascontiguousarray(pix, np.int64)
    dirs = np.zeros((len(pix), 3), np.float32)
    lib().orc_ray_dirs(_p(F), _p(R), _p(U), int(cam.width), int(cam.height), _p(pix), len(pix), _p(dirs))
    return dirs


@dataclass
class Frame:
    """Everything the oracle builds for one (line set, view)."""
    dims: tuple
    ing: Ingest
    words: np.ndarray
    status: int
    n_fragments: int
    occ: list
    blocking: np.ndarray
    vis: np.ndarray
    vis_levels: list
    offsets: np.ndarray
    ids: np.ndarray
    total: int
    eyeq: np.ndarray
    limit: int
    times: dict
    mode: int = VOX_CAPSULE  # membership mode the frame was built with


def build_frame(ls, eye, cull_mode, alpha=1.0, tau=1.0 / 256.0, literal=False, mode=VOX_CAPSULE) -> Frame:
    t = {}
    t0 = time.perf_counter()
    ing = ingest(ls)
    t["ingest"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    words, st, nf = voxelize(ing, ls.dims, literal, mode)
    t["voxelize"] = time.perf_counter() - t0
    st = st or ing.status
    t0 = time.perf_counter()
    occ = occupancy_pyramid(words)
    t["mips"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    blk = erode_blocking(occ[0])
    t["erode"] = time.perf_counter() - t0
    eq = eye_q(eye, ls)
    lim = cull_limit(cull_mode, alpha, tau)
    t0 = time.perf_counter()
    vis = visibility(words, blk, eq, lim)
    t["cull"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    vlev = visibility_pyramid(vis)
    t["cull_mips"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    offsets, ids, total = csr(ing, words, vis, literal, mode)
    t["lists"] = time.perf_counter() - t0
    return Frame(tuple(ls.dims), ing, words, st, nf, occ, blk, vis, vlev, offsets, ids, total, eq, lim, t,
                 _mode(literal, mode))


def recull_frame(fr: Frame, ls, eye, cull_mode, alpha=1.0, tau=1.0 / 256.0) -> Frame:
    """Culling, culling pyramid and lists of an already voxelized frame for another view."""
    t = {}
    eq = eye_q(eye, ls)
    lim = cull_limit(cull_mode, alpha, tau)
    t0 = time.perf_counter()
    vis = visibility(fr.words, fr.blocking, eq, lim)
    t["cull"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    vlev = visibility_pyramid(vis)
    t["cull_mips"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    offsets, ids, total = csr(fr.ing, fr.words, vis, mode=fr.mode)
    t["lists"] = time.perf_counter() - t0
    return Frame(fr.dims, fr.ing, fr.words, fr.status, fr.n_fragments, fr.occ, fr.blocking, vis, vlev, offsets, ids,
                 total, eq, lim, t, fr.mode)


@dataclass
class TraceResult:
    pix: np.ndarray
    id: np.ndarray
    t: np.ndarray        # voxel units
    depth: np.ndarray    # world units
    rgba: np.ndarray
    m_geom: np.ndarray
    m_face: np.ndarray
    n_comp: np.ndarray


def trace(fr: Frame, ls, cam, pix, mode, alpha=1.0, tau=1.0 / 256.0, brute=False, dirs=None,
          invoxel=False, seg_rgba=None, lit=None) -> TraceResult:
    """brute: test every segment; invoxel: the paper's per-voxel acceptance rule.  seg_rgba: None (colour =
    |unit tangent|, opacity alpha) or float32 [n_vertices, 4], the colour and opacity of segment i in row i.
    lit: None or the voxel-space shading (float64, shaped like the grid) that scales each hit's colour."""
    pix = np.ascontiguousarray(pix, np.int64)
    if dirs is None:
        dirs = ray_dirs(cam, pix)
    # the trace's eye is the quantized camera eye
    eq = eye_q(cam.eye, ls)
    n = len(pix)
    out_id = np.zeros(n, np.int64)
    out_t = np.zeros(n, np.float64)
    rgba = np.zeros((n, 4), np.float64)
    mg = np.zeros(n, np.float64)
    mf = np.zeros(n, np.float64)
    nc = np.zeros(n, np.int64)
    gx, gy, gz = fr.dims
    ids = fr.ids if fr.ids.size else np.zeros(1, np.uint32)
    if seg_rgba is not None:
        seg_rgba = np.ascontiguousarray(seg_rgba, np.float32).reshape(-1, 4)
    lit_arr = None if lit is None else np.ascontiguousarray(lit, np.float64)
    if lit_arr is not None and lit_arr.shape != fr.vis.shape:
        raise ValueError("lit must be shaped like the grid")
    if seg_rgba is not None and seg_rgba.shape[0] < fr.ing.q.shape[0]:
        raise ValueError("rgba needs one row per vertex")
    lib().orc_trace(gx, gy, gz, _p(fr.ing.q), _p(fr.ing.nrm), _p(fr.ing.interior), _p(fr.ing.seg_valid),
                    fr.ing.q.shape[0], fr.ing.rq, _p(fr.vis), _p(fr.words), _p(fr.offsets), _p(ids), _p(eq),
                    _p(np.ascontiguousarray(dirs, np.float32)), n, int(mode), float(alpha), float(tau),
                    None if seg_rgba is None else _p(seg_rgba), None if lit is None else _p(lit_arr),
                    2 if invoxel else int(brute), _p(out_id), _p(out_t), _p(rgba), _p(mg), _p(mf), _p(nc))
    return TraceResult(pix, out_id, out_t, out_t * float(ls.voxel_size), rgba, mg, mf, nc)


def num_threads() -> int:
    return int(lib().orc_num_threads())


# ---------------------------------------------------------------------------
# voxel-space shading (Section 3.4)


def shade_dirs(K):
    U = np.zeros((K, 3), np.int32)
    lib().orc_shade_dirs(int(K), _p(U))
    return U


def shade_light(light):
    L = np.zeros(3, np.int32)
    lib().orc_shade_light(_p(np.ascontiguousarray(light, np.float32)), _p(L))
    return L


def shade(occ, vis, n_cones=16, n_samples=4, light=(0.3, 0.5, 0.8), ambient=0.3):
    """Ambient occlusion, shadow and lit value of every visible voxel (float64 arrays shaped like vis).
    occ: the occupancy pyramid (level 0 first); vis: level-0 visibility."""
    G = _i32(vis.shape[::-1])
    lv = [np.ascontiguousarray(o, np.uint16) for o in occ[:n_samples + 1]]
    if len(lv) < n_samples + 1:
        raise ValueError("the pyramid has fewer levels than samples")
    ptrs = (C.c_void_p * len(lv))(*[o.ctypes.data for o in lv])
    U = shade_dirs(n_cones)
    L = shade_light(light)
    ao, sh, lit = (np.zeros(vis.shape, np.float64) for _ in range(3))
    lib().orc_shade(_p(G), ptrs, int(n_samples), _p(np.ascontiguousarray(vis, np.uint8)), int(n_cones), _p(U),
                    _p(L), float(ambient), _p(ao), _p(sh), _p(lit))
    return ao, sh, lit

