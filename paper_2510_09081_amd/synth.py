"""Seeded synthetic line sets and cameras (input generation only).

This module produces the inputs that both the HIP path and the CPU oracle
consume: FP32 polyline vertices, polyline offsets, a grid, a radius and a
camera.  It holds none of the rendering method's arithmetic (no quantization,
voxelization, culling or tracing); it only draws random polylines with the
shapes of the paper's workloads (Table 1: tractography bundles and flow
pathlines), which are not available here.

Every generator takes an explicit ``numpy.random.Generator`` (PCG64) so that a
workload is a pure function of its seed.  Coordinates are computed in float64
and cast once to float32; the float32 arrays are the single input of record.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import math

import numpy as np

CULL_NONE, CULL_OPAQUE, CULL_ALPHA = 0, 1, 2
MODE_OPAQUE, MODE_TRANSPARENT = 0, 1


@dataclass
class LineSet:
    """Polylines plus the grid they are voxelized into (world units)."""

    xyz: np.ndarray          # float32 [n_vertices, 3]
    offsets: np.ndarray      # int32 [n_polylines + 1]; polyline p = [offsets[p], offsets[p+1])
    radius: float            # capsule radius, world units (float32 value)
    origin: np.ndarray       # float32 [3], world position of the grid corner
    voxel_size: float        # world size of one voxel (float32 value)
    dims: tuple              # (Gx, Gy, Gz), each a multiple of 8

    @property
    def n_vertices(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_polylines(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_segments(self) -> int:
        return self.n_vertices - self.n_polylines


@dataclass
class Camera:
    """Pinhole camera in world units; vertical field of view in degrees."""

    eye: np.ndarray
    target: np.ndarray
    up: np.ndarray
    fovy_deg: float
    width: int
    height: int


@dataclass
class Pass:
    """One render pass of a frame: culling mode for the view, trace mode, alpha."""

    cull_mode: int
    trace_mode: int
    alpha: float
    tau: float = 1.0 / 256.0


@dataclass
class Workload:
    name: str
    lines: LineSet
    camera: Camera
    passes: list = field(default_factory=list)


# --------------------------------------------------------------------------
# helpers


def _f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32)


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _random_unit(rng, n):
    return _unit(rng.normal(size=(n, 3)))


def _offsets_from_lengths(n_vertices_per_poly):
    off = np.zeros(len(n_vertices_per_poly) + 1, dtype=np.int64)
    np.cumsum(n_vertices_per_poly, out=off[1:])
    return off.astype(np.int32)


def orbit_eye(centre, distance, theta_deg=60.0, phi_deg=30.0):
    """Eye position on a sphere around ``centre`` (polar angle from +z)."""
    th, ph = math.radians(theta_deg), math.radians(phi_deg)
    u = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    return np.asarray(centre, dtype=np.float64) + distance * u


# --------------------------------------------------------------------------
# generators (positions in "cube units": the unit cube maps to the grid)


def random_walk(rng, n_poly, n_seg, step_lo, step_hi, sigma_deg, lo=0.1, hi=0.9):
    """Random-walk polylines inside the unit cube.

    Start uniform in [lo, hi]^3, initial direction uniform on the sphere.  Each
    step has length U(step_lo, step_hi) (cube units) and turns by |N(0, sigma)|
    about a random axis perpendicular to the direction; walls of the unit cube
    reflect the walk specularly.
    Returns float64 [n_poly, n_seg + 1, 3].
    """
    sigma = math.radians(sigma_deg)
    p = rng.uniform(lo, hi, size=(n_poly, 3))
    d = _random_unit(rng, n_poly)
    out = np.empty((n_poly, n_seg + 1, 3))
    out[:, 0] = p
    for k in range(n_seg):
        ang = np.abs(rng.normal(0.0, sigma, size=n_poly))
        axis = rng.normal(size=(n_poly, 3))
        axis -= (axis * d).sum(1, keepdims=True) * d
        axis = _unit(axis)
        d = d * np.cos(ang)[:, None] + np.cross(axis, d) * np.sin(ang)[:, None]
        d = _unit(d)
        step = rng.uniform(step_lo, step_hi, size=n_poly)
        p = p + d * step[:, None]
        for c in range(3):
            below = p[:, c] < 0.0
            p[below, c] = -p[below, c]
            d[below, c] = -d[below, c]
            above = p[:, c] > 1.0
            p[above, c] = 2.0 - p[above, c]
            d[above, c] = -d[above, c]
        out[:, k + 1] = p
    return out


def _catmull_rom(ctrl, samples_per_span):
    """Uniform Catmull-Rom spline through ``ctrl`` (ends extended by reflection)."""
    c = np.asarray(ctrl, dtype=np.float64)
    pts = np.vstack([2 * c[0] - c[1], c, 2 * c[-1] - c[-2]])
    u = np.linspace(0.0, 1.0, samples_per_span, endpoint=False)[:, None]
    out = []
    for i in range(1, len(pts) - 2):
        p0, p1, p2, p3 = pts[i - 1], pts[i], pts[i + 1], pts[i + 2]
        out.append(0.5 * ((2 * p1) + (-p0 + p2) * u + (2 * p0 - 5 * p1 + 4 * p2 - p3) * u ** 2
                          + (-p0 + 3 * p1 - 3 * p2 + p3) * u ** 3))
    out.append(c[-1][None, :])
    return np.vstack(out)


def _rotation_minimizing_frame(x):
    """Double-reflection rotation-minimizing frame along sampled curve ``x``."""
    n = len(x)
    t = np.gradient(x, axis=0)
    t = _unit(t)
    ref = np.array([0.0, 0.0, 1.0]) if abs(t[0, 2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    r = np.empty_like(x)
    r0 = ref - np.dot(ref, t[0]) * t[0]
    r[0] = r0 / np.linalg.norm(r0)
    for i in range(n - 1):
        v1 = x[i + 1] - x[i]
        c1 = np.dot(v1, v1)
        if c1 == 0.0:
            r[i + 1] = r[i]
            continue
        rl = r[i] - (2.0 / c1) * np.dot(v1, r[i]) * v1
        tl = t[i] - (2.0 / c1) * np.dot(v1, t[i]) * v1
        v2 = t[i + 1] - tl
        c2 = np.dot(v2, v2)
        r[i + 1] = rl if c2 == 0.0 else rl - (2.0 / c2) * np.dot(v2, rl) * v2
    s = np.cross(t, r)
    return r, s


def bundles(rng, n_bundles, per_bundle, grid, step_vox=0.5, sigma_vox=3.0,
            len_lo=20, len_hi=200, jitter_vox=0.05):
    """Tractography-shaped bundles (cube units); returns (xyz float64 [n,3], n_vertices per polyline).

    Each bundle follows a Catmull-Rom centreline through 5 control points (first
    uniform in [0.15, 0.85]^3, each next one U(0.15, 0.30) away in a random
    direction, clamped to [0.1, 0.9]^3), parametrized by arc length.  Each
    polyline has U{len_lo..len_hi} segments spaced ``step_vox`` voxels along the
    centreline from a uniform start, a constant lateral offset N(0, sigma_vox^2)
    per axis of the rotation-minimizing normal frame, and N(0, jitter_vox^2)
    per-vertex jitter.
    """
    vox = 1.0 / grid
    chunks, nverts = [], []
    for _ in range(n_bundles):
        ctrl = [rng.uniform(0.15, 0.85, size=3)]
        for _k in range(4):
            d = _random_unit(rng, 1)[0]
            ctrl.append(np.clip(ctrl[-1] + rng.uniform(0.15, 0.30) * d, 0.1, 0.9))
        x = _catmull_rom(np.array(ctrl), 512)
        seg = np.linalg.norm(np.diff(x, axis=0), axis=1)
        arc = np.concatenate([[0.0], np.cumsum(seg)])
        total = arc[-1]
        nrm, bin_ = _rotation_minimizing_frame(x)
        nseg = rng.integers(len_lo, len_hi + 1, size=per_bundle)
        span = nseg * step_vox * vox
        start = rng.uniform(0.0, 1.0, size=per_bundle) * np.maximum(total - span, 0.0)
        off = rng.normal(0.0, sigma_vox * vox, size=(per_bundle, 2))
        nv = nseg + 1
        idx_poly = np.repeat(np.arange(per_bundle), nv)
        k = np.arange(nv.sum()) - np.repeat(np.cumsum(nv) - nv, nv)
        s = np.minimum(start[idx_poly] + k * step_vox * vox, total)
        pos = np.stack([np.interp(s, arc, x[:, c]) for c in range(3)], axis=1)
        fn = np.stack([np.interp(s, arc, nrm[:, c]) for c in range(3)], axis=1)
        fb = np.stack([np.interp(s, arc, bin_[:, c]) for c in range(3)], axis=1)
        pos += fn * off[idx_poly, 0:1] + fb * off[idx_poly, 1:2]
        pos += rng.normal(0.0, jitter_vox * vox, size=pos.shape)
        chunks.append(pos)
        nverts.append(nv)
    return np.vstack(chunks), np.concatenate(nverts)


def abc_velocity(p, A=math.sqrt(3.0), B=math.sqrt(2.0), C=1.0):
    x, y, z = p[..., 0], p[..., 1], p[..., 2]
    return np.stack([A * np.sin(z) + C * np.cos(y),
                     B * np.sin(x) + A * np.cos(z),
                     C * np.sin(y) + B * np.cos(x)], axis=-1)


def abc_trajectories(rng, n_seeds, n_steps, dt):
    """RK4 trajectories of the steady ABC flow; float64 [n_seeds, n_steps + 1, 3]."""
    p = rng.uniform(0.0, 2.0 * math.pi, size=(n_seeds, 3))
    out = np.empty((n_seeds, n_steps + 1, 3))
    out[:, 0] = p
    for k in range(n_steps):
        k1 = abc_velocity(p)
        k2 = abc_velocity(p + 0.5 * dt * k1)
        k3 = abc_velocity(p + 0.5 * dt * k2)
        k4 = abc_velocity(p + dt * k3)
        p = p + (dt / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
        out[:, k + 1] = p
    return out


# --------------------------------------------------------------------------
# workloads


def _unit_cube_lineset(pos_cube, nverts, G, radius_vox):
    vs = np.float32(1.0 / G)
    return LineSet(xyz=_f32(pos_cube.reshape(-1, 3)), offsets=_offsets_from_lengths(nverts),
                   radius=float(np.float32(radius_vox / G)), origin=np.zeros(3, np.float32),
                   voxel_size=float(vs), dims=(G, G, G))


def _camera_for_cube(W, H, theta=60.0, phi=30.0, up=(0.0, 0.0, 1.0), distance=2.0):
    c = np.array([0.5, 0.5, 0.5])
    return Camera(eye=orbit_eye(c, distance, theta, phi), target=c, up=np.array(up, float),
                  fovy_deg=60.0, width=W, height=H)


def random_walk_set(seed=0, n_poly=200, n_seg=50, G=64, radius_vox=0.5,
                    step_lo=0.5, step_hi=1.5, sigma_deg=10.0):
    rng = np.random.default_rng(seed)
    pos = random_walk(rng, n_poly, n_seg, step_lo / G, step_hi / G, sigma_deg)
    return _unit_cube_lineset(pos, np.full(n_poly, n_seg + 1), G, radius_vox)


def bundle_set(seed=1, n_bundles=20, per_bundle=2500, G=512, radius_vox=0.35, **kw):
    rng = np.random.default_rng(seed)
    pos, nv = bundles(rng, n_bundles, per_bundle, G, **kw)
    return _unit_cube_lineset(pos, nv, G, radius_vox)


def pathline_frames(seed=2, n_seeds=20000, seg_per_line=100, n_frames=120,
                    steps_per_frame=2, dt=0.05, G=256, radius_vox=0.5):
    """ABC pathlines; returns (trajectories, grid origin, voxel size, dims, radius).

    Frame f uses trajectory steps [f*steps_per_frame, f*steps_per_frame + seg_per_line].
    The grid is a cube of G^3 voxels covering every frame's vertices with one
    voxel of padding on each side.
    """
    rng = np.random.default_rng(seed)
    n_steps = (n_frames - 1) * steps_per_frame + seg_per_line
    traj = abc_trajectories(rng, n_seeds, n_steps, dt)
    lo, hi = traj.reshape(-1, 3).min(0), traj.reshape(-1, 3).max(0)
    ext = float((hi - lo).max())
    vs = np.float32(ext / (G - 2))
    origin = _f32(lo - float(vs))
    return traj, origin, float(vs), (G, G, G), float(np.float32(radius_vox * float(vs)))


def pathline_frame(frames, f, seg_per_line=100, steps_per_frame=2):
    traj, origin, vs, dims, radius = frames
    a = f * steps_per_frame
    pos = traj[:, a:a + seg_per_line + 1]
    n = pos.shape[0]
    return LineSet(xyz=_f32(pos.reshape(-1, 3)),
                   offsets=_offsets_from_lengths(np.full(n, seg_per_line + 1)),
                   radius=radius, origin=origin, voxel_size=vs, dims=dims)


def grid_camera(ls: LineSet, W, H, theta=60.0, phi=30.0, distance=2.0, up=(0.0, 0.0, 1.0)):
    """Camera orbiting the centre of the grid cube at ``distance`` cube widths."""
    ext = np.array(ls.dims, float) * ls.voxel_size
    c = ls.origin.astype(np.float64) + 0.5 * ext
    eye = orbit_eye(c, distance * float(ext.max()), theta, phi)
    return Camera(eye=eye, target=c, up=np.array(up, float), fovy_deg=60.0, width=W, height=H)


def batch_sets(seed=4, n_sets=64, lo=1e3, hi=1e6, W=512, H=512):
    """Uneven batch: log-uniform segment counts, mixed generators, per-set grid and camera."""
    rng = np.random.default_rng(seed)
    items = []
    for _ in range(n_sets):
        ns = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        G = int(8 * round(math.exp(rng.uniform(math.log(8), math.log(32)))))
        sub = int(rng.integers(0, 2**31 - 1))
        if rng.uniform() < 0.5:
            n_poly = max(1, ns // 50)
            ls = random_walk_set(seed=sub, n_poly=n_poly, n_seg=50, G=G, radius_vox=0.5)
        else:
            nb = max(1, math.ceil(ns / 110 / 2500))
            per = max(1, ns // (110 * nb))
            ls = bundle_set(seed=sub, n_bundles=nb, per_bundle=per, G=G, radius_vox=0.35)
        u = _random_unit(rng, 1)[0]
        up = (0.0, 1.0, 0.0) if abs(u[2]) > 0.99 else (0.0, 0.0, 1.0)
        c = np.array([0.5, 0.5, 0.5])
        cam = Camera(eye=c + 2.0 * u, target=c, up=np.array(up), fovy_deg=60.0, width=W, height=H)
        items.append(Workload(name=f"batch{len(items)}", lines=ls, camera=cam,
                              passes=[Pass(CULL_OPAQUE, MODE_OPAQUE, 1.0)]))
    return items


def decimate(ls: LineSet, n: int) -> LineSet:
    """Level of detail: every polyline keeps its vertices 0, n, 2n, ... and its last one, so segments become
    about n times longer (the segment-length sweep of the voxelizer comparison)."""
    if n <= 1:
        return ls
    keep, lengths = [], []
    for p in range(ls.n_polylines):
        a, b = int(ls.offsets[p]), int(ls.offsets[p + 1])
        idx = list(range(a, b, n))
        if idx[-1] != b - 1:
            idx.append(b - 1)
        keep.extend(idx)
        lengths.append(len(idx))
    return replace(ls, xyz=np.ascontiguousarray(ls.xyz[np.asarray(keep, np.int64)]),
                   offsets=_offsets_from_lengths(np.asarray(lengths)))


def regrid(ls: LineSet, G: int) -> LineSet:
    """The same world-space line set on a G^3 grid over the same cube (voxel size and radius in voxels scale)."""
    ext = float(ls.voxel_size) * max(ls.dims)
    return replace(ls, voxel_size=float(np.float32(ext / G)), dims=(G, G, G))


def workload(name: str) -> Workload:
    """Named workloads with the shapes of the benchmark configurations."""
    if name == "random_walk_10k":
        ls = random_walk_set(seed=0)
        return Workload(name, ls, _camera_for_cube(256, 256),
                        [Pass(CULL_NONE, MODE_OPAQUE, 1.0), Pass(CULL_NONE, MODE_TRANSPARENT, 0.3),
                         Pass(CULL_OPAQUE, MODE_OPAQUE, 1.0)])
    if name == "bundles_5m":
        ls = bundle_set(seed=1)
        return Workload(name, ls, _camera_for_cube(1920, 1080),
                        [Pass(CULL_OPAQUE, MODE_OPAQUE, 1.0), Pass(CULL_ALPHA, MODE_TRANSPARENT, 0.2)])
    if name == "bundles_small":
        # the bundle shape at a size the oracle finishes in seconds
        ls = bundle_set(seed=11, n_bundles=3, per_bundle=300, G=128)
        return Workload(name, ls, _camera_for_cube(320, 240),
                        [Pass(CULL_OPAQUE, MODE_OPAQUE, 1.0), Pass(CULL_ALPHA, MODE_TRANSPARENT, 0.2),
                         Pass(CULL_NONE, MODE_TRANSPARENT, 0.2)])
    raise KeyError(name)


def with_camera(w: Workload, **kw) -> Workload:
    return replace(w, camera=replace(w.camera, **kw))
