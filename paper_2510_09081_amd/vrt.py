"""ctypes binding of libvrt.so (argument marshalling only).

Every step of the path runs in the HIP library; this module converts Python
values into the C ABI structs of ``include/vrt.h`` and raises on any non-zero
status.  PyTorch supplies device memory and the stream.  There is no CPU
fallback: importing works without a GPU, but creating a context needs the
built library and a HIP device.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libvrt.so")

VRT_OK, VRT_ERR_INVALID_ARG, VRT_ERR_RANGE, VRT_ERR_NOT_BUILT = 0, 1, 2, 3
VRT_ERR_CAPACITY, VRT_ERR_COUNT_OVERFLOW, VRT_ERR_HIP = 4, 5, 6
CULL_NONE, CULL_OPAQUE, CULL_ALPHA = 0, 1, 2
TRACE_OPAQUE, TRACE_TRANSPARENT = 0, 1
FORM_PLAIN, FORM_FP16 = 0, 1
BATCH_PERSISTENT, BATCH_SEQUENTIAL, BATCH_STAGED, BATCH_SPLIT = 0, 1, 2, 3

EXPORTED = ["vrt_create", "vrt_destroy", "vrt_voxelize", "vrt_cull", "vrt_trace", "vrt_frame_status",
            "vrt_query_as", "vrt_debug_rays", "vrt_copy_to_host", "vrt_last_hip_error", "vrt_status_string",
            "vrt_profile_enable", "vrt_profile_read", "vrt_trace_stats_run", "vrt_graph_create",
            "vrt_graph_launch", "vrt_graph_destroy", "vrt_batch_create", "vrt_batch_run", "vrt_batch_context",
            "vrt_batch_destroy", "vrt_set_tune", "vrt_get_tune", "vrt_autotune", "vrt_autotune_grid",
            "vrt_frame_noalloc", "vrt_microbench", "vrt_sort_lists", "vrt_shade"]
MB_COPY, MB_ATOMIC_RANDOM, MB_ATOMIC_BRICK = 0, 1, 2
NOALLOC_MAX_VERTICES, NOALLOC_MAX_FRAGMENTS, NOALLOC_MAX_DIM, NOALLOC_MAX_PIXELS = 65536, 1 << 20, 64, 512 * 512


class VrtError(RuntimeError):
    def __init__(self, status, what, hip=0):
        self.status = status
        super().__init__(f"{what}: status {status} ({_status_string(status)})" + (f", hip error {hip}" if hip else ""))


class vrt_desc(C.Structure):
    _fields_ = [("max_vertices", C.c_int64), ("max_fragments", C.c_int64), ("max_dim", C.c_int32),
                ("device", C.c_int32), ("max_pixels", C.c_int64), ("form", C.c_int32), ("reserved", C.c_int32)]


class vrt_lines(C.Structure):
    _fields_ = [("xyz", C.c_void_p), ("poly_offsets", C.c_void_p), ("n_vertices", C.c_int64),
                ("n_polylines", C.c_int64), ("radius", C.c_float), ("alpha_default", C.c_float),
                ("rgba", C.c_void_p), ("voxelizer", C.c_int32), ("reserved", C.c_int32)]


VOX_CAPSULE, VOX_THIN, VOX_AABB = 0, 2, 3


def make_lines(xyz, offsets, radius, voxelizer=VOX_CAPSULE, rgba=None, alpha_default=0.0):
    """vrt_lines for device tensors xyz [n, 3] float32 and offsets [n_polylines + 1] int32; rgba: None or a
    device float32 tensor [n, 4] (colour and opacity of the segment starting at each vertex)."""
    return vrt_lines(_ptr(xyz), _ptr(offsets), int(xyz.shape[0]), int(offsets.shape[0] - 1), float(radius),
                     float(alpha_default), _ptr(rgba), int(voxelizer), 0)


class vrt_grid(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("voxel_size", C.c_float), ("dims", C.c_int32 * 3)]


class vrt_view(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("cull_mode", C.c_int32), ("alpha", C.c_float), ("tau", C.c_float)]


class vrt_camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("target", C.c_float * 3), ("up", C.c_float * 3), ("fovy_deg", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32), ("mode", C.c_int32), ("alpha", C.c_float),
                ("tau", C.c_float)]


class vrt_image(C.Structure):
    _fields_ = [("rgba", C.c_void_p), ("depth", C.c_void_p), ("first_id", C.c_void_p)]


class vrt_frame_info(C.Structure):
    _fields_ = [("device_status", C.c_int32), ("n_fragments", C.c_int64), ("n_listed", C.c_int64),
                ("n_bricks", C.c_int64), ("required_fragments", C.c_int64), ("n_occupied", C.c_int64),
                ("n_visible", C.c_int64)]


class vrt_as_view(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("n_levels", C.c_int32), ("n_bricks", C.c_int32),
                ("brick_list", C.c_void_p), ("words", C.c_void_p), ("occ", C.c_void_p * 4), ("occ_hi", C.c_void_p),
                ("blocking", C.c_void_p), ("vis", C.c_void_p * 4), ("vis_hi", C.c_void_p), ("list_end", C.c_void_p),
                ("ids", C.c_void_p), ("lit", C.c_void_p)]


class vrt_shading(C.Structure):
    _fields_ = [("light_dir", C.c_float * 3), ("n_cones", C.c_int32), ("n_samples", C.c_int32),
                ("ambient", C.c_float), ("enable", C.c_int32), ("reserved", C.c_int32)]


class vrt_batch_item(C.Structure):
    _fields_ = [("lines", vrt_lines), ("grid", vrt_grid), ("view", vrt_view), ("cam", vrt_camera),
                ("image", vrt_image)]


class vrt_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double)]


class vrt_trace_stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ["rays", "rays_hit", "cell_skips_64", "cell_skips_8", "voxel_steps",
                                         "list_visits", "capsule_tests", "kbuffer_passes", "distinct_list_voxels",
                                         "distinct_list_entries", "distinct_segments", "max_tests_per_ray"]]


_lib = None


class vrt_tune(C.Structure):
    _fields_ = [("march_threads", C.c_int32), ("shade_group", C.c_int32), ("shade_batch", C.c_int32),
                ("lane_keys", C.c_int32), ("shade_blocks", C.c_int32), ("reserved", C.c_int32 * 3)]


TUNE_FIELDS = ["march_threads", "shade_group", "shade_batch", "lane_keys", "shade_blocks"]


class vrt_tune_space(C.Structure):
    _fields_ = [("cam", C.POINTER(vrt_camera)), ("image", C.POINTER(vrt_image)), ("reps", C.c_int32),
                ("warmup", C.c_int32), ("sweeps", C.c_int32), ("reserved", C.c_int32), ("cache_path", C.c_char_p),
                ("key", C.c_char_p)]


class vrt_tune_result(C.Structure):
    _fields_ = [("best", vrt_tune), ("best_ms", C.c_float), ("start_ms", C.c_float), ("evaluated", C.c_int32),
                ("from_cache", C.c_int32)]


def load():
    """Loads libvrt.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2510_09081_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.vrt_create.argtypes = [C.POINTER(vrt_desc), C.POINTER(P)]
        L.vrt_destroy.argtypes = [P]
        L.vrt_voxelize.argtypes = [P, C.POINTER(vrt_lines), C.POINTER(vrt_grid), P]
        L.vrt_cull.argtypes = [P, C.POINTER(vrt_view), P]
        L.vrt_trace.argtypes = [P, C.POINTER(vrt_camera), C.POINTER(vrt_image), P]
        L.vrt_frame_status.argtypes = [P, C.POINTER(vrt_frame_info)]
        L.vrt_query_as.argtypes = [P, C.POINTER(vrt_as_view)]
        L.vrt_debug_rays.argtypes = [P, C.POINTER(vrt_camera), P, C.c_int64, P, P]
        L.vrt_copy_to_host.argtypes = [P, P, C.c_int64]
        L.vrt_profile_enable.argtypes = [P, C.c_int32]
        L.vrt_graph_create.argtypes = [P, C.POINTER(vrt_lines), C.POINTER(vrt_grid), C.POINTER(vrt_view),
                                       C.POINTER(vrt_camera), C.POINTER(vrt_image), C.c_int32, C.POINTER(P)]
        L.vrt_graph_launch.argtypes = [P, P]
        L.vrt_batch_create.argtypes = [C.POINTER(vrt_desc), C.c_int32, C.POINTER(P)]
        L.vrt_batch_run.argtypes = [P, C.POINTER(vrt_batch_item), C.c_int32, C.c_int32, P]
        L.vrt_batch_context.argtypes = [P, C.c_int32, C.POINTER(P)]
        L.vrt_batch_destroy.argtypes = [P]
        L.vrt_graph_destroy.argtypes = [P]
        L.vrt_trace_stats_run.argtypes = [P, C.POINTER(vrt_camera), C.POINTER(vrt_image), C.POINTER(vrt_trace_stats), P]
        L.vrt_profile_read.argtypes = [P, C.POINTER(vrt_kernel_time), C.c_int32, C.POINTER(C.c_int32)]
        L.vrt_set_tune.argtypes = [P, C.c_int32, C.POINTER(vrt_tune)]
        L.vrt_get_tune.argtypes = [P, C.c_int32, C.POINTER(vrt_tune)]
        L.vrt_autotune.argtypes = [P, C.POINTER(vrt_tune_space), C.POINTER(vrt_tune_result), P]
        L.vrt_autotune_grid.argtypes = [P, C.POINTER(vrt_lines), C.POINTER(vrt_grid), C.c_int32,
                                        C.POINTER(vrt_view), C.POINTER(vrt_camera), C.POINTER(vrt_image), C.c_int32,
                                        C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_float), P]
        L.vrt_frame_noalloc.argtypes = [C.POINTER(vrt_lines), C.POINTER(vrt_grid), C.POINTER(vrt_view),
                                        C.POINTER(vrt_camera), C.POINTER(vrt_image), C.POINTER(vrt_frame_info), P]
        L.vrt_microbench.argtypes = [C.c_int32, P, C.c_int64, C.c_int64, C.POINTER(C.c_float), P]
        L.vrt_sort_lists.argtypes = [P, P]
        L.vrt_shade.argtypes = [P, C.POINTER(vrt_shading), P]
        L.vrt_last_hip_error.restype = C.c_int32
        L.vrt_status_string.argtypes = [C.c_int32]
        L.vrt_status_string.restype = C.c_char_p
        for name in ["vrt_create", "vrt_destroy", "vrt_voxelize", "vrt_cull", "vrt_trace", "vrt_frame_status",
                     "vrt_query_as", "vrt_debug_rays", "vrt_copy_to_host", "vrt_profile_enable",
                     "vrt_profile_read", "vrt_trace_stats_run", "vrt_graph_create", "vrt_graph_launch",
                     "vrt_graph_destroy", "vrt_batch_create", "vrt_batch_run", "vrt_batch_context",
                     "vrt_batch_destroy", "vrt_set_tune", "vrt_get_tune", "vrt_autotune", "vrt_autotune_grid",
                     "vrt_frame_noalloc", "vrt_microbench", "vrt_sort_lists", "vrt_shade"]:
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def _status_string(s):
    try:
        return load().vrt_status_string(int(s)).decode()
    except Exception:  # noqa: BLE001 - only used to decorate an error message
        return "?"


def _check(status, what):
    if status != VRT_OK:
        hip = load().vrt_last_hip_error() if status == VRT_ERR_HIP else 0
        raise VrtError(status, what, hip)


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def copy_to_host(dev_ptr, nbytes, dtype, count):
    out = np.empty(count, dtype=dtype)
    if count:
        _check(load().vrt_copy_to_host(out.ctypes.data_as(C.c_void_p), C.c_void_p(dev_ptr), int(nbytes)),
               "vrt_copy_to_host")
    return out


def _f3(v):
    v = np.asarray(v, dtype=np.float32).reshape(3)
    return (C.c_float * 3)(*[float(x) for x in v])


def make_camera(eye, target, up, fovy_deg, width, height, mode=TRACE_OPAQUE, alpha=1.0, tau=1.0 / 256.0):
    return vrt_camera(_f3(eye), _f3(target), _f3(up), float(np.float32(fovy_deg)), int(width), int(height), int(mode),
                      float(alpha), float(tau))


def microbench(kind, buf, ops=0, stream=None):
    """Time (ms) of one memory-system microbenchmark launch over the device tensor buf (see vrt.h)."""
    ms = C.c_float()
    _check(load().vrt_microbench(int(kind), _ptr(buf), int(buf.numel() * buf.element_size()), int(ops),
                                 C.byref(ms), _stream_ptr(stream)), "vrt_microbench")
    return float(ms.value)


def _info_dict(info):
    return {"device_status": info.device_status, "n_fragments": info.n_fragments, "n_listed": info.n_listed,
            "n_bricks": info.n_bricks, "n_occupied": info.n_occupied, "n_visible": info.n_visible}


def frame_noalloc(xyz, offsets, radius, origin, voxel_size, dims, view, camera: vrt_camera, rgba, depth=None,
                  first_id=None, status=True, stream=None):
    """One frame (voxelize, cull, trace) in the library's fixed per-device arena, with no context and no
    allocation.  view = (eye, cull_mode, alpha, tau).  status: synchronize and return the frame totals
    (as Context.frame_status), else return None without synchronizing."""
    lines = make_lines(xyz, offsets, radius)
    grid = vrt_grid(_f3(origin), float(voxel_size), (C.c_int32 * 3)(*[int(x) for x in dims]))
    eye, mode, alpha, tau = view
    v = vrt_view(_f3(eye), int(mode), float(alpha), float(tau))
    img = vrt_image(_ptr(rgba), _ptr(depth), _ptr(first_id))
    info = vrt_frame_info()
    _check(load().vrt_frame_noalloc(C.byref(lines), C.byref(grid), C.byref(v), C.byref(camera), C.byref(img),
                                    C.byref(info) if status else None, _stream_ptr(stream)), "vrt_frame_noalloc")
    if not status:
        return None
    return _info_dict(info)


class Context:
    """One voxel ray tracing context: arenas sized at creation, reused per frame."""

    def __init__(self, max_vertices, max_fragments, max_dim, device=0, max_pixels=1920 * 1080, form=FORM_PLAIN):
        L = load()
        d = vrt_desc(int(max_vertices), int(max_fragments), int(max_dim), int(device), int(max_pixels), int(form), 0)
        h = C.c_void_p()
        _check(L.vrt_create(C.byref(d), C.byref(h)), "vrt_create")
        self._h = h
        self.device = device
        self.max_fragments = int(max_fragments)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(load().vrt_destroy(self._h), "vrt_destroy")
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def voxelize(self, xyz, offsets, radius, origin, voxel_size, dims, stream=None, voxelizer=VOX_CAPSULE,
                 rgba=None, alpha_default=0.0):
        """xyz: device float32 [n, 3]; offsets: device int32 [n_polylines + 1]; see make_lines."""
        lines = make_lines(xyz, offsets, radius, voxelizer, rgba, alpha_default)
        grid = vrt_grid(_f3(origin), float(voxel_size), (C.c_int32 * 3)(*[int(x) for x in dims]))
        _check(load().vrt_voxelize(self._h, C.byref(lines), C.byref(grid), _stream_ptr(stream)), "vrt_voxelize")

    def cull(self, eye, mode, alpha=1.0, tau=1.0 / 256.0, stream=None):
        view = vrt_view(_f3(eye), int(mode), float(alpha), float(tau))
        _check(load().vrt_cull(self._h, C.byref(view), _stream_ptr(stream)), "vrt_cull")

    def shade(self, light_dir=(0.3, 0.5, 0.8), n_cones=16, n_samples=4, ambient=0.3, enable=True, stream=None):
        """Voxel-space shading of the visible voxels (ambient occlusion + directional shadow); the following
        traces scale hit colours by it, until the next cull."""
        sh = vrt_shading(_f3(light_dir), int(n_cones), int(n_samples), float(ambient), int(bool(enable)), 0)
        _check(load().vrt_shade(self._h, C.byref(sh), _stream_ptr(stream)), "vrt_shade")

    def sort_lists(self, stream=None):
        """Sorts every visible voxel's list ascending by segment id (canonical order)."""
        _check(load().vrt_sort_lists(self._h, _stream_ptr(stream)), "vrt_sort_lists")

    def trace(self, camera: vrt_camera, rgba, depth=None, first_id=None, stream=None):
        img = vrt_image(_ptr(rgba), _ptr(depth), _ptr(first_id))
        _check(load().vrt_trace(self._h, C.byref(camera), C.byref(img), _stream_ptr(stream)), "vrt_trace")

    def trace_stats(self, camera: vrt_camera, rgba, depth=None, first_id=None, stream=None):
        """Work counters of one trace (synchronizes); also writes the image."""
        img = vrt_image(_ptr(rgba), _ptr(depth), _ptr(first_id))
        st = vrt_trace_stats()
        _check(load().vrt_trace_stats_run(self._h, C.byref(camera), C.byref(img), C.byref(st), _stream_ptr(stream)),
               "vrt_trace_stats_run")
        return {n: int(getattr(st, n)) for n, _ in vrt_trace_stats._fields_}

    def debug_rays(self, camera: vrt_camera, pixels, dirs, stream=None):
        _check(load().vrt_debug_rays(self._h, C.byref(camera), _ptr(pixels), int(pixels.shape[0]), _ptr(dirs),
                                     _stream_ptr(stream)), "vrt_debug_rays")

    def frame_status(self):
        info = vrt_frame_info()
        _check(load().vrt_frame_status(self._h, C.byref(info)), "vrt_frame_status")
        return _info_dict(info)

    def set_tune(self, mode, **shape):
        """Sets the tracer launch shape of trace mode `mode`; unnamed fields keep their current value."""
        t = vrt_tune()
        _check(load().vrt_get_tune(self._h, int(mode), C.byref(t)), "vrt_get_tune")
        for k, v in shape.items():
            if k not in TUNE_FIELDS:
                raise KeyError(k)
            setattr(t, k, int(v))
        _check(load().vrt_set_tune(self._h, int(mode), C.byref(t)), "vrt_set_tune")

    def get_tune(self, mode):
        t = vrt_tune()
        _check(load().vrt_get_tune(self._h, int(mode), C.byref(t)), "vrt_get_tune")
        return {k: int(getattr(t, k)) for k in TUNE_FIELDS}

    def autotune(self, camera: vrt_camera, rgba, depth=None, first_id=None, reps=3, warmup=1, sweeps=2,
                 cache_path=None, key=None, stream=None):
        """Times launch shapes of the camera's trace mode on the current structure and keeps the fastest
        (synchronizes).  Returns {"best": shape, "best_ms", "start_ms", "evaluated", "from_cache"}."""
        img = vrt_image(_ptr(rgba), _ptr(depth), _ptr(first_id))
        sp = vrt_tune_space(C.pointer(camera), C.pointer(img), int(reps), int(warmup), int(sweeps), 0,
                            None if cache_path is None else os.fsencode(cache_path),
                            None if key is None else str(key).encode())
        res = vrt_tune_result()
        _check(load().vrt_autotune(self._h, C.byref(sp), C.byref(res), _stream_ptr(stream)), "vrt_autotune")
        return {"best": {k: int(getattr(res.best, k)) for k in TUNE_FIELDS}, "best_ms": float(res.best_ms),
                "start_ms": float(res.start_ms), "evaluated": int(res.evaluated), "from_cache": bool(res.from_cache)}

    def autotune_grid(self, xyz, offsets, radius, grids, passes, reps=3, warmup=1, stream=None):
        """Times whole frames for each candidate grid (origin, voxel_size, dims); passes as in frame_graph.
        Returns (index of the fastest grid, [mean frame ms per grid, inf where it did not fit]).  Synchronizes;
        the context holds the last candidate's structure afterwards."""
        lines = make_lines(xyz, offsets, radius)
        gs = (vrt_grid * len(grids))()
        for i, (origin, voxel_size, dims) in enumerate(grids):
            gs[i] = vrt_grid(_f3(origin), float(voxel_size), (C.c_int32 * 3)(*[int(x) for x in dims]))
        views, cams, imgs = self._passes(passes)
        best = C.c_int32()
        ms = (C.c_float * len(grids))()
        _check(load().vrt_autotune_grid(self._h, C.byref(lines), gs, len(grids), views, cams, imgs, len(passes),
                                        int(reps), int(warmup), C.byref(best), ms, _stream_ptr(stream)),
               "vrt_autotune_grid")
        return int(best.value), [float(x) for x in ms]

    @staticmethod
    def _passes(passes):
        n = len(passes)
        views = (vrt_view * max(n, 1))()
        cams = (vrt_camera * max(n, 1))()
        imgs = (vrt_image * max(n, 1))()
        for i, (view, cam, rgba, depth, fid) in enumerate(passes):
            eye, mode, alpha, tau = view
            views[i] = vrt_view(_f3(eye), int(mode), float(alpha), float(tau))
            cams[i] = cam
            imgs[i] = vrt_image(_ptr(rgba), _ptr(depth), _ptr(fid))
        return views, cams, imgs

    def profile_enable(self, enable=True):
        _check(load().vrt_profile_enable(self._h, int(bool(enable))), "vrt_profile_enable")

    def profile_read(self):
        """{kernel name: (launches, total ms)} since the last read (synchronizes)."""
        buf = (vrt_kernel_time * 64)()
        n = C.c_int32()
        _check(load().vrt_profile_read(self._h, buf, 64, C.byref(n)), "vrt_profile_read")
        return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(n.value)}

    def frame_graph(self, xyz, offsets, radius, origin, voxel_size, dims, passes):
        """Captures one frame as a HIP graph.  passes: list of (view, camera, rgba, depth, first_id) with
        view = (eye, cull_mode, alpha, tau).  Returns a FrameGraph; keep the tensors alive while it exists."""
        lines = make_lines(xyz, offsets, radius)
        grid = vrt_grid(_f3(origin), float(voxel_size), (C.c_int32 * 3)(*[int(x) for x in dims]))
        n = len(passes)
        views, cams, imgs = self._passes(passes)
        h = C.c_void_p()
        _check(load().vrt_graph_create(self._h, C.byref(lines), C.byref(grid), views, cams, imgs, n, C.byref(h)),
               "vrt_graph_create")
        return FrameGraph(h, self, (xyz, offsets, passes))

    def query_as(self):
        v = vrt_as_view()
        _check(load().vrt_query_as(self._h, C.byref(v)), "vrt_query_as")
        return v


class FrameGraph:
    """A captured frame; launch() replays it on the current (or given) stream."""

    def __init__(self, handle, ctx, keepalive):
        self._h = handle
        self._ctx = ctx
        self._keep = keepalive

    def launch(self, stream=None):
        _check(load().vrt_graph_launch(self._h, _stream_ptr(stream)), "vrt_graph_launch")

    def close(self):
        if self._h and self._h.value:
            _check(load().vrt_graph_destroy(self._h), "vrt_graph_destroy")
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


class _Borrowed(Context):
    """A context owned by a batch (not destroyed by Python)."""

    def __init__(self, handle):  # noqa: D401 - no allocation here
        self._h = handle
        self.device = 0
        self.max_fragments = 0

    def close(self):
        self._h = C.c_void_p()


class Batch:
    """Many line sets built and traced together (one persistent launch, or set by set)."""

    def __init__(self, capacities, device=0, form=FORM_PLAIN):
        """capacities: list of (max_vertices, max_fragments, max_dim, max_pixels), one per set."""
        n = len(capacities)
        descs = (vrt_desc * n)()
        for i, (mv, mf, md, mp) in enumerate(capacities):
            descs[i] = vrt_desc(int(mv), int(mf), int(md), int(device), int(mp), int(form), 0)
        h = C.c_void_p()
        _check(load().vrt_batch_create(descs, n, C.byref(h)), "vrt_batch_create")
        self._h = h
        self.n = n

    def run(self, items, mode=BATCH_PERSISTENT, stream=None):
        """items: list of dicts with xyz, offsets, radius, origin, voxel_size, dims, view=(eye, mode, alpha, tau),
        camera (vrt_camera), rgba, depth, first_id."""
        arr = (vrt_batch_item * self.n)()
        for i, it in enumerate(items):
            x, o = it["xyz"], it["offsets"]
            eye, cm, al, tau = it["view"]
            arr[i] = vrt_batch_item(
                make_lines(x, o, it["radius"], it.get("voxelizer", VOX_CAPSULE), it.get("rgba_seg"),
                           it.get("alpha_default", 0.0)),
                vrt_grid(_f3(it["origin"]), float(it["voxel_size"]), (C.c_int32 * 3)(*[int(v) for v in it["dims"]])),
                vrt_view(_f3(eye), int(cm), float(al), float(tau)), it["camera"],
                vrt_image(_ptr(it["rgba"]), _ptr(it.get("depth")), _ptr(it.get("first_id"))))
        _check(load().vrt_batch_run(self._h, arr, self.n, int(mode), _stream_ptr(stream)), "vrt_batch_run")

    def context(self, i):
        h = C.c_void_p()
        _check(load().vrt_batch_context(self._h, int(i), C.byref(h)), "vrt_batch_context")
        return _Borrowed(h)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(load().vrt_batch_destroy(self._h), "vrt_batch_destroy")
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass
