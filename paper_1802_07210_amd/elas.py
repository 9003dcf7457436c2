"""Python binding of libelas_mi355x.so (argument marshalling only).

Every stage of the path runs in the library's HIP kernels and host code; this
module only converts torch tensors and numpy arrays to pointers. PyTorch is
used for device memory and streams.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libelas_mi355x.so")

ELAS_OK = 0
ERRORS = {-1: "ELAS_ERR_ARG", -2: "ELAS_ERR_OOM", -3: "ELAS_ERR_HIP",
          -4: "ELAS_ERR_UNSUPPORTED", -5: "ELAS_ERR_INTERNAL"}

EXPORTS = ("elas_params_default", "elas_create", "elas_destroy", "elas_process",
           "elas_get_stats", "elas_last_error", "elas_get_intermediate", "elas_triangulate",
           "elas_set_timing", "elas_get_timing", "elas_set_batch_flags", "elas_process_batch",
           "elas_get_tuned_variants", "elas_frame_bytes", "elas_server_config_default",
           "elas_server_create", "elas_server_submit", "elas_server_wait", "elas_server_poll",
           "elas_server_get_stats", "elas_server_last_error", "elas_server_destroy",
           "elas_server_submit_on", "elas_set_mesh_round_limit",
           "elas_get_batch_intermediate", "elas_process_noalloc", "elas_set_tile_variants",
           "elas_device_bytes")

BATCH_GRAPH = 1
BATCH_AUTOTUNE = 2


class ElasParams(C.Structure):
    _fields_ = [
        ("disp_min", C.c_int32), ("disp_max", C.c_int32),
        ("support_threshold", C.c_float), ("support_texture", C.c_int32),
        ("candidate_stepsize", C.c_int32), ("incon_window_size", C.c_int32),
        ("incon_threshold", C.c_int32), ("incon_min_support", C.c_int32),
        ("redun_max_dist", C.c_int32), ("redun_threshold", C.c_int32),
        ("grid_size", C.c_int32), ("beta", C.c_float), ("gamma", C.c_float),
        ("sigma", C.c_float), ("sradius", C.c_int32), ("match_texture", C.c_int32),
        ("lr_threshold", C.c_int32), ("full_search", C.c_int32),
        ("mesh_on_host", C.c_int32),
        ("descriptor", C.c_int32), ("census_support_window", C.c_int32),
        ("census_dense_window", C.c_int32), ("ambiguity", C.c_int32),
        ("redundancy", C.c_int32), ("support_subsample", C.c_int32),
        ("median_window", C.c_int32), ("add_corners", C.c_int32),
    ]


class ElasStats(C.Structure):
    _fields_ = [
        ("support_evals", C.c_int64), ("dense_evals", C.c_int64),
        ("n_support_left", C.c_int32), ("n_support_right", C.c_int32),
        ("n_tri_left", C.c_int32), ("n_tri_right", C.c_int32),
        ("host_mesh_ms", C.c_double),
        ("mesh_rounds", C.c_int32 * 2), ("mesh_flips", C.c_int32 * 2),
    ]


class ElasTiming(C.Structure):
    _fields_ = [
        ("descriptor_ms", C.c_float), ("support_ms", C.c_float), ("filter_ms", C.c_float),
        ("rows_ms", C.c_float), ("mesh_ms", C.c_float), ("raster_ms", C.c_float),
        ("dense_ms", C.c_float), ("lrcheck_ms", C.c_float), ("device_span_ms", C.c_float),
        ("host_wait_ms", C.c_double), ("host_mesh_ms", C.c_double),
    ]


class ElasPair(C.Structure):
    _fields_ = [
        ("left", C.c_void_p), ("right", C.c_void_p),
        ("w", C.c_int32), ("h", C.c_int32), ("stride", C.c_int32),
        ("disp_left", C.c_void_p), ("disp_right", C.c_void_p),
        ("params", C.c_void_p),
    ]


class ServerConfig(C.Structure):
    _fields_ = [("max_batch", C.c_int32), ("max_inflight", C.c_int32),
                ("memory_budget", C.c_int64), ("plain", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("batches", C.c_int64),
                ("batched_pairs", C.c_int64), ("peak_bytes_in_flight", C.c_int64),
                ("queued", C.c_int64), ("bytes_in_flight", C.c_int64),
                ("resident_bytes", C.c_int64), ("peak_resident_bytes", C.c_int64)]


# name -> (enum value, numpy dtype, trailing shape kind)
INTERMEDIATES = {
    "desc_left": (0, np.uint8), "desc_right": (1, np.uint8),
    "dcan_raw": (2, np.int16), "dcan_incon": (3, np.int16), "dcan_vert": (4, np.int16),
    "dcan_final": (5, np.int16),
    "support_left": (6, np.int32), "support_right": (7, np.int32), "corners": (8, np.int32),
    "tri_left": (9, np.int32), "tri_right": (10, np.int32),
    "plane_left": (11, np.float32), "plane_right": (12, np.float32),
    "owner_left": (13, np.int32), "owner_right": (14, np.int32),
    "dplane_left": (15, np.int16), "dplane_right": (16, np.int16),
    "grid_left": (17, np.uint64), "grid_right": (18, np.uint64),
    "raw_left": (19, np.int16), "raw_right": (20, np.int16),
    "lut": (21, np.int32),
    "census_dense_left": (22, np.uint64), "census_dense_right": (23, np.uint64),
    "census_support_left": (24, np.uint32), "census_support_right": (25, np.uint32),
    "checked_left": (26, np.int16), "checked_right": (27, np.int16),
}

_lib = None


class ElasError(RuntimeError):
    pass


def lib() -> C.CDLL:
    """Loads the HIP library; there is no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ElasError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.elas_params_default.argtypes = [C.POINTER(ElasParams)]
        L.elas_params_default.restype = None
        L.elas_create.argtypes = [C.POINTER(ElasParams), C.POINTER(vp)]
        L.elas_destroy.argtypes = [vp]
        L.elas_process.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp]
        L.elas_process_noalloc.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, vp,
                                           vp, vp]
        L.elas_get_stats.argtypes = [vp, C.POINTER(ElasStats)]
        L.elas_last_error.argtypes = [vp]
        L.elas_last_error.restype = C.c_char_p
        L.elas_get_intermediate.argtypes = [vp, C.c_int32, vp, C.c_int64, C.POINTER(C.c_int64)]
        L.elas_triangulate.argtypes = [vp, C.c_int32, vp, C.c_int32, C.c_int32, vp, vp]
        L.elas_set_timing.argtypes = [vp, C.c_int32]
        L.elas_get_timing.argtypes = [vp, C.POINTER(ElasTiming)]
        L.elas_set_batch_flags.argtypes = [vp, C.c_int32]
        L.elas_process_batch.argtypes = [vp, C.c_int32, C.POINTER(ElasPair), vp]
        L.elas_get_tuned_variants.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                              C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.elas_set_tile_variants.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                             C.c_int32]
        L.elas_frame_bytes.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_int64)]
        L.elas_device_bytes.argtypes = [vp, C.POINTER(C.c_int64)]
        L.elas_server_config_default.argtypes = [C.POINTER(ServerConfig)]
        L.elas_server_config_default.restype = None
        L.elas_server_create.argtypes = [vp, C.POINTER(ServerConfig), C.POINTER(vp)]
        L.elas_server_submit.argtypes = [vp, C.POINTER(ElasPair), C.POINTER(C.c_int64)]
        L.elas_server_submit_on.argtypes = [vp, C.POINTER(ElasPair), vp,
                                            C.POINTER(C.c_int64)]
        L.elas_set_mesh_round_limit.argtypes = [vp, C.c_int32]
        L.elas_get_batch_intermediate.argtypes = [vp, C.c_int32, C.c_int32, vp, C.c_int64,
                                                  C.POINTER(C.c_int64)]
        L.elas_server_wait.argtypes = [vp, C.c_int64, C.POINTER(C.c_double)]
        L.elas_server_poll.argtypes = [vp, C.c_int64, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_double)]
        L.elas_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
        L.elas_server_last_error.argtypes = [vp]
        L.elas_server_last_error.restype = C.c_char_p
        L.elas_server_destroy.argtypes = [vp]
        for name in EXPORTS:
            if name not in ("elas_params_default", "elas_last_error",
                            "elas_server_config_default", "elas_server_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def default_params(**overrides) -> ElasParams:
    p = ElasParams()
    lib().elas_params_default(C.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k) or k.startswith("_"):
            raise KeyError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def _check(rc: int, handle=None):
    if rc < 0:
        msg = lib().elas_last_error(handle)
        raise ElasError(f"{ERRORS.get(rc, rc)}: {msg.decode() if msg else ''}")
    return rc


def _np_ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def triangulate(pts: np.ndarray, corners, w: int, h: int) -> Tuple[np.ndarray, np.ndarray]:
    """Host mesh step: canonical triangles [ntri, 9] and planes [ntri, 3];
    ntri = 2n+2 with the four corners' d in `corners`, or, with corners None,
    the mesh of the points alone."""
    pts = np.ascontiguousarray(pts, np.int32).reshape(-1, 3)
    n = len(pts)
    cptr = None
    if corners is not None:
        corners = np.ascontiguousarray(corners, np.int32)
        cptr = _np_ptr(corners)
    recs = np.zeros((max(1, 2 * n + 2), 9), np.int32)
    planes = np.zeros((max(1, 2 * n + 2), 3), np.float32)
    nt = _check(lib().elas_triangulate(_np_ptr(pts), n, cptr, w, h,
                                       _np_ptr(recs), _np_ptr(planes)))
    return recs[:nt], planes[:nt]


class Elas:
    """One handle: parameters, the prior table and per-size device buffers."""

    def __init__(self, params: Optional[ElasParams] = None, **overrides):
        self.params = params if params is not None else default_params(**overrides)
        h = C.c_void_p()
        _check(lib().elas_create(C.byref(self.params), C.byref(h)))
        self._h = h
        self._shape = None

    def close(self):
        if getattr(self, "_h", None):
            lib().elas_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def process(self, left, right, out_left=None, out_right=None, stream=None):
        """left/right: torch.uint8 CUDA tensors [H, W] (rows may be padded:
        stride(0) >= W, stride(1) == 1, same layout for both). Returns int16
        [H, W] left and right disparity maps (-1 = invalid)."""
        import torch
        if left.dtype != torch.uint8 or right.dtype != torch.uint8:
            raise TypeError("images must be uint8")
        if not (left.is_cuda and right.is_cuda):
            raise TypeError("images must be device tensors")
        if left.dim() != 2 or left.shape != right.shape:
            raise ValueError("images must be 2-D and of equal shape")
        if left.stride(1) != 1 or right.stride(1) != 1 or left.stride(0) != right.stride(0):
            raise ValueError("images need unit column stride and equal row strides")
        H, W = left.shape
        stride = left.stride(0)
        if out_left is None:
            out_left = torch.empty((H, W), dtype=torch.int16, device=left.device)
        if out_right is None:
            out_right = torch.empty((H, W), dtype=torch.int16, device=left.device)
        for o in (out_left, out_right):
            if o.dtype != torch.int16 or not o.is_contiguous() or tuple(o.shape) != (H, W):
                raise ValueError("outputs must be contiguous int16 [H, W]")
        if stream is None:
            stream = torch.cuda.current_stream(left.device)
        s = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        _check(lib().elas_process(self._h, C.c_void_p(left.data_ptr()),
                                  C.c_void_p(right.data_ptr()), W, H, stride, C.c_void_p(s),
                                  C.c_void_p(out_left.data_ptr()),
                                  C.c_void_p(out_right.data_ptr())), self._h)
        self._shape = (H, W)
        return out_left, out_right

    def set_batch_flags(self, graph: bool = True, autotune: bool = True):
        flags = (BATCH_GRAPH if graph else 0) | (BATCH_AUTOTUNE if autotune else 0)
        _check(lib().elas_set_batch_flags(self._h, flags), self._h)

    def process_batch(self, items, stream=None):
        """items: sequence of (left, right, out_left, out_right) or
        (left, right, out_left, out_right, params_elas) with torch uint8 [H, W]
        images and int16 [H, W] outputs on the device; params_elas (an Elas)
        supplies that pair's parameters. All pairs run in one batched call."""
        import torch
        arr = (ElasPair * max(1, len(items)))()
        keep = []
        for i, it in enumerate(items):
            left, right, ol, orr = it[:4]
            ph = it[4].handle if len(it) > 4 and it[4] is not None else None
            for t in (left, right):
                if t.dtype != torch.uint8 or not t.is_cuda or t.dim() != 2 or t.stride(1) != 1:
                    raise ValueError("images must be uint8 [H, W] device tensors with unit column stride")
            if left.shape != right.shape or left.stride(0) != right.stride(0):
                raise ValueError("left and right must share shape and row stride")
            H, W = left.shape
            for o in (ol, orr):
                if o.dtype != torch.int16 or not o.is_contiguous() or tuple(o.shape) != (H, W):
                    raise ValueError("outputs must be contiguous int16 [H, W]")
            arr[i] = ElasPair(left.data_ptr(), right.data_ptr(), W, H, left.stride(0),
                              ol.data_ptr(), orr.data_ptr(), ph)
            keep.append(it)
        if stream is None:
            dev = items[0][0].device if items else torch.device("cuda:0")
            stream = torch.cuda.current_stream(dev)
        s = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        _check(lib().elas_process_batch(self._h, len(items), arr, C.c_void_p(s)), self._h)
        return [(it[2], it[3]) for it in keep]

    def frame_bytes(self, w: int, h: int) -> int:
        b = C.c_int64()
        _check(lib().elas_frame_bytes(self._h, w, h, C.byref(b)), self._h)
        return b.value

    def set_tile_variants(self, w: int, h: int, desc_rows: int, dense_rows: int,
                          support_run: int = 16):
        _check(lib().elas_set_tile_variants(self._h, w, h, desc_rows, dense_rows, support_run),
               self._h)

    def device_bytes(self) -> int:
        """Device bytes the handle holds (buffer sets of every size and stream)."""
        b = C.c_int64()
        _check(lib().elas_device_bytes(self._h, C.byref(b)), self._h)
        return b.value

    def tuned_variants(self, w: int, h: int):
        """(descriptor rows, dense rows, support run) chosen for (w, h)."""
        r, b, q = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().elas_get_tuned_variants(self._h, w, h, C.byref(r), C.byref(b), C.byref(q)),
               self._h)
        return r.value, b.value, q.value

    def stats(self) -> dict:
        st = ElasStats()
        _check(lib().elas_get_stats(self._h, C.byref(st)), self._h)
        out = {k: getattr(st, k) for k, _ in ElasStats._fields_}
        for k in ("mesh_rounds", "mesh_flips"):
            out[k] = list(out[k])
        return out

    def set_mesh_round_limit(self, rounds: int):
        """Test hook: caps the device mesh's flip rounds (a frame that needs
        more fails, reported as ELAS_ERR_INTERNAL by the next call)."""
        _check(lib().elas_set_mesh_round_limit(self._h, int(rounds)), self._h)

    def set_timing(self, enable: bool):
        _check(lib().elas_set_timing(self._h, int(bool(enable))), self._h)

    def timing(self) -> dict:
        t = ElasTiming()
        _check(lib().elas_get_timing(self._h, C.byref(t)), self._h)
        return {k: getattr(t, k) for k, _ in ElasTiming._fields_}

    def intermediate(self, name: str) -> np.ndarray:
        which, dtype = INTERMEDIATES[name]
        need = C.c_int64(0)
        _check(lib().elas_get_intermediate(self._h, which, None, 0, C.byref(need)), self._h)
        nbytes = int(need.value)
        buf = np.zeros(max(nbytes, 1), np.uint8)
        _check(lib().elas_get_intermediate(self._h, which, _np_ptr(buf), nbytes, None), self._h)
        return buf[:nbytes].view(dtype).copy()

    def batch_intermediate(self, pair: int, name: str) -> np.ndarray:
        """Stage `name` of pair `pair` of this handle's last batched call."""
        which, dtype = INTERMEDIATES[name]
        need = C.c_int64(0)
        L = lib()
        _check(L.elas_get_batch_intermediate(self._h, pair, which, None, 0, C.byref(need)),
               self._h)
        nbytes = int(need.value)
        buf = np.zeros(max(nbytes, 1), np.uint8)
        _check(L.elas_get_batch_intermediate(self._h, pair, which, _np_ptr(buf), nbytes, None),
               self._h)
        return buf[:nbytes].view(dtype).copy()


def _pair_of(left, right, out_left, out_right, params=None) -> ElasPair:
    import torch
    for t in (left, right):
        if t.dtype != torch.uint8 or not t.is_cuda or t.dim() != 2 or t.stride(1) != 1:
            raise ValueError("images must be uint8 [H, W] device tensors with unit column stride")
    if left.shape != right.shape or left.stride(0) != right.stride(0):
        raise ValueError("left and right must share shape and row stride")
    H, W = left.shape
    for o in (out_left, out_right):
        if o.dtype != torch.int16 or not o.is_contiguous() or tuple(o.shape) != (H, W):
            raise ValueError("outputs must be contiguous int16 [H, W]")
    return ElasPair(left.data_ptr(), right.data_ptr(), W, H, left.stride(0),
                    out_left.data_ptr(), out_right.data_ptr(),
                    params.handle if params is not None else None)


class Server:
    """Continuous-batching server over one handle (the handle and every
    parameter handle of submitted pairs belong to the server until close)."""

    def __init__(self, elas: "Elas", max_batch: int = 32, max_inflight: int = 3,
                 memory_budget: int = 32 << 30, plain: bool = False):
        cfg = ServerConfig()
        lib().elas_server_config_default(C.byref(cfg))
        cfg.max_batch, cfg.max_inflight = max_batch, max_inflight
        cfg.memory_budget, cfg.plain = memory_budget, int(bool(plain))
        s = C.c_void_p()
        rc = lib().elas_server_create(elas.handle, C.byref(cfg), C.byref(s))
        if rc < 0:
            raise ElasError(f"{ERRORS.get(rc, rc)}: {lib().elas_server_last_error(None).decode()}")
        self._s = s
        self._elas = elas
        self._keep = {}

    def _check(self, rc):
        if rc < 0:
            msg = lib().elas_server_last_error(self._s)
            raise ElasError(f"{ERRORS.get(rc, rc)}: {msg.decode() if msg else ''}")
        return rc

    def submit(self, left, right, out_left, out_right, params: "Elas" = None,
               stream=None) -> int:
        """Queues a pair; it runs after the work already on `stream` (default:
        torch's current stream, which wrote the tensors)."""
        import torch
        pr = _pair_of(left, right, out_left, out_right, params)
        if stream is None:
            stream = torch.cuda.current_stream(left.device)
        s = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        t = C.c_int64()
        self._check(lib().elas_server_submit_on(self._s, C.byref(pr), C.c_void_p(s),
                                                C.byref(t)))
        self._keep[t.value] = (left, right, out_left, out_right)
        return t.value

    def wait(self, ticket: int) -> float:
        ms = C.c_double()
        rc = lib().elas_server_wait(self._s, ticket, C.byref(ms))
        self._keep.pop(ticket, None)
        self._check(rc)
        return ms.value

    def poll(self, ticket: int):
        done, ms = C.c_int32(), C.c_double()
        rc = lib().elas_server_poll(self._s, ticket, C.byref(done), C.byref(ms))
        if done.value:
            self._keep.pop(ticket, None)
        self._check(rc)
        return (ms.value if done.value else None)

    def stats(self) -> dict:
        st = ServerStats()
        self._check(lib().elas_server_get_stats(self._s, C.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_s", None):
            lib().elas_server_destroy(self._s)
            self._s = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
