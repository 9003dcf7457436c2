"""ctypes wrapper of the plain C oracle (liborc_elas.so).

TEST INFRASTRUCTURE ONLY: the parity reference for the HIP library. Only the
tests, the smoke check and the benchmark's CPU-baseline leg import this.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liborc_elas.so")
SOURCES = ["elas_oracle_match.c", "elas_oracle_mesh.c", "elas_oracle_pipeline.c",
           "elas_oracle_variant.c"]

DEFAULTS = dict(
    disp_min=0, disp_max=127, support_threshold=0.85, support_texture=10,
    candidate_stepsize=5, incon_window_size=5, incon_threshold=5,
    incon_min_support=5, redun_max_dist=5, redun_threshold=1, grid_size=20,
    beta=0.02, gamma=3.0, sigma=1.0, sradius=2, match_texture=1,
    lr_threshold=2, full_search=0, descriptor=0, census_support_window=9,
    census_dense_window=5, ambiguity=0, redundancy=0, support_subsample=1,
    median_window=0, add_corners=1)


class OrcParams(C.Structure):
    _fields_ = [
        ("disp_min", C.c_int32), ("disp_max", C.c_int32),
        ("support_threshold", C.c_float), ("support_texture", C.c_int32),
        ("candidate_stepsize", C.c_int32), ("incon_window_size", C.c_int32),
        ("incon_threshold", C.c_int32), ("incon_min_support", C.c_int32),
        ("redun_max_dist", C.c_int32), ("redun_threshold", C.c_int32),
        ("grid_size", C.c_int32), ("beta", C.c_float), ("gamma", C.c_float),
        ("sigma", C.c_float), ("sradius", C.c_int32), ("match_texture", C.c_int32),
        ("lr_threshold", C.c_int32), ("full_search", C.c_int32),
        ("descriptor", C.c_int32), ("census_support_window", C.c_int32),
        ("census_dense_window", C.c_int32), ("ambiguity", C.c_int32),
        ("redundancy", C.c_int32), ("support_subsample", C.c_int32),
        ("median_window", C.c_int32), ("add_corners", C.c_int32),
    ]


_P8, _P16, _P32, _P64 = (C.POINTER(C.c_uint8), C.POINTER(C.c_int16),
                         C.POINTER(C.c_int32), C.POINTER(C.c_uint64))


class OrcTrace(C.Structure):
    _fields_ = [
        ("w", C.c_int32), ("h", C.c_int32), ("lw", C.c_int32), ("lh", C.c_int32),
        ("gw", C.c_int32), ("gh", C.c_int32), ("words", C.c_int32), ("D", C.c_int32),
        ("descL", _P8), ("descR", _P8),
        ("dcan_raw", _P16), ("dcan_incon", _P16), ("dcan_vert", _P16), ("dcan_final", _P16),
        ("nL", C.c_int32), ("nR", C.c_int32),
        ("ptsL", _P32), ("ptsR", _P32),
        ("cornersL", C.c_int32 * 4), ("cornersR", C.c_int32 * 4),
        ("ntriL", C.c_int32), ("ntriR", C.c_int32),
        ("recL", _P32), ("recR", _P32),
        ("planeL", C.POINTER(C.c_float)), ("planeR", C.POINTER(C.c_float)),
        ("ownerL", _P32), ("ownerR", _P32),
        ("dplaneL", _P16), ("dplaneR", _P16),
        ("gridL", _P64), ("gridR", _P64),
        ("lut", _P32),
        ("rawL", _P16), ("rawR", _P16),
        ("outL", _P16), ("outR", _P16),
        ("support_evals", C.c_int64), ("dense_evals", C.c_int64),
        ("stage_ms", C.c_double * 6),
        ("swords", C.c_int32), ("dwords", C.c_int32),
        ("csupL", C.POINTER(C.c_uint32)), ("csupR", C.POINTER(C.c_uint32)),
        ("cdenL", C.POINTER(C.c_uint32)), ("cdenR", C.POINTER(C.c_uint32)),
        ("chkL", _P16), ("chkR", _P16),
        ("nL_all", C.c_int32),
    ]


_lib = None


def build(force: bool = False) -> str:
    """Compiles the oracle with gcc (plain -O2, no fp contraction)."""
    import subprocess
    srcs = [os.path.join(_HERE, s) for s in SOURCES]
    hdr = os.path.join(_HERE, "elas_oracle.h")
    stale = (not os.path.exists(LIB_PATH) or
             max(os.path.getmtime(f) for f in srcs + [hdr]) > os.path.getmtime(LIB_PATH))
    if force or stale:
        tmp = LIB_PATH + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fPIC",
                        "-shared", *srcs, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.orc_sobel.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp, vp]
        L.orc_descriptors.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp]
        L.orc_prior_lut.argtypes = [C.POINTER(OrcParams), vp]
        L.orc_lattice.argtypes = [C.POINTER(OrcParams), C.c_int32, C.c_int32, vp, vp, vp, vp]
        L.orc_support_match.argtypes = [C.POINTER(OrcParams), vp, vp, C.c_int32, C.c_int32,
                                        vp, vp]
        L.orc_ratio_accept.argtypes = [C.c_float, C.c_int32, C.c_int32]
        L.orc_ratio_accept.restype = C.c_int32
        L.orc_filter_incon.argtypes = [C.POINTER(OrcParams), vp, C.c_int32, C.c_int32, vp]
        L.orc_filter_redun.argtypes = [C.POINTER(OrcParams), vp, C.c_int32, C.c_int32,
                                       C.c_int32, vp]
        L.orc_support_lists.argtypes = [C.POINTER(OrcParams), vp, C.c_int32, C.c_int32,
                                        C.c_int32, C.c_int32, vp, vp, vp, vp, vp, vp]
        L.orc_delaunay.argtypes = [vp, C.c_int32, vp]
        L.orc_delaunay.restype = C.c_int32
        L.orc_delaunay_points.argtypes = [vp, C.c_int32, vp]
        L.orc_delaunay_points.restype = C.c_int32
        L.orc_orient.argtypes = [vp, vp, vp]
        L.orc_orient.restype = C.c_int64
        L.orc_incircle.argtypes = [vp, vp, vp, vp]
        L.orc_incircle.restype = C.c_int64
        L.orc_canonical_triangles.argtypes = [vp, vp, C.c_int32, vp]
        L.orc_plane.argtypes = [vp, vp]
        L.orc_plane_map.argtypes = [C.POINTER(OrcParams), vp, vp, C.c_int32, C.c_int32,
                                    C.c_int32, vp, vp]
        L.orc_grid_dims.argtypes = [C.POINTER(OrcParams), C.c_int32, C.c_int32, vp, vp, vp]
        L.orc_grid.argtypes = [C.POINTER(OrcParams), vp, C.c_int32, C.c_int32, C.c_int32, vp]
        L.orc_dense.argtypes = [C.POINTER(OrcParams), vp, vp, vp, vp, C.c_int32, vp,
                                C.c_int32, C.c_int32, C.c_int32, vp]
        L.orc_dense.restype = C.c_int64
        L.orc_lrcheck.argtypes = [C.POINTER(OrcParams), vp, vp, C.c_int32, C.c_int32, vp, vp]
        L.orc_process.argtypes = [C.POINTER(OrcParams), vp, vp, C.c_int32, C.c_int32,
                                  C.c_int32, C.POINTER(OrcTrace)]
        L.orc_process.restype = C.c_int32
        L.orc_trace_free.argtypes = [C.POINTER(OrcTrace)]
        L.orc_census.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, C.c_int32]
        L.orc_hamming.argtypes = [vp, vp, C.c_int32]
        L.orc_hamming.restype = C.c_int32
        L.orc_census_texture.argtypes = [vp, C.c_int32]
        L.orc_census_texture.restype = C.c_int32
        L.orc_shiftsum_threshold.argtypes = [C.c_int32]
        L.orc_shiftsum_threshold.restype = C.c_int32
        L.orc_shiftsum_accept.argtypes = [C.c_int32, C.c_int32]
        L.orc_shiftsum_accept.restype = C.c_int32
        L.orc_support_accept.argtypes = [C.POINTER(OrcParams), C.c_int32, C.c_int32]
        L.orc_support_accept.restype = C.c_int32
        L.orc_support_match_census.argtypes = [C.POINTER(OrcParams), vp, vp, C.c_int32,
                                               C.c_int32, C.c_int32, vp, vp]
        L.orc_filter_redun_past.argtypes = [C.POINTER(OrcParams), vp, C.c_int32, C.c_int32,
                                            C.c_int32, vp]
        L.orc_subsample.argtypes = [vp, C.c_int32, C.c_int32]
        L.orc_subsample.restype = C.c_int32
        L.orc_dense_census.argtypes = [C.POINTER(OrcParams), vp, vp, C.c_int32, vp, vp,
                                       C.c_int32, vp, C.c_int32, C.c_int32, C.c_int32, vp]
        L.orc_dense_census.restype = C.c_int64
        L.orc_median.argtypes = [C.c_int32, vp, C.c_int32, C.c_int32, vp]
        _lib = L
    return _lib


def params(**overrides) -> OrcParams:
    d = dict(DEFAULTS)
    d.update(overrides)
    unknown = set(d) - set(DEFAULTS)
    if unknown:
        raise KeyError(f"unknown parameters: {sorted(unknown)}")
    return OrcParams(**d)


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- stages
def sobel(img: np.ndarray):
    h, w = img.shape
    img = np.ascontiguousarray(img, np.uint8)
    du = np.zeros((h, w), np.int16)
    dv = np.zeros((h, w), np.int16)
    lib().orc_sobel(_ptr(img), w, h, w, _ptr(du), _ptr(dv))
    return du, dv


def descriptors(img: np.ndarray) -> np.ndarray:
    h, w = img.shape
    img = np.ascontiguousarray(img, np.uint8)
    out = np.zeros((h, w, 16), np.uint8)
    lib().orc_descriptors(_ptr(img), w, h, w, _ptr(out))
    return out


def prior_lut(p: OrcParams) -> np.ndarray:
    D = p.disp_max - p.disp_min + 1
    out = np.zeros(D, np.int32)
    lib().orc_prior_lut(C.byref(p), _ptr(out))
    return out


def lattice(p: OrcParams, w: int, h: int):
    vals = [np.zeros(1, np.int32) for _ in range(4)]
    lib().orc_lattice(C.byref(p), w, h, *[_ptr(v) for v in vals])
    return tuple(int(v[0]) for v in vals)  # lw, lh, u0, v0


def support_match(p: OrcParams, descL: np.ndarray, descR: np.ndarray):
    h, w = descL.shape[:2]
    lw, lh, _, _ = lattice(p, w, h)
    out = np.zeros((lh, lw), np.int16)
    ev = np.zeros(1, np.int64)
    lib().orc_support_match(C.byref(p), _ptr(np.ascontiguousarray(descL)),
                            _ptr(np.ascontiguousarray(descR)), w, h, _ptr(out), _ptr(ev))
    return out, int(ev[0])


def ratio_accept(thr: float, m1: int, m2: int) -> bool:
    return bool(lib().orc_ratio_accept(thr, m1, m2))


def filter_incon(p: OrcParams, dcan: np.ndarray) -> np.ndarray:
    dcan = np.ascontiguousarray(dcan, np.int16)
    out = np.zeros_like(dcan)
    lib().orc_filter_incon(C.byref(p), _ptr(dcan), dcan.shape[1], dcan.shape[0], _ptr(out))
    return out


def filter_redun(p: OrcParams, dcan: np.ndarray, vertical: bool) -> np.ndarray:
    dcan = np.ascontiguousarray(dcan, np.int16)
    out = np.zeros_like(dcan)
    lib().orc_filter_redun(C.byref(p), _ptr(dcan), dcan.shape[1], dcan.shape[0],
                           int(vertical), _ptr(out))
    return out


def support_lists(p: OrcParams, dcan: np.ndarray, w: int, h: int):
    dcan = np.ascontiguousarray(dcan, np.int16)
    lh, lw = dcan.shape
    cap = max(1, lw * lh)
    pl = np.zeros((cap, 3), np.int32)
    pr = np.zeros((cap, 3), np.int32)
    nl = np.zeros(1, np.int32)
    nr = np.zeros(1, np.int32)
    cl = np.zeros(4, np.int32)
    cr = np.zeros(4, np.int32)
    lib().orc_support_lists(C.byref(p), _ptr(dcan), lw, lh, w, h, _ptr(pl), _ptr(nl),
                            _ptr(cl), _ptr(pr), _ptr(nr), _ptr(cr))
    return pl[:nl[0]].copy(), cl, pr[:nr[0]].copy(), cr


def orient(a, b, c) -> int:
    arr = [np.asarray(x, np.int32) for x in (a, b, c)]
    return int(lib().orc_orient(*[_ptr(x) for x in arr]))


def incircle(a, b, c, d) -> int:
    arr = [np.asarray(x, np.int32) for x in (a, b, c, d)]
    return int(lib().orc_incircle(*[_ptr(x) for x in arr]))


def delaunay(uv: np.ndarray) -> np.ndarray:
    """uv: [n, 2] points, corners first. Returns [ntri, 3] vertex indices."""
    uv = np.ascontiguousarray(uv, np.int32)
    n = uv.shape[0]
    tris = np.zeros((2 * n + 8, 3), np.int32)
    nt = lib().orc_delaunay(_ptr(uv), n, _ptr(tris))
    if nt < 0:
        raise ValueError("orc_delaunay rejected its input")
    return tris[:nt].copy()


def delaunay_points(uv: np.ndarray) -> np.ndarray:
    """uv: [n, 2] distinct points, no corners. Returns [ntri, 3] vertex
    indices (empty for collinear points)."""
    uv = np.ascontiguousarray(uv, np.int32).reshape(-1, 2)
    n = uv.shape[0]
    tris = np.zeros((max(1, 2 * n), 3), np.int32)
    nt = lib().orc_delaunay_points(_ptr(uv), n, _ptr(tris))
    if nt < 0:
        raise ValueError("orc_delaunay_points rejected its input")
    return tris[:nt].copy()


def canonical(uvd: np.ndarray, tris: np.ndarray):
    uvd = np.ascontiguousarray(uvd, np.int32)
    tris = np.ascontiguousarray(tris, np.int32)
    recs = np.zeros((max(1, len(tris)), 9), np.int32)
    lib().orc_canonical_triangles(_ptr(uvd), _ptr(tris), len(tris), _ptr(recs))
    return recs[:len(tris)].copy()


def plane(rec) -> np.ndarray:
    rec = np.ascontiguousarray(rec, np.int32)
    out = np.zeros(3, np.float32)
    lib().orc_plane(_ptr(rec), _ptr(out))
    return out


def plane_map(p: OrcParams, recs: np.ndarray, planes: np.ndarray, w: int, h: int):
    recs = np.ascontiguousarray(recs, np.int32)
    planes = np.ascontiguousarray(planes, np.float32)
    owner = np.zeros((h, w), np.int32)
    dp = np.zeros((h, w), np.int16)
    lib().orc_plane_map(C.byref(p), _ptr(recs), _ptr(planes), len(recs), w, h, _ptr(owner),
                        _ptr(dp))
    return owner, dp


def grid(p: OrcParams, pts: np.ndarray, w: int, h: int) -> np.ndarray:
    vals = [np.zeros(1, np.int32) for _ in range(3)]
    lib().orc_grid_dims(C.byref(p), w, h, *[_ptr(v) for v in vals])
    gw, gh, words = (int(v[0]) for v in vals)
    out = np.zeros((gh, gw, words), np.uint64)
    pts = np.ascontiguousarray(pts, np.int32).reshape(-1, 3)
    lib().orc_grid(C.byref(p), _ptr(pts), len(pts), w, h, _ptr(out))
    return out


def dense(p: OrcParams, desc_self, desc_other, dplane, grid_, has_list: bool, lut,
          right_frame: bool):
    h, w = desc_self.shape[:2]
    out = np.zeros((h, w), np.int16)
    ev = lib().orc_dense(C.byref(p), _ptr(np.ascontiguousarray(desc_self)),
                         _ptr(np.ascontiguousarray(desc_other)),
                         _ptr(np.ascontiguousarray(dplane, np.int16)),
                         _ptr(np.ascontiguousarray(grid_, np.uint64)), int(has_list),
                         _ptr(np.ascontiguousarray(lut, np.int32)), w, h, int(right_frame),
                         _ptr(out))
    return out, int(ev)


def lrcheck(p: OrcParams, rawL, rawR):
    h, w = rawL.shape
    oL = np.zeros((h, w), np.int16)
    oR = np.zeros((h, w), np.int16)
    lib().orc_lrcheck(C.byref(p), _ptr(np.ascontiguousarray(rawL, np.int16)),
                      _ptr(np.ascontiguousarray(rawR, np.int16)), w, h, _ptr(oL), _ptr(oR))
    return oL, oR


# ---------------------------------------------------------------- Section VI variant
def census_words(win: int) -> int:
    return (win * win + 31) // 32


def census(img: np.ndarray, win: int) -> np.ndarray:
    """[h, w, words] uint32 census descriptors of a win x win window."""
    img = np.ascontiguousarray(img, np.uint8)
    h, w = img.shape
    words = census_words(win)
    out = np.zeros((h, w, words), np.uint32)
    lib().orc_census(_ptr(img), w, h, w, win, _ptr(out), words)
    return out


def hamming(a: np.ndarray, b: np.ndarray) -> int:
    a = np.ascontiguousarray(a, np.uint32)
    b = np.ascontiguousarray(b, np.uint32)
    return int(lib().orc_hamming(_ptr(a), _ptr(b), a.size))


def census_texture(a: np.ndarray) -> int:
    a = np.ascontiguousarray(a, np.uint32)
    return int(lib().orc_census_texture(_ptr(a), a.size))


def shiftsum_threshold(m2: int) -> int:
    return int(lib().orc_shiftsum_threshold(m2))


def shiftsum_accept(m1: int, m2: int) -> bool:
    return bool(lib().orc_shiftsum_accept(m1, m2))


def support_accept(p: OrcParams, m1: int, m2: int) -> bool:
    return bool(lib().orc_support_accept(C.byref(p), m1, m2))


def support_match_census(p: OrcParams, csL: np.ndarray, csR: np.ndarray):
    h, w, words = csL.shape
    lw, lh, _, _ = lattice(p, w, h)
    out = np.zeros((lh, lw), np.int16)
    ev = np.zeros(1, np.int64)
    lib().orc_support_match_census(C.byref(p), _ptr(np.ascontiguousarray(csL, np.uint32)),
                                   _ptr(np.ascontiguousarray(csR, np.uint32)), words, w, h,
                                   _ptr(out), _ptr(ev))
    return out, int(ev[0])


def filter_redun_past(p: OrcParams, dcan: np.ndarray, vertical: bool) -> np.ndarray:
    dcan = np.ascontiguousarray(dcan, np.int16)
    out = np.zeros_like(dcan)
    lib().orc_filter_redun_past(C.byref(p), _ptr(dcan), dcan.shape[1], dcan.shape[0],
                                int(vertical), _ptr(out))
    return out


def subsample(pts: np.ndarray, k: int) -> np.ndarray:
    pts = np.array(pts, np.int32).reshape(-1, 3)
    n = lib().orc_subsample(_ptr(pts), len(pts), k)
    return pts[:n].copy()


def dense_census(p: OrcParams, c_self, c_other, dplane, grid_, has_list: bool, lut,
                 right_frame: bool):
    h, w, words = c_self.shape
    out = np.zeros((h, w), np.int16)
    ev = lib().orc_dense_census(C.byref(p), _ptr(np.ascontiguousarray(c_self, np.uint32)),
                                _ptr(np.ascontiguousarray(c_other, np.uint32)), words,
                                _ptr(np.ascontiguousarray(dplane, np.int16)),
                                _ptr(np.ascontiguousarray(grid_, np.uint64)), int(has_list),
                                _ptr(np.ascontiguousarray(lut, np.int32)), w, h,
                                int(right_frame), _ptr(out))
    return out, int(ev)


def median(win: int, disp: np.ndarray) -> np.ndarray:
    disp = np.ascontiguousarray(disp, np.int16)
    out = np.zeros_like(disp)
    lib().orc_median(win, _ptr(disp), disp.shape[1], disp.shape[0], _ptr(out))
    return out


# ---------------------------------------------------------------- pipeline
@dataclass
class Trace:
    w: int
    h: int
    descL: np.ndarray
    descR: np.ndarray
    dcan_raw: np.ndarray
    dcan_incon: np.ndarray
    dcan_vert: np.ndarray
    dcan_final: np.ndarray
    ptsL: np.ndarray
    ptsR: np.ndarray
    cornersL: np.ndarray
    cornersR: np.ndarray
    recL: np.ndarray
    recR: np.ndarray
    planeL: np.ndarray
    planeR: np.ndarray
    ownerL: np.ndarray
    ownerR: np.ndarray
    dplaneL: np.ndarray
    dplaneR: np.ndarray
    gridL: np.ndarray
    gridR: np.ndarray
    lut: np.ndarray
    rawL: np.ndarray
    rawR: np.ndarray
    outL: np.ndarray
    outR: np.ndarray
    support_evals: int
    dense_evals: int
    stage_ms: tuple
    csupL: np.ndarray
    csupR: np.ndarray
    cdenL: np.ndarray
    cdenR: np.ndarray
    chkL: np.ndarray
    chkR: np.ndarray
    nL_all: int


def _arr(ptr, shape, dtype):
    n = int(np.prod(shape))
    if n == 0 or not ptr:
        return np.zeros(shape, dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).view(dtype).reshape(shape).copy()


def process(p: OrcParams, left: np.ndarray, right: np.ndarray) -> Trace:
    left = np.ascontiguousarray(left, np.uint8)
    right = np.ascontiguousarray(right, np.uint8)
    h, w = left.shape
    t = OrcTrace()
    rc = lib().orc_process(C.byref(p), _ptr(left), _ptr(right), w, h, w, C.byref(t))
    if rc != 0:
        lib().orc_trace_free(C.byref(t))
        raise ValueError(f"orc_process failed with {rc}")
    try:
        lw, lh = t.lw, t.lh
        g = (t.gh, t.gw, t.words)
        out = Trace(
            w=w, h=h,
            descL=_arr(t.descL, (h, w, 16), np.uint8), descR=_arr(t.descR, (h, w, 16), np.uint8),
            dcan_raw=_arr(t.dcan_raw, (lh, lw), np.int16),
            dcan_incon=_arr(t.dcan_incon, (lh, lw), np.int16),
            dcan_vert=_arr(t.dcan_vert, (lh, lw), np.int16),
            dcan_final=_arr(t.dcan_final, (lh, lw), np.int16),
            ptsL=_arr(t.ptsL, (t.nL, 3), np.int32), ptsR=_arr(t.ptsR, (t.nR, 3), np.int32),
            cornersL=np.array(t.cornersL[:], np.int32),
            cornersR=np.array(t.cornersR[:], np.int32),
            recL=_arr(t.recL, (t.ntriL, 9), np.int32), recR=_arr(t.recR, (t.ntriR, 9), np.int32),
            planeL=_arr(t.planeL, (t.ntriL, 3), np.float32),
            planeR=_arr(t.planeR, (t.ntriR, 3), np.float32),
            ownerL=_arr(t.ownerL, (h, w), np.int32), ownerR=_arr(t.ownerR, (h, w), np.int32),
            dplaneL=_arr(t.dplaneL, (h, w), np.int16), dplaneR=_arr(t.dplaneR, (h, w), np.int16),
            gridL=_arr(t.gridL, g, np.uint64), gridR=_arr(t.gridR, g, np.uint64),
            lut=_arr(t.lut, (t.D,), np.int32),
            rawL=_arr(t.rawL, (h, w), np.int16), rawR=_arr(t.rawR, (h, w), np.int16),
            outL=_arr(t.outL, (h, w), np.int16), outR=_arr(t.outR, (h, w), np.int16),
            support_evals=int(t.support_evals), dense_evals=int(t.dense_evals),
            stage_ms=tuple(t.stage_ms[:]),
            csupL=_arr(t.csupL, (h, w, t.swords), np.uint32),
            csupR=_arr(t.csupR, (h, w, t.swords), np.uint32),
            cdenL=_arr(t.cdenL, (h, w, t.dwords), np.uint32),
            cdenR=_arr(t.cdenR, (h, w, t.dwords), np.uint32),
            chkL=_arr(t.chkL, (h, w), np.int16), chkR=_arr(t.chkR, (h, w), np.int16),
            nL_all=int(t.nL_all),
        )
    finally:
        lib().orc_trace_free(C.byref(t))
    return out
