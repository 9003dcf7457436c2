"""Seeded synthetic piecewise-planar stereo pairs.

This module only produces inputs. It holds none of the stereo method's
arithmetic; both the CPU oracle's tests and the GPU path's tests and benchmark
draw their images from it.

Scene model (stand-in for the KITTI 1242x375 and New Tsukuba 640x480 shapes
used in the paper's evaluation section; no dataset content is used):

* random numbers: SplitMix64 seeded with ``seed``; draw ``n`` (n = 0, 1, ...)
  is the published SplitMix64 output function applied to
  ``seed + (n + 1) * 0x9E3779B97F4A7C15``, consumed in the fixed order below.
  Uniform doubles are ``(x >> 11) * 2**-53``, bytes are ``x >> 56`` and
  Gaussians come from Box-Muller using both outputs of each pair.
* K Voronoi cells with seeds uniform in [0, W) x [0, H); each pixel takes the
  nearest seed (double precision, ties to the lower index).
* each cell is a slanted plane ``d = c + a (u - u_s) + b (v - v_s)`` relative
  to its seed, ``a, b ~ U[-A, A]``, ``c ~ U[c_lo, c_hi]``; ground truth is
  ``clamp(floor(d + 1/2), 0, D - 1)``. With ``ground`` the rows
  ``v >= floor(2H/3)`` are one plane ``d = c_g + b_g (v - floor(2H/3))``.
* left image: uniform byte noise, box-blurred 3x3 as ``(sum + 4) // 9`` with
  replicated edges, then 48x48 constant patches at uniform positions with a
  uniform byte value until at least ``flat_frac`` of the area is covered.
* right image: z-buffer warp ``R(u - GT, v) = L(u, v)`` where the larger
  disparity wins, holes filled with fresh noise, then
  ``clamp(floor(R + sigma * n + 1/2), 0, 255)`` with Gaussian ``n``.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


class SplitMix64:
    """Counter form of SplitMix64: draw n is mix(seed + (n+1)*gamma)."""

    def __init__(self, seed: int):
        self.seed = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        self.n = 0

    def u64(self, count: int) -> np.ndarray:
        idx = np.arange(self.n + 1, self.n + 1 + count, dtype=np.uint64)
        self.n += count
        with np.errstate(over="ignore"):
            z = self.seed + idx * _GAMMA
            z = (z ^ (z >> np.uint64(30))) * _M1
            z = (z ^ (z >> np.uint64(27))) * _M2
            z = z ^ (z >> np.uint64(31))
        return z

    def uniform(self, count: int) -> np.ndarray:
        return (self.u64(count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def bytes_(self, count: int) -> np.ndarray:
        return (self.u64(count) >> np.uint64(56)).astype(np.uint8)

    def normal(self, count: int) -> np.ndarray:
        pairs = (count + 1) // 2
        u = self.uniform(2 * pairs).reshape(pairs, 2)
        r = np.sqrt(-2.0 * np.log1p(-u[:, 0]))  # 1 - u1 lies in (0, 1]
        t = 2.0 * np.pi * u[:, 1]
        z = np.stack([r * np.cos(t), r * np.sin(t)], axis=1).reshape(-1)
        return z[:count]


@dataclass(frozen=True)
class SceneConfig:
    width: int
    height: int
    disp_range: int          # D; disparities 0..D-1
    planes: int              # K Voronoi cells
    slope: float             # A: |a|, |b| <= A
    c_lo: float
    c_hi: float
    noise_sigma: float       # Gaussian noise on the right image
    flat_frac: float         # textureless patch coverage target
    ground: bool = False     # bottom third replaced by one ground plane
    patch: int = 48
    seed: int = 0

    def with_seed(self, seed: int) -> "SceneConfig":
        return replace(self, seed=seed)


# The four workload shapes (320x240, 640x480, 1242x375 automotive, 1280x720).
QVGA = SceneConfig(320, 240, 64, 8, 0.05, 4.0, 59.0, 2.0, 0.10)
VGA = SceneConfig(640, 480, 128, 24, 0.05, 4.0, 123.0, 2.0, 0.10)
WIDE = SceneConfig(1242, 375, 256, 32, 0.08, 4.0, 251.0, 3.0, 0.15, ground=True)
HD = SceneConfig(1280, 720, 192, 32, 0.05, 4.0, 187.0, 2.0, 0.10)
SHAPES = {"320x240": QVGA, "640x480": VGA, "1242x375": WIDE, "1280x720": HD}


@dataclass
class StereoPair:
    left: np.ndarray         # uint8 [H, W]
    right: np.ndarray        # uint8 [H, W]
    gt_left: np.ndarray      # int32 [H, W] ground-truth disparity of the left view
    occluded: np.ndarray     # bool [H, W] left pixels not visible in the right view
    labels: np.ndarray       # int32 [H, W] plane index (K = ground plane)
    config: SceneConfig


def _box_blur3(img: np.ndarray) -> np.ndarray:
    p = np.pad(img.astype(np.int32), 1, mode="edge")
    h, w = img.shape
    s = np.zeros((h, w), np.int32)
    for dy in range(3):
        for dx in range(3):
            s += p[dy:dy + h, dx:dx + w]
    return ((s + 4) // 9).astype(np.uint8)


def make_pair(cfg: SceneConfig) -> StereoPair:
    W, H, D, K = cfg.width, cfg.height, cfg.disp_range, cfg.planes
    rng = SplitMix64(cfg.seed)

    # 1. Voronoi seeds and labels
    sd = rng.uniform(2 * K).reshape(K, 2)
    su = sd[:, 0] * W
    sv = sd[:, 1] * H
    uu = np.arange(W, dtype=np.float64)[None, :]
    vv = np.arange(H, dtype=np.float64)[:, None]
    labels = np.zeros((H, W), np.int32)
    best = np.full((H, W), np.inf)
    for k in range(K):
        dist = (uu - su[k]) ** 2 + (vv - sv[k]) ** 2
        closer = dist < best             # strict: ties keep the lower index
        best = np.where(closer, dist, best)
        labels = np.where(closer, k, labels)

    # 2. planes, seed-relative
    pl = rng.uniform(3 * K).reshape(K, 3)
    a = -cfg.slope + 2.0 * cfg.slope * pl[:, 0]
    b = -cfg.slope + 2.0 * cfg.slope * pl[:, 1]
    c = cfg.c_lo + (cfg.c_hi - cfg.c_lo) * pl[:, 2]
    disp = c[labels] + a[labels] * (uu - su[labels]) + b[labels] * (vv - sv[labels])
    if cfg.ground:
        g = rng.uniform(2)
        b_g = 0.04 + 0.04 * g[0]
        c_g = 4.0 + 119.0 * g[1]
        v0 = (2 * H) // 3
        rows = np.arange(H)[:, None] >= v0
        dg = c_g + b_g * (vv - v0) + 0.0 * uu
        disp = np.where(rows, dg, disp)
        labels = np.where(rows, K, labels)
    gt = np.clip(np.floor(disp + 0.5), 0, D - 1).astype(np.int32)

    # 3. left texture and flat patches
    left = _box_blur3(rng.bytes_(W * H).reshape(H, W))
    ps = min(cfg.patch, W, H)
    covered = np.zeros((H, W), bool)
    target = cfg.flat_frac * W * H
    guard = 0
    while covered.sum() < target and guard < 100000:
        r = rng.uniform(2)
        x0 = int(np.floor(r[0] * (W - ps + 1)))
        y0 = int(np.floor(r[1] * (H - ps + 1)))
        val = rng.bytes_(1)[0]
        left[y0:y0 + ps, x0:x0 + ps] = val
        covered[y0:y0 + ps, x0:x0 + ps] = True
        guard += 1

    # 4. z-buffer warp into the right view: larger disparity wins
    vgrid = np.broadcast_to(np.arange(H)[:, None], (H, W))
    ugrid = np.broadcast_to(np.arange(W)[None, :], (H, W))
    ut = ugrid - gt
    ok = ut >= 0
    key = (vgrid * W + ut)[ok]
    packed = (gt[ok].astype(np.int64) << 20) | ugrid[ok].astype(np.int64)
    zbuf = np.full(H * W, -1, np.int64)
    np.maximum.at(zbuf, key, packed)
    fresh = rng.bytes_(W * H)
    right = fresh.reshape(H, W).copy()
    hit = zbuf >= 0
    src_u = (zbuf[hit] & ((1 << 20) - 1)).astype(np.int64)
    src_v = np.nonzero(hit)[0] // W
    right.reshape(-1)[hit] = left[src_v, src_u]
    winner = np.zeros(H * W, bool)
    winner_idx = src_v * W + src_u
    winner[winner_idx] = True
    occluded = ~winner.reshape(H, W)

    # 5. sensor noise on the right view only
    noise = rng.normal(W * H).reshape(H, W)
    if cfg.noise_sigma > 0:
        right = np.clip(np.floor(right.astype(np.float64) + cfg.noise_sigma * noise + 0.5),
                        0, 255).astype(np.uint8)
    return StereoPair(left=left, right=right, gt_left=gt, occluded=occluded,
                      labels=labels, config=cfg)


def shifted_pair(width: int, height: int, d0: int, seed: int = 0):
    """Textured noise L and R(u, v) = L(u + d0, v) where defined (constant disparity).

    Columns of R with u + d0 >= W hold texture that does not occur in L.
    """
    rng = SplitMix64(seed)
    big = _box_blur3(rng.bytes_((width + d0) * height).reshape(height, width + d0))
    left = np.ascontiguousarray(big[:, :width])
    right = np.ascontiguousarray(big[:, d0:d0 + width])
    return left, right


def batch_shapes(n: int, seed: int = 0):
    """Resolution index of each of n pairs, uniform over the four shapes."""
    rng = SplitMix64(seed)
    r = rng.uniform(n)
    names = list(SHAPES)
    return [names[int(np.floor(x * len(names)))] for x in r]


def sparse_layout_pair(width: int, height: int, kind: str, d0: int, seed: int = 0):
    """Flat pair (R(u, v) = L(u + d0, v)) with noise texture only where a
    support lattice of step 10 should find points: 'vline' one point per row,
    all on one column; 'two' two such columns; 'diag' one point per row on a
    staircase; 'spot' a single point; 'hline' every point in one row."""
    rng = SplitMix64(seed)
    left = np.full((height, width), 90, np.uint8)

    def tex(v0, v1, u0, u1):
        left[v0:v1, u0:u1] = rng.bytes_((v1 - v0) * (u1 - u0)).reshape(v1 - v0, u1 - u0)

    if kind == "vline":
        tex(8, height - 8, 48, 53)
    elif kind == "two":
        tex(8, height - 8, 38, 43)
        tex(18, height - 18, 78, 83)
    elif kind == "diag":
        for i, v in enumerate(range(10, height - 10, 10)):
            tex(v - 2, v + 3, 28 + 10 * (i % 6), 33 + 10 * (i % 6))
    elif kind == "spot":
        tex(38, 43, 58, 63)
    elif kind == "hline":
        tex(38, 43, d0 + 10, width - 10)
    else:
        raise ValueError(kind)
    right = np.full_like(left, 90)
    right[:, :width - d0] = left[:, d0:]
    return left, right
