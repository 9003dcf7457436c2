"""Pins of the oracle's grid vectors, dense matching and final check.

* dense: exhaustive per-pixel energy minimisation written independently with
  numpy, on tiny images, with the candidate set forced to every disparity and
  with random plane maps and grid masks;
* grid: hand-built point sets;
* left/right check: hand-built maps.
"""
import numpy as np
import pytest

import synth
from oracle import ref


def exhaustive(desc_self, desc_other, dplane, lut, cand_mask, dmin, right, match_texture):
    """E(d) for every d, then argmin with the smallest d on ties."""
    h, w = desc_self.shape[:2]
    D = cand_mask.shape[-1]
    out = np.full((h, w), -1, np.int16)
    count = 0
    s = desc_self.astype(np.int32)
    o = desc_other.astype(np.int32)
    tex = np.abs(s - 128).sum(-1)
    for v in range(2, h - 2):
        for u in range(2, w - 2):
            if tex[v, u] < match_texture:
                continue
            best, bestE = -1, None
            for k in range(D):
                d = dmin + k
                uo = u + d if right else u - d
                if uo < 2 or uo > w - 3 or not cand_mask[v, u, k]:
                    continue
                count += 1
                E = int(np.abs(s[v, u] - o[v, uo]).sum())
                if dplane[v, u] >= 0:
                    E += int(lut[abs(d - dplane[v, u])])
                if bestE is None or E < bestE:
                    best, bestE = d, E
            out[v, u] = best
    return out, count


def tiny_pair(seed, w=24, h=16, d=8):
    cfg = synth.SceneConfig(w, h, d, 2, 0.05, 1.0, d - 2.0, 2.0, 0.0, seed=seed)
    pr = synth.make_pair(cfg)
    return ref.descriptors(pr.left), ref.descriptors(pr.right)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("right", [False, True])
def test_full_search_no_prior_is_exhaustive_argmin(seed, right):
    dl, dr = tiny_pair(seed)
    p = ref.params(disp_max=7, full_search=1)
    h, w = dl.shape[:2]
    dplane = np.full((h, w), -1, np.int16)
    grid = np.zeros((1, 2, 1), np.uint64)
    lut = ref.prior_lut(p)
    self_, other = (dr, dl) if right else (dl, dr)
    got, ev = ref.dense(p, self_, other, dplane, grid, False, lut, right)
    exp, cnt = exhaustive(self_, other, dplane, lut, np.ones((h, w, 8), bool), 0, right, 1)
    assert np.array_equal(got, exp)
    assert ev == cnt


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("right", [False, True])
def test_full_search_with_plane_prior(seed, right):
    dl, dr = tiny_pair(seed, w=30, h=18, d=12)
    p = ref.params(disp_min=2, disp_max=13, full_search=1, grid_size=7)
    h, w = dl.shape[:2]
    rng = np.random.default_rng(seed)
    dplane = rng.integers(2, 14, size=(h, w)).astype(np.int16)
    gw, gh = -(-w // 7), -(-h // 7)
    grid = np.zeros((gh, gw, 1), np.uint64)
    lut = ref.prior_lut(p)
    self_, other = (dr, dl) if right else (dl, dr)
    got, ev = ref.dense(p, self_, other, dplane, grid, True, lut, right)
    exp, cnt = exhaustive(self_, other, dplane, lut, np.ones((h, w, 12), bool), 2, right, 1)
    assert np.array_equal(got, exp)
    assert ev == cnt


@pytest.mark.parametrize("seed", range(4))
def test_restricted_candidates_plane_window_union_grid(seed):
    dl, dr = tiny_pair(seed, w=40, h=20, d=16)
    g = 6
    p = ref.params(disp_max=15, grid_size=g, sradius=1, match_texture=30)
    h, w = dl.shape[:2]
    rng = np.random.default_rng(10 + seed)
    dplane = rng.integers(0, 16, size=(h, w)).astype(np.int16)
    dplane[rng.random((h, w)) < 0.2] = -1          # some pixels without a plane
    gw, gh = -(-w // g), -(-h // g)
    bits = rng.random((gh, gw, 16)) < 0.2
    grid = np.zeros((gh, gw, 1), np.uint64)
    for k in range(16):
        grid[..., 0] |= (bits[..., k].astype(np.uint64) << np.uint64(k))
    mask = np.zeros((h, w, 16), bool)
    for v in range(h):
        for u in range(w):
            mask[v, u] = bits[v // g, u // g]
            if dplane[v, u] >= 0:
                lo, hi = max(0, dplane[v, u] - 1), min(15, dplane[v, u] + 1)
                mask[v, u, lo:hi + 1] = True
    lut = ref.prior_lut(p)
    got, ev = ref.dense(p, dl, dr, dplane, grid, True, lut, False)
    exp, cnt = exhaustive(dl, dr, dplane, lut, mask, 0, False, 30)
    assert np.array_equal(got, exp)
    assert ev == cnt


def test_grid_pools_plus_minus_one_per_cell():
    p = ref.params(disp_min=0, disp_max=69, grid_size=20)
    pts = np.array([[5, 5, 0], [19, 19, 10], [20, 5, 69], [45, 30, 33], [46, 31, 35]], np.int32)
    g = ref.grid(p, pts, 60, 40)
    assert g.shape == (2, 3, 2)

    def bits(cell):
        words = cell.tolist()
        return {k for k in range(70) if (words[k // 64] >> (k % 64)) & 1}

    assert bits(g[0, 0]) == {0, 1, 9, 10, 11}          # d-1 = -1 is outside the range
    assert bits(g[0, 1]) == {68, 69}                   # 70 is outside the range
    assert bits(g[1, 2]) == {32, 33, 34, 35, 36}
    assert bits(g[0, 2]) == set() and bits(g[1, 0]) == set()


def test_lrcheck_hand_built():
    p = ref.params(lr_threshold=2)
    L = np.full((1, 12), -1, np.int16)
    R = np.full((1, 12), -1, np.int16)
    L[0, 8] = 5            # partner R[3]
    R[0, 3] = 7            # |7 - 5| = 2: consistent both ways? R[3] -> L[10]
    L[0, 10] = 6           # partner R[4] is invalid -> dropped
    L[0, 11] = 2           # partner R[9] = 5 -> |5-2| > 2 -> dropped
    R[0, 9] = 5
    oL, oR = ref.lrcheck(p, L, R)
    assert oL[0].tolist() == [-1] * 8 + [5, -1, -1, -1]
    # R[3] = 7 looks at L[10] = 6 -> kept; R[9] = 5 looks at L[14]: outside -> dropped
    assert oR[0].tolist() == [-1, -1, -1, 7] + [-1] * 8
