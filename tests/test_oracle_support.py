"""Pins of the oracle's support matching: the FP32 ratio test, lattice
geometry, closed-form constant-disparity pairs, periodic (ambiguous) texture
and the exact mirror symmetry of the search."""
import numpy as np
import pytest

import synth
from oracle import ref


def test_ratio_test_is_strict_fp32():
    thr = 0.85
    assert not ref.ratio_accept(thr, 0, 0)          # flat texture: ambiguous
    assert ref.ratio_accept(thr, 0, 1)
    # 0.85f * 100 rounds to exactly 85.0f, so m1 = 85 is not strictly below it
    assert not ref.ratio_accept(thr, 85, 100)
    assert ref.ratio_accept(thr, 84, 100)
    assert not ref.ratio_accept(thr, 100, 100)
    # 0.85f = 0.850000023841858; 0.85f * 20000 = 17000.000476837 -> 17000.0f
    assert not ref.ratio_accept(thr, 17000, 20000)
    assert ref.ratio_accept(thr, 16999, 20000)


@pytest.mark.parametrize("w,h,s,expect", [
    (640, 480, 5, (127, 95, 5, 5)),
    (320, 240, 5, (63, 47, 5, 5)),
    (1242, 375, 5, (247, 74, 5, 5)),
    (1280, 720, 5, (255, 143, 5, 5)),
    (30, 20, 1, (22, 12, 4, 4)),
    (9, 9, 1, (1, 1, 4, 4)),
    (9, 9, 5, (0, 0, 5, 5)),
    (14, 14, 3, (2, 2, 6, 6)),
])
def test_lattice_geometry(w, h, s, expect):
    assert ref.lattice(ref.params(candidate_stepsize=s), w, h) == expect


def _support(p, L, R):
    dl, dr = ref.descriptors(L), ref.descriptors(R)
    return ref.support_match(p, dl, dr)


@pytest.mark.parametrize("d0,seed", [(7, 0), (13, 1), (21, 2)])
def test_constant_disparity_support_points(d0, seed):
    # R(u, v) = L(u + d0, v): the true disparity costs 0 wherever it is
    # admissible (u - 4 >= d0) and its right window is clear of the border
    # gradients (u - d0 - 4 >= 1); there every accepted point must be d0.
    # Further left d0 is not admissible and a smaller d may win.
    L, R = synth.shifted_pair(160, 80, d0, seed=seed)
    p = ref.params(disp_max=31)
    dcan, ev = _support(p, L, R)
    lw, lh, u0, v0 = ref.lattice(p, 160, 80)
    us = u0 + 5 * np.arange(lw)
    inner = np.broadcast_to(us >= d0 + 5, dcan.shape)
    valid = (dcan >= 0) & inner
    assert valid.sum() > 0.8 * inner.sum()
    assert np.all(dcan[valid] == d0)
    not_adm = np.broadcast_to(us < d0 + 4, dcan.shape)
    assert np.all(dcan[(dcan >= 0) & not_adm] < d0)
    assert ev > 0


def test_periodic_texture_is_ambiguous():
    # period 8 along u: cost(d0) = cost(d0 + 8) = 0 -> m1 = m2 -> rejected
    rng = synth.SplitMix64(5)
    tile = rng.bytes_(8 * 60).reshape(60, 8)
    big = np.tile(tile, (1, 30))
    big = synth._box_blur3(big)
    d0 = 10
    L = np.ascontiguousarray(big[:, 8:8 + 200])
    R = np.ascontiguousarray(big[:, 8 + d0:8 + d0 + 200 - 0])
    R = np.ascontiguousarray(np.pad(R, ((0, 0), (0, 200 - R.shape[1])), mode="wrap")[:, :200])
    p = ref.params(disp_max=31)
    dcan, _ = _support(p, L, R)
    lw, lh, u0, v0 = ref.lattice(p, 200, 60)
    us = u0 + 5 * np.arange(lw)
    far = us >= 40   # both d = 2 and d = 10 admissible and away from borders
    assert np.all(dcan[:, far] == -1)
    # the same texture without the repetition is matched
    L2, R2 = synth.shifted_pair(200, 60, d0, seed=5)
    dcan2, _ = _support(p, L2, R2)
    assert (dcan2[:, far] == d0).sum() > 0.5 * dcan2[:, far].size


def test_flat_image_has_no_support():
    L = np.full((40, 60), 77, np.uint8)
    dcan, ev = _support(ref.params(disp_max=15), L, L)
    assert np.all(dcan == -1)
    assert ev == 0          # the texture test stops every search


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_support_search_mirror_symmetry(seed):
    # With a unit lattice and an exact left/right tolerance, swapping the views
    # and flipping them maps every accepted (u, v, d) to (w-1-(u-d), v, d).
    cfg = synth.SceneConfig(72, 40, 32, 3, 0.05, 4.0, 27.0, 2.0, 0.0, seed=seed)
    pair = synth.make_pair(cfg)
    p = ref.params(candidate_stepsize=1, lr_threshold=0, disp_max=31)
    w = cfg.width
    d1, _ = _support(p, pair.left, pair.right)
    d2, _ = _support(p, np.ascontiguousarray(pair.right[:, ::-1]),
                     np.ascontiguousarray(pair.left[:, ::-1]))
    lw, lh, u0, v0 = ref.lattice(p, w, cfg.height)
    a = {(w - 1 - (u0 + k - d), v0 + l, int(d)) for (l, k), d in np.ndenumerate(d1) if d >= 0}
    b = {(u0 + k, v0 + l, int(d)) for (l, k), d in np.ndenumerate(d2) if d >= 0}
    assert len(a) > 50
    assert a == b


def test_lr_check_rejects_occluded_points():
    # The left view contains a strip that the right view does not (it was
    # overwritten with fresh texture). Points on it find no consistent
    # reverse match; points elsewhere are unaffected.
    L, R = synth.shifted_pair(160, 60, 9, seed=4)
    R = R.copy()
    rng = synth.SplitMix64(77)
    R[:, 60:90] = synth._box_blur3(rng.bytes_(60 * 30).reshape(60, 30))
    p = ref.params(disp_max=31)
    dcan, _ = _support(p, L, R)
    lw, lh, u0, v0 = ref.lattice(p, 160, 60)
    us = u0 + 5 * np.arange(lw)
    # left columns whose 9x9 window maps entirely into the overwritten strip
    hidden = (us - 9 - 4 >= 60) & (us - 9 + 4 < 90)
    assert np.all(dcan[:, hidden] != 9)
    clean = (us - 9 - 4 >= 100)
    assert (dcan[:, clean] == 9).mean() > 0.8
