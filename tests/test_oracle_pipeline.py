"""Whole-pipeline pins of the oracle.

* constant disparity: the closed-form result on the interior;
* noise-free planar scenes: ground-truth recovery within +-1;
* mirror symmetry: exact for the dense stage given mirrored priors,
  approximate for the whole pipeline (lexicographic tie rules and the support
  filters' lattice neighbourhoods are not mirror-symmetric);
* invariants: value range, left/right partner consistency, determinism.
"""
import numpy as np
import pytest
from scipy import ndimage

import synth
from oracle import ref


@pytest.mark.parametrize("d0,W,H", [(9, 160, 64), (18, 200, 50), (30, 256, 40)])
def test_constant_disparity_closed_form(d0, W, H):
    L, R = synth.shifted_pair(W, H, d0, seed=d0)
    p = ref.params(disp_max=63)
    t = ref.process(p, L, R)
    # precondition: the support stage found only the true disparity (a lattice
    # column with u - 4 < d0 cannot reach d0 and may pick a smaller d; the
    # cases here are chosen so that no such point survives the filters)
    assert len(t.ptsL) > 0
    assert np.all(t.ptsL[:, 2] == d0) and np.all(t.ptsR[:, 2] == d0)
    assert np.all(t.cornersL == d0) and np.all(t.cornersR == d0)
    # every plane is a = b = 0, c = d0, so the prior matrix is d0 everywhere
    assert np.all(t.planeL == np.float32([0, 0, d0])) and np.all(t.planeR == np.float32([0, 0, d0]))
    assert np.all(t.dplaneL == d0) and np.all(t.dplaneR == d0)
    # E(d0) = SAD 0 + P[0] = -14 beats every other candidate (>= 0 + P[1] = -9)
    tex = np.abs(t.descL.astype(np.int32) - 128).sum(-1)
    u = np.arange(W)[None, :].repeat(H, 0)
    v = np.arange(H)[:, None].repeat(W, 1)
    region = (u >= d0 + 3) & (u <= W - 4) & (v >= 2) & (v <= H - 3) & (tex >= 1)
    assert np.all(t.outL[region] == d0)
    assert np.all(t.rawL[region] == d0)


def _far_from_edges(labels, r):
    lab = labels
    edge = np.zeros_like(lab, bool)
    dh = lab[:, 1:] != lab[:, :-1]
    dvv = lab[1:] != lab[:-1]
    edge[:, 1:] |= dh
    edge[:, :-1] |= dh
    edge[1:] |= dvv
    edge[:-1] |= dvv
    return ndimage.distance_transform_cdt(~edge, metric="chessboard") >= r


# Thresholds calibrated once on the oracle over these six seeds (worst case
# 87.5 % valid, 97.1 % within +-1; mean 99.0 % within +-1), then frozen.
@pytest.mark.parametrize("seed", range(6))
def test_noise_free_planar_scene_recovers_ground_truth(seed):
    cfg = synth.SceneConfig(320, 240, 64, 8, 0.05, 4.0, 59.0, 0.0, 0.0, seed=seed)
    pr = synth.make_pair(cfg)
    t = ref.process(ref.params(disp_max=63), pr.left, pr.right)
    H, W = pr.labels.shape
    u = np.arange(W)[None, :].repeat(H, 0)
    v = np.arange(H)[:, None].repeat(W, 1)
    region = (_far_from_edges(pr.labels, 8) & ~pr.occluded & (u >= 63 + 8) & (u <= W - 9)
              & (v >= 8) & (v <= H - 9))
    valid = t.outL >= 0
    sel = region & valid
    acc = (np.abs(t.outL[sel].astype(int) - pr.gt_left[sel]) <= 1).mean()
    assert valid[region].mean() >= 0.85
    assert acc >= 0.97


def test_dense_stage_is_exactly_mirror_symmetric():
    # given the right view's prior matrix and grid, mirrored, the left-view
    # dense stage on the swapped and flipped pair reproduces the right-view
    # result flipped (grid cells mirror exactly because w is a multiple of g)
    pr = synth.make_pair(synth.QVGA.with_seed(4))
    p = ref.params(disp_max=63)
    t = ref.process(p, pr.left, pr.right)
    dl = ref.descriptors(np.ascontiguousarray(pr.right[:, ::-1]))
    dr = ref.descriptors(np.ascontiguousarray(pr.left[:, ::-1]))
    dp = np.ascontiguousarray(t.dplaneR[:, ::-1])
    grid = np.ascontiguousarray(t.gridR[:, ::-1])
    got, ev = ref.dense(p, dl, dr, dp, grid, True, t.lut, False)
    assert np.array_equal(got, t.rawR[:, ::-1])
    _, evR = ref.dense(p, t.descR, t.descL, t.dplaneR, t.gridR, True, t.lut, True)
    assert ev == evR


@pytest.mark.parametrize("seed", [0, 1])
def test_pipeline_mirror_agreement(seed):
    # unit lattice, w = 320 a multiple of g = 20 (values observed: 99.6-99.7 %
    # on pixels valid in both maps, 98.4-98.9 % on pixels valid in either)
    pr = synth.make_pair(synth.QVGA.with_seed(seed))
    p = ref.params(disp_max=63, candidate_stepsize=1)
    a = ref.process(p, pr.left, pr.right)
    b = ref.process(p, np.ascontiguousarray(pr.right[:, ::-1]),
                    np.ascontiguousarray(pr.left[:, ::-1]))
    A, B = b.outL, a.outR[:, ::-1]
    both = (A >= 0) & (B >= 0)
    either = (A >= 0) | (B >= 0)
    assert (A[both] == B[both]).mean() >= 0.99
    assert (A[either] == B[either]).mean() >= 0.98


@pytest.mark.parametrize("shape", ["320x240", "640x480"])
def test_invariants_and_determinism(shape):
    cfg = synth.SHAPES[shape]
    pr = synth.make_pair(cfg.with_seed(3))
    p = ref.params(disp_max=cfg.disp_range - 1)
    t = ref.process(p, pr.left, pr.right)
    for m in (t.outL, t.outR, t.rawL, t.rawR):
        vals = m[m >= 0]
        assert np.all(m >= -1) and vals.max() <= cfg.disp_range - 1
    H, W = t.outL.shape
    for v, u in zip(*np.nonzero(t.outL >= 0)):
        d = t.outL[v, u]
        e = t.rawR[v, u - d]
        assert e >= 0 and abs(int(e) - int(d)) <= p.lr_threshold
    # the final maps are the raw maps with some pixels removed
    keep = t.outL >= 0
    assert np.array_equal(t.outL[keep], t.rawL[keep])
    t2 = ref.process(p, pr.left, pr.right)
    assert np.array_equal(t.outL, t2.outL) and np.array_equal(t.outR, t2.outR)
    assert t.dense_evals == t2.dense_evals and t.support_evals == t2.support_evals


def test_flat_pair_has_no_support_and_no_output():
    L = np.full((40, 64), 90, np.uint8)
    t = ref.process(ref.params(disp_max=15), L, L)
    assert len(t.ptsL) == 0 and len(t.recL) == 0
    assert np.all(t.dplaneL == -1) and np.all(t.outL == -1) and np.all(t.outR == -1)
    assert t.dense_evals == 0


def test_empty_support_with_full_search_still_matches():
    # texture too weak for support points (threshold raised), full search on
    L, R = synth.shifted_pair(64, 32, 5, seed=2)
    t = ref.process(ref.params(disp_max=15, support_texture=10 ** 6, full_search=1), L, R)
    assert len(t.ptsL) == 0
    inner = t.rawL[2:-2, 5 + 3:64 - 4]
    assert (inner == 5).mean() > 0.95


def test_rejects_bad_arguments():
    L = np.zeros((8, 20), np.uint8)
    with pytest.raises(ValueError):
        ref.process(ref.params(), L, L)           # height < 9
    L = np.zeros((20, 20), np.uint8)
    with pytest.raises(ValueError):
        ref.process(ref.params(disp_min=0, disp_max=256), L, L)
    with pytest.raises(ValueError):
        ref.process(ref.params(beta=0.0), L, L)
