"""Pins of the oracle's gradient and descriptor stage against closed forms,
hand-derived impulse responses and the mirror symmetry of the definition."""
import numpy as np
import pytest

import synth
from oracle import ref


def test_sobel_linear_ramp_closed_form():
    # I = 3u + 2v + 10: the 3x3 Sobel pair responds with 8 x the slope.
    h, w = 20, 30
    v, u = np.mgrid[0:h, 0:w]
    img = (3 * u + 2 * v + 10).astype(np.uint8)
    du, dv = ref.sobel(img)
    assert np.all(du[1:-1, 1:-1] == 24)
    assert np.all(dv[1:-1, 1:-1] == 16)
    border = np.ones((h, w), bool)
    border[1:-1, 1:-1] = False
    assert np.all(du[border] == 0) and np.all(dv[border] == 0)


def test_sobel_impulse_response_signs():
    # A single bright pixel: columns to its left see it on their right side.
    img = np.zeros((9, 9), np.uint8)
    img[4, 4] = 100
    du, dv = ref.sobel(img)
    assert du[4, 3] == 200 and du[4, 5] == -200
    assert du[3, 3] == 100 and du[5, 3] == 100 and du[3, 5] == -100
    assert du[4, 4] == 0 and du[3, 4] == 0
    assert dv[3, 4] == 200 and dv[5, 4] == -200
    assert dv[3, 3] == 100 and dv[5, 5] == -100
    assert dv[4, 4] == 0 and dv[4, 3] == 0


def test_quantisation_truncates_toward_zero_and_clamps():
    # impulse of 7: the pixel diagonally below-right has du = dv = -7, which
    # quantises to -1 (truncation), byte 127; floor division would give 126.
    img = np.zeros((12, 12), np.uint8)
    img[4, 4] = 7
    d = ref.descriptors(img)
    du, dv = ref.sobel(img)
    assert du[5, 5] == -7 and dv[5, 5] == -7
    # descriptor at (u, v) = (6, 5): byte 1 is du at (u-1, v) = (5, 5)
    assert d[5, 6, 1] == 127
    # step edge 0 | 255: du = 4*255 = 1020 -> 255 -> clamp 127 -> byte 255
    step = np.zeros((12, 12), np.uint8)
    step[:, 6:] = 255
    d = ref.descriptors(step)
    # descriptor at u = 4: byte 3 samples du at u+2 = 6 where the edge is (5|6)
    du, _ = ref.sobel(step)
    assert du[5, 5] == 1020 and du[5, 6] == 1020
    assert d[5, 4, 3] == 255
    inv = (255 - step).astype(np.uint8)
    d2 = ref.descriptors(inv)
    assert d2[5, 4, 3] == 1


def test_descriptor_layout_from_impulse():
    # impulse 100 at (x0, y0) = (8, 8); hand-derived gradient bytes:
    # du(7, 8) = 200 -> q 50 -> 178 ; du(9, 8) = -200 -> 78 ; du(7, 7) = 100 -> 153
    img = np.zeros((17, 17), np.uint8)
    img[8, 8] = 100
    d = ref.descriptors(img)
    # pixel (u, v) = (9, 8): byte 0 = du(u-2, v) = du(7, 8)
    assert d[8, 9, 0] == 178
    # pixel (u, v) = (5, 8): byte 3 = du(u+2, v) = du(7, 8)
    assert d[8, 5, 3] == 178
    # pixel (u, v) = (8, 9): byte 4 = du(u-1, v-2) = du(7, 7) = 100 -> 153
    assert d[9, 8, 4] == 153
    # dv(8, 7) = 200 -> 178: pixel (8, 9) byte 8 = dv(u, v-2) = dv(8, 7)
    assert d[9, 8, 8] == 178
    # pixel (10, 8): byte 12 = dv(u-2, v-1) = dv(8, 7) = 200 -> 178
    assert d[8, 10, 12] == 178


def test_descriptor_undefined_border_is_zero():
    img = synth.shifted_pair(24, 20, 3, seed=1)[0]
    d = ref.descriptors(img)
    inner = np.zeros((20, 24), bool)
    inner[2:-2, 2:-2] = True
    assert np.all(d[~inner] == 0)
    assert np.all(d[inner] >= 1)


HFLIP = [3, 2, 1, 0, 5, 4, 7, 6, 8, 9, 10, 11, 13, 12, 15, 14]
VFLIP = [0, 1, 2, 3, 6, 7, 4, 5, 11, 10, 9, 8, 14, 15, 12, 13]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_descriptor_horizontal_mirror(seed):
    # flipping u negates du and mirrors the sample pattern: the descriptor at
    # the mirrored pixel is the permuted complement on the du half.
    img = synth.make_pair(synth.QVGA.with_seed(seed)).left[:60, :90]
    d = ref.descriptors(img)
    dm = ref.descriptors(np.ascontiguousarray(img[:, ::-1]))
    dm = dm[:, ::-1][..., HFLIP].astype(np.int32)
    exp = d.astype(np.int32)
    defined = exp[..., 0] > 0
    exp_du = 256 - exp[..., :8]
    assert np.array_equal(dm[..., :8][defined], exp_du[defined])
    assert np.array_equal(dm[..., 8:][defined], exp[..., 8:][defined])


@pytest.mark.parametrize("seed", [0, 3])
def test_descriptor_vertical_mirror(seed):
    img = synth.make_pair(synth.QVGA.with_seed(seed)).left[:70, :50]
    d = ref.descriptors(img).astype(np.int32)
    dm = ref.descriptors(np.ascontiguousarray(img[::-1, :]))
    dm = dm[::-1, :][..., VFLIP].astype(np.int32)
    defined = d[..., 0] > 0
    assert np.array_equal(dm[..., :8][defined], d[..., :8][defined])
    assert np.array_equal(dm[..., 8:][defined], (256 - d[..., 8:])[defined])
