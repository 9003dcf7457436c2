"""Pins of the Section VI variant and the optional steps in the oracle:
census descriptors and Hamming costs (Section VI-A), the shift-sum ambiguity
threshold (Section VI-B, eq. 3), past-only redundancy (Section VI-C, Fig. 7),
support down-sampling (Section VII-B) and the median post-filter
(Section VIII).

Each expected value is a closed form worked out from the definition (ramp
images whose darker neighbours are known in advance, runs of equal values
whose survivors follow from the filter rule, multiples of 32 for eq. 3), a
library routine that computes the same quantity independently (numpy's
popcount, scipy's median filter on fully valid windows), or an invariant the
definition implies (monotone intensity maps, antisymmetry, translation).
"""
import numpy as np
import pytest
from scipy import ndimage

import synth
from oracle import ref

WINDOWS = [3, 5, 7, 9, 11, 13]


def bits_of(words: np.ndarray, nbits: int) -> np.ndarray:
    """Unpacks census words into a bool vector, bit i = word i//32, bit i%32."""
    out = np.zeros(nbits, bool)
    for i in range(nbits):
        out[i] = (int(words[i // 32]) >> (i % 32)) & 1
    return out


def offsets(win):
    r = win // 2
    return [(dx, dy) for dy in range(-r, r + 1) for dx in range(-r, r + 1)]


# ---------------------------------------------------------------- census
@pytest.mark.parametrize("win", WINDOWS)
def test_census_row_ramp_interior_sets_the_leading_bits(win):
    # I(u, v) = v*w + u: the darker neighbours are the rows above and the
    # pixels to the left on the centre row, i.e. exactly the window offsets
    # that precede the centre in row-major order
    h, w = 15, 16
    img = (np.arange(h)[:, None] * w + np.arange(w)[None, :]).astype(np.uint8)
    c = ref.census(img, win)
    assert c.shape == (h, w, ref.census_words(win))
    r = win // 2
    n = win * win
    want = np.arange(n) < (n - 1) // 2
    for v in range(r, h - r):
        for u in range(r, w - r):
            assert np.array_equal(bits_of(c[v, u], n), want), (u, v)
    # padding bits of the last word stay clear
    if n % 32:
        assert np.all((c[..., -1] >> np.uint32(n % 32)) == 0)


@pytest.mark.parametrize("win", [5, 9, 13])
def test_census_column_ramp_fixes_the_bit_order(win):
    # I(u, v) = u*h + v: darker = columns to the left, and above on the centre
    # column; a transposed bit order would fail this and pass the row ramp
    h, w = 15, 16
    img = (np.arange(w)[None, :] * h + np.arange(h)[:, None]).astype(np.uint8)
    c = ref.census(img, win)
    want = np.array([dx < 0 or (dx == 0 and dy < 0) for dx, dy in offsets(win)])
    r = win // 2
    for v in range(r, h - r):
        for u in range(r, w - r):
            assert np.array_equal(bits_of(c[v, u], win * win), want)


@pytest.mark.parametrize("win", [3, 9, 13])
def test_census_outside_neighbours_are_zero_bits(win):
    h, w = 15, 16
    img = (np.arange(h)[:, None] * w + np.arange(w)[None, :]).astype(np.uint8)
    c = ref.census(img, win)
    n = win * win
    # top-left pixel is the darkest: no bit at all
    assert not bits_of(c[0, 0], n).any()
    # bottom-right pixel is the brightest: every in-image neighbour is darker,
    # every outside one is a 0 bit
    want = np.array([dx <= 0 and dy <= 0 and (dx, dy) != (0, 0) for dx, dy in offsets(win)])
    assert np.array_equal(bits_of(c[h - 1, w - 1], n), want)
    # a pixel on the right border: the columns beyond the image are 0 bits
    v = 7
    want = np.array([(dy < 0 or (dy == 0 and dx < 0)) and dx <= 0 and 0 <= v + dy < h
                     for dx, dy in offsets(win)])
    assert np.array_equal(bits_of(c[v, w - 1], n), want)


def test_census_constant_image_is_zero():
    img = np.full((20, 24), 77, np.uint8)
    for win in WINDOWS:
        assert not ref.census(img, win).any()


def test_census_invariant_under_increasing_intensity_maps():
    # census depends only on the order of intensities
    rng = np.random.default_rng(3)
    img = rng.integers(0, 80, (30, 40), dtype=np.uint8)
    x = np.arange(80)
    m = (x + x * x // 40).astype(np.uint8)            # strictly increasing, nonlinear
    assert np.all(np.diff(m.astype(int)) > 0)
    for win in (5, 9, 13):
        assert np.array_equal(ref.census(img, win), ref.census(m[img], win))


def test_census_antisymmetry_of_pairs():
    # for two in-image pixels p, q = p + (dx, dy): bit (dx, dy) of p and bit
    # (-dx, -dy) of q are never both set, and exactly one is set unless the
    # intensities are equal
    rng = np.random.default_rng(5)
    img = (rng.integers(0, 6, (18, 21)) * 40).astype(np.uint8)   # many ties
    win = 7
    c = ref.census(img, win)
    offs = offsets(win)
    idx = {o: i for i, o in enumerate(offs)}
    h, w = img.shape
    for v in range(h):
        for u in range(w):
            bp = bits_of(c[v, u], win * win)
            for (dx, dy), i in idx.items():
                x, y = u + dx, v + dy
                if (dx, dy) == (0, 0) or not (0 <= x < w and 0 <= y < h):
                    continue
                bq = bits_of(c[y, x], win * win)[idx[(-dx, -dy)]]
                assert not (bp[i] and bq)
                assert (bp[i] or bq) == (img[y, x] != img[v, u])


def test_census_translation():
    d0 = 7
    L, R = synth.shifted_pair(60, 30, d0, seed=2)
    for win in (5, 9):
        cL, cR = ref.census(L, win), ref.census(R, win)
        r = win // 2
        # windows fully inside both images: R(u - d0) = L(u)
        for v in range(r, 30 - r):
            for u in range(d0 + r, 60 - r):
                assert np.array_equal(cL[v, u], cR[v, u - d0])


def test_hamming_and_texture_match_numpy_popcount():
    rng = np.random.default_rng(9)
    for words in (1, 2, 3, 4, 6):
        for _ in range(50):
            a = rng.integers(0, 2 ** 32, words, dtype=np.uint64).astype(np.uint32)
            b = rng.integers(0, 2 ** 32, words, dtype=np.uint64).astype(np.uint32)
            assert ref.hamming(a, b) == int(np.bitwise_count(a ^ b).sum())
            assert ref.census_texture(a) == int(np.bitwise_count(a).sum())
            assert ref.hamming(a, a) == 0


# ---------------------------------------------------------------- shift-sum
def test_shiftsum_multiples_of_32_give_29_32():
    for k in range(0, 2000):
        assert ref.shiftsum_threshold(32 * k) == 29 * k


def test_shiftsum_bounds_and_monotone():
    prev = -1
    for m2 in range(0, 5000):
        t = ref.shiftsum_threshold(m2)
        # four truncated terms: within 4 below 29/32 m2, never above it
        assert 32 * t <= 29 * m2 < 32 * t + 4 * 32
        assert t >= prev
        prev = t


def test_shiftsum_accept_hand_values():
    # m2 = 100: 50 + 25 + 12 + 3 = 90
    assert ref.shiftsum_threshold(100) == 90
    assert ref.shiftsum_accept(90, 100) and not ref.shiftsum_accept(91, 100)
    # m2 = 10: 5 + 2 + 1 + 0 = 8
    assert ref.shiftsum_accept(8, 10) and not ref.shiftsum_accept(9, 10)
    # a tie m1 = m2 is rejected except at 0 (0 <= 0, the comparison of eq. 2)
    assert not ref.shiftsum_accept(1, 1) and not ref.shiftsum_accept(7, 7)
    assert ref.shiftsum_accept(0, 0)


def test_support_accept_follows_the_parameter():
    p0 = ref.params(support_threshold=0.85)
    p1 = ref.params(support_threshold=0.85, ambiguity=1)
    # 85 < 0.85 * 100 fails (strict, FP32); 85 <= 90 passes eq. 3
    assert not ref.support_accept(p0, 85, 100)
    assert ref.support_accept(p1, 85, 100)
    assert ref.support_accept(p0, 84, 100) and ref.support_accept(p1, 84, 100)
    assert not ref.support_accept(p0, 0, 0) and ref.support_accept(p1, 0, 0)


# ---------------------------------------------------------------- past-only redundancy
def test_past_only_run_keeps_one_every_r_plus_1():
    # Fig. 7: a run of equal values along a row; looking both ways removes
    # every interior value, looking back only keeps one every r + 1 steps
    p = ref.params(redun_max_dist=5, redun_threshold=1)
    a = np.full((3, 20), -1, np.int16)
    a[1, :] = 33
    past = ref.filter_redun_past(p, a, vertical=False)
    both = ref.filter_redun(p, a, vertical=False)
    assert np.array_equal(np.nonzero(past[1] >= 0)[0], np.arange(0, 20, 6))
    assert np.array_equal(np.nonzero(both[1] >= 0)[0], [0, 19])
    assert np.all(past[[0, 2]] == -1)


def test_past_only_survivors_not_inputs_decide():
    # position 6 sees positions 1..5, all removed by position 0: it survives.
    # A rule that read the unfiltered input would remove it.
    p = ref.params(redun_max_dist=5, redun_threshold=1)
    a = np.full((1, 7), 20, np.int16)
    out = ref.filter_redun_past(p, a, vertical=False)
    assert out[0].tolist() == [20, -1, -1, -1, -1, -1, 20]


def test_past_only_threshold_and_invalid_gaps():
    p = ref.params(redun_max_dist=3, redun_threshold=1)
    a = np.array([[10, 11, 12, -1, 14, 10]], np.int16)
    # 11: |10-11| = 1 -> removed; 12: 10 kept at distance 2, |12-10| = 2 -> kept;
    # 14: back 3 = {12, -1, 11(removed)} -> |14-12| = 2 -> kept;
    # 10: back 3 = {-1, 14, 12} -> kept (10 at distance 5 is out of reach)
    assert ref.filter_redun_past(p, a, vertical=False)[0].tolist() == [10, -1, 12, -1, 14, 10]


def test_past_only_vertical_runs_down_columns():
    p = ref.params(redun_max_dist=2, redun_threshold=0)
    a = np.full((7, 3), -1, np.int16)
    a[:, 1] = 5
    a[:, 2] = np.arange(7)
    out = ref.filter_redun_past(p, a, vertical=True)
    assert out[:, 1].tolist() == [5, -1, -1, 5, -1, -1, 5]
    assert np.array_equal(out[:, 2], a[:, 2])            # all distinct: untouched
    assert np.all(out[:, 0] == -1)
    # the same lattice transposed through the horizontal pass
    assert np.array_equal(ref.filter_redun_past(p, a.T.copy(), vertical=False), out.T)


# ---------------------------------------------------------------- down-sampling
def test_subsample_every_kth():
    pts = np.arange(30, dtype=np.int32).reshape(10, 3)
    assert np.array_equal(ref.subsample(pts, 1), pts)
    assert np.array_equal(ref.subsample(pts, 3), pts[[0, 3, 6, 9]])
    assert np.array_equal(ref.subsample(pts, 10), pts[:1])
    assert np.array_equal(ref.subsample(pts, 64), pts[:1])
    assert len(ref.subsample(pts[:0], 4)) == 0


@pytest.mark.parametrize("k", [2, 8, 14])
def test_pipeline_subsample_thins_the_left_list(k):
    pair = synth.make_pair(synth.SceneConfig(200, 120, 32, 4, 0.05, 4.0, 27.0, 2.0, 0.1,
                                             seed=k))
    full = ref.process(ref.params(disp_max=31), pair.left, pair.right)
    sub = ref.process(ref.params(disp_max=31, support_subsample=k), pair.left, pair.right)
    assert np.array_equal(sub.dcan_final, full.dcan_final)
    assert sub.nL_all == len(full.ptsL)
    assert np.array_equal(sub.ptsL, full.ptsL[::k])
    # right list: the kept points seen from the right view, one per pixel,
    # the larger disparity where two land on the same pixel
    proj = {}
    for u, v, d in sub.ptsL:
        key = (u - d, v)
        proj[key] = max(proj.get(key, -1), d)
    want = sorted((v, u, d) for (u, v), d in proj.items())
    assert [(v, u, d) for u, v, d in sub.ptsR] == want


# ---------------------------------------------------------------- median
def test_median_matches_scipy_on_fully_valid_windows():
    rng = np.random.default_rng(4)
    disp = rng.integers(0, 100, (25, 31)).astype(np.int16)
    for win in (3, 5):
        got = ref.median(win, disp)
        want = ndimage.median_filter(disp, size=win, mode="nearest")
        r = win // 2
        assert np.array_equal(got[r:-r, r:-r], want[r:-r, r:-r])


def test_median_invalid_pixels_and_clipping():
    disp = np.full((5, 6), -1, np.int16)
    disp[0, 0], disp[0, 1], disp[1, 0], disp[1, 1] = 5, 1, 9, 7
    out = ref.median(3, disp)
    # corner window clipped to 2x2: sorted 1 5 7 9, lower median 5
    assert out[0, 0] == 5
    # (1, 1) sees the same four valid values in its 3x3 window
    assert out[1, 1] == 5
    # invalid centre stays invalid even with valid neighbours
    assert out[2, 2] == -1 and out[0, 2] == -1
    # (0, 1): 2x3 window holds 5 1 9 7 and invalid -> lower median 5
    assert out[0, 1] == 5


def test_median_removes_salt_keeps_ramps_and_identity_when_off():
    base = np.tile(np.arange(20, dtype=np.int16), (12, 1))
    salt = base.copy()
    salt[6, 10] = 90
    for win in (3, 5):
        r = win // 2
        assert np.array_equal(ref.median(win, salt)[r:-r, r:-r], base[r:-r, r:-r])
        assert np.array_equal(ref.median(win, base)[r:-r, r:-r], base[r:-r, r:-r])
    for win in (0, 1):
        assert np.array_equal(ref.median(win, salt), salt)


# ---------------------------------------------------------------- census matching
def test_census_support_matching_finds_a_constant_shift():
    d0 = 12
    W, H = 120, 60
    L, R = synth.shifted_pair(W, H, d0, seed=11)
    for amb in (0, 1):
        p = ref.params(disp_max=31, descriptor=1, ambiguity=amb, support_texture=0)
        for win in (5, 9, 13):
            cL, cR = ref.census(L, win), ref.census(R, win)
            dcan, _ = ref.support_match_census(p, cL, cR)
            lw, lh, u0, v0 = ref.lattice(p, W, H)
            r = win // 2
            checked = 0
            for l in range(lh):
                for k in range(lw):
                    u = u0 + 5 * k
                    # the true disparity is in the search range and both
                    # windows lie inside the images
                    if u - 4 >= d0 and u - d0 - r >= 0 and u + r <= W - 1:
                        # a 5x5 census of this smooth texture can repeat along
                        # the row (a second zero-cost disparity): the point is
                        # then rejected, never matched wrongly
                        if win == 5:
                            assert dcan[l, k] in (d0, -1), (win, u)
                        else:
                            assert dcan[l, k] == d0, (win, u)
                        checked += 1
            assert checked > 0


def test_census_dense_full_search_finds_a_constant_shift():
    d0 = 9
    W, H = 80, 30
    L, R = synth.shifted_pair(W, H, d0, seed=13)
    p = ref.params(disp_max=31, descriptor=1, full_search=1, match_texture=0)
    lut = ref.prior_lut(p)
    gw, gh = (W + 19) // 20, (H + 19) // 20
    grid = np.zeros((gh, gw, 1), np.uint64)
    dp = np.full((H, W), -1, np.int16)
    for win in (3, 5, 7):
        cL, cR = ref.census(L, win), ref.census(R, win)
        out, ev = ref.dense_census(p, cL, cR, dp, grid, False, lut, False)
        r = win // 2
        u = np.arange(W)[None, :].repeat(H, 0)
        v = np.arange(H)[:, None].repeat(W, 1)
        region = (u >= d0 + max(2, r)) & (u <= W - 1 - max(2, r)) & (v >= 2) & (v <= H - 3)
        # d0 costs 0 there, so the result is the smallest zero-cost disparity:
        # never above d0, and d0 itself wherever the census does not repeat
        got = out[region]
        assert np.all((got >= 0) & (got <= d0))
        for (vv, uu), d in zip(np.argwhere(region), got):
            assert ref.hamming(cL[vv, uu], cR[vv, uu - d]) == 0
        if win == 7:
            assert np.mean(got == d0) > 0.95
        assert ev > 0


def test_census_pipeline_constant_disparity():
    d0 = 14
    W, H = 200, 64
    L, R = synth.shifted_pair(W, H, d0, seed=21)
    p = ref.params(disp_max=63, descriptor=1, ambiguity=1, support_texture=0,
                   match_texture=0)
    t = ref.process(p, L, R)
    assert len(t.ptsL) > 0
    assert np.all(t.ptsL[:, 2] == d0)
    assert np.all(t.dplaneL == d0) and np.all(t.dplaneR == d0)
    r = p.census_dense_window // 2
    u = np.arange(W)[None, :].repeat(H, 0)
    v = np.arange(H)[:, None].repeat(W, 1)
    region = (u >= d0 + max(2, r)) & (u <= W - 1 - max(2, r)) & (v >= 2) & (v <= H - 3)
    assert np.all(t.rawL[region] == d0)
    assert np.all(t.outL[region] == d0)


def test_variant_parameters_validated():
    L = np.zeros((20, 20), np.uint8)
    for bad in (dict(descriptor=2), dict(descriptor=1, census_support_window=4),
                dict(descriptor=1, census_support_window=15),
                dict(descriptor=1, census_dense_window=9), dict(ambiguity=3),
                dict(redundancy=2), dict(support_subsample=0),
                dict(support_subsample=65), dict(median_window=7)):
        with pytest.raises(ValueError):
            ref.process(ref.params(disp_max=15, **bad), L, L)


def test_median_in_the_pipeline_filters_the_checked_maps():
    pair = synth.make_pair(synth.SceneConfig(160, 100, 32, 4, 0.05, 4.0, 27.0, 2.0, 0.1,
                                             seed=3))
    plain = ref.process(ref.params(disp_max=31), pair.left, pair.right)
    med = ref.process(ref.params(disp_max=31, median_window=5), pair.left, pair.right)
    assert np.array_equal(med.chkL, plain.outL) and np.array_equal(med.chkR, plain.outR)
    assert np.array_equal(med.outL, ref.median(5, plain.outL))
    assert np.array_equal(med.outR, ref.median(5, plain.outR))
    assert np.array_equal(plain.chkL, plain.outL)
