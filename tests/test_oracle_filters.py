"""Pins of the support filters and support lists on hand-built lattices
(expected outputs worked out by hand from the stated rules)."""
import numpy as np
import pytest

from oracle import ref

P = ref.params()   # window 5, threshold 5, min support 5, redundancy 5 / 1


def lat(h, w):
    return np.full((h, w), -1, np.int16)


def test_incon_isolated_point_removed_cluster_kept():
    a = lat(15, 15)
    a[7, 7] = 40
    assert np.all(ref.filter_incon(P, a) == -1)
    a[6:9, 6:9] = 40                         # 3x3 block: 8 neighbours each
    out = ref.filter_incon(P, a)
    assert np.all(out[6:9, 6:9] == 40)


def test_incon_self_not_counted_and_threshold():
    a = lat(15, 15)
    a[7, 7] = 40
    a[7, 8:12] = 40                          # 4 consistent others: 4 < 5
    out = ref.filter_incon(P, a)
    assert out[7, 7] == -1
    a[7, 12] = 45                            # |45 - 40| = 5 <= 5: now 5 others
    out = ref.filter_incon(P, a)
    assert out[7, 7] == 40
    a[7, 12] = 46                            # 6 > 5: back to 4
    assert ref.filter_incon(P, a)[7, 7] == -1


def test_incon_window_is_in_lattice_units():
    a = lat(20, 20)
    a[10, 10] = 30
    for k in range(5):                        # five supporters exactly 5 steps away
        a[5 + k, 15] = 30
    assert ref.filter_incon(P, a)[10, 10] == 30
    b = lat(20, 20)
    b[10, 10] = 30
    for k in range(5):                        # six steps away: outside
        b[5 + k, 16] = 30
    assert ref.filter_incon(P, b)[10, 10] == -1


def test_incon_reads_unfiltered_input():
    # a chain where every point has exactly 5 supporters only when the points
    # that themselves fail are still counted (simultaneous update)
    a = lat(3, 13)
    a[1, 0:7] = 20          # endpoints have 5 supporters within +-5 along the row
    out = ref.filter_incon(P, a)
    assert np.all(out[1, 0:7] == 20)
    a2 = lat(3, 13)
    a2[1, 0:6] = 20         # 5 others each at most (k=0 sees 1..5)
    out2 = ref.filter_incon(P, a2)
    assert np.all(out2[1, 0:6] == 20)
    a3 = lat(3, 13)
    a3[1, 0:5] = 20         # only 4 others
    assert np.all(ref.filter_incon(P, a3) == -1)


def test_redundancy_vertical_run_keeps_endpoints():
    a = lat(10, 3)
    a[1:8, 1] = 50
    out = ref.filter_redun(P, a, vertical=True)
    assert out[1, 1] == 50 and out[7, 1] == 50
    assert np.all(out[2:7, 1] == -1)
    # the horizontal pass leaves a vertical run alone
    assert np.array_equal(ref.filter_redun(P, a, vertical=False), a)


def test_redundancy_threshold_and_distance():
    a = lat(1, 20)
    a[0, [0, 5, 10]] = [30, 31, 32]          # neighbours differ by 1: redundant
    out = ref.filter_redun(P, a, vertical=False)
    assert list(out[0, [0, 5, 10]]) == [30, -1, 32]
    b = lat(1, 20)
    b[0, [0, 5, 10]] = [30, 32, 30]          # differ by 2: not redundant
    assert np.array_equal(ref.filter_redun(P, b, vertical=False), b)
    c = lat(1, 20)
    c[0, [0, 6, 12]] = 30                     # 6 steps apart: beyond the range
    assert np.array_equal(ref.filter_redun(P, c, vertical=False), c)


def test_redundancy_needs_both_sides():
    a = lat(1, 12)
    a[0, [3, 4]] = 60                         # neighbour only on one side each
    assert np.array_equal(ref.filter_redun(P, a, vertical=False), a)


def test_support_lists_right_view_and_corners():
    # lattice of a 60x40 image with s = 5: u = 5..55, v = 5..35
    p = ref.params(disp_max=31)
    lw, lh, u0, v0 = ref.lattice(p, 60, 40)
    d = lat(lh, lw)
    # (u, v) = (20, 10) d 10 -> right (10, 10); (u, v) = (25, 10) d 15 -> (10, 10)
    d[1, 3] = 10
    d[1, 4] = 15
    d[5, 9] = 4             # (50, 30) -> (46, 30)
    d[0, 0] = 0             # (5, 5) -> (5, 5)
    ptsL, cL, ptsR, cR = ref.support_lists(p, d, 60, 40)
    assert ptsL.tolist() == [[5, 5, 0], [20, 10, 10], [25, 10, 15], [50, 30, 4]]
    # collision at (10, 10): the larger disparity (nearer surface) wins
    assert ptsR.tolist() == [[5, 5, 0], [10, 10, 15], [46, 30, 4]]
    # corners: (0,0) nearest (5,5); (59,0): (25,10) at 34^2+10^2 = 1256 vs
    # (50,30) at 81+900 = 981 -> d 4; (0,39): (5,5) 25+1156 = 1181, (20,10)
    # 400+841 = 1241 -> d 0; (59,39) -> (50,30) d 4
    assert cL.tolist() == [0, 4, 0, 4]
    # right view: (0,39) is nearer (10,10) (100+841 = 941) than (5,5) (1181);
    # (59,0): (46,30) at 169+900 = 1069 vs (10,10) at 2401+100 -> d 4
    assert cR.tolist() == [0, 4, 15, 4]


def test_corner_tie_goes_to_earlier_point():
    p = ref.params(disp_max=31)
    lw, lh, u0, v0 = ref.lattice(p, 41, 41)
    d = lat(lh, lw)
    # (20, 10) and (10, 20) are both at distance^2 500 from (0, 0)
    d[(10 - v0) // 5, (20 - u0) // 5] = 7
    d[(20 - v0) // 5, (10 - u0) // 5] = 9
    ptsL, cL, _, _ = ref.support_lists(p, d, 41, 41)
    assert ptsL.tolist() == [[20, 10, 7], [10, 20, 9]]
    assert cL[0] == 7
