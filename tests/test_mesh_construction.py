"""Facts about the starting triangulation that the device mesh relies on
(Section III-A: Delaunay triangulation of the support points), checked here
on the CPU from their definitions.

* Band zipper = merge. Between two horizontal rows of points the zipper that
  picks each diagonal by the exact in-circle test emits the same triangles,
  in the same order, as a merge of the two rows' edge u-sums (lower edge
  first on ties: the four points are co-circular, and that gives the
  diagonal from the (v, u)-smallest of them, the canonical fan). The device
  places each band triangle by that merge.
* Band twins. In that order, a row edge joins the triangle of the band below
  (local vertex 2) and of the band above (local vertex 0), and consecutive
  triangles of a band share their diagonal: local vertex 0 of a top-edge
  triangle or 2 of a bottom-edge one, against 1 of the next. The device sets
  these neighbours directly and searches only the rest.
"""
import random

import pytest


def incircle(a, b, c, d):
    """> 0 iff d is strictly inside the circle through the counter-clockwise
    a, b, c (exact integer determinant)."""
    du, dv = d
    ax, ay = a[0] - du, a[1] - dv
    bx, by = b[0] - du, b[1] - dv
    cx, cy = c[0] - du, c[1] - dv
    la, lb, lc = ax * ax + ay * ay, bx * bx + by * by, cx * cx + cy * cy
    return la * (bx * cy - by * cx) + lb * (cx * ay - cy * ax) + lc * (ax * by - ay * bx)


def zipper(A, B):
    """Sequential band zipper: advance on the upper row while the next lower
    point lies strictly outside the circle of the current upper edge (on it:
    the lower row advances, the canonical fan diagonal)."""
    out, i, j = [], 0, 0
    while i + 1 < len(A) or j + 1 < len(B):
        if i + 1 >= len(A):
            upper = False
        elif j + 1 >= len(B):
            upper = True
        else:
            upper = incircle(A[i], A[i + 1], B[j], B[j + 1]) < 0
        if upper:
            out.append(("top", i, j))
            i += 1
        else:
            out.append(("bot", i, j))
            j += 1
    return out


def merge(A, B):
    """The same band by ranks: upper edge i sits at slot i + #(lower sums at
    or below its sum), lower edge j at j + #(upper sums below its sum)."""
    S = [A[i][0] + A[i + 1][0] for i in range(len(A) - 1)]
    T = [B[j][0] + B[j + 1][0] for j in range(len(B) - 1)]
    slots = {}
    for i, s in enumerate(S):
        j = sum(1 for t in T if t <= s)
        slots[i + j] = ("top", i, j)
    for j, t in enumerate(T):
        i = sum(1 for s in S if s < t)
        slots[i + j] = ("bot", i, j)
    assert sorted(slots) == list(range(len(A) + len(B) - 2))
    return [slots[k] for k in range(len(slots))]


def random_row(rng, W, count, v, step):
    us = sorted(rng.sample(range(0, W, step), min(count, len(range(0, W, step)))))
    return [(u, v) for u in us]


@pytest.mark.parametrize("seed", range(4))
def test_band_zipper_is_a_merge_of_edge_sums(seed):
    rng = random.Random(seed)
    n = 0
    for _ in range(4000):
        W = rng.choice([12, 30, 640])
        step = rng.choice([1, 5])  # step 1 on narrow rows makes tied sums common
        va = rng.randint(0, 400)
        A = random_row(rng, W, rng.randint(1, 10), va, step)
        B = random_row(rng, W, rng.randint(1, 10), va + rng.choice([1, 5, 35]), step)
        if len(A) + len(B) < 3:
            continue
        assert zipper(A, B) == merge(A, B), (A, B)
        n += 1
    assert n > 3000


def test_tied_sums_take_the_lower_edge_first():
    # u-sums 0+4 = 4 above and 1+3 = 4 below: B[1] lies exactly on the circle.
    # The lower edge first gives the diagonal A[0]-B[1], from the
    # (v, u)-smallest point A[0]: the canonical fan of the co-circular cell
    A, B = [(0, 0), (4, 0)], [(1, 5), (3, 5)]
    assert incircle(A[0], A[1], B[0], B[1]) == 0
    assert zipper(A, B) == merge(A, B) == [("bot", 0, 0), ("top", 0, 1)]


def band_mesh(rows):
    """Triangles of all bands (rows[0] and rows[-1] are the corner rows) by
    the merge, as rank triples, with the neighbours the construction fixes."""
    off = [0]
    for s in range(len(rows) - 1):
        off.append(off[-1] + len(rows[s]) + len(rows[s + 1]) - 2)
    tris, kind, row_edge = [None] * off[-1], [None] * off[-1], {}
    for s in range(len(rows) - 1):
        A, B = rows[s], rows[s + 1]
        for k, (typ, i, j) in enumerate(merge([(u, 0) for _, u in A], [(u, 1) for _, u in B])):
            t = off[s] + k
            if typ == "top":
                tris[t] = (A[i][0], A[i + 1][0], B[j][0])
                row_edge[(s, i, "below")] = t
            else:
                tris[t] = (A[i][0], B[j + 1][0], B[j][0])
                row_edge[(s + 1, j, "above")] = t
            kind[t] = typ
    known = {}
    for s in range(len(rows) - 1):
        for t in range(off[s], off[s + 1] - 1):
            li = 0 if kind[t] == "top" else 2
            known[(t, li)] = (t + 1, 1)
            known[(t + 1, 1)] = (t, li)
    for (r, i, side), t in row_edge.items():
        if side == "below" and (r, i, "above") in row_edge:
            ta = row_edge[(r, i, "above")]
            known[(t, 2)] = (ta, 0)
            known[(ta, 0)] = (t, 2)
    return tris, known


def twins(tris):
    """Neighbour of every half-edge by brute force: half-edge k of triangle t
    runs from vertex k+1 to vertex k+2, its twin the other way."""
    he = {}
    for t, v in enumerate(tris):
        for k in range(3):
            he[(v[(k + 1) % 3], v[(k + 2) % 3])] = (t, k)
    return {tk: he[(b, a)] for (a, b), tk in he.items() if (b, a) in he}


@pytest.mark.parametrize("seed", range(3))
def test_band_twins_from_the_construction(seed):
    rng = random.Random(100 + seed)
    for _ in range(1500):
        W = rng.choice([30, 640])
        rows, r = [[(0, 0), (1, W - 1)]], 2
        for _ in range(rng.randint(1, 6)):
            us = sorted(rng.sample(range(W), rng.randint(1, 6)))
            rows.append([(r + i, u) for i, u in enumerate(us)])
            r += len(us)
        rows.append([(r, 0), (r + 1, W - 1)])
        tris, known = band_mesh(rows)
        truth = twins(tris)
        for key, val in known.items():
            assert truth.get(key) == val, (rows, key, val, truth.get(key))
        # every half-edge is covered but the two side edges of each band with
        # triangles (two one-point rows bound an empty band) and the top and
        # bottom corner edges
        bands = sum(1 for s in range(len(rows) - 1) if len(rows[s]) + len(rows[s + 1]) > 2)
        assert len(known) == 3 * len(tris) - 2 * bands - 2
