"""Pins of the oracle's triangulation, planes and prior raster.

* Delaunay: an O(n^4) brute force (empty circumcircles + the fan rule for
  co-circular cells) on random lattice subsets and forced co-circular sets.
* predicates: hand-evaluated signs.
* planes: triangles cut from integer-coefficient planes give exact a, b, c.
* raster: per-pixel test of every triangle on tiny images.
"""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import ref


def _incircle(a, b, c, d):
    adx, ady = a[0] - d[0], a[1] - d[1]
    bdx, bdy = b[0] - d[0], b[1] - d[1]
    cdx, cdy = c[0] - d[0], c[1] - d[1]
    return ((adx * adx + ady * ady) * (bdx * cdy - cdx * bdy)
            - (bdx * bdx + bdy * bdy) * (adx * cdy - cdx * ady)
            + (cdx * cdx + cdy * cdy) * (adx * bdy - bdx * ady))


def _orient(a, b, c):
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def brute_force_delaunay(pts):
    """Every triangle with an empty circumcircle; a circle through k > 3
    points contributes the fan from its (v, u)-smallest point."""
    pts = [tuple(map(int, p)) for p in pts]
    n = len(pts)
    out = set()
    for i, j, k in itertools.combinations(range(n), 3):
        a, b, c = pts[i], pts[j], pts[k]
        o = _orient(a, b, c)
        if o == 0:
            continue
        if o < 0:
            b, c = c, b
        on, inside = [i, j, k], False
        for m in range(n):
            if m in (i, j, k):
                continue
            s = _incircle(a, b, c, pts[m])
            if s > 0:
                inside = True
                break
            if s == 0:
                on.append(m)
        if inside:
            continue
        if len(on) == 3:
            out.add(tuple(sorted(on)))
            continue
        # circumcentre, then circular order of the co-circular set
        ax, ay = a
        bx, by = b
        cx, cy = c
        dd = 2.0 * (ax * (by - cy) + bx * (cy - ay) + cx * (ay - by))
        ux = ((ax * ax + ay * ay) * (by - cy) + (bx * bx + by * by) * (cy - ay)
              + (cx * cx + cy * cy) * (ay - by)) / dd
        uy = ((ax * ax + ay * ay) * (cx - bx) + (bx * bx + by * by) * (ax - cx)
              + (cx * cx + cy * cy) * (bx - ax)) / dd
        m = min(on, key=lambda q: (pts[q][1], pts[q][0]))
        ang = lambda q: math.atan2(pts[q][1] - uy, pts[q][0] - ux)
        ring = sorted(on, key=ang)
        r0 = ring.index(m)
        chain = ring[r0 + 1:] + ring[:r0]       # circular order starting after m
        fan = {tuple(sorted((m, chain[t], chain[t + 1]))) for t in range(len(chain) - 1)}
        key = tuple(sorted((i, j, k)))
        if key in fan:
            out.add(key)
    return out


def corners(W, H):
    return [(0, 0), (W - 1, 0), (0, H - 1), (W - 1, H - 1)]


def run_oracle(pts):
    tris = ref.delaunay(np.array(pts, np.int32))
    return {tuple(sorted(t)) for t in tris.tolist()}, tris


def check_valid(pts, tris):
    pts = np.array(pts)
    for t in tris:
        assert _orient(*[tuple(pts[q]) for q in t]) > 0
    W1, H1 = pts[1][0], pts[2][1]
    area2 = sum(_orient(*[tuple(pts[q]) for q in t]) for t in tris)
    assert area2 == 2 * W1 * H1                 # the triangles tile the image rectangle
    assert len(tris) == 2 * len(pts) - 6        # Euler, four hull vertices


@pytest.mark.parametrize("seed", range(12))
def test_delaunay_matches_brute_force_on_lattice_subsets(seed):
    rng = np.random.default_rng(seed)
    W, H = 46, 36
    cand = [(u, v) for v in range(5, H - 4, 5) for u in range(5, W - 4, 5)]
    k = int(rng.integers(3, min(30, len(cand))))
    sel = rng.choice(len(cand), size=k, replace=False)
    pts = corners(W, H) + [cand[s] for s in sorted(sel)]
    got, tris = run_oracle(pts)
    check_valid(pts, tris)
    assert got == brute_force_delaunay(pts)


@pytest.mark.parametrize("seed", range(6))
def test_delaunay_matches_brute_force_on_random_points(seed):
    rng = np.random.default_rng(100 + seed)
    W, H = 60, 45
    allp = {(int(u), int(v)) for u, v in zip(rng.integers(1, W - 1, 40), rng.integers(1, H - 1, 40))}
    pts = corners(W, H) + sorted(allp, key=lambda p: (p[1], p[0]))[:30]
    got, tris = run_oracle(pts)
    check_valid(pts, tris)
    assert got == brute_force_delaunay(pts)


def test_full_lattice_rectangle_fans():
    # every lattice square is a co-circular cell: split from its top-left
    W, H = 31, 26
    pts = corners(W, H) + [(u, v) for v in (5, 10, 15, 20) for u in (5, 10, 15, 20, 25)]
    got, tris = run_oracle(pts)
    check_valid(pts, tris)
    assert got == brute_force_delaunay(pts)
    idx = {p: i for i, p in enumerate(pts)}
    for v in (5, 10, 15):
        for u in (5, 10, 15, 20):
            tl, tr, bl, br = idx[(u, v)], idx[(u + 5, v)], idx[(u, v + 5)], idx[(u + 5, v + 5)]
            assert tuple(sorted((tl, tr, br))) in got
            assert tuple(sorted((tl, br, bl))) in got


@pytest.mark.parametrize("with_centre", [False, True])
def test_twelve_point_circle(with_centre):
    # (+-3, +-4), (+-4, +-3), (+-5, 0), (0, +-5) scaled by 5 about (50, 50)
    base = [(3, 4), (4, 3), (5, 0), (4, -3), (3, -4), (0, -5), (-3, -4), (-4, -3),
            (-5, 0), (-4, 3), (-3, 4), (0, 5)]
    ring = [(50 + 5 * x, 50 + 5 * y) for x, y in base]
    pts = corners(101, 101) + ring + ([(50, 50)] if with_centre else [])
    got, tris = run_oracle(pts)
    check_valid(pts, tris)
    assert got == brute_force_delaunay(pts)
    if not with_centre:
        top = pts.index((50, 25))                # (v, u)-smallest point of the ring
        inner = [t for t in got if all(q >= 4 for q in t)]
        assert len(inner) == 10 and all(top in t for t in inner)


def test_delaunay_independent_of_insertion_order():
    W, H = 46, 36
    cand = [(u, v) for v in range(5, H - 4, 5) for u in range(5, W - 4, 5)]
    rng = np.random.default_rng(7)
    pts = corners(W, H) + cand
    a, _ = run_oracle(pts)
    perm = rng.permutation(len(cand))
    pts2 = corners(W, H) + [cand[i] for i in perm]
    b, _ = run_oracle(pts2)
    remap = {i + 4: pts2.index(cand[i]) for i in range(len(cand))}
    remap.update({i: i for i in range(4)})
    assert {tuple(sorted(remap[q] for q in t)) for t in a} == b


def test_predicate_signs():
    a, b, c = (1, 0), (0, 1), (-1, 0)           # positive orientation
    assert ref.orient(a, b, c) == 2
    assert ref.orient(a, c, b) == -2
    assert ref.incircle(a, b, c, (0, 0)) > 0     # centre is inside
    assert ref.incircle(a, b, c, (0, -1)) == 0   # on the unit circle
    assert ref.incircle(a, b, c, (2, 2)) < 0
    # large coordinates stay exact
    big = [(0, 0), (8191, 0), (8191, 8191)]
    assert ref.incircle(*big, (0, 8191)) == 0
    assert ref.incircle(*big, (1, 8190)) > 0


def test_delaunay_rejects_bad_input():
    with pytest.raises(ValueError):
        ref.delaunay(np.array([(0, 0), (9, 0), (0, 9), (9, 9), (9, 4)], np.int32))


# ------------------------------------------------------------------ planes
@pytest.mark.parametrize("p_,q_,r_,k", [(3, -5, 40, 3), (-7, 2, 11, 4), (0, 0, 17, 0),
                                        (1, 1, 0, 1), (-13, 9, 200, 5)])
def test_plane_exact_for_dyadic_planes(p_, q_, r_, k):
    # d = (p/2^k) u + (q/2^k) v + r at vertices where d is an integer
    s = 2 ** k
    verts = [(0, 0), (3 * s, s), (s, 4 * s)]
    rec = []
    for u, v in verts:
        num = p_ * u + q_ * v
        assert num % s == 0
        rec += [u + 10 * s, v + 7 * s, num // s + r_ - (p_ * 10 * s + q_ * 7 * s) // s]
    # re-express with the shifted origin: d = a u + b v + c
    a, b = p_ / s, q_ / s
    c = rec[2] - a * rec[0] - b * rec[1]
    got = ref.plane(rec)
    assert got[0] == np.float32(a) and got[1] == np.float32(b) and got[2] == np.float32(c)
    # vertex order does not matter
    perm = rec[3:6] + rec[6:9] + rec[0:3]
    assert np.array_equal(ref.plane(perm), got)


def test_plane_map_constant_and_rounding():
    # one plane d = 0.5 u through all triangles -> floor(0.5u + 0.5)
    W, H = 21, 11
    pts = corners(W, H) + [(10, 5)]
    uvd = np.array([(u, v, 0) for u, v in pts], np.int32)
    uvd[:, 2] = [0, 10, 0, 10, 5]
    tris = ref.delaunay(uvd[:, :2])
    recs = ref.canonical(uvd, tris)
    planes = np.array([ref.plane(r) for r in recs])
    assert np.allclose(planes, [[0.5, 0.0, 0.0]] * len(recs))
    p = ref.params(disp_max=7)
    owner, dp = ref.plane_map(p, recs, planes, W, H)
    u = np.arange(W)[None, :].repeat(H, 0)
    assert np.array_equal(dp, np.clip(np.floor(0.5 * u + 0.5), 0, 7).astype(np.int16))
    assert np.all(owner >= 0)


@pytest.mark.parametrize("seed", range(4))
def test_plane_map_owner_is_first_containing_triangle(seed):
    rng = np.random.default_rng(seed)
    W, H = 36, 26
    cand = [(u, v) for v in range(5, H - 4, 5) for u in range(5, W - 4, 5)]
    sel = rng.choice(len(cand), size=8, replace=False)
    pts = corners(W, H) + [cand[s] for s in sorted(sel)]
    uvd = np.array([(u, v, int(rng.integers(0, 40))) for u, v in pts], np.int32)
    tris = ref.delaunay(uvd[:, :2])
    recs = ref.canonical(uvd, tris)
    # canonical order: vertices sorted by (v, u), records sorted
    keys = [tuple((r[3 * i + 1], r[3 * i]) for i in range(3)) for r in recs.tolist()]
    assert keys == sorted(keys) and all(list(k) == sorted(k) for k in keys)
    planes = np.array([ref.plane(r) for r in recs], np.float32)
    p = ref.params(disp_max=63)
    owner, dp = ref.plane_map(p, recs, planes, W, H)
    for v in range(H):
        for u in range(W):
            first = -1
            for t, r in enumerate(recs.tolist()):
                A, B, C = (r[0], r[1]), (r[3], r[4]), (r[6], r[7])
                if _orient(A, B, C) < 0:
                    B, C = C, B
                if _orient(A, B, (u, v)) >= 0 and _orient(B, C, (u, v)) >= 0 and \
                        _orient(C, A, (u, v)) >= 0:
                    first = t
                    break
            assert owner[v, u] == first
            a, b, c = planes[first]
            mu = np.float32(np.float32(np.float32(a * np.float32(u)) + np.float32(b * np.float32(v))) + c)
            exp = int(np.floor(np.float32(mu + np.float32(0.5))))
            assert dp[v, u] == min(max(exp, 0), 63)


# ---- the mesh of the support points alone (add_corners = 0) -----------------

def hull_boundary(pts):
    """Points on the convex hull boundary (vertices and collinear points on
    its edges), and twice the hull's area: Andrew's monotone chain, then each
    point tested against the hull's edges."""
    P = sorted(set(map(tuple, pts)))
    if len(P) < 3:
        return set(P), 0

    def chain(seq):
        out = []
        for p in seq:
            while len(out) >= 2 and _orient(out[-2], out[-1], p) <= 0:
                out.pop()
            out.append(p)
        return out

    H = chain(P)[:-1] + chain(P[::-1])[:-1]
    area2 = abs(sum(H[i][0] * H[(i + 1) % len(H)][1] - H[(i + 1) % len(H)][0] * H[i][1]
                    for i in range(len(H))))
    on = set()
    for p in P:
        for i in range(len(H)):
            a, b = H[i], H[(i + 1) % len(H)]
            if _orient(a, b, p) == 0 and min(a[0], b[0]) <= p[0] <= max(a[0], b[0]) \
                    and min(a[1], b[1]) <= p[1] <= max(a[1], b[1]):
                on.add(p)
    return on, area2


def check_valid_points(pts, tris):
    for t in tris:
        assert _orient(*[tuple(pts[q]) for q in t]) > 0
    on, area2 = hull_boundary(pts)
    assert sum(_orient(*[tuple(pts[q]) for q in t]) for t in tris) == area2  # tiles the hull
    assert len(tris) == 2 * len(pts) - 2 - len(on)                           # Euler


@pytest.mark.parametrize("seed", range(10))
def test_points_alone_match_brute_force_on_lattice_subsets(seed):
    rng = np.random.default_rng(300 + seed)
    cand = [(u, v) for v in range(5, 41, 5) for u in range(5, 51, 5)]
    k = int(rng.integers(4, 28))
    sel = rng.choice(len(cand), size=k, replace=False)
    pts = [cand[s] for s in sorted(sel)]
    tris = ref.delaunay_points(np.array(pts))
    if len(tris):
        check_valid_points(pts, tris)
    assert {tuple(sorted(t)) for t in tris.tolist()} == brute_force_delaunay(pts)


@pytest.mark.parametrize("seed", range(6))
def test_points_alone_match_brute_force_on_random_points(seed):
    rng = np.random.default_rng(400 + seed)
    allp = {(int(u), int(v)) for u, v in zip(rng.integers(1, 60, 40), rng.integers(1, 45, 40))}
    pts = sorted(allp, key=lambda p: (p[1], p[0]))[:28]
    tris = ref.delaunay_points(np.array(pts))
    check_valid_points(pts, tris)
    assert {tuple(sorted(t)) for t in tris.tolist()} == brute_force_delaunay(pts)


def test_points_alone_degenerate_sets():
    assert len(ref.delaunay_points(np.zeros((0, 2), np.int32))) == 0
    assert len(ref.delaunay_points(np.array([(3, 4), (9, 4)]))) == 0
    assert len(ref.delaunay_points(np.array([(5, 5), (10, 5), (20, 5), (40, 5)]))) == 0
    assert len(ref.delaunay_points(np.array([(5, 5), (10, 10), (15, 15)]))) == 0
    # a row and one point below: a fan of triangles from that point
    pts = [(5, 5), (10, 5), (15, 5), (20, 5), (12, 9)]
    tris = ref.delaunay_points(np.array(pts))
    assert {tuple(sorted(t)) for t in tris.tolist()} == {(0, 1, 4), (1, 2, 4), (2, 3, 4)}
    with pytest.raises(ValueError):
        ref.delaunay_points(np.array([(5, 5), (5, 5), (7, 8)]))


@pytest.mark.parametrize("with_centre", [False, True])
def test_points_alone_twelve_point_circle(with_centre):
    c = (30, 30)
    ring = [(c[0] + 5 * x, c[1] + 5 * y) for x, y in
            [(3, 4), (4, 3), (5, 0), (4, -3), (3, -4), (0, -5), (-3, -4), (-4, -3), (-5, 0),
             (-4, 3), (-3, 4), (0, 5)]]
    pts = ring + ([c] if with_centre else [])
    tris = ref.delaunay_points(np.array(pts))
    check_valid_points(pts, tris)
    assert {tuple(sorted(t)) for t in tris.tolist()} == brute_force_delaunay(pts)


def test_pipeline_without_corners_has_priors_exactly_on_the_hull():
    cfg = synth.QVGA.with_seed(2)
    pr = synth.make_pair(cfg)
    t1 = ref.process(ref.params(disp_max=63), pr.left, pr.right)
    t0 = ref.process(ref.params(disp_max=63, add_corners=0), pr.left, pr.right)
    # the stages before the mesh do not change; no corners are reported
    assert np.array_equal(t0.ptsL, t1.ptsL) and np.array_equal(t0.gridL, t1.gridL)
    assert np.all(t0.cornersL == -1) and np.all(t0.cornersR == -1)
    for pts, rec, dpl in ((t0.ptsL, t0.recL, t0.dplaneL), (t0.ptsR, t0.recR, t0.dplaneR)):
        on, _ = hull_boundary(pts[:, :2])
        assert len(rec) == 2 * len(pts) - 2 - len(on)
        # a pixel has a plane prior iff it lies in the hull of the points
        H, W = dpl.shape
        P = sorted(set(map(tuple, pts[:, :2].tolist())))

        def half(seq):
            out = []
            for p in seq:
                while len(out) >= 2 and _orient(out[-2], out[-1], p) <= 0:
                    out.pop()
                out.append(p)
            return out

        hull = half(P)[:-1] + half(P[::-1])[:-1]
        vv, uu = np.mgrid[0:H, 0:W]
        inside = np.ones((H, W), bool)
        for i in range(len(hull)):
            a, b = hull[i], hull[(i + 1) % len(hull)]
            o = (b[0] - a[0]) * (vv - a[1]) - (b[1] - a[1]) * (uu - a[0])
            inside &= o >= 0
        assert np.array_equal(dpl >= 0, inside)
