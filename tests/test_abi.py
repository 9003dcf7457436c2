"""The C-ABI library on the CPU: it loads, exports every declared symbol,
validates arguments without touching a GPU, and its host mesh step agrees
with the oracle's (independently written) triangulation bit for bit."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from oracle import ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def E():
    import paper_1802_07210_amd as pkg
    if not os.path.exists(pkg.elas.LIB_PATH):
        from paper_1802_07210_amd import build
        build.build()
    return pkg


def declared_functions():
    text = open(os.path.join(ROOT, "include", "elas.h")).read()
    return sorted(set(re.findall(r"ELAS_API\s+[\w\s\*]+?\b(elas_\w+)\s*\(", text)))


def test_exports_every_declared_symbol(E):
    names = declared_functions()
    assert len(names) >= 8
    L = C.CDLL(E.elas.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(E.elas.EXPORTS)


def test_defaults_match_the_workload_parameters(E):
    p = E.default_params()
    assert (p.disp_min, p.disp_max) == (0, 127)
    assert p.support_threshold == np.float32(0.85) and p.support_texture == 10
    assert p.candidate_stepsize == 5 and p.incon_window_size == 5
    assert p.incon_threshold == 5 and p.incon_min_support == 5
    assert p.grid_size == 20 and p.beta == np.float32(0.02)
    assert p.gamma == 3 and p.sigma == 1 and p.sradius == 2
    assert p.match_texture == 1 and p.lr_threshold == 2 and p.full_search == 0
    # the embedded variant and the optional steps are off by default
    assert (p.descriptor, p.ambiguity, p.redundancy) == (0, 0, 0)
    assert (p.census_support_window, p.census_dense_window) == (9, 5)
    assert p.support_subsample == 1 and p.median_window == 0
    assert p.add_corners == 1


def test_param_struct_mirrors_the_oracle_fields():
    # every oracle parameter exists in the C-ABI struct under the same name
    from oracle import ref
    import paper_1802_07210_amd.elas as el
    names = {n for n, _ in el.ElasParams._fields_}
    assert set(ref.DEFAULTS) <= names


@pytest.mark.parametrize("bad", [
    dict(disp_min=-1), dict(disp_min=10, disp_max=9), dict(disp_max=256),
    dict(candidate_stepsize=0), dict(grid_size=0), dict(beta=0.0), dict(gamma=-1.0),
    dict(sigma=float("nan")), dict(incon_window_size=-1), dict(full_search=2),
    dict(sradius=-3), dict(descriptor=2), dict(ambiguity=-1), dict(redundancy=2),
    dict(descriptor=1, census_support_window=8), dict(descriptor=1, census_support_window=15),
    dict(descriptor=1, census_dense_window=1), dict(descriptor=1, census_dense_window=9),
    dict(support_subsample=0), dict(support_subsample=65), dict(median_window=2),
    dict(median_window=7), dict(add_corners=2), dict(add_corners=-1),
])
def test_create_rejects_bad_parameters(E, bad):
    with pytest.raises(E.ElasError, match="ELAS_ERR_ARG"):
        E.Elas(**bad)


def test_create_rejects_prior_out_of_key_range(E):
    with pytest.raises(E.ElasError, match="ELAS_ERR_UNSUPPORTED"):
        E.Elas(beta=1e-8)   # lut[0] = -ln(4/3)/beta is about -2.9e7


def test_create_accepts_edge_parameters(E):
    for kw in (dict(disp_max=255), dict(disp_min=7, disp_max=7), dict(candidate_stepsize=1),
               dict(full_search=1), dict(disp_min=3, disp_max=200),
               dict(descriptor=1, census_support_window=13, census_dense_window=7),
               dict(descriptor=1, census_support_window=3, census_dense_window=3),
               dict(ambiguity=1, redundancy=1, support_subsample=64, median_window=5),
               dict(median_window=1), dict(redundancy=1, redun_max_dist=16),
               dict(add_corners=0)):
        e = E.Elas(**kw)
        e.close()


def test_noalloc_rejects_a_mesh_without_corners_before_any_hip_call(E):
    # the points-alone mesh is built on the host, which the entry point that
    # allocates nothing does not do
    e = E.Elas(add_corners=0)
    buf = C.c_void_p(0x1000)    # never dereferenced: validation fails first
    assert E.elas.lib().elas_process_noalloc(e.handle, buf, buf, 64, 64, 64, None, buf,
                                             buf) == -4
    assert b"corners" in E.elas.lib().elas_last_error(e.handle)
    e.close()


def test_process_rejects_bad_arguments_before_any_hip_call(E):
    L = E.elas.lib()
    e = E.Elas()
    h = e.handle
    buf = C.c_void_p(0x1000)    # never dereferenced: validation fails first
    assert L.elas_process(h, None, buf, 64, 64, 64, None, buf, buf) == -1
    assert L.elas_process(h, buf, buf, 8, 64, 64, None, buf, buf) == -1
    assert L.elas_process(h, buf, buf, 64, 8193, 64, None, buf, buf) == -1
    assert L.elas_process(h, buf, buf, 64, 64, 63, None, buf, buf) == -1
    assert b"stride" in L.elas_last_error(h)
    assert L.elas_process(None, buf, buf, 64, 64, 64, None, buf, buf) == -1
    # no completed call yet
    st = E.elas.ElasStats()
    assert L.elas_get_stats(h, C.byref(st)) == -1
    need = C.c_int64()
    assert L.elas_get_intermediate(h, 0, None, 0, C.byref(need)) == -1
    e.close()


def test_triangulate_rejects_bad_input(E):
    with pytest.raises(E.ElasError):
        E.triangulate(np.array([[0, 5, 3]]), [1, 1, 1, 1], 20, 20)     # on the border
    with pytest.raises(E.ElasError):
        E.triangulate(np.array([[5, 5, 3], [5, 5, 4]]), [1, 1, 1, 1], 20, 20)  # duplicate
    with pytest.raises(E.ElasError):
        E.triangulate(np.zeros((0, 3)), [1, 1, 1, 1], 20, 20)


@pytest.mark.parametrize("shape", list(synth.SHAPES))
def test_host_mesh_matches_oracle(E, shape):
    cfg = synth.SHAPES[shape]
    for seed in range(2):
        pr = synth.make_pair(cfg.with_seed(seed))
        t = ref.process(ref.params(disp_max=cfg.disp_range - 1), pr.left, pr.right)
        for pts, cor, recs, planes in ((t.ptsL, t.cornersL, t.recL, t.planeL),
                                       (t.ptsR, t.cornersR, t.recR, t.planeR)):
            r2, p2 = E.triangulate(pts, cor, cfg.width, cfg.height)
            assert np.array_equal(r2, recs)
            assert np.array_equal(p2.view(np.uint32), planes.view(np.uint32))


@pytest.mark.parametrize("seed", range(8))
def test_host_mesh_matches_oracle_on_dense_cocircular_lattices(E, seed):
    # dense lattice subsets: many co-circular cells, exercises the fan rule
    rng = np.random.default_rng(seed)
    W, H = 101, 81
    cand = [(u, v) for v in range(5, H - 4, 5) for u in range(5, W - 4, 5)]
    k = int(rng.integers(10, len(cand)))
    sel = sorted(rng.choice(len(cand), size=k, replace=False))
    pts = np.array([(cand[i][0], cand[i][1], int(rng.integers(0, 64))) for i in sel], np.int32)
    corners = rng.integers(0, 64, 4).astype(np.int32)
    uvd = np.concatenate([np.array([[0, 0, corners[0]], [W - 1, 0, corners[1]],
                                    [0, H - 1, corners[2]], [W - 1, H - 1, corners[3]]],
                                   np.int32), pts])
    tris = ref.delaunay(uvd[:, :2])
    recs = ref.canonical(uvd, tris)
    planes = np.array([ref.plane(r) for r in recs], np.float32)
    r2, p2 = E.triangulate(pts, corners, W, H)
    assert np.array_equal(r2, recs)
    assert np.array_equal(p2.view(np.uint32), planes.view(np.uint32))


def _points_alone(rng, W, H, k, lattice):
    if lattice:  # many co-circular cells and collinear hull runs
        cand = [(u, v) for v in range(0, H, 5) for u in range(0, W, 5)]
    else:
        cand = [(u, v) for v in range(H) for u in range(W)]
    sel = sorted(rng.choice(len(cand), size=k, replace=False))
    return np.array([(cand[i][0], cand[i][1], int(rng.integers(0, 64))) for i in sel], np.int32)


@pytest.mark.parametrize("seed", range(12))
def test_host_mesh_of_points_alone_matches_oracle(E, seed):
    # no corners: the library's sweep + flips against the oracle's gift
    # wrapping, lattice subsets (co-circular cells, hull runs touching the
    # image border) and random points
    rng = np.random.default_rng(100 + seed)
    W, H = 101, 81
    for lattice in (True, False):
        k = int(rng.integers(3, 300 if lattice else 150))
        pts = _points_alone(rng, W, H, k, lattice)
        tris = ref.delaunay_points(pts[:, :2])
        recs = ref.canonical(pts, tris)
        planes = np.array([ref.plane(r) for r in recs], np.float32).reshape(-1, 3)
        r2, p2 = E.triangulate(pts, None, W, H)
        assert np.array_equal(r2, recs), (seed, lattice, k)
        assert np.array_equal(p2.view(np.uint32), planes.view(np.uint32))


def test_host_mesh_of_points_alone_degenerate(E):
    # fewer than three points, collinear points: no triangles
    for pts in ([[3, 3, 1]], [[3, 3, 1], [9, 4, 2]], [[0, 0, 1], [5, 5, 2], [10, 10, 3], [20, 20, 4]],
                [[4, 7, 1], [9, 7, 1], [30, 7, 1]]):
        r, p = E.triangulate(np.array(pts, np.int32), None, 40, 40)
        assert len(r) == 0 and len(p) == 0
    # a collinear run then one point off it: a fan of n - 2 triangles
    pts = np.array([[u, 10, 5] for u in range(0, 40, 4)] + [[17, 30, 9]], np.int32)
    r, _ = E.triangulate(pts, None, 40, 40)
    assert len(r) == len(pts) - 2
    assert np.array_equal(r, ref.canonical(pts, ref.delaunay_points(pts[:, :2])))
    # points on the border are allowed without corners, not with them
    E.triangulate(np.array([[0, 0, 1], [39, 0, 2], [0, 39, 3]], np.int32), None, 40, 40)
    with pytest.raises(E.ElasError):
        E.triangulate(np.array([[0, 0, 1], [39, 0, 2], [0, 39, 3]], np.int32), [1, 1, 1, 1], 40, 40)
    with pytest.raises(E.ElasError):
        E.triangulate(np.array([[5, 5, 1], [5, 5, 2], [9, 1, 3]], np.int32), None, 40, 40)


@pytest.mark.parametrize("shape", list(synth.SHAPES))
def test_host_mesh_of_points_alone_on_pipeline_lists(E, shape):
    cfg = synth.SHAPES[shape]
    pr = synth.make_pair(cfg.with_seed(5))
    t = ref.process(ref.params(disp_max=cfg.disp_range - 1, add_corners=0), pr.left, pr.right)
    assert list(t.cornersL) == [-1] * 4 and list(t.cornersR) == [-1] * 4
    for pts, recs, planes in ((t.ptsL, t.recL, t.planeL), (t.ptsR, t.recR, t.planeR)):
        r2, p2 = E.triangulate(pts, None, cfg.width, cfg.height)
        assert np.array_equal(r2, recs)
        assert np.array_equal(p2.view(np.uint32), planes.view(np.uint32))
