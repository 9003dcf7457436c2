"""Parity of the HIP path with the CPU oracle, element by element: every
intermediate stage and both output maps must match exactly (zero mismatching
pixels; the arithmetic is integer except the FP32 ratio test and plane mean,
which both sides evaluate with the same operations in the same order)."""
import numpy as np
import pytest

import synth
from oracle import ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def E():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_07210_amd as pkg
    return pkg


def run_pair(E, left, right, stride=None, **kw):
    h, w = left.shape
    dev = torch.device("cuda:0")
    if stride is None or stride == w:
        L = torch.from_numpy(np.ascontiguousarray(left)).to(dev)
        R = torch.from_numpy(np.ascontiguousarray(right)).to(dev)
    else:
        padL = np.full((h, stride), 7, np.uint8)
        padR = np.full((h, stride), 9, np.uint8)
        padL[:, :w] = left
        padR[:, :w] = right
        L = torch.from_numpy(padL).to(dev)[:, :w]
        R = torch.from_numpy(padR).to(dev)[:, :w]
    e = E.Elas(**kw)
    oL, oR = e.process(L, R)
    torch.cuda.synchronize()
    return e, oL.cpu().numpy(), oR.cpu().numpy()


def run_and_compare(E, left, right, **kw):
    e, oL, oR = run_pair(E, left, right, **kw)
    return compare(e, ref.process(oracle_params(kw), left, right), oL, oR)


def compare(e, t, outL, outR):
    """Returns a list of (stage, mismatch count) for every stage that differs."""
    h, w = t.outL.shape
    bad = []

    def chk(name, got, exp):
        got = np.asarray(got)
        exp = np.asarray(exp)
        if got.shape != exp.shape:
            bad.append((name, f"shape {got.shape} vs {exp.shape}"))
            return
        n = int(np.count_nonzero(got != exp))
        if n:
            bad.append((name, n))

    lh, lw = t.dcan_raw.shape
    prm = e.params
    if prm.descriptor == 1:
        # dense census: one uint64 per pixel; support census: the lattice rows,
        # 4*q words per pixel, zero-padded beyond the oracle's words
        for side, cden, csup in (("left", t.cdenL, t.csupL), ("right", t.cdenR, t.csupR)):
            exp = cden[..., 0].astype(np.uint64)
            if cden.shape[-1] > 1:
                exp |= cden[..., 1].astype(np.uint64) << np.uint64(32)
            chk(f"census_dense_{side}", e.intermediate(f"census_dense_{side}").reshape(h, w), exp)
            if lh:
                step = prm.candidate_stepsize
                rows = ((4 + step - 1) // step) * step + step * np.arange(lh)
                got = e.intermediate(f"census_support_{side}").reshape(lh, w, -1)
                nw = csup.shape[-1]
                chk(f"census_support_{side}", got[..., :nw], csup[rows])
                chk(f"census_support_pad_{side}", got[..., nw:], np.zeros_like(got[..., nw:]))
    else:
        chk("desc_left", e.intermediate("desc_left").reshape(h, w, 16), t.descL)
        chk("desc_right", e.intermediate("desc_right").reshape(h, w, 16), t.descR)
    if prm.median_window > 1:
        chk("checked_left", e.intermediate("checked_left").reshape(h, w), t.chkL)
        chk("checked_right", e.intermediate("checked_right").reshape(h, w), t.chkR)
    for nm, arr in (("dcan_raw", t.dcan_raw), ("dcan_incon", t.dcan_incon),
                    ("dcan_vert", t.dcan_vert), ("dcan_final", t.dcan_final)):
        chk(nm, e.intermediate(nm).reshape(lh, lw), arr)
    chk("support_left", e.intermediate("support_left").reshape(-1, 3), t.ptsL)
    chk("support_right", e.intermediate("support_right").reshape(-1, 3), t.ptsR)
    chk("corners", e.intermediate("corners"), np.concatenate([t.cornersL, t.cornersR]))
    chk("tri_left", e.intermediate("tri_left").reshape(-1, 9), t.recL)
    chk("tri_right", e.intermediate("tri_right").reshape(-1, 9), t.recR)
    chk("plane_left", e.intermediate("plane_left").reshape(-1, 3).view(np.uint32),
        t.planeL.view(np.uint32))
    chk("plane_right", e.intermediate("plane_right").reshape(-1, 3).view(np.uint32),
        t.planeR.view(np.uint32))
    for side, own in (("left", t.ownerL), ("right", t.ownerR)):
        got = e.intermediate(f"owner_{side}").reshape(h, w)
        got = np.where(got == 0x7FFFFFFF, -1, got)
        chk(f"owner_{side}", got, own)
    chk("dplane_left", e.intermediate("dplane_left").reshape(h, w), t.dplaneL)
    chk("dplane_right", e.intermediate("dplane_right").reshape(h, w), t.dplaneR)
    if len(t.ptsL):
        chk("grid_left", e.intermediate("grid_left").reshape(t.gridL.shape), t.gridL)
        chk("grid_right", e.intermediate("grid_right").reshape(t.gridR.shape), t.gridR)
    chk("raw_left", e.intermediate("raw_left").reshape(h, w), t.rawL)
    chk("raw_right", e.intermediate("raw_right").reshape(h, w), t.rawR)
    chk("lut", e.intermediate("lut"), t.lut)
    chk("out_left", outL, t.outL)
    chk("out_right", outR, t.outR)
    st = e.stats()
    chk("support_evals", st["support_evals"], t.support_evals)
    chk("dense_evals", st["dense_evals"], t.dense_evals)
    chk("n_support", (st["n_support_left"], st["n_support_right"]), (len(t.ptsL), len(t.ptsR)))
    chk("n_tri", (st["n_tri_left"], st["n_tri_right"]), (len(t.recL), len(t.recR)))
    return bad


def oracle_params(kw):
    return ref.params(**{k: v for k, v in kw.items() if k != "mesh_on_host"})


@pytest.mark.parametrize("mesh_on_host", [0, 1])
@pytest.mark.parametrize("shape", ["320x240", "640x480", "1242x375", "1280x720"])
def test_workload_shapes_bit_exact(E, shape, mesh_on_host):
    cfg = synth.SHAPES[shape]
    pair = synth.make_pair(cfg)
    kw = dict(disp_max=cfg.disp_range - 1)
    e, oL, oR = run_pair(E, pair.left, pair.right, mesh_on_host=mesh_on_host, **kw)
    t = ref.process(oracle_params(kw), pair.left, pair.right)
    assert compare(e, t, oL, oR) == []
    assert (oL >= 0).mean() > 0.4


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_qvga_seeds_bit_exact(E, seed):
    cfg = synth.QVGA.with_seed(seed)
    pair = synth.make_pair(cfg)
    kw = dict(disp_max=63)
    e, oL, oR = run_pair(E, pair.left, pair.right, **kw)
    assert compare(e, ref.process(oracle_params(kw), pair.left, pair.right), oL, oR) == []


SMALL = [
    # (w, h, D, extra params)
    (9, 9, 4, {}),
    (13, 11, 8, {}),
    (37, 23, 16, {}),
    (97, 61, 32, {}),
    (131, 77, 64, {}),
    (200, 50, 256, {}),
    (65, 40, 100, {}),                         # D > w
    (70, 33, 1, {}),                           # a single disparity: no support points
    (90, 45, 20, dict(disp_min=5)),
    (96, 48, 24, dict(full_search=1)),
    (96, 48, 24, dict(candidate_stepsize=1)),
    (123, 57, 48, dict(candidate_stepsize=3, grid_size=7, sradius=0)),
    (150, 70, 40, dict(incon_window_size=2, incon_min_support=2, redun_max_dist=2,
                       redun_threshold=0, lr_threshold=0)),
    (77, 66, 30, dict(support_threshold=0.95, support_texture=0, match_texture=0)),
    (111, 64, 33, dict(gamma=1.5, sigma=2.5, beta=0.01)),
]


@pytest.mark.parametrize("mesh_on_host", [0, 1])
@pytest.mark.parametrize("w,h,D,extra", SMALL)
def test_small_and_ragged_sizes(E, w, h, D, extra, mesh_on_host):
    dmin = extra.get("disp_min", 0)
    cfg = synth.SceneConfig(w, h, max(D, 4), 3, 0.05, 1.0, max(2.0, D - 3.0), 2.0, 0.1,
                            seed=w * 7 + h)
    pair = synth.make_pair(cfg)
    kw = dict(extra)
    kw["disp_max"] = dmin + D - 1
    e, oL, oR = run_pair(E, pair.left, pair.right, mesh_on_host=mesh_on_host, **kw)
    assert compare(e, ref.process(oracle_params(kw), pair.left, pair.right), oL, oR) == []


@pytest.mark.parametrize("stride", [64 + 3, 128, 333])
def test_padded_rows(E, stride):
    cfg = synth.SceneConfig(61, 45, 24, 3, 0.05, 2.0, 20.0, 2.0, 0.1, seed=stride)
    pair = synth.make_pair(cfg)
    kw = dict(disp_max=23)
    e, oL, oR = run_pair(E, pair.left, pair.right, stride=stride, **kw)
    assert compare(e, ref.process(oracle_params(kw), pair.left, pair.right), oL, oR) == []


def test_flat_pair(E):
    L = np.full((40, 64), 90, np.uint8)
    kw = dict(disp_max=15)
    e, oL, oR = run_pair(E, L, L, **kw)
    t = ref.process(oracle_params(kw), L, L)
    assert compare(e, t, oL, oR) == []
    assert np.all(oL == -1) and e.stats()["n_support_left"] == 0


def test_flat_pair_full_search(E):
    L, R = synth.shifted_pair(64, 32, 5, seed=2)
    kw = dict(disp_max=15, support_texture=10 ** 6, full_search=1)
    e, oL, oR = run_pair(E, L, R, **kw)
    assert compare(e, ref.process(oracle_params(kw), L, R), oL, oR) == []


@pytest.mark.parametrize("d0", [9, 30])
def test_constant_disparity(E, d0):
    L, R = synth.shifted_pair(256, 40, d0, seed=d0)
    kw = dict(disp_max=63)
    e, oL, oR = run_pair(E, L, R, **kw)
    assert compare(e, ref.process(oracle_params(kw), L, R), oL, oR) == []


def test_handle_reuse_across_sizes_and_determinism(E):
    dev = torch.device("cuda:0")
    e = E.Elas(disp_max=63)
    shapes = [(320, 240), (97, 61), (320, 240), (200, 120)]
    first = {}
    for i, (w, h) in enumerate(shapes):
        cfg = synth.SceneConfig(w, h, 64, 5, 0.05, 4.0, 59.0, 2.0, 0.1, seed=i % 3)
        pair = synth.make_pair(cfg)
        L = torch.from_numpy(pair.left).to(dev)
        R = torch.from_numpy(pair.right).to(dev)
        oL, oR = e.process(L, R)
        torch.cuda.synchronize()
        t = ref.process(ref.params(disp_max=63), pair.left, pair.right)
        assert compare(e, t, oL.cpu().numpy(), oR.cpu().numpy()) == []
        key = (w, h, i % 3)
        if key in first:
            assert np.array_equal(first[key], oL.cpu().numpy())
        first[key] = oL.cpu().numpy()


def test_nondefault_stream(E):
    dev = torch.device("cuda:0")
    pair = synth.make_pair(synth.QVGA.with_seed(9))
    s = torch.cuda.Stream(device=dev)
    e = E.Elas(disp_max=63)
    with torch.cuda.stream(s):
        L = torch.from_numpy(pair.left).to(dev)
        R = torch.from_numpy(pair.right).to(dev)
        oL, oR = e.process(L, R, stream=s)
    s.synchronize()
    t = ref.process(ref.params(disp_max=63), pair.left, pair.right)
    assert compare(e, t, oL.cpu().numpy(), oR.cpu().numpy()) == []


@pytest.mark.parametrize("seed", range(6))
def test_dense_support_sets_exercise_the_device_mesh(E, seed):
    # weak filtering keeps most lattice points: thousands of support points,
    # long runs of co-circular lattice squares, the global-memory mesh path
    # for the larger cases
    cfg = synth.SceneConfig(320 + 64 * seed, 240, 64, 6, 0.05, 4.0, 59.0, 2.0, 0.05, seed=seed)
    pair = synth.make_pair(cfg)
    kw = dict(disp_max=63, incon_min_support=0, redun_max_dist=0,
              candidate_stepsize=[5, 4, 3, 5, 4, 6][seed])
    assert run_and_compare(E, pair.left, pair.right, **kw) == []


@pytest.mark.parametrize("mesh_on_host", [0, 1])
@pytest.mark.parametrize("kind", ["vline", "two", "diag", "spot", "hline"])
def test_sparse_support_layouts(E, kind, mesh_on_host):
    # few support points in degenerate layouts: single-point rows (empty
    # bands), a collinear chain, one point, one row
    L, R = synth.sparse_layout_pair(128, 96, kind, 9, seed=3)
    kw = dict(disp_max=31, redun_max_dist=0, incon_min_support=0, candidate_stepsize=10,
              mesh_on_host=mesh_on_host)
    t = ref.process(oracle_params(kw), L, R)
    n = len(t.ptsL)
    assert {"vline": n >= 6, "two": n >= 10, "diag": n >= 6, "spot": n == 1,
            "hline": n >= 8}[kind]
    e, oL, oR = run_pair(E, L, R, **kw)
    assert compare(e, t, oL, oR) == []


@pytest.mark.parametrize("mesh_on_host", [0, 1])
def test_unit_lattice_both_mesh_modes(E, mesh_on_host):
    cfg = synth.SceneConfig(96, 72, 32, 4, 0.05, 4.0, 27.0, 2.0, 0.05, seed=5)
    pair = synth.make_pair(cfg)
    kw = dict(disp_max=31, candidate_stepsize=1, mesh_on_host=mesh_on_host)
    assert run_and_compare(E, pair.left, pair.right, **kw) == []


def test_concurrent_streams_each_frame_bit_exact(E):
    # frames on different streams use separate buffers and overlap on the
    # device; each result must equal the oracle's for its own pair
    dev = torch.device("cuda:0")
    e = E.Elas(disp_max=63)
    cfgs = [synth.QVGA.with_seed(s) for s in (11, 12, 13)]
    pairs = [synth.make_pair(c) for c in cfgs]
    streams = [torch.cuda.Stream(device=dev) for _ in pairs]
    ins = [(torch.from_numpy(p.left).to(dev), torch.from_numpy(p.right).to(dev)) for p in pairs]
    outs = [(torch.empty(p.left.shape, dtype=torch.int16, device=dev),
             torch.empty(p.left.shape, dtype=torch.int16, device=dev)) for p in pairs]
    torch.cuda.synchronize()
    for rep in range(3):
        for (L, R), s, (oL, oR) in zip(ins, streams, outs):
            e.process(L, R, oL, oR, stream=s)
    torch.cuda.synchronize()
    for p, (oL, oR) in zip(pairs, outs):
        t = ref.process(ref.params(disp_max=63), p.left, p.right)
        assert np.array_equal(oL.cpu().numpy(), t.outL)
        assert np.array_equal(oR.cpu().numpy(), t.outR)


# The mesh of the support points alone (add_corners = 0, Section III-A): it is
# built on the host; pixels outside the hull have no plane prior.
@pytest.mark.parametrize("shape", ["320x240", "640x480", "1242x375", "1280x720"])
def test_workload_shapes_without_corners(E, shape):
    cfg = synth.SHAPES[shape]
    pair = synth.make_pair(cfg.with_seed(3))
    kw = dict(disp_max=cfg.disp_range - 1, add_corners=0)
    e, oL, oR = run_pair(E, pair.left, pair.right, **kw)
    t = ref.process(oracle_params(kw), pair.left, pair.right)
    assert (t.ownerL < 0).any() and list(t.cornersL) == [-1] * 4
    assert compare(e, t, oL, oR) == []


@pytest.mark.parametrize("kind", ["vline", "two", "diag", "spot", "hline"])
def test_sparse_support_layouts_without_corners(E, kind):
    # collinear support (vline, hline) and a single point give no triangles:
    # no pixel has a plane prior, the grid vectors alone give candidates
    L, R = synth.sparse_layout_pair(128, 96, kind, 9, seed=3)
    kw = dict(disp_max=31, redun_max_dist=0, incon_min_support=0, candidate_stepsize=10,
              add_corners=0)
    t = ref.process(oracle_params(kw), L, R)
    if kind in ("vline", "hline", "spot"):
        assert len(t.recL) == 0
    e, oL, oR = run_pair(E, L, R, **kw)
    assert compare(e, t, oL, oR) == []


@pytest.mark.parametrize("w,h,D,extra", SMALL[:9])
def test_small_sizes_without_corners(E, w, h, D, extra):
    dmin = extra.get("disp_min", 0)
    cfg = synth.SceneConfig(w, h, max(D, 4), 3, 0.05, 1.0, max(2.0, D - 3.0), 2.0, 0.1,
                            seed=w * 7 + h)
    pair = synth.make_pair(cfg)
    kw = dict(extra, add_corners=0)
    kw["disp_max"] = dmin + D - 1
    e, oL, oR = run_pair(E, pair.left, pair.right, **kw)
    assert compare(e, ref.process(oracle_params(kw), pair.left, pair.right), oL, oR) == []
