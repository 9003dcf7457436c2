"""Batched processing (one launch per stage for many pairs of mixed sizes and
disparity ranges, graph capture and replay, tile autotuning): every pair's
maps must equal the oracle's for that pair, exactly."""
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


# (w, h, D, seed): sizes, ragged tiles and several disparity ranges
MIX = [(320, 240, 64, 0), (97, 61, 64, 1), (200, 120, 32, 2), (320, 240, 64, 3),
       (131, 77, 128, 4), (256, 96, 256, 5), (97, 61, 64, 6)]


def make_mix(seed_shift=0):
    pairs = []
    for w, h, D, seed in MIX:
        cfg = synth.SceneConfig(w, h, D, 4, 0.05, 4.0, max(5.0, D - 5.0), 2.0, 0.1,
                                seed=seed + seed_shift)
        pairs.append((synth.make_pair(cfg), D))
    return pairs


def run_batch(E, pairs, graph, autotune, reps=1, stream=None, handles=None):
    dev = torch.device("cuda:0")
    base = E.Elas(disp_max=63) if handles is None else handles[64]
    base.set_batch_flags(graph=graph, autotune=autotune)
    hs = handles if handles is not None else {D: E.Elas(disp_max=D - 1) for D in {64, 32, 128, 256}}
    items, outs = [], []
    for p, D in pairs:
        L = torch.from_numpy(p.left).to(dev)
        R = torch.from_numpy(p.right).to(dev)
        oL = torch.full(p.left.shape, -7, dtype=torch.int16, device=dev)
        oR = torch.full(p.left.shape, -7, dtype=torch.int16, device=dev)
        items.append((L, R, oL, oR, hs[D]))
        outs.append((oL, oR))
    torch.cuda.synchronize()
    for _ in range(reps):
        base.process_batch(items, stream=stream)
    torch.cuda.synchronize()
    return [(a.cpu().numpy(), b.cpu().numpy()) for a, b in outs], base, hs


def check(pairs, got):
    for (p, D), (oL, oR) in zip(pairs, got):
        t = ref.process(ref.params(disp_max=D - 1), p.left, p.right)
        assert np.array_equal(oL, t.outL), (p.left.shape, D)
        assert np.array_equal(oR, t.outR), (p.left.shape, D)


@pytest.mark.parametrize("graph,autotune", [(False, False), (True, False), (False, True),
                                            (True, True)])
def test_batch_mixed_sizes_bit_exact(E, graph, autotune):
    pairs = make_mix()
    got, base, hs = run_batch(E, pairs, graph, autotune, reps=2)
    check(pairs, got)
    if autotune:  # the batch handle keeps the choice per (w, h, D); it has D = 64
        for p, D in pairs:
            if D == 64:
                h, w = p.left.shape
                rows, batch, run = base.tuned_variants(w, h)
                assert rows in (4, 8, 16) and batch in (1, 2, 4)  # dense rows per block
                assert run in (16, 32)  # support lattice points per block


def test_uniform_and_mixed_batches_alternate_on_one_handle(E):
    # equal frames find a block's frame by a multiply, mixed ones by search;
    # each batch shape keeps its own captured graph, replayed in turn
    uni = []
    for i in range(4):
        cfg = synth.SceneConfig(320, 240, 64, 4, 0.05, 4.0, 59.0, 2.0, 0.1, seed=40 + i)
        uni.append((synth.make_pair(cfg), 64))
    mix = make_mix(seed_shift=20)
    want = {}
    for name, pairs in (("uni", uni), ("mix", mix)):
        want[name] = [ref.process(ref.params(disp_max=D - 1), p.left, p.right) for p, D in pairs]
    handles = {D: E.Elas(disp_max=D - 1) for D in {64, 32, 128, 256}}
    for rep in range(2):
        for name, pairs in (("uni", uni), ("mix", mix)):
            got, _, _ = run_batch(E, pairs, True, False, handles=handles)
            for (p, D), t, (oL, oR) in zip(pairs, want[name], got):
                assert np.array_equal(oL, t.outL), (name, rep, p.left.shape, D)
                assert np.array_equal(oR, t.outR), (name, rep, p.left.shape, D)


def test_batch_graph_replay_with_new_inputs(E):
    # the same batch shape replays its captured graph; the frame table is
    # uploaded per call, so new images and outputs are picked up
    dev = torch.device("cuda:0")
    hs = {D: E.Elas(disp_max=D - 1) for D in {64, 32, 128, 256}}
    for shift in (0, 100, 200):
        pairs = make_mix(shift)
        got, _, _ = run_batch(E, pairs, True, shift > 0, handles=hs)
        check(pairs, got)


def test_timed_batch_reports_stage_times_and_same_maps(E):
    # with timing on, the batch is launched directly with events around each
    # launch: the maps still equal the oracle's, every stage of the path has a
    # positive time, and the stage times fit in the span
    hs = {D: E.Elas(disp_max=D - 1) for D in {64, 32, 128, 256}}
    base = hs[64]
    base.set_timing(True)
    pairs = make_mix(11)
    got, _, _ = run_batch(E, pairs, True, False, handles=hs)
    check(pairs, got)
    t = base.timing()
    stages = ["descriptor", "support", "filter", "rows", "mesh", "raster", "dense", "lrcheck"]
    for s in stages:
        assert t[s + "_ms"] > 0.0, s
    assert sum(t[s + "_ms"] for s in stages) <= t["device_span_ms"] * 1.001 + 1e-3
    assert t["host_wait_ms"] == 0.0 and t["host_mesh_ms"] == 0.0
    # a plain call afterwards reports its own stages again
    dev = torch.device("cuda:0")
    p, D = pairs[0]
    hs[D].set_timing(True)
    hs[D].process(torch.from_numpy(p.left).to(dev), torch.from_numpy(p.right).to(dev))
    t1 = hs[D].timing()
    assert t1["dense_ms"] > 0.0 and t1["device_span_ms"] > 0.0


def test_batch_equals_single_calls(E):
    dev = torch.device("cuda:0")
    pairs = make_mix(7)
    got, _, hs = run_batch(E, pairs, True, True)
    for (p, D), (oL, oR) in zip(pairs, got):
        L = torch.from_numpy(p.left).to(dev)
        R = torch.from_numpy(p.right).to(dev)
        sL, sR = hs[D].process(L, R)
        torch.cuda.synchronize()
        assert np.array_equal(sL.cpu().numpy(), oL)
        assert np.array_equal(sR.cpu().numpy(), oR)


@pytest.mark.parametrize("graph", [False, True])
def test_batch_of_one_pair(E, graph):
    # one frame: its block count is the whole grid, and every block finds
    # frame 0 by the multiply
    for (w, h, D, seed) in [(320, 240, 64, 3), (97, 61, 64, 6), (256, 96, 256, 5)]:
        cfg = synth.SceneConfig(w, h, D, 4, 0.05, 4.0, max(5.0, D - 5.0), 2.0, 0.1, seed=seed)
        pairs = [(synth.make_pair(cfg), D)]
        got, _, _ = run_batch(E, pairs, graph, False, reps=2)
        check(pairs, got)


def test_batch_of_many_equal_small_pairs(E):
    # 48 frames of one shape in one call: the frame of a block by the
    # multiply, across many frame boundaries
    pairs = []
    for i in range(48):
        cfg = synth.SceneConfig(97, 61, 64, 4, 0.05, 4.0, 59.0, 2.0, 0.1, seed=200 + i)
        pairs.append((synth.make_pair(cfg), 64))
    got, _, _ = run_batch(E, pairs, True, False, reps=2)
    check(pairs, got)


def test_batch_with_host_mesh_pairs(E):
    # a pair wider than the device mesh limit goes through the host mesh path
    dev = torch.device("cuda:0")
    wide = synth.SceneConfig(4100, 12, 32, 3, 0.05, 2.0, 27.0, 2.0, 0.1, seed=3)
    small = synth.SceneConfig(96, 64, 32, 3, 0.05, 2.0, 27.0, 2.0, 0.1, seed=4)
    pairs = [(synth.make_pair(wide), 32), (synth.make_pair(small), 32)]
    hs = {32: E.Elas(disp_max=31)}
    base = hs[32]
    base.set_batch_flags(graph=True, autotune=False)
    items, outs = [], []
    for p, D in pairs:
        L = torch.from_numpy(p.left).to(dev)
        R = torch.from_numpy(p.right).to(dev)
        oL = torch.empty(p.left.shape, dtype=torch.int16, device=dev)
        oR = torch.empty(p.left.shape, dtype=torch.int16, device=dev)
        items.append((L, R, oL, oR))
        outs.append((oL, oR))
    base.process_batch(items)
    torch.cuda.synchronize()
    check(pairs, [(a.cpu().numpy(), b.cpu().numpy()) for a, b in outs])


def test_batches_on_two_streams_concurrently(E):
    dev = torch.device("cuda:0")
    hs = {D: E.Elas(disp_max=D - 1) for D in {64, 32, 128, 256}}
    s1, s2 = torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)
    p1, p2 = make_mix(11), make_mix(12)
    base = hs[64]
    base.set_batch_flags(graph=True, autotune=False)

    def items_of(pairs):
        its, outs = [], []
        for p, D in pairs:
            L = torch.from_numpy(p.left).to(dev)
            R = torch.from_numpy(p.right).to(dev)
            oL = torch.empty(p.left.shape, dtype=torch.int16, device=dev)
            oR = torch.empty(p.left.shape, dtype=torch.int16, device=dev)
            its.append((L, R, oL, oR, hs[D]))
            outs.append((oL, oR))
        return its, outs

    i1, o1 = items_of(p1)
    i2, o2 = items_of(p2)
    torch.cuda.synchronize()
    for _ in range(2):
        base.process_batch(i1, stream=s1)
        base.process_batch(i2, stream=s2)
    torch.cuda.synchronize()
    check(p1, [(a.cpu().numpy(), b.cpu().numpy()) for a, b in o1])
    check(p2, [(a.cpu().numpy(), b.cpu().numpy()) for a, b in o2])


@pytest.mark.parametrize("graph", [False, True])
def test_batch_sparse_support_layouts(E, graph):
    # degenerate support layouts (empty bands, a collinear chain, one point,
    # one row) next to an ordinary pair in one batched call, through the
    # batched device mesh; each pair's maps equal the oracle's
    dev = torch.device("cuda:0")
    sparse = dict(disp_max=31, redun_max_dist=0, incon_min_support=0, candidate_stepsize=10)
    plain = dict(disp_max=63)
    hs, hp = E.Elas(**sparse), E.Elas(**plain)
    cases = [(synth.sparse_layout_pair(128, 96, k, 9, seed=3), sparse, hs)
             for k in ("vline", "two", "diag", "spot", "hline")]
    p = synth.make_pair(synth.SceneConfig(160, 96, 64, 4, 0.05, 4.0, 59.0, 2.0, 0.1, seed=21))
    cases.append(((p.left, p.right), plain, hp))
    hp.set_batch_flags(graph=graph, autotune=False)
    items, outs = [], []
    for (left, right), _, h in cases:
        L = torch.from_numpy(left).to(dev)
        R = torch.from_numpy(right).to(dev)
        oL = torch.full(left.shape, -7, dtype=torch.int16, device=dev)
        oR = torch.full(left.shape, -7, dtype=torch.int16, device=dev)
        items.append((L, R, oL, oR, h))
        outs.append((oL, oR))
    for _ in range(2):
        hp.process_batch(items)
    torch.cuda.synchronize()
    for ((left, right), kw, _), (oL, oR) in zip(cases, outs):
        t = ref.process(ref.params(**kw), left, right)
        assert np.array_equal(oL.cpu().numpy(), t.outL), kw
        assert np.array_equal(oR.cpu().numpy(), t.outR), kw


def test_batch_argument_errors(E):
    e = E.Elas(disp_max=63)
    with pytest.raises(E.ElasError):
        e.process_batch([(torch.zeros((4, 4), dtype=torch.uint8, device="cuda:0"),
                          torch.zeros((4, 4), dtype=torch.uint8, device="cuda:0"),
                          torch.zeros((4, 4), dtype=torch.int16, device="cuda:0"),
                          torch.zeros((4, 4), dtype=torch.int16, device="cuda:0"))])
    e.process_batch([])  # an empty batch is a no-op


def test_batch_with_pairs_meshed_without_corners(E):
    # pairs whose handle meshes the support points alone go through the host
    # mesh path inside the batch, next to device-meshed pairs
    dev = torch.device("cuda:0")
    hc = E.Elas(disp_max=63)
    hn = E.Elas(disp_max=63, add_corners=0)
    hc.set_batch_flags(graph=True, autotune=False)
    pairs = make_mix(30)[:4]
    items, outs, want = [], [], []
    for k, (p, D) in enumerate(pairs):
        if D != 64:
            continue
        for h, ac in ((hc, 1), (hn, 0)):
            L = torch.from_numpy(p.left).to(dev)
            R = torch.from_numpy(p.right).to(dev)
            oL = torch.full(p.left.shape, -7, dtype=torch.int16, device=dev)
            oR = torch.full(p.left.shape, -7, dtype=torch.int16, device=dev)
            items.append((L, R, oL, oR, h))
            outs.append((oL, oR))
            want.append((p, ac))
    torch.cuda.synchronize()
    for _ in range(2):
        hc.process_batch(items)
    torch.cuda.synchronize()
    for (p, ac), (oL, oR) in zip(want, outs):
        t = ref.process(ref.params(disp_max=63, add_corners=ac), p.left, p.right)
        assert np.array_equal(oL.cpu().numpy(), t.outL), ac
        assert np.array_equal(oR.cpu().numpy(), t.outR), ac


@pytest.mark.parametrize("run", [8, 16, 32])
def test_support_run_lengths_bit_exact(E, run):
    # the support stage's lattice points per workgroup, fixed per size: single
    # calls and a batch give the oracle's maps with each
    dev = torch.device("cuda:0")
    pairs = make_mix(40)
    hs = {D: E.Elas(disp_max=D - 1) for D in {64, 32, 128, 256}}
    for p, D in pairs:
        h, w = p.left.shape
        hs[D].set_tile_variants(w, h, 8, 2, run)
        assert hs[D].tuned_variants(w, h) == (8, 2, run)
    got, _, _ = run_batch(E, pairs, True, False, handles=hs)
    check(pairs, got)
    p, D = pairs[5]
    L = torch.from_numpy(p.left).to(dev)
    R = torch.from_numpy(p.right).to(dev)
    sL, sR = hs[D].process(L, R)
    torch.cuda.synchronize()
    t = ref.process(ref.params(disp_max=D - 1), p.left, p.right)
    assert np.array_equal(sL.cpu().numpy(), t.outL)
    assert np.array_equal(sR.cpu().numpy(), t.outR)


@pytest.mark.parametrize("graph", [False, True])
def test_dense_support_many_triangles_per_band(E, graph):
    # a unit lattice with the support filters off keeps ~12 k points and
    # ~24 k triangles per view, ~1200-1400 of them over every 4-row raster
    # band: the batched raster gathers and rasterises each band in several
    # passes, the single-frame raster in many gather steps. Batched (beside an
    # ordinary pair) and single calls both give the oracle's maps.
    dev = torch.device("cuda:0")
    dense = dict(disp_max=31, candidate_stepsize=1, redun_max_dist=0, incon_min_support=0)
    plain = dict(disp_max=63)
    hd, hp = E.Elas(**dense), E.Elas(**plain)
    pd = synth.make_pair(synth.SceneConfig(160, 120, 32, 4, 0.05, 4.0, 27.0, 2.0, 0.05, seed=5))
    pp = synth.make_pair(synth.SceneConfig(160, 96, 64, 4, 0.05, 4.0, 59.0, 2.0, 0.1, seed=21))
    cases = [(pd, dense, hd), (pp, plain, hp)]
    hp.set_batch_flags(graph=graph, autotune=False)
    items, outs = [], []
    for p, _, h in cases:
        L = torch.from_numpy(p.left).to(dev)
        R = torch.from_numpy(p.right).to(dev)
        oL = torch.full(p.left.shape, -7, dtype=torch.int16, device=dev)
        oR = torch.full(p.left.shape, -7, dtype=torch.int16, device=dev)
        items.append((L, R, oL, oR, h))
        outs.append((oL, oR))
    for _ in range(2):
        hp.process_batch(items)
    sL, sR = hd.process(items[0][0], items[0][1])
    torch.cuda.synchronize()
    refs = [ref.process(ref.params(**kw), p.left, p.right) for p, kw, _ in cases]
    assert len(refs[0].recL) > 20000 and len(refs[0].recR) > 20000
    for t, (oL, oR) in zip(refs, outs):
        assert np.array_equal(oL.cpu().numpy(), t.outL)
        assert np.array_equal(oR.cpu().numpy(), t.outR)
    assert np.array_equal(sL.cpu().numpy(), refs[0].outL)
    assert np.array_equal(sR.cpu().numpy(), refs[0].outR)
