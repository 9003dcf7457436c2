"""Parity of the HIP path with the oracle for the embedded variant and the
optional steps: census descriptors with Hamming costs (Section VI-A), the
shift-sum ambiguity test (eq. 3), past-only redundancy (Section VI-C), support
down-sampling (Section VII-B) and the median post-filter (Section VIII).
Every intermediate and both maps must match exactly, in single calls and in
batches that mix parameter sets."""
import numpy as np
import pytest

import synth
from oracle import ref
from test_gpu_parity import compare, oracle_params, run_pair

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def E():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_07210_amd as pkg
    return pkg


def qvga(seed=0):
    return synth.make_pair(synth.QVGA.with_seed(seed))


def check(E, pair, stride=None, **kw):
    print("case", pair.left.shape, kw, flush=True)
    e, oL, oR = run_pair(E, pair.left, pair.right, stride=stride, **kw)
    t = ref.process(oracle_params(kw), pair.left, pair.right)
    assert compare(e, t, oL, oR) == []
    return t, oL


@pytest.mark.parametrize("ws,wd", [(3, 3), (5, 5), (7, 3), (9, 5), (11, 7), (13, 5), (13, 7)])
@pytest.mark.parametrize("amb", [0, 1])
def test_census_windows_bit_exact(E, ws, wd, amb):
    # a 3x3 census has at most 8 set bits: the default texture test (10)
    # would reject every point, so that case runs without it
    t, oL = check(E, qvga(ws), disp_max=63, descriptor=1, census_support_window=ws,
                  census_dense_window=wd, ambiguity=amb, support_texture=10 if ws > 3 else 0)
    assert len(t.ptsL) > 0


def test_census_literal_thresholds_bit_exact(E):
    # no texture tests at all (the paper's census pipeline has none)
    t, oL = check(E, qvga(3), disp_max=63, descriptor=1, ambiguity=1, support_texture=0,
                  match_texture=0)
    assert (oL >= 0).mean() > 0.4


def test_shiftsum_on_gradient_descriptors_bit_exact(E):
    check(E, qvga(4), disp_max=63, ambiguity=1)


@pytest.mark.parametrize("r", [0, 1, 3, 5, 8, 9, 16])
def test_past_only_redundancy_bit_exact(E, r):
    t, _ = check(E, qvga(5), disp_max=63, redundancy=1, redun_max_dist=r)
    if r:
        assert np.count_nonzero(t.dcan_final >= 0) < np.count_nonzero(t.dcan_incon >= 0)


@pytest.mark.parametrize("k", [1, 2, 8, 14, 32, 64])
def test_support_subsample_bit_exact(E, k):
    t, _ = check(E, qvga(6), disp_max=63, support_subsample=k)
    assert len(t.ptsL) == (t.nL_all + k - 1) // k


@pytest.mark.parametrize("win", [1, 3, 5])
def test_median_bit_exact(E, win):
    check(E, qvga(7), disp_max=63, median_window=win)


@pytest.mark.parametrize("mesh_on_host", [0, 1])
@pytest.mark.parametrize("shape", ["640x480", "1242x375"])
def test_embedded_configuration_full_size(E, shape, mesh_on_host):
    # the paper's most accurate KITTI configuration: census 9x9 / 5x5, eq. 3,
    # past-only redundancy, 1/8 of the support points, median filter
    cfg = synth.SHAPES[shape]
    pair = synth.make_pair(cfg)
    t, oL = check(E, pair, disp_max=cfg.disp_range - 1, descriptor=1, census_support_window=9,
                  census_dense_window=5, ambiguity=1, redundancy=1, support_subsample=8,
                  median_window=5, mesh_on_host=mesh_on_host)
    assert (oL >= 0).mean() > 0.4


@pytest.mark.parametrize("w,h", [(9, 9), (12, 10), (97, 61), (131, 77)])
def test_census_small_and_ragged_sizes(E, w, h):
    cfg = synth.SceneConfig(w, h, 16, 3, 0.05, 2.0, 11.0, 2.0, 0.1, seed=w + h)
    pair = synth.make_pair(cfg)
    check(E, pair, disp_max=15, descriptor=1, census_support_window=13, census_dense_window=7,
          ambiguity=1, redundancy=1, support_subsample=3, median_window=3)


def test_census_padded_rows(E):
    check(E, qvga(8), stride=352, disp_max=63, descriptor=1, median_window=3)


def test_census_wide_disparity_range(E):
    cfg = synth.SHAPES["1242x375"].with_seed(9)
    pair = synth.make_pair(cfg)
    check(E, pair, disp_max=255, descriptor=1, census_support_window=13, ambiguity=1)


def test_batch_mixing_variant_and_default_parameters(E):
    dev = torch.device("cuda:0")
    hs = {
        "base": E.Elas(disp_max=63),
        "census": E.Elas(disp_max=63, descriptor=1, ambiguity=1, redundancy=1,
                         support_subsample=8, median_window=5),
        "c13": E.Elas(disp_max=31, descriptor=1, census_support_window=13,
                      census_dense_window=7, median_window=3),
        "sub": E.Elas(disp_max=63, support_subsample=14, redundancy=1),
    }
    kws = {
        "base": dict(disp_max=63),
        "census": dict(disp_max=63, descriptor=1, ambiguity=1, redundancy=1,
                       support_subsample=8, median_window=5),
        "c13": dict(disp_max=31, descriptor=1, census_support_window=13, census_dense_window=7,
                    median_window=3),
        "sub": dict(disp_max=63, support_subsample=14, redundancy=1),
    }
    order = ["census", "base", "c13", "sub", "census", "c13"]
    pairs = []
    for i, name in enumerate(order):
        D = kws[name]["disp_max"] + 1
        w, h = (320, 240) if i % 2 == 0 else (200, 130)
        cfg = synth.SceneConfig(w, h, D, 4, 0.05, 4.0, max(5.0, D - 5.0), 2.0, 0.1, seed=40 + i)
        pairs.append((synth.make_pair(cfg), name))
    for graph, autotune in ((False, False), (True, True)):
        base = hs["base"]
        base.set_batch_flags(graph=graph, autotune=autotune)
        items, outs = [], []
        for p, name in pairs:
            L = torch.from_numpy(p.left).to(dev)
            R = torch.from_numpy(p.right).to(dev)
            oL = torch.full(p.left.shape, -7, dtype=torch.int16, device=dev)
            oR = torch.full(p.left.shape, -7, dtype=torch.int16, device=dev)
            items.append((L, R, oL, oR, hs[name]))
            outs.append((oL, oR))
        torch.cuda.synchronize()
        for _ in range(2):
            base.process_batch(items)
        torch.cuda.synchronize()
        for (p, name), (oL, oR) in zip(pairs, outs):
            t = ref.process(ref.params(**kws[name]), p.left, p.right)
            assert np.array_equal(oL.cpu().numpy(), t.outL), (name, graph)
            assert np.array_equal(oR.cpu().numpy(), t.outR), (name, graph)
