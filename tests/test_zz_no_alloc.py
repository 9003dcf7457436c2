"""elas_process_noalloc, the entry point that allocates nothing, called
through the C-ABI: its maps equal elas_process's bit for bit (and so the
oracle's) on two calls in a row, the second with a smaller frame, so the
scratch array's leftovers from the larger frame cannot leak into the
smaller one. Frames above the array's limit are refused before any work."""
import ctypes as C

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


def call_noalloc(E, e, L, R, oL, oR, stream):
    H, W = L.shape
    rc = E.elas.lib().elas_process_noalloc(
        e.handle, C.c_void_p(L.data_ptr()), C.c_void_p(R.data_ptr()), W, H, L.stride(0),
        C.c_void_p(stream.cuda_stream), C.c_void_p(oL.data_ptr()), C.c_void_p(oR.data_ptr()))
    return rc


def test_noalloc_equals_process_large_then_small(E):
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    cases = [(synth.HD.with_seed(3), 192), (synth.QVGA.with_seed(4), 64)]
    for cfg, D in cases:
        p = synth.make_pair(cfg)
        print(f"noalloc: {cfg.width}x{cfg.height} D={D}", flush=True)
        L = torch.from_numpy(p.left).to(dev)
        R = torch.from_numpy(p.right).to(dev)
        e = E.Elas(disp_max=D - 1)
        refL, refR = e.process(L, R)
        torch.cuda.synchronize()
        oL = torch.full_like(refL, -9)
        oR = torch.full_like(refR, -9)
        torch.cuda.synchronize()
        assert call_noalloc(E, e, L, R, oL, oR, stream) == 0, E.elas.lib().elas_last_error(e.handle)
        stream.synchronize()
        assert torch.equal(oL, refL) and torch.equal(oR, refR)
        st = e.stats()  # reads the scratch array's header and counts
        t = ref.process(ref.params(disp_max=D - 1), p.left, p.right)
        assert np.array_equal(oL.cpu().numpy(), t.outL)
        assert np.array_equal(oR.cpu().numpy(), t.outR)
        assert st["dense_evals"] == t.dense_evals and st["n_tri_left"] == len(t.recL)
        assert np.array_equal(e.intermediate("raw_left").reshape(t.rawL.shape), t.rawL)


def test_noalloc_rejects_frames_above_the_limit(E):
    e = E.Elas(disp_max=255)
    dev = torch.device("cuda:0")
    img = torch.zeros((4096, 4096), dtype=torch.uint8, device=dev)
    out = torch.zeros((4096, 4096), dtype=torch.int16, device=dev)
    rc = call_noalloc(E, e, img, img, out, out, torch.cuda.current_stream(dev))
    assert rc == -1
    assert b"scratch" in E.elas.lib().elas_last_error(e.handle)
    e2 = E.Elas(disp_max=63, mesh_on_host=1)
    small = torch.zeros((64, 64), dtype=torch.uint8, device=dev)
    so = torch.zeros((64, 64), dtype=torch.int16, device=dev)
    assert call_noalloc(E, e2, small, small, so, so, torch.cuda.current_stream(dev)) == -4
