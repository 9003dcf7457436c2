"""A device mesh that gives up is an error, never a silent mesh-less frame.

The flip rounds of the device mesh are capped from the host (a test hook), so
the kernel's own bounded loop stops early and every kernel exits normally.
The failing frame is then matched without plane priors; the library must
report ELAS_ERR_INTERNAL: once, on the next call of the handle (single and
batched calls) or from elas_get_stats, and through the failing ticket of a
server. Afterwards the handle works again and matches the oracle."""
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


def pair_tensors(seed, w=320, h=240, D=64):
    cfg = synth.SceneConfig(w, h, D, 8, 0.05, 4.0, D - 5.0, 2.0, 0.1, seed=seed)
    p = synth.make_pair(cfg)
    dev = torch.device("cuda:0")
    return p, D, torch.from_numpy(p.left).to(dev), torch.from_numpy(p.right).to(dev)


def oracle_equal(p, D, oL, oR):
    t = ref.process(ref.params(disp_max=D - 1), p.left, p.right)
    return np.array_equal(oL.cpu().numpy(), t.outL) and np.array_equal(oR.cpu().numpy(), t.outR)


def test_round_limit_rejects_zero(E):
    e = E.Elas(disp_max=63)
    with pytest.raises(E.ElasError, match="ELAS_ERR_ARG"):
        e.set_mesh_round_limit(0)


def test_single_call_failure_reported_by_stats_and_next_call(E):
    p, D, L, R = pair_tensors(0)
    e = E.Elas(disp_max=D - 1)
    e.set_mesh_round_limit(1)
    e.process(L, R)                      # enqueues; the failure happens on the device
    torch.cuda.synchronize()
    with pytest.raises(E.ElasError, match="ELAS_ERR_INTERNAL"):
        e.stats()
    # the next call reports a failure that finished before it, once
    e.process(L, R)
    torch.cuda.synchronize()
    with pytest.raises(E.ElasError, match="ELAS_ERR_INTERNAL"):
        e.process(L, R)
    torch.cuda.synchronize()
    # back to the default limit: the handle works and matches the oracle (the
    # call that reported the failure did no work of its own)
    e.set_mesh_round_limit(32000)
    oL, oR = e.process(L, R)
    torch.cuda.synchronize()
    st = e.stats()
    assert st["n_tri_left"] > 0 and st["n_tri_right"] > 0
    assert oracle_equal(p, D, oL, oR)


def test_batched_failure_reported_on_the_calling_handle(E):
    dev = torch.device("cuda:0")
    bad = E.Elas(disp_max=63)
    bad.set_mesh_round_limit(1)
    good = E.Elas(disp_max=63)
    base = E.Elas(disp_max=63)
    for graph in (False, True):
        base.set_batch_flags(graph=graph, autotune=False)
        items = []
        for seed, h in ((1, bad), (2, good)):
            p, D, L, R = pair_tensors(seed)
            oL = torch.empty_like(L, dtype=torch.int16)
            oR = torch.empty_like(L, dtype=torch.int16)
            items.append((L, R, oL, oR, h))
        base.process_batch(items)
        torch.cuda.synchronize()
        with pytest.raises(E.ElasError, match="ELAS_ERR_INTERNAL"):
            base.process_batch(items)
        torch.cuda.synchronize()
        # reported once: the handle is usable again (with only good pairs)
        p, D, L, R = pair_tensors(3)
        oL = torch.empty_like(L, dtype=torch.int16)
        oR = torch.empty_like(L, dtype=torch.int16)
        base.process_batch([(L, R, oL, oR, good)])
        torch.cuda.synchronize()
        assert oracle_equal(p, D, oL, oR)
    del dev


def test_server_fails_only_the_failing_ticket(E):
    bad = E.Elas(disp_max=63)
    bad.set_mesh_round_limit(1)
    good = E.Elas(disp_max=63)
    for plain in (False, True):
        srv = E.Server(E.Elas(disp_max=63), max_batch=4, max_inflight=2, plain=plain)
        reqs = []
        for seed, h in ((4, good), (5, bad), (6, good)):
            p, D, L, R = pair_tensors(seed)
            oL = torch.empty_like(L, dtype=torch.int16)
            oR = torch.empty_like(L, dtype=torch.int16)
            reqs.append((p, D, oL, oR, h, srv.submit(L, R, oL, oR, h)))
        for p, D, oL, oR, h, t in reqs:
            if h is bad:
                with pytest.raises(E.ElasError, match="ELAS_ERR_INTERNAL"):
                    srv.wait(t)
            else:
                srv.wait(t)
                assert oracle_equal(p, D, oL, oR)
        srv.close()
