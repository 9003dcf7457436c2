"""The continuous-batching server: every result equals the oracle's, the
same whether the pair runs alone or in a mix of sizes arriving while others
are on the device; admission respects the memory budget."""
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


SIZES = [(320, 240, 64), (131, 77, 32), (256, 96, 128)]


def requests(n, shift=0):
    dev = torch.device("cuda:0")
    out = []
    for i in range(n):
        w, h, D = SIZES[i % len(SIZES)]
        cfg = synth.SceneConfig(w, h, D, 4, 0.05, 4.0, D - 5.0, 2.0, 0.1, seed=100 + i + shift)
        p = synth.make_pair(cfg)
        L = torch.from_numpy(p.left).to(dev)
        R = torch.from_numpy(p.right).to(dev)
        oL = torch.full((h, w), -9, dtype=torch.int16, device=dev)
        oR = torch.full((h, w), -9, dtype=torch.int16, device=dev)
        out.append((p, D, L, R, oL, oR))
    return out


def oracle_check(reqs):
    for p, D, _, _, oL, oR in reqs:
        t = ref.process(ref.params(disp_max=D - 1), p.left, p.right)
        assert np.array_equal(oL.cpu().numpy(), t.outL)
        assert np.array_equal(oR.cpu().numpy(), t.outR)


def handles(E):
    return {D: E.Elas(disp_max=D - 1) for _, _, D in SIZES}


def test_server_mix_equals_alone_and_oracle(E):
    hs = handles(E)
    base = E.Elas(disp_max=63)
    srv = E.Server(base, max_batch=4, max_inflight=3)
    mix = requests(12)
    torch.cuda.synchronize()
    # two waves: the second arrives while the first is on the device
    tickets = [srv.submit(L, R, oL, oR, hs[D]) for _, D, L, R, oL, oR in mix[:6]]
    tickets += [srv.submit(L, R, oL, oR, hs[D]) for _, D, L, R, oL, oR in mix[6:]]
    lat = [srv.wait(t) for t in tickets]
    assert all(x >= 0 for x in lat)
    st = srv.stats()
    assert st["completed"] == 12 and st["queued"] == 0 and st["bytes_in_flight"] == 0
    mixed = [(oL.clone(), oR.clone()) for *_, oL, oR in mix]
    oracle_check(mix)
    # the same pairs alone, one at a time
    for (_, D, L, R, oL, oR) in mix:
        oL.fill_(-9)
        oR.fill_(-9)
        srv.wait(srv.submit(L, R, oL, oR, hs[D]))
    for (*_, oL, oR), (mL, mR) in zip(mix, mixed):
        assert torch.equal(oL, mL) and torch.equal(oR, mR)
    srv.close()


def test_server_admission_budget(E):
    hs = handles(E)
    base = E.Elas(disp_max=63)
    one = hs[64].frame_bytes(320, 240)
    srv = E.Server(base, max_batch=16, max_inflight=4, memory_budget=int(2.5 * one))
    reqs = [r for r in requests(9) if r[1] == 64]  # the 320x240 pairs
    tickets = [srv.submit(L, R, oL, oR, hs[D]) for _, D, L, R, oL, oR in reqs]
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    assert st["peak_bytes_in_flight"] <= int(2.5 * one)
    assert st["peak_resident_bytes"] <= int(2.5 * one)
    assert st["batches"] >= 2  # at most two 320x240 buffer sets fit at once
    assert st["resident_bytes"] <= int(2.5 * one)
    oracle_check(reqs)
    with pytest.raises(E.ElasError):  # larger than the whole budget
        srv.submit(torch.zeros((1000, 1000), dtype=torch.uint8, device="cuda:0"),
                   torch.zeros((1000, 1000), dtype=torch.uint8, device="cuda:0"),
                   torch.zeros((1000, 1000), dtype=torch.int16, device="cuda:0"),
                   torch.zeros((1000, 1000), dtype=torch.int16, device="cuda:0"), hs[64])
    srv.close()
    # the handles (theirs again once the server is closed) hold what the
    # server accounted for, plus small batch tables
    held = sum(h.device_bytes() for h in hs.values()) + base.device_bytes()
    assert held <= st["resident_bytes"] + (1 << 20)


def test_server_plain_mode(E):
    hs = handles(E)
    base = E.Elas(disp_max=63)
    srv = E.Server(base, plain=True)
    reqs = requests(6, shift=20)
    tickets = [srv.submit(L, R, oL, oR, hs[D]) for _, D, L, R, oL, oR in reqs]
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    assert st["batches"] == 6 and st["batched_pairs"] == 6
    oracle_check(reqs)
    srv.close()


def test_server_poll_and_unknown_ticket(E):
    hs = handles(E)
    base = E.Elas(disp_max=63)
    srv = E.Server(base, max_batch=8, max_inflight=2)
    _, D, L, R, oL, oR = requests(1, shift=40)[0]
    t = srv.submit(L, R, oL, oR, hs[D])
    got = None
    for _ in range(100000):
        got = srv.poll(t)
        if got is not None:
            break
    if got is None:
        got = srv.wait(t)
    assert got >= 0
    with pytest.raises(E.ElasError):
        srv.wait(t)  # a ticket is reported once
    srv.close()


def test_server_budget_with_full_size_frames(E):
    # the four full workload shapes under a budget of three 1280x720 buffer
    # sets: new sets are admitted against the budget, idle streams' sets are
    # released when the oldest pair needs room, and what the library holds
    # never exceeds it; every result equals the oracle's
    import synth as S
    names = list(S.SHAPES)
    hs = {S.SHAPES[n].disp_range: E.Elas(disp_max=S.SHAPES[n].disp_range - 1) for n in names}
    base = E.Elas(disp_max=127)
    big = hs[192].frame_bytes(1280, 720)
    budget = 3 * big
    srv = E.Server(base, max_batch=8, max_inflight=3, memory_budget=budget)
    dev = torch.device("cuda:0")
    reqs = []
    for k in range(12):
        cfg = S.SHAPES[names[k % 4]].with_seed(500 + k)
        p = S.make_pair(cfg)
        L = torch.from_numpy(p.left).to(dev)
        R = torch.from_numpy(p.right).to(dev)
        oL = torch.full(p.left.shape, -9, dtype=torch.int16, device=dev)
        oR = torch.full(p.left.shape, -9, dtype=torch.int16, device=dev)
        reqs.append((p, cfg.disp_range, L, R, oL, oR))
    tickets = [srv.submit(L, R, oL, oR, hs[D]) for _, D, L, R, oL, oR in reqs]
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    assert st["completed"] == 12
    assert st["peak_resident_bytes"] <= budget
    srv.close()
    held = sum(h.device_bytes() for h in hs.values()) + base.device_bytes()
    assert held <= st["resident_bytes"] + (1 << 20) <= budget + (1 << 20)
    for p, D, _, _, oL, oR in reqs:
        t = ref.process(ref.params(disp_max=D - 1), p.left, p.right)
        assert np.array_equal(oL.cpu().numpy(), t.outL)
        assert np.array_equal(oR.cpu().numpy(), t.outR)
