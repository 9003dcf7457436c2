"""Integer identities the kernels use in place of divisions (no GPU): a
multiply by a rounded-up reciprocal and a shift must give the exact floor
quotient over the whole range each kernel relies on."""
import numpy as np
import pytest


def ceil_div(a, b):
    return (a + b - 1) // b


@pytest.mark.parametrize("bpf", [2, 3, 5, 7, 480, 1440, 2860, 11520, 40000, 65535, 65536])
def test_batch_frame_index_by_multiply(bpf):
    # frame of block b in a batch of frames with bpf blocks each:
    # umulhi(b, ceil(2^32 / bpf)) == b // bpf whenever b * bpf < 2^32
    bmul = ceil_div(1 << 32, bpf)
    assert bmul < (1 << 32)
    top = ((1 << 32) - 1) // bpf  # the largest b the launcher admits
    b = np.unique(np.concatenate([
        np.arange(0, min(top, 200_000) + 1, dtype=np.uint64),
        np.linspace(0, top, 100_001).astype(np.uint64),
        np.array([top], np.uint64),
        # block indices just below and at every frame boundary near the top
        (np.arange(max(0, top // bpf - 50), top // bpf + 1, dtype=np.uint64) * np.uint64(bpf)),
    ]))
    b = b[b <= top]
    q = (b * np.uint64(bmul)) >> np.uint64(32)
    assert np.array_equal(q, b // np.uint64(bpf))


@pytest.mark.parametrize("w", [9, 97, 320, 640, 1242, 1280, 4096, 8191, 8192])
def test_pixel_row_by_multiply(w):
    # row of pixel index px: (px * ceil(2^40 / w)) >> 40 == px // w while
    # px * w < 2^40, which holds for every image the API admits (w, h <= 8192,
    # so px < 2^26)
    rowmul = ceil_div(1 << 40, w)
    rng = np.random.default_rng(w)
    px = [int(x) for x in rng.integers(0, 1 << 27, 20_000)]
    px += [k * w + r for k in range(0, (1 << 27) // w, max(1, (1 << 27) // w // 500))
           for r in (0, w - 1) if k * w + r < (1 << 27)]
    px += [(1 << 27) - 1]
    for x in px:
        assert (x * rowmul) >> 40 == x // w, (w, x)


@pytest.mark.parametrize("gs", [1, 2, 3, 7, 20, 33, 100])
def test_grid_region_by_multiply(gs):
    # x / grid_size == umulhi(2x, ceil(2^31 / grid_size)) for 0 <= x < 2^31 / grid_size
    gdiv = ceil_div(1 << 31, gs)
    top = (1 << 31) // gs - 1
    x = np.unique(np.concatenate([np.arange(0, min(top, 300_000) + 1, dtype=np.uint64),
                                  np.linspace(0, top, 50_001).astype(np.uint64)]))
    q = ((np.uint64(2) * x) * np.uint64(gdiv)) >> np.uint64(32)
    assert np.array_equal(q, x // np.uint64(gs))
