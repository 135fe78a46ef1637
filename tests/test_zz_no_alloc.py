"""hrrm_rank2d_noalloc (through the C ABI) against hrrm_rank2d on the same
inputs: two calls in a row, the second with a smaller image, for the window
kernel with rows left to the tiered kernel (its tile flags live in the fixed
array), the window kernel alone, the tiered kernel alone, and the adaptive
tree; plus the size limit of the fixed array."""
import numpy as np
import pytest

from gpu_util import announce, first_mismatch, to_dev, to_host
from paper_1105_3829_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hrrm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_3829_amd as m
    m.lib()
    return m


CASES = [
    # name, image maker, r, variant, window_rows (None = default tile)
    ("noise u16, rows left to the tiered kernel", lambda h, w, s: datagen.uniform_u16(h, w, seed=s),
     6, "plain", 8),
    ("x-ray u16, window kernel", lambda h, w, s: datagen.xray_u16(h, w, seed=s), 15, "plain", None),
    ("x-ray u16, tiered kernel", lambda h, w, s: datagen.xray_u16(h, w, seed=s), 4, "plain", None),
    ("x-ray u16 adaptive", lambda h, w, s: datagen.xray_u16(h, w, seed=s), 9, "adaptive", None),
    ("low-key u8", lambda h, w, s: datagen.lowkey_u8(h, w, seed=s), 8, "plain", None),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_rank2d(hrrm, case):
    import torch
    name, make, r, variant, window_rows = case
    ctx = hrrm.Context(0)
    code = None
    for call, (h, w) in enumerate([(300, 520), (130, 200)]):
        img = make(h, w, 500 + call)
        code = hrrm.U16 if img.dtype == np.uint16 else hrrm.U8
        if window_rows is not None:
            ctx.set_tile(code, 2, r, variant, window_rows=window_rows)
        n = (2 * r + 1) ** 2
        for rank in ((n - 1) // 2, n // 5):
            announce("noalloc", name, "call", call, (h, w), "r=%d" % r, "rank=%d" % rank)
            src = to_dev(img)
            want = to_host(ctx.rank2d(src, r, rank=rank, variant=variant))
            out = torch.zeros_like(src)
            got = to_host(ctx.rank2d_noalloc(src, r, rank=rank, variant=variant, out=out))
            assert np.array_equal(got, want), (call, rank, first_mismatch(got, want))
    if window_rows is not None:
        ctx.set_tile(code, 2, r, variant)
    ctx.close()


def test_noalloc_size_limit(hrrm):
    import torch
    ctx = hrrm.Context(0)
    # ceil(w / 256) * ceil(h / 16) tiles: 2 x 32769 > 65536
    src = torch.zeros((16 * 32769, 300), dtype=torch.uint8, device="cuda:0")
    ctx.set_tile(hrrm.U8, 2, 8, "plain", window_rows=16)
    with pytest.raises(hrrm.HrrmError) as ei:
        ctx.rank2d_noalloc(src, 8)
    assert ei.value.code == hrrm.EUNSUPPORTED and "tiles" in str(ei.value)
    ctx.set_tile(hrrm.U8, 2, 8, "plain")
    with pytest.raises(hrrm.HrrmError) as ei:
        ctx.rank2d_noalloc(src[:64], 8, variant="full")
    assert ei.value.code == hrrm.EUNSUPPORTED
    ctx.close()
