"""Exhaustive tiny images on the GPU: every 2x3 and 3x2 image over a
three-value alphabet (the extremes and a middle value), 8- and 16-bit, for
r = 0..3, through the single-image entry point and the batched launch, each
compared bit for bit with the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import announce, to_dev, to_host
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


@pytest.mark.parametrize("dt,alphabet", [(np.uint8, (0, 128, 255)),
                                         (np.uint16, (0, 4095, 65535))])
@pytest.mark.parametrize("shape", [(2, 3), (3, 2)])
def test_every_tiny_image(hrrm, dt, alphabet, shape):
    import torch
    imgs = datagen.enumerate_images(shape[0], shape[1], alphabet).astype(dt)
    srcs = [to_dev(i) for i in imgs]
    for r in range(4):
        announce("exhaustive", dt.__name__, shape, "r=%d" % r, len(imgs))
        want = [oracle.median2d(i, r) for i in imgs]
        outs = hrrm.median2d_batched(srcs, [r] * len(srcs))
        torch.cuda.synchronize()
        bad = [k for k, (o, w) in enumerate(zip(outs, want)) if not np.array_equal(to_host(o), w)]
        assert not bad, ("batched", r, imgs[bad[0]], to_host(outs[bad[0]]), want[bad[0]])
        for k in range(0, len(imgs), 37):  # a spread of single-image launches
            got = to_host(hrrm.median2d(srcs[k], r))
            assert np.array_equal(got, want[k]), ("single", r, imgs[k], got, want[k])
