"""Stream capture: after hrrm_ctx_reserve, median calls recorded into a HIP
graph (through torch.cuda.graph) give the eager results on every replay, with
eager work on the same buffers between the replays."""
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


def test_captured_calls_replay_like_eager(hrrm):
    import torch
    ctx = hrrm.Context(0)
    img16 = to_dev(datagen.xray_u16(300, 700, seed=170))
    img8 = to_dev(datagen.lowkey_u8(250, 600, seed=171))
    ctx.reserve(hrrm.U16, img16.numel(), 9, "adaptive")
    cases = [("u16 plain", img16, "plain"), ("u16 adaptive", img16, "adaptive"),
             ("u8 plain", img8, "plain"), ("u8 full", img8, "full")]
    want = {name: to_host(ctx.median2d(src, 9, variant=v)) for name, src, v in cases}
    outs = {name: torch.empty_like(src) for name, src, _ in cases}
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on a side stream before capture
        for name, src, v in cases:
            ctx.median2d(src, 9, variant=v, out=outs[name])
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    announce("capture")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for name, src, v in cases:
            ctx.median2d(src, 9, variant=v, out=outs[name])
    for rep in range(3):
        for o in outs.values():
            o.zero_()
        ctx.median2d(img8, 2, out=torch.empty_like(img8))  # unrelated eager work
        torch.cuda.synchronize()
        announce("replay", rep)
        g.replay()
        torch.cuda.synchronize()
        for name, o in outs.items():
            got = to_host(o)
            assert np.array_equal(got, want[name]), (rep, name, first_mismatch(got, want[name]))


def test_capture_without_warmup_after_reserve(hrrm):
    # reserve raises every kernel build's LDS limit, so calls captured with no
    # eager call before them (builds for six, four and three workgroups per
    # CU, 3-D, wave-private slots) record only launches
    import torch
    ctx = hrrm.Context(0)
    img16 = to_dev(datagen.xray_u16(200, 600, seed=172))
    img8 = to_dev(datagen.lowkey_u8(180, 520, seed=173))
    vol = to_dev(datagen.xray_volume_u16(4, 40, 300, seed=174))
    ctx.reserve(hrrm.U16, img16.numel(), 12, "plain")
    c = ctx.get_tile(hrrm.U16, 2, 12)
    c.wave_slots = 1
    ctx.set_tile(hrrm.U16, 2, 12, "plain", c)
    calls = [("u16 r=2", lambda o: ctx.median2d(img16, 2, out=o), img16),
             ("u8 r=3", lambda o: ctx.median2d(img8, 3, out=o), img8),
             ("u8 r=20", lambda o: ctx.median2d(img8, 20, out=o), img8),
             ("u16 r=12 wave slots", lambda o: ctx.median2d(img16, 12, out=o), img16),
             ("3-D r=1", lambda o: ctx.median3d(vol, 1, out=o), vol)]
    outs = {name: torch.empty_like(src) for name, _, src in calls}
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    announce("capture without warm-up")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        for name, fn, _ in calls:
            fn(outs[name])
    want = {}
    for name, fn, src in calls:
        o = torch.empty_like(src)
        fn(o)
        want[name] = to_host(o)
    for rep in range(2):
        for o in outs.values():
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for name, o in outs.items():
            got = to_host(o)
            assert np.array_equal(got, want[name]), (rep, name, first_mismatch(got, want[name]))
    ctx.set_tile(hrrm.U16, 2, 12, "plain", None)
