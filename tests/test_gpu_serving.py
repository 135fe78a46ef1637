"""Batched persistent launch and the continuous-batching server on the GPU.

Every output must be bit-identical to the oracle (small images) and to the
same image filtered alone by hrrm_median2d (tolerance 0)."""
import time

import numpy as np
import pytest

import oracle
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


def _mixed_images(seed, n, max_side=300):
    g = np.random.default_rng(seed)
    out = []
    for i in range(n):
        h = int(g.integers(1, max_side))
        w = int(g.integers(1, max_side))
        r = int(g.choice([0, 1, 2, 3, 7, 15, 31]))
        if g.integers(0, 2):
            img = datagen.uniform_u8(h, w, seed=seed * 100 + i)
        else:
            img = datagen.xray_u16(h, w, seed=seed * 100 + i)
        out.append((img, r))
    return out


@pytest.mark.parametrize("use_stream", [False, True])
def test_batched_matches_oracle(hrrm, use_stream):
    import torch
    ctx = hrrm.Context(0)
    stream = torch.cuda.Stream() if use_stream else None
    for rep in range(3):  # graph replays with different batches
        imgs = _mixed_images(10 * rep + int(use_stream), 12)
        announce("batched", "stream" if use_stream else "default", rep,
                 [(i.shape, i.dtype.name, r) for i, r in imgs])
        srcs = [to_dev(i) for i, _ in imgs]
        outs = [torch.empty_like(s) for s in srcs]
        torch.cuda.synchronize()  # inputs were written on the default stream
        ctx.median2d_batched(srcs, [r for _, r in imgs], outs=outs, stream=stream)
        torch.cuda.synchronize()
        for (img, r), o in zip(imgs, outs):
            got = to_host(o)
            want = oracle.median2d(img, r)
            assert np.array_equal(got, want), (img.shape, r, first_mismatch(got, want))


def test_batched_large_mix_equals_alone(hrrm):
    import torch
    ctx = hrrm.Context(0)
    g = np.random.default_rng(5)
    imgs = []
    for i in range(20):
        h, w = int(g.integers(256, 1200)), int(g.integers(256, 1200))
        r = int(g.choice([1, 2, 3, 7, 15, 31]))
        img = datagen.uniform_u8(h, w, seed=i) if i % 2 else datagen.xray_u16(h, w, seed=i)
        imgs.append((img, r))
    srcs = [to_dev(i) for i, _ in imgs]
    outs = [torch.empty_like(s) for s in srcs]
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    ctx.median2d_batched(srcs, [r for _, r in imgs], outs=outs, stream=stream)
    torch.cuda.synchronize()
    for (img, r), s, o in zip(imgs, srcs, outs):
        alone = to_host(ctx.median2d(s, r))
        assert np.array_equal(to_host(o), alone), (img.shape, r)
    # sampled oracle check on the largest image
    k = max(range(len(imgs)), key=lambda i: imgs[i][0].size)
    img, r = imgs[k]
    ys = g.integers(0, img.shape[0], 2000)
    xs = g.integers(0, img.shape[1], 2000)
    assert np.array_equal(to_host(outs[k])[ys, xs], oracle.rank2d_at(img, r, xs, ys))


def test_batched_window_images_only(hrrm):
    # batches whose every image takes the grey-level-window kernel (no
    # persistent launch), of both element types, degenerate shapes included;
    # two batches in a row reuse the staging and flag buffers
    import torch
    ctx = hrrm.Context(0)
    stream = torch.cuda.Stream()
    shapes = [[(1, 1), (64, 1), (2, 300), (130, 257), (300, 64), (33, 65)],
              [(5, 7), (257, 130), (1, 500), (96, 96)]]
    for rep, sh in enumerate(shapes):
        imgs = []
        for i, (h, w) in enumerate(sh):
            if i % 2:
                imgs.append((datagen.uniform_u8(h, w, seed=50 + i + 10 * rep), [1, 7, 15, 24][i % 4]))
            else:
                imgs.append((datagen.xray_u16(h, w, seed=60 + i + 10 * rep), [7, 15, 31, 32][i % 4]))
        announce("batched window-only", rep, [(i.shape, i.dtype.name, r) for i, r in imgs])
        srcs = [to_dev(i) for i, _ in imgs]
        outs = [torch.empty_like(s) for s in srcs]
        torch.cuda.synchronize()
        ctx.median2d_batched(srcs, [r for _, r in imgs], outs=outs, stream=stream)
        torch.cuda.synchronize()
        for (img, r), o in zip(imgs, outs):
            got = to_host(o)
            want = oracle.median2d(img, r)
            assert np.array_equal(got, want), (img.shape, r, first_mismatch(got, want))


def test_batched_large_images_run_alone(hrrm):
    # images large enough to fill the GPU on their own run as single launches
    # inside a batch (window and tiered kernels), the others are packed; every
    # output equals the image filtered alone, and sampled pixels the oracle
    import torch
    ctx = hrrm.Context(0)
    g = np.random.default_rng(12)
    imgs = [(datagen.xray_u16(2048, 4096, seed=90), 15), (datagen.uniform_u8(3000, 3000, seed=91), 3),
            (datagen.xray_u16(1024, 4096, seed=92), 2), (datagen.xray_u16(300, 500, seed=93), 15),
            (datagen.uniform_u8(200, 700, seed=94), 31), (datagen.xray_u16(100, 90, seed=95), 1)]
    announce("batched solo + packed", [(i.shape, i.dtype.name, r) for i, r in imgs])
    srcs = [to_dev(i) for i, _ in imgs]
    outs = [torch.empty_like(s) for s in srcs]
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(2):  # twice: the flag buffers are reused
        ctx.median2d_batched(srcs, [r for _, r in imgs], outs=outs, stream=stream)
        torch.cuda.synchronize()
        for (img, r), s, o in zip(imgs, srcs, outs):
            alone = to_host(ctx.median2d(s, r))
            assert np.array_equal(to_host(o), alone), (img.shape, r)
    for (img, r), o in zip(imgs, outs):
        ys = g.integers(0, img.shape[0], 500)
        xs = g.integers(0, img.shape[1], 500)
        assert np.array_equal(to_host(o)[ys, xs], oracle.rank2d_at(img, r, xs, ys)), (img.shape, r)


def test_batched_persistent_launch(hrrm):
    # enough small images of the tiered kernel's radii (16-bit r <= 3, 8-bit
    # r = 31, r = 0) that the batch packs them into the persistent launch
    import torch
    ctx = hrrm.Context(0)
    g = np.random.default_rng(21)
    imgs = []
    for i in range(24):
        h, w = int(g.integers(1, 260)), int(g.integers(1, 300))
        if i % 3 == 2:
            imgs.append((datagen.uniform_u8(h, w, seed=700 + i), int(g.choice([0, 31]))))
        else:
            imgs.append((datagen.xray_u16(h, w, seed=700 + i), int(g.choice([0, 1, 2, 3]))))
    announce("batched persistent", [(i.shape, i.dtype.name, r) for i, r in imgs])
    srcs = [to_dev(i) for i, _ in imgs]
    outs = [torch.empty_like(s) for s in srcs]
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(2):  # graph replay
        ctx.median2d_batched(srcs, [r for _, r in imgs], outs=outs, stream=stream)
        torch.cuda.synchronize()
        for (img, r), o in zip(imgs, outs):
            got = to_host(o)
            want = oracle.median2d(img, r)
            assert np.array_equal(got, want), (img.shape, r, first_mismatch(got, want))


def test_batched_rejects_bad_image(hrrm):
    import torch
    ctx = hrrm.Context(0)
    a = to_dev(datagen.uniform_u8(10, 10))
    with pytest.raises(hrrm.HrrmError):
        ctx.median2d_batched([a], [200])
    with pytest.raises(hrrm.HrrmError):
        ctx.median2d_batched([a], [-1])


def _run_server(hrrm, imgs, per_image=False, budget=1 << 30):
    ctx = hrrm.Context(0)
    srv = hrrm.Server(ctx, budget, per_image=per_image)
    tickets = [srv.submit(img, r) for img, r in imgs]
    outs = {}
    deadline = time.time() + 60
    while len(outs) < len(tickets):
        for t in tickets:
            if t in outs:
                continue
            res = srv.poll(t)
            if res is not None:
                assert res["status"] == 0
                assert res["t_submit"] <= res["t_admit"] <= res["t_done"]
                outs[t] = srv.fetch(res).numpy()
                srv.release(t)
        assert time.time() < deadline, "server did not finish"
        time.sleep(0.001)
    srv.close()
    return [outs[t] for t in tickets]


@pytest.mark.parametrize("per_image", [False, True])
def test_server_results_mix_equal_alone(hrrm, per_image):
    imgs = _mixed_images(7 + int(per_image), 40)
    announce("server", "per-image" if per_image else "batched", len(imgs))
    got = _run_server(hrrm, imgs, per_image)
    ctx = hrrm.Context(0)
    for (img, r), o in zip(imgs, got):
        alone = to_host(ctx.median2d(to_dev(img), r))
        assert np.array_equal(o, alone), (img.shape, r)
        assert np.array_equal(o, oracle.median2d(img, r)), (img.shape, r)


def test_server_concurrent_clients(hrrm):
    # four client threads submit, poll and release at once while a fifth
    # drains: the worker uploads and launches outside the lock these calls
    # take, and every result must still equal the oracle's
    import threading
    ctx = hrrm.Context(0)
    srv = hrrm.Server(ctx, 1 << 30)
    jobs = [_mixed_images(40 + k, 15) for k in range(4)]
    announce("server", "concurrent clients", [len(j) for j in jobs])
    results = [None] * len(jobs)
    errors = []
    stop = threading.Event()

    def client(k):
        try:
            g = np.random.default_rng(k)
            tickets = []
            for img, r in jobs[k]:
                tickets.append(srv.submit(img, r))
                time.sleep(float(g.uniform(0, 0.002)))
            outs = {}
            deadline = time.time() + 60
            while len(outs) < len(tickets):
                for t in tickets:
                    if t not in outs:
                        res = srv.poll(t)
                        if res is not None:
                            assert res["status"] == 0
                            outs[t] = srv.fetch(res).numpy()
                            srv.release(t)
                assert time.time() < deadline, "server did not finish"
                time.sleep(0.001)
            results[k] = [outs[t] for t in tickets]
        except Exception as e:  # reported by the main thread
            errors.append(e)

    def drainer():
        while not stop.is_set():
            srv.drain(64)
            time.sleep(0.0005)

    threads = [threading.Thread(target=client, args=(k,)) for k in range(len(jobs))]
    d = threading.Thread(target=drainer)
    d.start()
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    stop.set()
    d.join()
    srv.close()
    assert not errors, errors
    for job, got in zip(jobs, results):
        for (img, r), o in zip(job, got):
            assert np.array_equal(o, oracle.median2d(img, r)), (img.shape, r)


def test_server_small_budget_admits_in_turn(hrrm):
    # a budget that holds only a couple of requests at once: later requests wait
    # for earlier outputs to be released, and everything still completes
    imgs = [(datagen.xray_u16(400, 500, seed=i), 5) for i in range(8)]
    got = _run_server(hrrm, imgs, budget=2 * 2 * 400 * 512 * 2 + 4096)
    for (img, r), o in zip(imgs, got):
        assert np.array_equal(o, oracle.median2d(img, r))


def test_server_errors_and_cancel(hrrm):
    ctx = hrrm.Context(0)
    srv = hrrm.Server(ctx, 1 << 20, max_inflight=1, max_queue=2)
    big = datagen.uniform_u8(1024, 1024)
    with pytest.raises(hrrm.HrrmError) as e:
        srv.submit(big, 1)  # input + output exceed the budget: can never fit
    assert e.value.code == hrrm.ENOMEM
    small = datagen.uniform_u8(64, 64)
    t1 = srv.submit(small, 1)
    t2 = srv.submit(small, 1)
    t3 = None
    try:
        t3 = srv.submit(small, 1)
    except hrrm.HrrmError as err:
        assert err.code == hrrm.EAGAIN  # queue of 2 is full (unless t1 was admitted already)
    # with max_inflight = 1, t2 waits until t1 is released: it can be cancelled
    while srv.poll(t1) is None:
        time.sleep(0.001)
    assert srv.cancel(t2) is True
    srv.release(t1)
    if t3 is not None:
        while srv.poll(t3) is None:
            time.sleep(0.001)
        srv.release(t3)
    with pytest.raises(hrrm.HrrmError):
        srv.poll(t2)  # cancelled tickets are gone
    srv.close()
