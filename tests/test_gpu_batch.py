"""GPU parity of the batched codec (dct_batch_plan / dct_batch_run): every image
of a batch of uneven sizes and quality scales, bit for bit against the oracle,
for both chunk sizes and for one-workgroup-per-chunk and persistent grids;
replays of a captured HIP graph; and the tuner's choice."""
import sys

import numpy as np
import pytest


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hip():
    from paper_1306_1373_amd import codec
    codec.load()
    return codec


def make_batch(n, seed, max_side=400):
    import torch
    from paper_1306_1373_amd.synth import synth_image
    rng = np.random.default_rng(seed)
    imgs, srcs, dsts, qs = [], [], [], []
    sizes = [(1, 1), (8, 8), (9, 7), (max_side, 3)] + [tuple(int(v) for v in rng.integers(1, max_side + 1, 2))
                                                      for _ in range(n - 4)]
    for k, (W, H) in enumerate(sizes):
        img = synth_image(W, H, 500 + k, float(rng.uniform(0, 10)))
        pitch = ((W + 7) // 8) * 8 + 8 * int(rng.integers(0, 3))
        buf = torch.full((H, pitch), 0xA5, dtype=torch.uint8, device="cuda")
        buf[:, :W] = torch.from_numpy(img).cuda()
        out = torch.full((H, pitch + 8), 0x5A, dtype=torch.uint8, device="cuda")
        imgs.append(img)
        srcs.append(buf[:, :W])
        dsts.append(out[:, :W])
        qs.append(int(rng.choice([1, 2, 4, 8, 16, 1024])))
    return imgs, srcs, dsts, qs


def check(oracle_mod, imgs, dsts, qs, sse):
    sse = sse.cpu().numpy()
    for k, (img, d, q) in enumerate(zip(imgs, dsts, qs)):
        rec, s = oracle_mod.cordic_codec(img, q)
        full = d.as_strided((d.shape[0], d.stride(0)), (d.stride(0), 1)).cpu().numpy()
        assert np.array_equal(full[:, :img.shape[1]], rec), k
        assert np.all(full[:, img.shape[1]:] == 0x5A), k          # pad untouched
        assert int(sse[k]) == s, k


@pytest.mark.parametrize("chunk,threads,grid", [(512, None, 0), (256, None, 0), (512, None, 3), (256, None, 7),
                                               (1024, 256, 0), (2048, 512, 5), (1024, 512, 0), (512, 256, 9)])
def test_batch_bit_exact(hip, oracle_mod, chunk, threads, grid):
    # every tile size and workgroup size: a workgroup of `threads` lanes codes a
    # tile of `chunk` blocks in chunk / threads passes
    imgs, srcs, dsts, qs = make_batch(40, 90 + chunk + grid)
    batch = hip.Batch(srcs, dsts, qs, chunk=chunk)
    sse = batch.run(grid, threads=threads)
    check(oracle_mod, imgs, dsts, qs, sse)
    say(f"[gpu] batch chunk {chunk} threads {threads} grid {grid}: {batch.total_chunks} chunks, "
        f"{len(imgs)} images exact")
    batch.release()


def test_batch_matches_single_image_calls(hip):
    imgs, srcs, dsts, qs = make_batch(12, 7, max_side=1100)
    batch = hip.Batch(srcs, dsts, qs)
    sse = batch.run().cpu().numpy()
    for k, (s, q) in enumerate(zip(srcs, qs)):
        d, s1 = hip.dct_codec(s, q)
        assert np.array_equal(d.cpu().numpy(), dsts[k].cpu().numpy())
        assert int(s1.cpu()[0]) == int(sse[k])


def test_batch_graph_replays(hip, oracle_mod):
    import torch
    imgs, srcs, dsts, qs = make_batch(24, 31)
    batch = hip.Batch(srcs, dsts, qs)
    eager = batch.run().clone()
    ref = [d.cpu().numpy().copy() for d in dsts]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        sse_g = torch.zeros_like(eager)
        with torch.cuda.graph(graph, stream=side):
            batch.run(sse=sse_g)
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(3):
        for d in dsts:
            d.fill_(rep + 1)                      # the replay must rewrite every pixel
        sse_g.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(sse_g, eager), rep
        for d, r in zip(dsts, ref):
            assert np.array_equal(d.cpu().numpy(), r), rep
        _ = (eager.float() * 2).sum().item()     # eager work between replays
    check(oracle_mod, imgs, dsts, qs, sse_g)


def test_unplanned_workspace_rejected(hip):
    import ctypes as C
    import torch
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda")
    sse = torch.zeros(4, dtype=torch.int64, device="cuda")
    assert hip.load().dct_batch_run(C.c_void_p(ws.data_ptr()), 0, C.c_void_p(sse.data_ptr()), None) == \
        hip.DCT_ERR_INVALID
    imgs, srcs, dsts, qs = make_batch(5, 3)
    batch = hip.Batch(srcs, dsts, qs, chunk=256)
    for bad in (128, 512, 1024):          # not 256 or 512, or more lanes than the tile
        with pytest.raises(hip.DctError):
            batch.run(threads=bad)
    batch.release()
    with pytest.raises(hip.DctError):
        batch.run()


def test_tuner_returns_a_measured_configuration(hip, oracle_mod):
    from paper_1306_1373_amd.autotune import tune_batch
    imgs, srcs, dsts, qs = make_batch(30, 17, max_side=900)
    res, batch = tune_batch(srcs, dsts, qs, grids=(0, 64, 512), reps=2)
    assert (res.chunk, res.threads, res.grid) in res.table and res.ms == min(res.table.values())
    assert len(res.table) == 21         # tiles 256: one lane count; 512, 1024, 2048: two; three grids each
    sse = batch.run(res.grid, threads=res.threads)
    check(oracle_mod, imgs, dsts, qs, sse)
