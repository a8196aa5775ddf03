"""Launch-shape tuner for the batched codec (dct_batch_run_threads).

The batched kernel has three free launch parameters: the tile (`chunk`, the
blocks a workgroup codes at a time: 256, 512, 1024 or 2048), the workgroup size
(256 or 512 lanes, one block per lane, at most the tile; a workgroup codes its
tile in tile / lanes passes), and the grid (one workgroup per tile, or a
persistent grid whose workgroups walk the tiles with a fixed stride).  The
tuner plans the batch once per tile size, times every (lanes, grid) on the real
batch with HIP events on the current stream, and returns the fastest
configuration.  Every configuration computes the same bytes; the tuner only
measures time.
"""
from dataclasses import dataclass, field


@dataclass
class TuneResult:
    chunk: int
    grid: int
    ms: float
    table: dict = field(default_factory=dict)   # (chunk, threads, grid) -> ms
    threads: int = 0


def tune_batch(srcs, dsts, qs, chunks=(256, 512, 1024, 2048), threads=(256, 512),
               grids=(0, 1024, 2048, 4096, 8192), reps: int = 3):
    """Time dct_batch_run_threads over chunks x threads x grids; returns (TuneResult,
    planned Batch of the winner)."""
    import torch

    from . import codec
    table, batches = {}, {}
    for chunk in chunks:
        batch = codec.Batch(srcs, dsts, qs, chunk=chunk)
        batches[chunk] = batch
        for lanes in threads:
            if lanes > chunk:
                continue
            for grid in grids:
                batch.run(grid, threads=lanes)             # warm
                torch.cuda.synchronize()
                t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                t0.record()
                for _ in range(reps):
                    batch.run(grid, threads=lanes)
                t1.record()
                torch.cuda.synchronize()
                table[(chunk, lanes, grid)] = t0.elapsed_time(t1) / reps
    (chunk, lanes, grid), ms = min(table.items(), key=lambda kv: kv[1])
    for c, b in batches.items():
        if c != chunk:
            b.release()
    return TuneResult(chunk, grid, ms, table, lanes), batches[chunk]
