"""Launch-shape tuner for the batched codec (dct_batch_run).

The batched kernel has two free launch parameters: the workgroup chunk (256 or
512 blocks, one lane per block) and the grid (one workgroup per chunk, or a
persistent grid whose workgroups walk the chunks with a fixed stride).  The
tuner plans the batch once per chunk size, times every grid on the real batch
with HIP events on the current stream, and returns the fastest configuration.
Every configuration computes the same bytes; the tuner only measures time.
"""
from dataclasses import dataclass, field


@dataclass
class TuneResult:
    chunk: int
    grid: int
    ms: float
    table: dict = field(default_factory=dict)   # (chunk, grid) -> ms


def tune_batch(srcs, dsts, qs, chunks=(256, 512), grids=(0, 1024, 2048, 4096, 8192), reps: int = 3):
    """Time dct_batch_run over chunks x grids; returns (TuneResult, planned Batch of the winner)."""
    import torch

    from . import codec
    table, batches = {}, {}
    for chunk in chunks:
        batch = codec.Batch(srcs, dsts, qs, chunk=chunk)
        batches[chunk] = batch
        for grid in grids:
            batch.run(grid)                       # warm
            torch.cuda.synchronize()
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(reps):
                batch.run(grid)
            t1.record()
            torch.cuda.synchronize()
            table[(chunk, grid)] = t0.elapsed_time(t1) / reps
    (chunk, grid), ms = min(table.items(), key=lambda kv: kv[1])
    for c, b in batches.items():
        if c != chunk:
            b.release()
    return TuneResult(chunk, grid, ms, table), batches[chunk]
