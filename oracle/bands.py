"""Run the oracle's image-level recipe functions on horizontal bands in threads.

TEST INFRASTRUCTURE ONLY (tests and the benchmark's CPU baseline).  Blocks are
independent and every band but the last is a whole number of block rows, so a
band's blocks are exactly the image's blocks of those rows; the last band holds
the image's last row, so edge replication is unchanged.  ctypes releases the
GIL during each call, so the bands run on separate cores.  No arithmetic of
the codec is done here.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import cordic_codec, cordic_forward, cordic_inverse, exact_codec, grid, recipe_codec


def _bands(H: int, nbands: int):
    rows = (H + 7) // 8
    per = max(1, -(-rows // nbands))
    out = []
    for r0 in range(0, rows, per):
        r1 = min(rows, r0 + per)
        out.append((r0 * 8, min(H, r1 * 8), r0, r1))
    return out


def codec_bands(img: np.ndarray, qs: int, threads: int = 8, want_q: bool = False, recipe=None):
    """(reconstruction, sse[, qcoef]) of the recipe codec (the default recipe, or
    recipe = (n, F, G)), band-parallel."""
    H, W = img.shape
    bw, _ = grid(W, H)
    rec = np.empty((H, W), np.uint8)
    q = np.empty((bw * ((H + 7) // 8), 64), np.int16) if want_q else None

    def run(b):
        y0, y1, r0, r1 = b
        band = np.ascontiguousarray(img[y0:y1])
        out = cordic_codec(band, qs, want_q=want_q) if recipe is None else \
            recipe_codec(*recipe, band, qs, want_q=want_q)
        rec[y0:y1] = out[0]
        if want_q:
            q[r0 * bw:r1 * bw] = out[2]
        return out[1]

    with ThreadPoolExecutor(max_workers=threads) as ex:
        sse = sum(ex.map(run, _bands(H, threads * 4)))
    return (rec, sse, q) if want_q else (rec, sse)


def forward_bands(img: np.ndarray, threads: int = 8) -> np.ndarray:
    H, W = img.shape
    bw, bh = grid(W, H)
    coef = np.empty((bw * bh, 64), np.int32)

    def run(b):
        y0, y1, r0, r1 = b
        coef[r0 * bw:r1 * bw] = cordic_forward(np.ascontiguousarray(img[y0:y1]))

    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(run, _bands(H, threads * 4)))
    return coef


def inverse_bands(qcoef: np.ndarray, qs: int, W: int, H: int, threads: int = 8) -> np.ndarray:
    bw, _ = grid(W, H)
    rec = np.empty((H, W), np.uint8)

    def run(b):
        y0, y1, r0, r1 = b
        rec[y0:y1] = cordic_inverse(np.ascontiguousarray(qcoef[r0 * bw:r1 * bw]), qs, W, y1 - y0)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(run, _bands(H, threads * 4)))
    return rec


def exact_codec_bands(img: np.ndarray, qs: int, threads: int = 8) -> np.ndarray:
    """The exact FP64 codec (reconstruction only), band-parallel."""
    H, W = img.shape
    rec = np.empty((H, W), np.uint8)

    def run(b):
        y0, y1, r0, r1 = b
        rec[y0:y1] = exact_codec(np.ascontiguousarray(img[y0:y1]), qs)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(run, _bands(H, threads * 4)))
    return rec
