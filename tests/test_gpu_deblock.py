"""GPU parity of the learned deblocking post-filter against the FP64 oracle
(oracle/deblock.c), entry by entry:

  * the forward pass and the inference entry point per pixel, within the
    tolerance deblock_bounds.py derives from FP16 activation storage and FP32
    accumulation (output pixels outside that tolerance of a rounding boundary
    must agree exactly), on small crops and on a whole 1024 x 1024 decoded
    image, the inference workload's shape;
  * every one of the 19,105 gradient entries within its own tolerance, on small
    crops and on 32 crops of 64 x 64 (the training workload's shape, where the
    weight-gradient passes run at their largest workgroup count);
  * Adam, the initialisation (Philox4x32-10 + Box-Muller, recomputed here), the
    fallback rule, the identity filter bit for bit, and a short training run
    that must lower the loss and raise held-out PSNR.

The tolerances are validated on the CPU in test_deblock_bounds.py: an emulation
of this arithmetic stays inside them and planted kernel mistakes break them.
"""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import deblock_bounds as dbb
from philox_ref import philox4x32_10


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]
NAMES = [("W1", 288), ("b1", 32), ("W2", 9216), ("b2", 32), ("W3", 9216), ("b3", 32), ("W4", 288), ("b4", 1)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hip():
    from paper_1306_1373_amd import codec
    codec.load()
    return codec


def fp16_round(p):
    return np.asarray(p, np.float32).astype(np.float16).astype(np.float64)


def coded_pair(W, H, seed, qs):
    """(original, decoded) uint8 images: a synthetic image and its codec output (oracle)."""
    import oracle
    from paper_1306_1373_amd.synth import synth_image
    img = synth_image(W, H, seed, 5.0)
    rec, _ = oracle.cordic_codec(img, qs)
    return img, rec


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def crops_of(plane, pos, h, w):
    """Crops of a plane at top-left positions pos, zero outside the plane (as the kernels read them)."""
    out = np.zeros((len(pos), h, w), np.float64)
    for k, (r, c) in enumerate(pos):
        sub = plane[r:r + h, c:c + w]
        out[k, :sub.shape[0], :sub.shape[1]] = sub
    return out


def oracle_loss_grad(oracle_mod, pq, x, t, threads=8):
    """The oracle's loss and gradient of a batch, its crops split over threads
    (each part's mean is weighted by its share of the pixels)."""
    parts = np.array_split(np.arange(len(x)), min(threads, len(x)))
    with ThreadPoolExecutor(len(parts)) as pool:
        res = list(pool.map(lambda ix: oracle_mod.db_loss_grad(pq, x[ix], t[ix]), parts))
    n = len(x)
    loss = sum(len(ix) / n * r[0] for ix, r in zip(parts, res))
    grad = sum(len(ix) / n * r[1] for ix, r in zip(parts, res))
    return loss, grad


def check_gradient(hip, oracle_mod, orig, dec, pos, h, w, params, label):
    pq = fp16_round(params)
    db = hip.Deblocker(params)
    g, loss = db.compute_grad(to_dev(dec), to_dev(orig), to_dev(pos), h, w)
    g = g.cpu().numpy().astype(np.float64)
    x = crops_of(dec, pos, h, w) / 255.0
    t = crops_of(orig, pos, h, w) / 255.0
    loss_ref, g_ref = oracle_loss_grad(oracle_mod, pq, x, t)
    E = dbb.Exact(pq, x, t)
    tol = dbb.gradient_tolerance(E)
    ratio = np.abs(g - g_ref) / tol
    o = 0
    for name, n in NAMES:
        r = ratio[o:o + n]
        say(f"[gpu] {label} grad {name}: worst err/tolerance {r.max():.3f}, median tolerance/|g| "
            f"{np.median(tol[o:o + n] / np.maximum(np.abs(g_ref[o:o + n]), 1e-30)):.2e}")
        o += n
    say(f"[gpu] {label} loss {float(loss.cpu()[0]):.6e} vs {loss_ref:.6e}")
    assert abs(float(loss.cpu()[0]) - loss_ref) <= 1e-4 * loss_ref + 1e-12
    bad = np.flatnonzero(ratio > 1.0)
    assert bad.size == 0, f"{bad.size} entries outside their tolerance, first {bad[:8]}"


def test_forward_matches_oracle(hip, oracle_mod):
    orig, dec = coded_pair(96, 80, 3, 16)
    params = dbb.he_params(5)
    pq = fp16_round(params)
    pos = np.array([[0, 0], [16, 40], [64, 56], [70, 70]], np.int32)   # the last crop leaves the plane
    h = w = 24
    db = hip.Deblocker(params)
    y = db.forward(to_dev(dec), to_dev(pos), h, w).cpu().numpy()
    x = crops_of(dec, pos, h, w) / 255.0
    for k in range(len(pos)):
        y_ref, _ = oracle_mod.db_forward(pq, x[k])
        tol = dbb.forward_tolerance(dbb.Exact(pq, x[k:k + 1]))[0]
        err = np.abs(y[k] - y_ref)
        say(f"[gpu] deblock forward crop {k}: max err {err.max():.2e}, worst err/tolerance {(err / tol).max():.2f}")
        assert np.all(err <= tol)


def test_gradient_entrywise_small_crops(hip, oracle_mod):
    orig, dec = coded_pair(128, 96, 4, 16)
    rng = np.random.default_rng(8)
    h = w = 16
    pos = np.stack([rng.integers(0, 96 - h, 6), rng.integers(0, 128 - w, 6)], axis=1).astype(np.int32)
    pos[5] = (90, 120)                                  # partly outside the plane: zero there
    check_gradient(hip, oracle_mod, orig, dec, pos, h, w, dbb.he_params(7), "6 x 16^2")


def test_gradient_entrywise_training_shape(hip, oracle_mod):
    # the training workload's step: 32 crops of 64 x 64 of 1024 x 1024 decoded
    # images (131,072 pixels: the weight-gradient passes at their largest grid)
    import oracle
    from paper_1306_1373_amd.synth import synth_image
    S, h = 1024, 64
    imgs = [synth_image(S, S, 60 + k, 4.0 + k) for k in range(2)]
    orig = np.concatenate(imgs)
    dec = np.concatenate([oracle.cordic_codec(im, 8 + 16 * k)[0] for k, im in enumerate(imgs)])
    rng = np.random.default_rng(9)
    b = rng.integers(0, 2, 32)
    pos = np.stack([b * S + rng.integers(0, S - h + 1, 32), rng.integers(0, S - h + 1, 32)], axis=1).astype(np.int32)
    check_gradient(hip, oracle_mod, orig, dec, pos, h, h, dbb.he_params(11), "32 x 64^2")


def test_adam_matches_oracle(hip, oracle_mod):
    import torch
    rng = np.random.default_rng(9)
    n = 19105
    p = rng.normal(size=n)
    db = hip.Deblocker(p.astype(np.float32))
    m64, v64, p64 = np.zeros(n), np.zeros(n), p.astype(np.float32).astype(np.float64)
    for step in range(1, 6):
        g = rng.normal(size=n).astype(np.float32)
        db.grad.copy_(torch.from_numpy(g))
        db.adam(1e-3)
        oracle_mod.adam_step(p64, m64, v64, g.astype(np.float64), 1e-3, step=step)
        got = db.params.cpu().numpy().astype(np.float64)
        assert np.abs(got - p64).max() <= 1e-6 * step, step


def forward_bands(oracle_mod, pq, x, band=64, threads=16):
    """(y, tolerance) of the oracle's forward pass over a whole image, computed in
    bands of rows with a four-row margin (the network's reach) cut away again."""
    H = x.shape[0]

    def work(r0):
        r1 = min(H, r0 + band)
        a, b = max(0, r0 - 4), min(H, r1 + 4)
        y, _ = oracle_mod.db_forward(pq, x[a:b])
        tol = dbb.forward_tolerance(dbb.Exact(pq, x[a:b][None]))[0]
        return r0, y[r0 - a:r1 - a], tol[r0 - a:r1 - a]

    y = np.empty_like(x)
    tol = np.empty_like(x)
    with ThreadPoolExecutor(threads) as pool:
        for r0, yb, tb in pool.map(work, range(0, H, band)):
            y[r0:r0 + yb.shape[0]] = yb
            tol[r0:r0 + tb.shape[0]] = tb
    return y, tol


def padded_plane(hip, a):
    """A device plane holding a (H, W) uint8 image with its pitch rounded up to a
    multiple of 8 (the ABI's rule); pad bytes hold 0xA5."""
    import torch
    H, W = a.shape
    pitch = (W + 7) // 8 * 8
    buf = torch.full((H, pitch), 0xA5, dtype=torch.uint8, device="cuda")
    buf[:, :W] = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return buf[:, :W]


def check_apply(hip, oracle_mod, dec, params, label):
    pq = fp16_round(params)
    db = hip.Deblocker(params)
    out = db.apply(padded_plane(hip, dec)).cpu().numpy().astype(np.int64)
    x = dec.astype(np.float64) / 255.0
    y_ref, tol = forward_bands(oracle_mod, pq, x)
    v = 255.0 * y_ref + 0.5
    ref = np.clip(np.floor(v), 0, 255)
    near = np.abs(v - np.round(v)) <= 255.0 * tol          # within the tolerance of a rounding boundary
    ok = (out == ref) | (near & (np.abs(out - ref) <= 1))
    say(f"[gpu] deblock apply {label}: {int((out != ref).sum())} of {out.size} pixels differ, all at a "
        f"rounding boundary; {int(near.sum())} pixels within reach of one")
    assert np.all(ok), np.argwhere(~ok)[:8]


def test_apply_matches_oracle_pixels(hip, oracle_mod):
    orig, dec = coded_pair(72, 40, 6, 16)
    check_apply(hip, oracle_mod, dec, dbb.he_params(10), "72 x 40")


@pytest.mark.parametrize("W,H", [(1, 1), (29, 29), (57, 57), (200, 13), (28, 28), (85, 79)])
def test_apply_ragged_tiles(hip, oracle_mod, W, H):
    # planes that are not whole numbers of the inference kernel's 28 x 28 tiles,
    # one smaller than a tile, one exactly one tile
    orig, dec = coded_pair(W, H, 20 + W, 16)
    check_apply(hip, oracle_mod, dec, dbb.he_params(21), f"{W} x {H}")


@pytest.mark.parametrize("W,H", [(1024, 1024), (85, 79)])
def test_fused_apply_equals_layer_kernels(hip, W, H):
    # the one-launch inference computes every float as the one-layer kernels of
    # the training forward pass do: its pixels are the rounding of their y (the
    # final 255 y + 1/2 taken with one rounding, as a fused multiply-add, or two)
    orig, dec = coded_pair(W, H, 30 + H, 20)
    db = hip.Deblocker(dbb.he_params(23))
    d = padded_plane(hip, dec)
    out = db.apply(d).cpu().numpy().astype(np.int64)
    y = db.forward(d, None, H, W).cpu().numpy()[0]
    one = np.float32(np.float64(y) * 255.0 + 0.5)
    two = np.float32(np.float32(255.0) * y) + np.float32(0.5)
    r1, r2 = (np.clip(np.floor(v), 0, 255).astype(np.int64) for v in (one, two))
    ok = (out == r1) | (out == r2)
    say(f"[gpu] fused apply {W} x {H}: {int((r1 != r2).sum())} pixels where the two roundings differ")
    assert np.all(ok), np.argwhere(~ok)[:8]


def test_apply_matches_oracle_1024(hip, oracle_mod):
    # the inference workload's shape: one 1024 x 1024 decoded image, every pixel
    orig, dec = coded_pair(1024, 1024, 12, 24)
    check_apply(hip, oracle_mod, dec, dbb.he_params(13), "1024 x 1024")


@pytest.mark.parametrize("W,H,n", [(85, 79, 3), (29, 27, 5), (1024, 1024, 2), (1, 1, 4)])
def test_apply_stack_equals_single_images(hip, W, H, n):
    # n images stacked vertically in one plane, filtered in one launch: each must
    # come out byte for byte as its own dct_deblock_apply call gives it (its own
    # zero padding at the seams), and nothing past the stack is written
    import torch
    db = hip.Deblocker(dbb.he_params(31))
    decs = [coded_pair(W, H, 40 + k, 16)[1] for k in range(n)]
    stack = padded_plane(hip, np.concatenate(decs, axis=0))
    pitch = (W + 7) // 8 * 8
    buf = torch.full((n * H + 2, pitch), 0x5A, dtype=torch.uint8, device="cuda")
    out = db.apply_stack(stack, n, out=buf[:n * H, :W]).cpu().numpy()
    assert bool((buf[n * H:] == 0x5A).all())
    for k in range(n):
        one = db.apply(padded_plane(hip, decs[k])).cpu().numpy()
        assert np.array_equal(out[k * H:(k + 1) * H], one), (W, H, n, k)
    say(f"[gpu] deblock apply stack {n} x {W} x {H}: equal to single-image calls")


def test_init_is_philox_box_muller(hip):
    seed = 0x1234_5678_9ABC_DEF0
    a = hip.Deblocker(seed=seed).params.cpu().numpy()
    b = hip.Deblocker(seed=seed).params.cpu().numpy()
    c = hip.Deblocker(seed=seed + 1).params.cpu().numpy()
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    for lo, hi in ((288, 320), (9536, 9568), (18784, 19105)):       # biases and the output layer
        assert np.all(a[lo:hi] == 0.0)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    rng = np.random.default_rng(3)
    for k in sorted(set(rng.integers(0, 18784, 300)) | {0, 287, 320, 9535, 9568, 18783}):
        if 288 <= k < 320 or 9536 <= k < 9568:
            continue
        x = philox4x32_10([int(k), 0, 0, 0], key)
        u1, u2 = (x[0] + 1.0) * 2.0 ** -32, x[1] * 2.0 ** -32
        sd = (2.0 / 9.0) ** 0.5 if k < 288 else (2.0 / 288.0) ** 0.5
        ref = np.float32(sd * np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2))
        assert abs(float(a[k]) - float(ref)) <= 2e-6 * max(1.0, abs(float(ref))), k
    w2 = a[320:9536]
    assert abs(w2.mean()) < 0.01 and abs(w2.std() / (2.0 / 288.0) ** 0.5 - 1.0) < 0.03


def test_identity_filter_is_exact(hip):
    orig, dec = coded_pair(104, 60, 11, 8)
    db = hip.Deblocker(seed=3)           # untrained: zero output layer
    out = db.apply(to_dev(dec)).cpu().numpy()
    assert np.array_equal(out, dec)


def test_select_keeps_or_zeroes(hip):
    import torch
    params = dbb.he_params(14)
    db = hip.Deblocker(params)
    plain = torch.tensor([1000, 2000, 50, 7], dtype=torch.int64, device="cuda")
    better = torch.tensor([800, 1500, 50, 6], dtype=torch.int64, device="cuda")
    gain, kept = db.select(plain, better)
    ref = np.mean([10 * np.log10(a / b) for a, b in ((1000, 800), (2000, 1500), (50, 50), (7, 6))])
    assert kept and abs(gain - ref) < 1e-12
    assert np.array_equal(db.params.cpu().numpy(), params)
    worse = torch.tensor([1200, 2100, 60, 7], dtype=torch.int64, device="cuda")
    gain, kept = db.select(plain, worse)
    assert not kept and gain < 0
    p = db.params.cpu().numpy()
    assert np.all(p[18816:] == 0.0) and np.array_equal(p[:18816], params[:18816])
    orig, dec = coded_pair(64, 48, 15, 16)
    assert np.array_equal(db.apply(to_dev(dec)).cpu().numpy(), dec)     # the fallback is the decoded image
    gain, kept = hip.Deblocker(params).select(plain, torch.zeros(4, dtype=torch.int64, device="cuda"))
    assert kept and gain == float("inf")


def test_short_training_improves_psnr(hip, oracle_mod):
    from paper_1306_1373_amd.synth import synth_image
    qs, S, n_img = 24, 256, 6
    imgs = [synth_image(S, S, 40 + k, 4.0) for k in range(n_img + 1)]
    recs = [oracle_mod.cordic_codec(im, qs)[0] for im in imgs]
    dec = to_dev(np.concatenate(recs[:n_img]))
    org = to_dev(np.concatenate(imgs[:n_img]))
    db = hip.Deblocker(seed=0)
    rng = np.random.default_rng(12)
    h = w = 48
    first = None
    for step in range(300):
        b = rng.integers(0, n_img, 16)
        pos = np.stack([b * S + rng.integers(0, S - h, 16), rng.integers(0, S - w, 16)], axis=1).astype(np.int32)
        loss = float(db.train_step(dec, org, to_dev(pos), h, w, lr=2e-3).cpu()[0])
        first = loss if first is None else first
    say(f"[gpu] deblock training loss {first:.3e} -> {loss:.3e}")
    assert loss < 0.9 * first
    out = db.apply(to_dev(recs[n_img])).cpu().numpy()
    gain = oracle_mod.psnr(imgs[n_img], out) - oracle_mod.psnr(imgs[n_img], recs[n_img])
    say(f"[gpu] held-out PSNR gain {gain:.3f} dB")
    assert gain > 0.0
