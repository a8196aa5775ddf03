"""Seeded synthetic grayscale images: the shared input of the codec and its oracle.

This module holds no part of the codec's arithmetic.  It stands in for the
paper's photographic test images (Lena and Cable-car, Sec. 4), which are not
available, with images of the same sizes and a similar mix of smooth shading,
oriented texture at several scales, and sensor-like noise.

Generator G(W, H, seed, sigma), NumPy ``default_rng(seed)`` (PCG64), draws in
this order:

1. for k = 1..6: period P_k = exp(U[ln 4, ln 128]), angle theta_k ~ U[0, pi),
   phase phi_k ~ U[0, 2 pi), amplitude A_k ~ U[10, 30];
2. gradient g_x, g_y ~ U[-40, 40];
3. noise N(0, sigma^2) over the H x W grid, drawn row-major in bands of
   ``_BAND`` rows.

    I(x, y) = 128 + sum_k A_k sin(2 pi (x cos theta_k + y sin theta_k) / P_k + phi_k)
                  + g_x (x / W - 1/2) + g_y (y / H - 1/2) + noise

rounded half to even (``rint``), clipped to [0, 255], stored as uint8.  Each
sinusoid is evaluated as sin(a x) cos(b y + phi) + cos(a x) sin(b y + phi) so
that the cost is O(W + H) transcendentals plus a few multiply-adds per pixel;
that evaluation order is part of the definition, and golden SHA-256 digests in
the tests pin the bytes.
"""
import hashlib

import numpy as np

_BAND = 256


def synth_image(W: int, H: int, seed: int, sigma: float = 5.0) -> np.ndarray:
    """One (H, W) uint8 image from generator G."""
    if W < 1 or H < 1:
        raise ValueError("W and H must be positive")
    rng = np.random.default_rng(seed)
    per, ang, pha, amp = [], [], [], []
    for _ in range(6):
        per.append(np.exp(rng.uniform(np.log(4.0), np.log(128.0))))
        ang.append(rng.uniform(0.0, np.pi))
        pha.append(rng.uniform(0.0, 2.0 * np.pi))
        amp.append(rng.uniform(10.0, 30.0))
    gx = rng.uniform(-40.0, 40.0)
    gy = rng.uniform(-40.0, 40.0)

    x = np.arange(W, dtype=np.float64)
    sx, cx = [], []
    for k in range(6):
        a = 2.0 * np.pi * np.cos(ang[k]) / per[k]
        sx.append(amp[k] * np.sin(a * x))
        cx.append(amp[k] * np.cos(a * x))
    ramp_x = gx * (x / W - 0.5)

    out = np.empty((H, W), np.uint8)
    for y0 in range(0, H, _BAND):
        y1 = min(H, y0 + _BAND)
        y = np.arange(y0, y1, dtype=np.float64)
        acc = np.empty((y1 - y0, W), np.float64)
        acc[...] = 128.0 + ramp_x[None, :] + (gy * (y / H - 0.5))[:, None]
        for k in range(6):
            b = 2.0 * np.pi * np.sin(ang[k]) * y / per[k] + pha[k]
            acc += np.cos(b)[:, None] * sx[k][None, :]
            acc += np.sin(b)[:, None] * cx[k][None, :]
        if sigma > 0:
            acc += rng.normal(0.0, sigma, size=(y1 - y0, W))
        np.rint(acc, out=acc)
        np.clip(acc, 0.0, 255.0, out=acc)
        out[y0:y1] = acc.astype(np.uint8)
    return out


def synth_rgb(W: int, H: int, seed: int, sigma: float = 5.0) -> np.ndarray:
    """An (H, W, 3) uint8 RGB image: a luminance image from G(W, H, seed, sigma)
    and two chroma images from G(W, H, seed + 1000, sigma) and G(W, H, seed + 2000,
    sigma), combined as R = L + 0.3 (C1 - 128), G = L - 0.2 (C1 - 128) - 0.2 (C2 - 128),
    B = L + 0.3 (C2 - 128), rounded half to even and clipped to [0, 255]."""
    L = synth_image(W, H, seed, sigma).astype(np.float64)
    c1 = synth_image(W, H, seed + 1000, sigma).astype(np.float64) - 128.0
    c2 = synth_image(W, H, seed + 2000, sigma).astype(np.float64) - 128.0
    rgb = np.stack([L + 0.3 * c1, L - 0.2 * c1 - 0.2 * c2, L + 0.3 * c2], axis=-1)
    return np.clip(np.rint(rgb), 0, 255).astype(np.uint8)


def synth_image_device(W: int, H: int, seed: int, sigma: float, out) -> None:
    """Write an image of generator G's family into the (H, W) uint8 device tensor
    ``out``, computed on the device (for batches too large to generate on the
    host): the same six random sinusoids, gradient and Gaussian noise, with the
    parameters and the noise drawn from torch's device generator seeded with
    ``seed``, evaluated in float32, rounded half to even and clipped.  The bytes
    are deterministic for a given device and torch build, not equal to G's;
    consumers that compare against the oracle copy them back."""
    import math

    import torch
    dev = out.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    u = torch.rand(26, generator=gen, device=dev, dtype=torch.float64).cpu().tolist()
    x = torch.arange(W, device=dev, dtype=torch.float32)
    y = torch.arange(H, device=dev, dtype=torch.float32)
    gx, gy = -40.0 + 80.0 * u[24], -40.0 + 80.0 * u[25]
    acc = (128.0 + gx * (x / W - 0.5))[None, :] + (gy * (y / H - 0.5))[:, None]
    for k in range(6):
        per = math.exp(math.log(4.0) + u[4 * k] * (math.log(128.0) - math.log(4.0)))
        ang, pha, amp = u[4 * k + 1] * math.pi, u[4 * k + 2] * 2.0 * math.pi, 10.0 + 20.0 * u[4 * k + 3]
        a = 2.0 * math.pi * math.cos(ang) / per
        b = 2.0 * math.pi * math.sin(ang) * y / per + pha
        acc = acc + torch.cos(b)[:, None] * (amp * torch.sin(a * x))[None, :]
        acc = acc + torch.sin(b)[:, None] * (amp * torch.cos(a * x))[None, :]
    if sigma > 0:
        acc = acc + sigma * torch.randn((H, W), generator=gen, device=dev, dtype=torch.float32)
    out.copy_(torch.clamp(torch.round(acc), 0.0, 255.0).to(torch.uint8))


def sigma_for_seed(seed: int) -> float:
    """Noise level of the 8192 x 8192 workload: sigma = 2 + 8 s / 7 for s = 0..7."""
    return 2.0 + 8.0 * (seed % 8) / 7.0


def digest(img: np.ndarray) -> str:
    """SHA-256 of the image bytes together with its shape."""
    h = hashlib.sha256()
    h.update(np.asarray(img.shape, np.int64).tobytes())
    h.update(np.ascontiguousarray(img).tobytes())
    return h.hexdigest()


def pad_plane(img: np.ndarray, stride: int, fill: int = 0xA5) -> np.ndarray:
    """Copy img into rows of ``stride`` bytes (stride >= W); returns the (H, W)
    view of the padded buffer.  The pad bytes hold ``fill`` so a reader that
    strays into them is noticed."""
    H, W = img.shape
    if stride < W:
        raise ValueError("stride < W")
    buf = np.full((H, stride), fill, np.uint8)
    buf[:, :W] = img
    return buf[:, :W]
