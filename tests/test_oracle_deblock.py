"""Pins of the deblocking network's oracle (deblock.c): the convolution against
SciPy and closed forms, the network's structure, the exact gradient against
central finite differences, and Adam's first step in closed form."""
import numpy as np
import pytest
import scipy.signal as ss


def rand_params(oracle_mod, rng, scale=0.3):
    p = rng.normal(0.0, scale, oracle_mod.db_nparam())
    return p


def test_parameter_count(oracle_mod):
    assert oracle_mod.db_nparam() == 19105 == (9 * 32 + 32) + 2 * (9 * 32 * 32 + 32) + (9 * 32 + 1)


def test_conv_matches_scipy_correlate(oracle_mod):
    rng = np.random.default_rng(61)
    x = rng.normal(size=(3, 9, 13))
    w = rng.normal(size=(2, 3, 3, 3))
    b = rng.normal(size=2)
    y = oracle_mod.conv3x3(x, w, b)
    for co in range(2):
        ref = b[co] + sum(ss.correlate2d(x[ci], w[co, ci], mode="same", boundary="fill", fillvalue=0.0)
                          for ci in range(3))
        assert np.allclose(y[co], ref, atol=1e-12)


def test_conv_identity_and_shift(oracle_mod):
    rng = np.random.default_rng(62)
    x = rng.normal(size=(1, 6, 7))
    w = np.zeros((1, 1, 3, 3))
    w[0, 0, 1, 1] = 1.0
    assert np.array_equal(oracle_mod.conv3x3(x, w)[0], x[0])
    w = np.zeros((1, 1, 3, 3))
    w[0, 0, 0, 1] = 1.0            # tap above: y[r][c] = x[r-1][c], zero in row 0
    y = oracle_mod.conv3x3(x, w)[0]
    assert np.array_equal(y[1:], x[0, :-1]) and not np.any(y[0])


def test_zero_network_is_identity(oracle_mod):
    rng = np.random.default_rng(63)
    x = rng.uniform(size=(8, 11))
    y, acts = oracle_mod.db_forward(np.zeros(oracle_mod.db_nparam()), x)
    assert np.array_equal(y, x) and not np.any(acts)


def test_forward_structure_by_hand(oracle_mod):
    # the network written out with SciPy on a small image
    rng = np.random.default_rng(64)
    p = rand_params(oracle_mod, rng)
    x = rng.uniform(size=(5, 6))
    sizes = [(32, 1), (32, 32), (32, 32), (1, 32)]
    o, layers = 0, []
    for co, ci in sizes:
        w = p[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = p[o:o + co]
        o += co
        layers.append((w, b))

    def conv(a, w, b):
        return np.stack([b[k] + sum(ss.correlate2d(a[i], w[k, i], mode="same") for i in range(a.shape[0]))
                         for k in range(w.shape[0])])

    a = x[None]
    for w, b in layers[:3]:
        a = np.maximum(conv(a, w, b), 0.0)
    y_ref = x + conv(a, *layers[3])[0]
    y, _ = oracle_mod.db_forward(p, x)
    assert np.allclose(y, y_ref, atol=1e-10)


@pytest.mark.parametrize("seed", [65, 66])
def test_gradient_matches_finite_differences(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    p = rand_params(oracle_mod, rng, 0.25)
    x = rng.uniform(size=(2, 5, 6))
    t = np.clip(x + rng.normal(0, 0.05, x.shape), 0, 1)
    loss, g = oracle_mod.db_loss_grad(p, x, t)
    # every bias, and a sample of weights of every layer
    idx = list(range(288, 320)) + list(range(9536, 9568)) + list(range(18784, 18816)) + [19104]
    idx += list(rng.choice(288, 12, replace=False)) + list(320 + rng.choice(9216, 20, replace=False))
    idx += list(9568 + rng.choice(9216, 20, replace=False)) + list(18816 + rng.choice(288, 12, replace=False))
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (oracle_mod.db_loss_grad(pp, x, t, want_grad=False)[0] -
              oracle_mod.db_loss_grad(pm, x, t, want_grad=False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, fd, g[k])


def test_conv_input_gradient_matches_finite_differences(oracle_mod):
    rng = np.random.default_rng(67)
    x = rng.normal(size=(3, 4, 5))
    w = rng.normal(size=(2, 3, 3, 3))
    gy = rng.normal(size=(2, 4, 5))
    gx, gw, gb = oracle_mod.conv3x3_bwd(x, w, gy)
    f = lambda xx: float((oracle_mod.conv3x3(xx, w) * gy).sum())
    for k in rng.choice(x.size, 15, replace=False):
        e = np.zeros(x.size)
        e[k] = 1e-6
        fd = (f(x + e.reshape(x.shape)) - f(x - e.reshape(x.shape))) / 2e-6
        assert abs(fd - gx.reshape(-1)[k]) < 1e-6
    assert np.allclose(gb, gy.sum(axis=(1, 2)))


def test_adam_first_step_closed_form(oracle_mod):
    rng = np.random.default_rng(68)
    g = rng.normal(size=50)
    p = rng.normal(size=50)
    m, v = np.zeros(50), np.zeros(50)
    p0 = p.copy()
    oracle_mod.adam_step(p, m, v, g, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, step=1)
    assert np.allclose(p, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # second step with the same gradient moves by the same amount again
    p1 = p.copy()
    oracle_mod.adam_step(p, m, v, g, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, step=2)
    assert np.allclose(p1 - p, 1e-3 * g / (np.abs(g) + 1e-8), atol=1e-12)


def test_training_reduces_loss(oracle_mod):
    # a few Adam steps on blocky images lower the loss below that of the identity
    rng = np.random.default_rng(69)
    t = rng.uniform(0.3, 0.7, size=(2, 8, 8))
    x = np.round(t * 255 / 16) * 16 / 255        # coarse quantization of the targets
    p = rand_params(oracle_mod, rng, 0.05)
    p[18816:19104] = 0.0                           # start at the identity
    m, v = np.zeros_like(p), np.zeros_like(p)
    l0, _ = oracle_mod.db_loss_grad(p, x, t, want_grad=False)
    for step in range(1, 41):
        loss, g = oracle_mod.db_loss_grad(p, x, t)
        oracle_mod.adam_step(p, m, v, g, lr=2e-3, step=step)
    l1, _ = oracle_mod.db_loss_grad(p, x, t, want_grad=False)
    assert l1 < 0.7 * l0
