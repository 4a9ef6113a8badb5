"""Pins of the FP64 U-Net oracle against facts fixed outside it: brute-force
index loops, a library correlation, adjoint identities, finite differences of
the loss, the IEEE bfloat16 rounding rule and Adam's closed form for a
constant gradient."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import unet
from paper_2204_07019_amd import inputs


def test_bf16_rounding_rule():
    # bfloat16 keeps 8 significant bits: ulp(1) = 2^-7; ties go to the even mantissa.
    vals = np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-8, 1 + 2**-8 + 2**-20, -2.5, 3.0e38, 1e-40])
    want = np.array([1.0, 1.0, 1 + 2**-6, 1 + 2**-7, -2.5, 2.9980e38, 0.0])
    got = unet.bf16(vals)
    assert got[:5].tolist() == want[:5].tolist()
    assert abs(got[5] / 3.0e38 - 1) < 2**-8
    assert abs(got[6]) < 1.2e-40
    assert np.isnan(unet.bf16(np.nan))


def test_conv3d_brute_force():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 4, 5, 3))
    w = rng.standard_normal((27, 3, 2))
    b = rng.standard_normal(2)
    y = unet.conv3d(x, w, b)
    N, D, H, W, _ = x.shape
    ref = np.zeros((N, D, H, W, 2))
    for n in range(N):
        for k in range(D):
            for j in range(H):
                for i in range(W):
                    for co in range(2):
                        s = b[co]
                        for a in (-1, 0, 1):
                            for bb in (-1, 0, 1):
                                for c in (-1, 0, 1):
                                    kk, jj, ii = k + a, j + bb, i + c
                                    if 0 <= kk < D and 0 <= jj < H and 0 <= ii < W:
                                        tap = 9 * (a + 1) + 3 * (bb + 1) + (c + 1)
                                        s += sum(x[n, kk, jj, ii, ci] * w[tap, ci, co] for ci in range(3))
                        ref[n, k, j, i, co] = s
    np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-13)


def test_conv3d_matches_library_correlation():
    # One channel in and out: the convolution is scipy's correlation with zero fill.
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 6, 5, 7, 1))
    k = rng.standard_normal((3, 3, 3))
    y = unet.conv3d(x, k.reshape(27, 1, 1))
    ref = ndimage.correlate(x[0, ..., 0], k, mode="constant", cval=0.0)
    np.testing.assert_allclose(y[0, ..., 0], ref, rtol=1e-12, atol=1e-12)


def test_adjoints():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 4, 6, 8, 3))
    g = rng.standard_normal((2, 4, 6, 8, 5))
    w = rng.standard_normal((27, 3, 5))
    lhs = np.sum(unet.conv3d(x, w) * g)
    assert np.isclose(lhs, np.sum(x * unet.conv3d_dgrad(g, w)), rtol=1e-12)
    assert np.isclose(lhs, np.sum(w * unet.conv3d_wgrad(x, g)), rtol=1e-12)
    gc = rng.standard_normal((2, 2, 3, 4, 3))
    assert np.isclose(np.sum(unet.pool(x) * gc), np.sum(x * unet.pool_adjoint(gc)), rtol=1e-12)
    assert np.isclose(np.sum(unet.up(gc) * x), np.sum(gc * unet.up_adjoint(x)), rtol=1e-12)
    # pooling a constant is the constant; upsampling then pooling is the identity
    np.testing.assert_allclose(unet.pool(np.full((1, 4, 4, 4, 2), 3.5)), 3.5)
    np.testing.assert_allclose(unet.pool(unet.up(gc)), gc, rtol=1e-14)


def test_param_layout_roundtrip():
    theta = inputs.unet_init(5).astype(np.float64)
    assert theta.size == unet.n_params()
    np.testing.assert_array_equal(unet.pack(unet.unpack(theta)), theta)
    p = unet.unpack(theta)
    assert np.all(p["e0a"][0][:, 4:, :] == 0.0)       # padded input channels carry no weight
    assert p["d1a"][0].shape == (27, 96, 32) and p["head"][0].shape == (16,)


def test_loss_gradient_matches_finite_differences():
    # Plain FP64 network (no bfloat16 rounding): the analytic gradient must
    # match central differences of the loss in every layer.
    x, t = inputs.unet_batch(1, 4, 4, 8, seed=7)
    theta = inputs.unet_init(8).astype(np.float64)
    rng = np.random.default_rng(9)
    theta[:-17] += 0.05 * rng.standard_normal(theta.size - 17) * (theta[:-17] != 0)
    loss, grad, _ = unet.loss_and_grad(theta, x, t, bf16_round=False)
    offs, o = {}, 0
    for name, ci, co in unet.LAYERS:
        offs[name] = (o, o + 27 * ci * co, o + 27 * ci * co + co)
        o += 27 * ci * co + co
    idx = []
    for name in offs:
        w0, b0, e0 = offs[name]
        nz = np.nonzero(grad[w0:b0])[0]
        idx += list(w0 + rng.choice(nz, 3, replace=False)) + [b0 + int(rng.integers(0, e0 - b0))]
    idx += [o + 3, o + 16]
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp = unet.loss_and_grad(tp, x, t, bf16_round=False)[0]
        lm = unet.loss_and_grad(tm, x, t, bf16_round=False)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(abs(fd), 1e-3 * abs(loss)), (i, fd, grad[i])


def test_bf16_network_close_to_fp64_network():
    # Rounding at the stored points perturbs the output by a few bfloat16 ulps.
    x, t = inputs.unet_batch(2, 8, 8, 8, seed=4)
    theta = inputs.unet_init(3).astype(np.float64)
    y64 = unet.forward(theta, x, bf16_round=False)[0]
    y16 = unet.forward(theta, x, bf16_round=True)[0]
    rel = np.linalg.norm(y16 - y64) / np.linalg.norm(y64)
    assert 1e-5 < rel < 5e-2


def test_adam_constant_gradient_closed_form():
    # With a constant gradient the bias-corrected moments are exact: m^ = g,
    # v^ = g^2, so every step moves theta by lr * g / (|g| + eps).
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th = np.array([1.0, 1.0, -1.0, 5.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 1e-2, 1e-8
    for t in range(1, 6):
        th, m, v = unet.adam(th, g, m, v, t, lr, eps=eps)
    np.testing.assert_allclose(th, np.array([1.0, 1.0, -1.0, 5.0]) - 5 * lr * g / (np.abs(g) + eps),
                               rtol=1e-12, atol=1e-15)


def test_training_reduces_loss():
    x, t = inputs.unet_batch(1, 8, 8, 8, seed=12)
    theta = inputs.unet_init(13).astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = None
    for it in range(1, 16):
        loss, g, _ = unet.loss_and_grad(theta, x, t, bf16_round=False)
        l0 = loss if l0 is None else l0
        theta, m, v = unet.adam(theta, g, m, v, it, 3e-3)
    assert loss < 0.5 * l0
