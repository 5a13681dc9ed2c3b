"""Pins of the surrogate's FP64 reference: gradients by central finite
differences, BF16 rounding on exactly representable and tie cases, GELU
against its integral definition, and Adam minimising a quadratic."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle.mlp_oracle import (MLPOracle, adam_step, bf16, decode_maps, ensemble_mean_spread, gelu, gelu_grad,
                               inside_box, predicted_error)


def _net(rng, n_in=7, width=6, depth=2, n_out=5):
    K0p = (n_in + 31) // 32 * 32
    dims = [K0p] + [width] * depth + [n_out]
    Ws, bs = [], []
    for l in range(len(dims) - 1):
        W = rng.normal(size=(dims[l], dims[l + 1])) / math.sqrt(dims[l])
        if l == 0:
            W[n_in:] = 0.0
        Ws.append(W)
        bs.append(rng.normal(size=dims[l + 1]) * 0.1)
    xm, xs = rng.normal(size=n_in), rng.uniform(0.5, 2.0, n_in)
    ym, ys = rng.normal(size=n_out), rng.uniform(0.5, 2.0, n_out)
    return MLPOracle(Ws, bs, xm, xs, ym, ys, n_in)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    o = _net(rng)
    x = rng.normal(size=(4, 7))
    y = rng.normal(size=(4, 5))
    loss, dW, db, _ = o.loss_and_grads(x, y, rounded=False)
    h = 1e-6
    for l in range(len(o.Ws)):
        for _ in range(6):
            i = rng.integers(o.n_in if l == 0 else o.Ws[l].shape[0])
            j = rng.integers(o.Ws[l].shape[1])
            o.Ws[l][i, j] += h
            lp = o.loss_and_grads(x, y, rounded=False)[0]
            o.Ws[l][i, j] -= 2 * h
            lm = o.loss_and_grads(x, y, rounded=False)[0]
            o.Ws[l][i, j] += h
            fd = (lp - lm) / (2 * h)
            assert dW[l][i, j] == pytest.approx(fd, rel=1e-5, abs=1e-10)
        j = rng.integers(len(o.bs[l]))
        o.bs[l][j] += h
        lp = o.loss_and_grads(x, y, rounded=False)[0]
        o.bs[l][j] -= 2 * h
        lm = o.loss_and_grads(x, y, rounded=False)[0]
        o.bs[l][j] += h
        assert db[l][j] == pytest.approx((lp - lm) / (2 * h), rel=1e-5, abs=1e-10)


def test_bf16_rounding():
    # exactly representable values are unchanged
    exact = np.array([0.0, 1.0, -2.5, 3.0e-3 * 0 + 0.0078125, 65280.0])
    assert np.array_equal(bf16(exact), exact)
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1.0)
    assert bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    # 1 + 3*2^-8 is halfway between 1+2^-7 and 1+2^-6: even is 1+2^-6
    assert bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6
    # unit roundoff of an 8-significant-bit format: 2^-8
    v = np.random.default_rng(1).normal(size=10000)
    assert np.max(np.abs(bf16(v) - v) / np.abs(v)) <= 2.0 ** -8


def test_gelu_is_x_times_normal_cdf():
    for x in (-3.0, -0.7, 0.0, 0.4, 2.2):
        phi, _ = integrate.quad(lambda t: math.exp(-t * t / 2) / math.sqrt(2 * math.pi), -np.inf, x)
        assert gelu(np.array(x)) == pytest.approx(x * phi, abs=1e-12)
        h = 1e-6
        assert gelu_grad(np.array(x)) == pytest.approx((gelu(np.array(x + h)) - gelu(np.array(x - h))) / (2 * h),
                                                       rel=1e-7, abs=1e-9)


def test_adam_minimises_a_quadratic():
    w = np.array([3.0, -2.0])
    m = np.zeros(2)
    v = np.zeros(2)
    for t in range(1, 3001):
        g = 2 * (w - np.array([0.5, 1.5]))
        w, m, v = adam_step(w, m, v, g, t, lr=1e-2)
    assert np.allclose(w, [0.5, 1.5], atol=1e-3)


def test_decoupled_weight_decay():
    """With zero gradients the decoupled decay alone acts: w_t = w_0 (1 - lr wd)^t.
    With a quadratic loss toward a, the decay pulls the end point from a
    toward 0 (same sign as a, smaller magnitude)."""
    w0 = np.array([1.5, -0.25])
    w, m, v = w0.copy(), np.zeros(2), np.zeros(2)
    for t in range(1, 101):
        w, m, v = adam_step(w, m, v, np.zeros(2), t, lr=1e-2, wd=0.5)
    assert np.allclose(w, w0 * (1 - 1e-2 * 0.5) ** 100, rtol=1e-12)
    # a decayed quadratic fit ends between 0 and the undecayed optimum
    a = np.array([0.5, 1.5])
    w, m, v = np.array([3.0, -2.0]), np.zeros(2), np.zeros(2)
    for t in range(1, 5001):
        w, m, v = adam_step(w, m, v, 2 * (w - a), t, lr=1e-3, wd=0.1)
    assert np.all(np.abs(w) < np.abs(a)) and np.all(w * a > 0)


def test_adam_first_two_steps_closed_form():
    """Kingma & Ba's bias correction makes the first step lr g / (|g| + eps)
    whatever the gradient's scale; a second step with the same gradient
    repeats it, one with the opposite gradient moves back by
    lr (1 - b1) / (1 + b1) g / (|g| + eps) (m_2 = -(1 - b1)^2 g,
    v_2 = (1 - b2^2) g^2).  A missing or shifted correction changes both."""
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    for g0 in (1e-6, 3e-3, 1.0, -250.0, 4e5):
        g = np.array([g0])
        w1, m, v = adam_step(np.zeros(1), np.zeros(1), np.zeros(1), g, 1, lr, b1, b2, eps)
        unit = g / (np.abs(g) + eps)
        assert w1[0] == pytest.approx(-lr * unit[0], rel=1e-9)
        w2, _, _ = adam_step(w1, m, v, g, 2, lr, b1, b2, eps)
        assert w2[0] - w1[0] == pytest.approx(-lr * unit[0], rel=1e-9)
        w2, _, _ = adam_step(w1, m, v, -g, 2, lr, b1, b2, eps)
        assert w2[0] - w1[0] == pytest.approx(lr * (1 - b1) / (1 + b1) * unit[0], rel=1e-9)


def test_decode_inverts_the_map_encoding():
    """A map encoded as (its unit-norm shape, log of its norm) decodes to
    itself, for maps spanning many orders of magnitude."""
    rng = np.random.default_rng(3)
    nc = 37
    heat = rng.gamma(2.0, 1.0, (3, nc)) * np.array([[1e9], [1e14], [3e16]])
    dens = rng.uniform(0.2, 1.0, (3, nc)) * 1e24
    enc = np.zeros((3, 2 * nc + 2))
    for k, Y in enumerate((heat, dens)):
        n = np.linalg.norm(Y, axis=1)
        enc[:, k * nc:(k + 1) * nc] = Y / n[:, None]
        enc[:, 2 * nc + k] = np.log(n)
    out = decode_maps(enc, nc)
    assert np.allclose(out[:, :nc], heat, rtol=1e-13, atol=0)
    assert np.allclose(out[:, nc:], dens, rtol=1e-13, atol=0)


def test_predicted_error_closed_forms():
    """Two members whose shapes are s +- d and log-norms l +- e: the sample
    spread is sqrt(2)|d| and sqrt(2)|e|, so the predicted error of a map is
    calib hypot(sqrt(2)|d| / |s|, sqrt(2)|e|); identical members give 0."""
    nc = 50
    rng = np.random.default_rng(8)
    s = rng.normal(size=(2, nc)); s /= np.linalg.norm(s, axis=1)[:, None]
    d = [0.01 * rng.normal(size=nc), 0.03 * rng.normal(size=nc)]
    e = [0.002, 0.0005]
    base = np.concatenate([s[0], s[1], [1.0, 2.0]])
    delta = np.concatenate([d[0], d[1], e])
    mean, spread = ensemble_mean_spread(np.stack([base + delta, base - delta])[:, None, :])
    assert np.allclose(mean[0], base, rtol=0, atol=1e-15)
    assert np.allclose(spread[0], math.sqrt(2) * np.abs(delta), rtol=1e-12)
    want = max(math.hypot(math.sqrt(2) * np.linalg.norm(d[k]) / np.linalg.norm(s[k]), math.sqrt(2) * e[k])
               for k in range(2))
    assert predicted_error(mean, spread, nc, 1.7)[0] == pytest.approx(1.7 * want, rel=1e-12)
    m0, s0 = ensemble_mean_spread(np.stack([base, base, base])[:, None, :])
    assert predicted_error(m0, s0, nc, 3.0)[0] < 1e-15


def test_training_box():
    lo, hi = np.array([0.0, -3.0, 17.0]), np.array([1.0, 0.0, 19.0])
    assert inside_box([0.5, -1.0, 18.0], lo, hi)
    assert inside_box([1.0 + 5e-7, -3.0, 19.0], lo, hi)          # within the 1e-6 widening
    assert not inside_box([1.0 + 2e-6, -3.0, 19.0], lo, hi)
    assert not inside_box([0.5, 0.1, 18.0], lo, hi)
