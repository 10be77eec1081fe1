"""Pins of the selector's float64 reference (features, network gradient,
Adam) against closed forms and finite differences."""

import numpy as np
import pytest

from oracle import selector as S


def test_parameter_count():
    assert S.NPARAM == 5443


def test_features_of_a_diagonal_matrix_closed_form():
    d = np.array([1.0, 2.0, 4.0, 8.0])
    a = np.diag(d)
    f = S.features(a)
    fro = np.sqrt(np.sum(d ** 2))
    rms = fro / 2.0
    assert f[0] == pytest.approx(0.2)
    assert f[1] == 1.0
    assert f[2] == pytest.approx(-1.0)
    assert f[3] == pytest.approx(np.log10(8.0 / rms))
    assert f[4] == pytest.approx(np.log10(1.0 / rms))
    assert f[5] == 0.0
    g = 1.0 / rms  # min(d_i - 0) / rms
    assert f[6] == pytest.approx(g / (1 + g))
    assert f[7] == 0.0
    assert f[8] == pytest.approx(np.log10(8.0))
    assert f[9] == pytest.approx(np.log10(8.0))
    assert f[10] == pytest.approx(np.log10(8.0 / fro))
    assert f[11] == pytest.approx(np.log10(8.0 / fro))
    assert f[12] == pytest.approx(np.log10(1 + 4 * fro ** 2 / 15.0 ** 2))
    assert f[13] == pytest.approx(1.0)
    assert f[14] == pytest.approx(15.0 / (2 * fro))
    assert f[15] == pytest.approx(np.log10(8.0))


def test_features_detect_asymmetry_and_negative_diagonal():
    a = np.array([[-1.0, 2.0], [0.0, 3.0]])
    f = S.features(a)
    assert f[1] == 0.0
    fro = np.sqrt(14.0)
    assert f[2] == pytest.approx(np.log10(np.sqrt(8.0) / fro + 1e-16) / 16)
    assert f[5] == 0.5
    # rows: (-1 - 2) and (3 - 0): min = -3
    g = -3.0 / (fro / np.sqrt(2))
    assert f[6] == pytest.approx(g / (1 + abs(g)))
    assert f[7] == 0.5
    assert f[13] == pytest.approx((1.0 + 9.0) / 14.0)  # tr(A^2) = sum of eigenvalues^2


def test_features_scale_invariance_of_the_ratios():
    rng = np.random.Generator(np.random.PCG64(3))
    a = rng.standard_normal((20, 20)) + 5 * np.eye(20)
    f1, f2 = S.features(a), S.features(1e3 * a)
    assert np.allclose(f1, f2, atol=1e-12)


def test_mlp_gradient_matches_central_differences():
    rng = np.random.Generator(np.random.PCG64(11))
    p = 0.3 * rng.standard_normal(S.NPARAM)
    x = rng.standard_normal((7, S.NFEAT))
    y = rng.standard_normal((7, S.NOUT))
    _, g = S.mlp_loss_grad(p, x, y)
    idx = rng.choice(S.NPARAM, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(S.NPARAM)
        e[i] = h
        lp, _ = S.mlp_loss_grad(p + e, x, y)
        lm, _ = S.mlp_loss_grad(p - e, x, y)
        fd = (lp - lm) / (2 * h)
        # central differences carry O(h^2) and rounding O(eps/h) errors
        assert g[i] == pytest.approx(fd, rel=1e-4, abs=1e-8)


def test_mlp_forward_tiny_hand_example():
    p = np.zeros(S.NPARAM)
    w1, b1, w2, b2, w3, b3 = S.unpack(p)  # views into a copy; rebuild explicitly
    o = 0
    p[0] = 2.0            # W1[0, 0]
    o = S.H * S.NFEAT
    p[o + 0] = -1.0       # b1[0]
    o += S.H
    p[o + 0] = 3.0        # W2[0, 0]
    o += S.H * S.H + S.H
    p[o + 0] = 0.5        # W3[0, 0]
    p[o + S.H + 1] = 4.0  # W3[1, 1] (h2[1] stays 0)
    o += S.NOUT * S.H
    p[o + 2] = 7.0        # b3[2]
    x = np.zeros((1, S.NFEAT))
    x[0, 0] = 1.5
    _, _, out = S.mlp_forward(p, x)
    # h1[0] = relu(2*1.5 - 1) = 2, h2[0] = relu(3*2) = 6, out = (0.5*6, 0, 7)
    assert np.allclose(out, [[3.0, 0.0, 7.0]])


def test_adam_first_step_moves_by_lr_times_sign():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -5.0, 1e-3])
    p1, m, v = S.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # first bias-corrected step is lr * g / (|g| + eps)
    assert np.allclose(p1, p - 0.01 * np.sign(g), atol=1e-7)
