"""Pins of the CPU reference network (oracle/cnn.py) to things other than
itself: a library correlation routine, the exact (erf) GELU, finite
differences, Adam's closed-form first steps, and the invariants the guess
must keep (mass, translation equivariance, reduction to extrapolation)."""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.special as sps

from oracle import cnn as N


def rnd(shape, seed, scale=1.0):
    return np.random.default_rng(seed).standard_normal(shape) * scale


def test_conv_is_periodic_correlation():
    """Against scipy.ndimage.correlate with wrap-around boundaries, on a
    non-square grid (catches swapped axes, flipped taps, wrong wrap)."""
    x = rnd((5, 7, 3), 1)
    W = rnd((3, 3, 3, 4), 2)
    b = rnd((4,), 3)
    got = N.conv(x, W, b)
    for co in range(4):
        ref = b[co] + sum(ndi.correlate(x[..., ci], W[:, :, ci, co], mode="wrap")
                          for ci in range(3))
        assert np.max(np.abs(got[..., co] - ref)) < 1e-12


def test_conv_single_tap_is_a_shift():
    x = rnd((6, 8, 1), 4)
    W = np.zeros((3, 3, 1, 1))
    W[2, 0, 0, 0] = 1.0  # offset (+1 in y, -1 in x)
    got = N.conv(x, W, np.zeros(1))[..., 0]
    ref = np.array([[x[(j + 1) % 6, (i - 1) % 8, 0] for i in range(8)] for j in range(6)])
    assert np.array_equal(got, ref)


def test_gelu_against_erf_form():
    """The tanh form approximates x Phi(x) (Phi the normal CDF) to within
    about 5e-4 everywhere; it is exactly odd-symmetric around x Phi(x) = x/2
    at 0 and tends to x and 0 at the ends."""
    x = np.linspace(-8, 8, 20001)
    exact = 0.5 * x * (1.0 + sps.erf(x / math.sqrt(2.0)))
    assert np.max(np.abs(N.gelu(x) - exact)) < 5e-4
    assert N.gelu(np.array([0.0]))[0] == 0.0
    assert abs(N.gelu(np.array([30.0]))[0] - 30.0) < 1e-12
    assert abs(N.gelu(np.array([-30.0]))[0]) < 1e-12
    assert N.gelu_grad(np.array([0.0]))[0] == 0.5


def test_gelu_grad_finite_difference():
    x = np.linspace(-5, 5, 101)
    h = 1e-6
    fd = (N.gelu(x + h) - N.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(N.gelu_grad(x) - fd)) < 1e-8


def samples(n, m, count, seed, dt=0.05):
    """(phi^{n-1}, phi^n, psi^n, phi^{n+1}) with psi^n near the difference quotient."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        a = 0.1 + 0.1 * rng.standard_normal((n, m))
        b = a + 0.01 * rng.standard_normal((n, m))
        p = (b - a) / dt + 0.05 * rng.standard_normal((n, m))
        c = b + (b - a) + 0.002 * rng.standard_normal((n, m))
        out.append((a, b, p, c))
    return out


def test_gradient_finite_difference():
    """Backward pass against central differences of the loss on a sample of
    parameters from every weight and bias array (relative 1e-6)."""
    blob = N.init_blob(5, zero_last=False)
    blob = N.with_params(blob, blob[N.HEADER:] * 0.7)
    S = samples(6, 8, 2, 6)
    loss, g = N.loss_and_grad(blob, S)
    rng = np.random.default_rng(7)
    off = 0
    picks = []
    for name, shape in N.layout():
        cnt = int(np.prod(shape))
        picks += list(off + rng.choice(cnt, size=min(cnt, 12), replace=False))
        off += cnt
    theta = blob[N.HEADER:].astype(np.float64)
    for k in picks:
        h = 1e-3 * max(1e-2, abs(theta[k]))
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        # float32 blobs cannot hold the perturbation exactly: use the stored values
        bp, bm = N.with_params(blob, tp), N.with_params(blob, tm)
        hp = float(bp[N.HEADER + k]) - float(blob[N.HEADER + k])
        hm = float(blob[N.HEADER + k]) - float(bm[N.HEADER + k])
        fd = (N.loss_and_grad(bp, S)[0] - N.loss_and_grad(bm, S)[0]) / (hp + hm)
        assert abs(fd - g[k]) <= 2e-5 * max(abs(g[k]), 1e-3 * np.max(np.abs(g))), (k, fd, g[k])


def test_adam_closed_form():
    """With bias correction, Adam's first step moves every parameter by
    lr * g / (|g| + eps) and a constant gradient keeps that step size."""
    g = np.array([0.3, -2.0, 1e-3, -5e-2])
    th = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    lr = 1e-2
    for t in range(1, 6):
        th, m, v = N.adam(th, g, m, v, t, lr)
        np.testing.assert_allclose(th, -t * lr * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_guess_keeps_mass_and_reduces_to_extrapolation():
    a, b, p, _ = samples(8, 8, 1, 9)[0]
    blob = N.init_blob(10, zero_last=False)
    g = N.guess(blob, a, b, p)
    # the mean of the extrapolation (= mean phi^n for solver data, which conserve it)
    assert abs(np.mean(g) - np.mean(2 * b - a)) < 1e-15
    zero = N.init_blob(10, zero_last=True)
    assert np.array_equal(N.guess(zero, a, b, p), 2 * b - a)
    # no motion at all: the guess is phi^n whatever the weights
    assert np.allclose(N.guess(blob, b, b, p), b, atol=1e-15, rtol=0)


def test_psi_input_is_the_velocity_mismatch():
    """x2 vanishes when psi^n equals the difference quotient (always so for the
    first-order scheme, eq. discrete_1_b), so psi then has no influence."""
    a, b, p, _ = samples(8, 8, 1, 13)[0]
    x, _ = N.inputs(a, b, (b - a) / 0.05, 0.05, 2.0)
    assert np.max(np.abs(x[..., 2])) < 1e-12
    x, _ = N.inputs(a, b, p, 0.05, 2.0)
    assert np.max(np.abs(x[..., 2])) > 0.01


def test_guess_is_translation_equivariant():
    a, b, p, _ = samples(8, 16, 1, 11)[0]
    blob = N.init_blob(12, zero_last=False)
    g = N.guess(blob, a, b, p)
    r = lambda f: np.roll(f, (3, 5), (0, 1))  # noqa: E731
    gs = N.guess(blob, r(a), r(b), r(p))
    assert np.max(np.abs(r(g) - gs)) < 1e-13


def test_blob_layout():
    assert N.n_params() == 19681
    blob = N.init_blob(1, dt=0.05)
    p, s_in, s_out = N.unpack(blob)
    assert (s_in, s_out) == (2.0, 1.0)
    assert abs(N.dt_of(blob) - 0.05) < 1e-8
    assert np.array_equal(N.pack(p, s_in, s_out, N.dt_of(blob)), blob)
    with pytest.raises(ValueError):
        N.unpack(blob[:-1])
